// C-ABI entry points: plans (one tensor or a batch of tensors of different
// shapes), their device tables, work-item lists and workspace layout, and the
// per-call orchestration of the randomized t-SVT and of the ADMM iteration.
//
// A plan is a list of tensors cut into transformed face slices.  Every stage of
// the t-SVT is one launch over all slices of all tensors: the kernels find a
// slice's operands through the device slice table and take their work from an
// item list built here, so a batch of uneven tensors costs the same number of
// launches as one tensor.  The whole launch sequence can be replayed as one
// HIP graph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"

namespace ht {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int ensure_dynamic_lds(const void* kernel, size_t bytes) {
  static std::mutex mu;
  static std::set<std::pair<int, const void*>> done;
  int dev = 0;
  HT_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({dev, kernel})) return HT_OK;
  HT_CHECK_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done.insert({dev, kernel});
  return HT_OK;
}

// Writes the sketch call index into the workspace (first node of a replayed graph).
__global__ void k_set_call(int32_t* slot, int32_t v) {
  if (threadIdx.x == 0) *slot = v;
}

}  // namespace ht

using namespace ht;

// Named regions of the workspace (for introspection by the tests).
enum { WS_A = 0, WS_OMEGA, WS_Y, WS_Z, WS_K, WS_QK, WS_C, WS_LNEW, WS_XIN, WS_STATE, WS_GP1, WS_GP2, WS_WK, WS_CALL,
       WS_WK2, WS_WKF, WS_SIG, WS_KEPT, WS_ANORM, WS_FEAT, WS_LSTATE, WS_STATUS, WS_RED, WS_GSQ, WS_OMH, WS_YH,
       WS_ZH, WS_COUNT };

// Block partials of the RSE reduction of the solver (two doubles per block).
constexpr int kRseBlocks = 1024;

// Optional per-stage timing with HIP events recorded on the launch stream.
enum { ST_TRANSFORM_FWD = 0, ST_OMEGA, ST_SKETCH_NN, ST_CHOLQR, ST_SKETCH_TN, ST_SMALLSVD, ST_RECON_QK, ST_RECON_NT,
       ST_TRANSFORM_INV, ST_ADMM_UPDATE, ST_COUNT };

struct Profiler {
  bool on = false;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
};

struct TensorHost {
  int order;
  int64_t dims[HT_MAX_ORDER];
  int64_t n1, n2, P, N;
  int r, p, l, k;
  int64_t x;       // offset in the packed buffers
  int64_t a;       // offset of its slices in A / C
  int64_t slice0;  // first slice in the slice table
  int cplx;        // unitary DFT on every transformed mode
  int64_t nslots;  // slices kept in A (canonical members of conjugate pairs when cplx)
  int64_t cmap;    // offset of its slot map (cplx)
  ModeTable fwd, inv;
};

struct ItemList {
  int64_t off;  // into the device item array
  int n;
};

// Key of a recorded graph: everything the launch sequence captures by value.
struct GraphKey {
  const void* X;
  void* out;
  void* ws;
  const double* tau_dev;
  double tau;
  int kind;
  double p0, p1;
  double* sigma;
  int* kept;
  hipStream_t stream;
  bool operator==(const GraphKey& o) const {
    return X == o.X && out == o.out && ws == o.ws && tau_dev == o.tau_dev && tau == o.tau && kind == o.kind &&
           p0 == o.p0 && p1 == o.p1 && sigma == o.sigma && kept == o.kept && stream == o.stream;
  }
};

struct GraphCache {
  bool valid = false;
  GraphKey key{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t call_node = nullptr;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    call_node = nullptr;
    valid = false;
  }
};

constexpr int kNumClasses = 5;
constexpr int kClassBound[kNumClasses] = {16, 32, 48, 64, HT_MAX_WIDTH};

struct ht_plan {
  bool batch;
  int precision, q;
  uint64_t seed;
  uint32_t stream_id;
  int device;
  std::vector<TensorHost> tens;
  int64_t Ntot, Ptot;
  int lmax, kmax;
  int64_t max_n2l;
  int prod_rows;     // output rows per product workgroup (64 or 128)
  size_t tf_budget;  // LDS bytes of one transform tile
  size_t tf_lds;
  int tf_nf;      // first-mode length of the fused DFT transform, shared by every tensor (0: general form)
  size_t tf_map;  // LDS bytes of the slot map the fused DFT transform keeps next to its tile
  std::vector<SliceDesc> h_slices;
  int64_t Atot;   // elements of the A / C regions
  bool cplx;      // every tensor under the unitary DFT (complex slices)
  int mode_nmax;  // longest transformed mode of the plan
  int32_t* d_cmap;
  TensorDesc* d_tens;
  SliceDesc* d_slices;
  int2* d_items;
  double* table64;
  float* table32;
  ItemList it_nn[2], it_tn[2], it_oy, it_oz, it_qk, it_nt, it_tf;  // [0]: 64-row tiles, [1]: 128-row tiles
  ItemList it_nns;  // nn items of the streaming product (256-row tiles)
  ItemList it_cp[2];  // BF16 products of complex slices: nn, tn items of kCplxProdRows complex rows
  ItemList it_cqk, it_cnt;  // complex reconstruction (strips x column-tile groups)
  ItemList it_asy, it_asz;  // complex CholeskyQR apply: 64-row tiles of Y (n1 rows), Z (n2 rows) in slice order
  ItemList it_t16;  // transform items when every tensor has two transformed modes of length 16 (else empty)
  // Width classes (bounds kClassBound) of plans whose slices differ in width:
  // orthonormalization items and small-SVD slices per class, so that each
  // launch is compiled for its own largest width (fixed widths only).
  bool class_split;
  int class_lmax[kNumClasses];
  ItemList it_oyc[kNumClasses], it_ozc[kNumClasses], it_svc[kNumClasses];
  bool nn_stream;   // FP32 real slices the streaming nn product can take
  int max_n2;
  int tf_capacity;
  size_t off[WS_COUNT];
  size_t size[WS_COUNT];
  size_t tsvt_bytes, admm_bytes;
  Profiler* prof;
  bool graph_on;
  GraphCache* graph;
  int learn_mode;            // 0 off, 1 track (fixed widths, features recorded), 2 predicted widths
  const float* learn_theta;  // network parameters (device, caller-owned)
  int force_fallback;        // redo every predicted slice at the fixed width
  const void* truth;         // ground truth of the solver's RSE (device, caller-owned) or null
};

namespace {

size_t elem_bytes(int precision) { return precision == HT_FP64 ? 8 : 4; }
int64_t align4(int64_t x) { return (x + 3) & ~int64_t(3); }

int check_penalty(const ht_penalty* pen) {
  if (!pen) HT_FAIL(HT_ERR_INVALID_ARG, "penalty is NULL");
  const double a = pen->p0, b = pen->p1;
  switch (pen->kind) {
    case HT_PEN_L1:
      return HT_OK;
    case HT_PEN_MCP:
      if (!(a > 0.0) || !std::isfinite(a)) HT_FAIL(HT_ERR_INVALID_ARG, "MCP needs gamma = p0 > 0");
      return HT_OK;
    case HT_PEN_SCAD:
      if (!(a > 2.0) || !(b > 0.0) || !std::isfinite(a) || !std::isfinite(b))
        HT_FAIL(HT_ERR_INVALID_ARG, "SCAD needs a = p0 > 2 and b = p1 > 0");
      return HT_OK;
    case HT_PEN_LOG:
      if (!(a > 0.0) || !std::isfinite(a)) HT_FAIL(HT_ERR_INVALID_ARG, "LOG needs eps = p0 > 0");
      return HT_OK;
    case HT_PEN_CAPPED_L1:
      if (!(a > 0.0) || !std::isfinite(a)) HT_FAIL(HT_ERR_INVALID_ARG, "CAPPED_L1 needs theta = p0 > 0");
      return HT_OK;
    case HT_PEN_FIRM:
      if (!(a > 1.0) || !std::isfinite(a)) HT_FAIL(HT_ERR_INVALID_ARG, "FIRM needs the threshold ratio a = p0 > 1");
      return HT_OK;
    default:
      HT_FAIL(HT_ERR_INVALID_ARG, "unknown penalty kind");
  }
}

Penalty to_dev(const ht_penalty* p) { return Penalty{p->kind, p->p0, p->p1}; }

void dct2_ortho(int n, std::vector<double>& U) {
  U.assign((size_t)n * n, 0.0);
  for (int kk = 0; kk < n; ++kk)
    for (int m = 0; m < n; ++m) {
      double v = std::cos(M_PI * (2.0 * m + 1.0) * kk / (2.0 * n)) * std::sqrt(2.0 / n);
      if (kk == 0) v *= 1.0 / std::sqrt(2.0);
      U[(size_t)kk * n + m] = v;
    }
}

void free_plan(ht_plan* pl) {
  if (!pl) return;
  if (pl->graph) {
    pl->graph->reset();
    delete pl->graph;
  }
  if (pl->prof) {
    for (auto& r : pl->prof->recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    delete pl->prof;
  }
  if (pl->table64) (void)hipFree(pl->table64);
  if (pl->table32) (void)hipFree(pl->table32);
  if (pl->d_tens) (void)hipFree(pl->d_tens);
  if (pl->d_slices) (void)hipFree(pl->d_slices);
  if (pl->d_items) (void)hipFree(pl->d_items);
  if (pl->d_cmap) (void)hipFree(pl->d_cmap);
  delete pl;
}

// Validate one tensor description and append its transform matrices (forward
// U_k, then inverse U_k^T / alpha_k, row-major) to tab.
int add_tensor(const ht_plan_desc* d, std::vector<double>& tab, TensorHost& t) {
  if (d->order < 2 || d->order > HT_MAX_ORDER) HT_FAIL(HT_ERR_INVALID_ARG, "order must be in [2, 8]");
  if (d->r < 1 || d->p < 0 || d->q < 0) HT_FAIL(HT_ERR_INVALID_ARG, "need r >= 1, p >= 0, q >= 0");
  t.order = d->order;
  int64_t P = 1;
  for (int i = 0; i < d->order; ++i) {
    if (d->dims[i] < 1) HT_FAIL(HT_ERR_INVALID_ARG, "dims must be >= 1");
    t.dims[i] = d->dims[i];
    if (i >= 2) P *= d->dims[i];
  }
  t.n1 = d->dims[0];
  t.n2 = d->dims[1];
  t.P = P;
  if (t.n1 * t.n2 > (int64_t)INT32_MAX || P > (int64_t)INT32_MAX / 4)
    HT_FAIL(HT_ERR_UNSUPPORTED, "face slice above 2^31 elements or too many slices");
  t.N = t.n1 * t.n2 * P;
  t.r = d->r;
  t.p = d->p;
  t.l = (int)std::min<int64_t>(std::min<int64_t>((int64_t)d->r + d->p, t.n1), t.n2);
  t.k = std::min(d->r, t.l);
  if (t.l > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width min(r+p, n1, n2) above HT_MAX_WIDTH");
  int ndft = 0;
  for (int m = 0; m < d->order - 2; ++m)
    ndft += d->transform[m + 2] == HT_DFT_UNITARY || d->transform[m + 2] == HT_DFT_UNNORMALIZED;
  if (ndft > 0 && ndft != d->order - 2)
    HT_FAIL(HT_ERR_UNSUPPORTED, "a DFT must be the transform of every mode 3..d (no mixing with real kinds)");
  t.cplx = ndft > 0;
  if (t.cplx && t.l > kMaxComplexWidth)
    HT_FAIL(HT_ERR_UNSUPPORTED, "complex slices need a sketch width l = min(r + p, n1, n2) <= 64");
  if (t.cplx && (2 * t.n1 * t.n2 > (int64_t)INT32_MAX))
    HT_FAIL(HT_ERR_UNSUPPORTED, "complex face slice above 2^31 elements");
  t.fwd.nmodes = t.inv.nmodes = d->order - 2;
  int stride = 1;
  for (int m = 0; m < d->order - 2; ++m) {
    const int n = (int)d->dims[m + 2];
    const int kind = d->transform[m + 2];
    if (n > HT_MAX_MODE) HT_FAIL(HT_ERR_UNSUPPORTED, "transformed mode longer than HT_MAX_MODE");
    std::vector<double> U;
    double alpha = 1.0;
    if (kind == HT_DCT2_ORTHO) {
      dct2_ortho(n, U);
    } else if (kind == HT_CUSTOM_REAL) {
      if (!d->custom[m + 2]) HT_FAIL(HT_ERR_INVALID_ARG, "CUSTOM_REAL transform needs a matrix");
      U.assign(d->custom[m + 2], d->custom[m + 2] + (size_t)n * n);
      double tr = 0.0;
      for (size_t i = 0; i < U.size(); ++i) tr += U[i] * U[i];
      alpha = tr / n;
      double err = 0.0;
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          double sdot = 0.0;
          for (int c = 0; c < n; ++c) sdot += U[(size_t)a * n + c] * U[(size_t)b * n + c];
          err = std::max(err, std::fabs(sdot - (a == b ? alpha : 0.0)));
        }
      if (!(alpha > 0.0) || err > 1e-10 * alpha)
        HT_FAIL(HT_ERR_INVALID_ARG, "CUSTOM_REAL matrix must satisfy U U^T = alpha I");
    } else if (kind == HT_DFT_UNITARY || kind == HT_DFT_UNNORMALIZED) {
      // interleaved (re, im): forward F[k][m] = exp(-2 pi i k m / n) s_f, inverse
      // F^H s_i with (s_f, s_i) = (1/sqrt n, 1/sqrt n) unitary, (1, 1/n) unnormalized
      const bool unit = kind == HT_DFT_UNITARY;
      const double sc = unit ? 1.0 / std::sqrt((double)n) : 1.0;
      const double sci = unit ? sc : 1.0 / n;
      t.fwd.n[m] = t.inv.n[m] = n;
      t.fwd.stride[m] = t.inv.stride[m] = stride;
      stride *= n;
      t.fwd.off[m] = (int)tab.size();
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          const double ang = -2.0 * M_PI * (double)((int64_t)a * b % n) / n;
          tab.push_back(std::cos(ang) * sc);
          tab.push_back(std::sin(ang) * sc);
        }
      t.inv.off[m] = (int)tab.size();
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {  // conj(F[b][a])
          const double ang = -2.0 * M_PI * (double)((int64_t)b * a % n) / n;
          tab.push_back(std::cos(ang) * sci);
          tab.push_back(-std::sin(ang) * sci);
        }
      continue;
    } else {
      HT_FAIL(HT_ERR_INVALID_ARG, "unknown transform kind");
    }
    t.fwd.n[m] = t.inv.n[m] = n;
    t.fwd.stride[m] = t.inv.stride[m] = stride;
    stride *= n;
    t.fwd.off[m] = (int)tab.size();
    tab.insert(tab.end(), U.begin(), U.end());
    t.inv.off[m] = (int)tab.size();
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) tab.push_back(U[(size_t)b * n + a] / alpha);
  }
  // the inverse applies mode d first, then d-1, ..., 3 (the mode products
  // commute, so the order does not change the result)
  ModeTable rev = t.inv;
  const int nm = t.inv.nmodes;
  for (int m = 0; m < nm; ++m) {
    rev.n[m] = t.inv.n[nm - 1 - m];
    rev.stride[m] = t.inv.stride[nm - 1 - m];
    rev.off[m] = t.inv.off[nm - 1 - m];
  }
  t.inv = rev;
  return HT_OK;
}

// Order per-slice item groups so that all items of a group run on one XCD.
// The dispatcher hands workgroups to the 8 XCDs round-robin in launch order,
// so the items of XCD x go to positions x, x + 8, x + 16, ...; groups are
// assigned largest first to the least-loaded XCD.  Tiles of one slice share
// its thin operands, which then stay in that XCD's L2.
std::vector<int2> xcd_grouped(const std::vector<std::vector<int2>>& groups, const std::vector<double>& cost) {
  constexpr int NX = 8;
  std::vector<int> order(groups.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return cost[a] * groups[a].size() > cost[b] * groups[b].size();
  });
  std::vector<std::vector<int2>> q(NX);
  std::vector<double> load(NX, 0.0);
  for (int g : order) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    q[x].insert(q[x].end(), groups[g].begin(), groups[g].end());
    load[x] += cost[g] * groups[g].size();
  }
  std::vector<int2> out;
  size_t longest = 0;
  for (auto& v : q) longest = std::max(longest, v.size());
  for (size_t i = 0; i < longest; ++i)
    for (int x = 0; x < NX; ++x)
      if (i < q[x].size()) out.push_back(q[x][i]);
  return out;
}

// Tiles of `rows` rows over dimension n of every slice (n = n1 or n2).
std::vector<int2> row_items(const ht_plan* pl, bool over_n2, int rows, bool cost_is_other_dim) {
  std::vector<std::vector<int2>> groups(pl->Ptot);
  std::vector<double> cost(pl->Ptot);
  for (int64_t s = 0; s < pl->Ptot; ++s) {
    const SliceDesc& d = pl->h_slices[s];
    const int n = over_n2 ? d.n2 : d.n1;
    for (int r0 = 0; r0 < n; r0 += rows) groups[s].push_back(make_int2((int)s, r0));
    cost[s] = cost_is_other_dim ? (double)(over_n2 ? d.n1 : d.n2) : 1.0;
  }
  return xcd_grouped(groups, cost);
}

// 64-row tiles over dimension n1 (or n2) of every slice, in slice order.
std::vector<int2> slice_order_tiles(const ht_plan* pl, bool over_n2) {
  std::vector<int2> items;
  for (int64_t s = 0; s < pl->Ptot; ++s) {
    const SliceDesc& d = pl->h_slices[s];
    const int n = over_n2 ? d.n2 : d.n1;
    for (int r0 = 0; r0 < n; r0 += 64) items.push_back(make_int2((int)s, r0));
  }
  return items;
}

// Complex reconstruction items: strips of kCmulRows complex rows times groups
// of kCmulGroup column tiles (QK = Q1 K': one group, its l <= 64 columns).
std::vector<int2> cmul_items(const ht_plan* pl, bool full) {
  std::vector<std::vector<int2>> groups(pl->Ptot);
  std::vector<double> cost(pl->Ptot, 1.0);
  for (int64_t s = 0; s < pl->Ptot; ++s) {
    const SliceDesc& d = pl->h_slices[s];
    const int ncg = full ? (int)ceil_div(ceil_div(d.n2, 64), kCmulGroup) : 1;
    const int nstrips = (int)ceil_div(d.n1, kCmulRows);
    for (int t = 0; t < nstrips * ncg; ++t) groups[s].push_back(make_int2((int)s, t));
  }
  return xcd_grouped(groups, cost);
}

std::vector<int2> nt_items(const ht_plan* pl) {
  std::vector<std::vector<int2>> groups(pl->Ptot);
  std::vector<double> cost(pl->Ptot, 1.0);
  for (int64_t s = 0; s < pl->Ptot; ++s) {
    const SliceDesc& d = pl->h_slices[s];
    const int nt = (int)(ceil_div(d.n1, 64) * ceil_div(d.n2, 64));
    for (int t = 0; t < nt; ++t) groups[s].push_back(make_int2((int)s, t));
  }
  return xcd_grouped(groups, cost);
}

// Items of the two-modes-of-16 transform, or none when some tensor does not
// qualify (FP64, complex slices, other mode lengths, ragged or huge slices).
std::vector<int2> t16_items(const ht_plan* pl) {
  std::vector<int2> items;
  if (pl->precision == HT_FP64 || pl->cplx) return items;
  for (const TensorHost& th : pl->tens) {
    const int64_t NT = th.n1 * th.n2;
    for (const ModeTable* mt : {&th.fwd, &th.inv})
      if (mt->nmodes != 2 || mt->n[0] != 16 || mt->n[1] != 16 || mt->stride[0] * mt->stride[1] != 16)
        return items;  // strides {1, 16}, or {16, 1} for the inverse (mode 4 first)
    if (th.cplx || th.P != 256 || NT % 16 != 0 || NT >= (int64_t(1) << 24) || th.x % 2 || th.a % 2) return items;
  }
  for (size_t t = 0; t < pl->tens.size(); ++t) {
    const int64_t NT = pl->tens[t].n1 * pl->tens[t].n2;
    for (int64_t t0 = 0; t0 < NT; t0 += kT16Tube) items.push_back(make_int2((int)t, (int)t0));
  }
  return items;
}

// The two-modes-of-16 transform applies to this plan and to these buffers
// (8-byte pairs in, 8- or 4-byte pairs out).
bool use_t16(const ht_plan* pl, const void* in, const void* out, size_t out_elem) {
  return pl->it_t16.n > 0 && reinterpret_cast<uintptr_t>(in) % 8 == 0 &&
         reinterpret_cast<uintptr_t>(out) % (2 * out_elem) == 0;
}

// Transform tiles of every tensor for an LDS budget; fills TP and the LDS size.
int tf_items(ht_plan* pl, size_t budget, std::vector<int2>& items, std::vector<int>& tps, size_t& lds) {
  const size_t es = elem_bytes(pl->precision);
  items.clear();
  tps.clear();
  lds = 0;
  for (size_t t = 0; t < pl->tens.size(); ++t) {
    const TensorHost& th = pl->tens[t];
    const size_t tes = th.cplx ? 2 * es : es;  // complex tiles hold two planes
    const int TP = transform_tile_width(th.P, tes, budget);
    if (TP == 0) HT_FAIL(HT_ERR_UNSUPPORTED, "too many face slices for the transform tile");
    tps.push_back(TP);
    lds = std::max(lds, (size_t)TP * th.P * tes);
    const int64_t NT = th.n1 * th.n2;
    for (int64_t t0 = 0; t0 < NT; t0 += TP) items.push_back(make_int2((int)t, (int)t0));
  }
  return HT_OK;
}

// Modes of the fused DFT transform of a mode table: the shortest mode goes
// first (length <= 8), the longest last, and every mode must have a
// power-of-two length <= 32; otherwise -1 (general form).
void pick_fused_modes(ModeTable& mt) {
  mt.first = mt.last = -1;
  if (mt.nmodes < 2) return;
  auto pow2 = [](int n) { return n >= 2 && (n & (n - 1)) == 0; };
  int f = 0, l = 0;
  for (int m = 0; m < mt.nmodes; ++m) {
    if (!pow2(mt.n[m])) return;
    if (mt.n[m] < mt.n[f]) f = m;
  }
  l = f == 0 ? 1 : 0;
  for (int m = 0; m < mt.nmodes; ++m)
    if (m != f && mt.n[m] > mt.n[l]) l = m;
  if (mt.n[f] > 8 || mt.n[l] > 32) return;
  mt.first = f;
  mt.last = l;
}

int upload_tensors(ht_plan* pl, const std::vector<int>& tps) {
  std::vector<TensorDesc> td(pl->tens.size());
  const int64_t V = 16 / (int64_t)elem_bytes(pl->precision);  // elements per 16-byte access
  pl->tf_nf = 0;
  pl->tf_map = 0;
  bool fused = pl->cplx;
  for (size_t t = 0; t < pl->tens.size(); ++t) {
    const TensorHost& th = pl->tens[t];
    TensorDesc& d = td[t];
    std::memset(&d, 0, sizeof(d));
    d.x = th.x;
    d.a = th.a;
    d.NT = th.n1 * th.n2;
    d.cmap = th.cmap;
    d.cplx = th.cplx;
    d.n1 = (int32_t)th.n1;
    d.nslots = (int32_t)th.nslots;
    d.P = (int32_t)th.P;
    d.TP = tps[t];
    int lg = 0;
    while ((1 << lg) < d.TP) ++lg;
    d.lgTP = lg;
    d.slice0 = (int32_t)th.slice0;
    d.fwd = th.fwd;
    d.inv = th.inv;
    pick_fused_modes(d.fwd);
    pick_fused_modes(d.inv);
    // 16-byte tile loads need V consecutive tube positions in one column of every slice and slot
    const bool vec = d.TP % V == 0 && d.NT % V == 0 && d.n1 % V == 0 && d.x % V == 0 && d.a % V == 0;
    if (d.fwd.first < 0 || d.inv.first < 0 || !vec) {
      fused = false;
    } else {
      const int nf = d.fwd.n[d.fwd.first];
      if (d.inv.n[d.inv.first] != nf || (pl->tf_nf != 0 && pl->tf_nf != nf)) fused = false;
      pl->tf_nf = nf;
      pl->tf_map = std::max(pl->tf_map, (size_t)align4(d.P) * sizeof(int32_t));
    }
  }
  if (!fused) pl->tf_nf = 0;
  if (!fused) pl->tf_map = 0;
  HT_CHECK_HIP(hipMemcpy(pl->d_tens, td.data(), td.size() * sizeof(TensorDesc), hipMemcpyHostToDevice));
  return HT_OK;
}

// (Re)build the transform tiling for an LDS budget and upload it.
int set_transform_budget(ht_plan* pl, size_t budget) {
  std::vector<int2> items;
  std::vector<int> tps;
  size_t lds = 0;
  int rc = tf_items(pl, budget, items, tps, lds);
  if (rc) return rc;
  if ((int)items.size() > pl->tf_capacity) HT_FAIL(HT_ERR_UNSUPPORTED, "transform budget below the planned minimum");
  if ((rc = upload_tensors(pl, tps))) return rc;
  HT_CHECK_HIP(hipMemcpy(pl->d_items + pl->it_tf.off, items.data(), items.size() * sizeof(int2),
                         hipMemcpyHostToDevice));
  pl->it_tf.n = (int)items.size();
  pl->tf_budget = budget;
  pl->tf_lds = lds;
  if (pl->graph) pl->graph->reset();
  return HT_OK;
}

constexpr size_t kTfBudgets[] = {32 * 1024, 64 * 1024, 128 * 1024};

void layout(ht_plan* pl, int64_t nY, int64_t nZ, int64_t nK, int64_t nG1, int64_t nG2) {
  const size_t es = elem_bytes(pl->precision);
  pl->size[WS_A] = (size_t)pl->Atot * (pl->precision == HT_BF16_MIXED ? 2 : es);
  pl->size[WS_OMEGA] = (size_t)nZ * es;
  pl->size[WS_Y] = (size_t)nY * es;
  pl->size[WS_Z] = (size_t)nZ * es;
  pl->size[WS_K] = (size_t)nK * es;
  pl->size[WS_QK] = (size_t)nY * es;
  pl->size[WS_C] = (size_t)pl->Atot * es;
  pl->size[WS_GP1] = (size_t)nG1 * sizeof(double);
  pl->size[WS_GP2] = (size_t)nG2 * sizeof(double);
  pl->size[WS_WK] = (size_t)pl->Ptot * sizeof(int2);
  pl->size[WS_CALL] = 256;
  pl->size[WS_WK2] = (size_t)pl->Ptot * sizeof(int2);
  pl->size[WS_WKF] = (size_t)pl->Ptot * sizeof(int2);
  pl->size[WS_SIG] = (size_t)pl->Ptot * pl->lmax * sizeof(double);
  pl->size[WS_KEPT] = (size_t)pl->Ptot * sizeof(int);
  pl->size[WS_ANORM] = (size_t)pl->Ptot * 2 * sizeof(double);
  pl->size[WS_FEAT] = (size_t)pl->Ptot * 32 * sizeof(float);
  pl->size[WS_LSTATE] = 256;
  pl->size[WS_STATUS] = (size_t)pl->Ptot * sizeof(int);
  pl->size[WS_RED] = (size_t)kRseBlocks * 2 * sizeof(double);
  {  // squared group norms of the tube-wise / slice-wise sparse update (single-tensor solvers)
    int64_t g = 1;
    for (const TensorHost& th : pl->tens) g = std::max<int64_t>(g, std::max<int64_t>(th.n1 * th.n2, th.P));
    pl->size[WS_GSQ] = (size_t)g * sizeof(double);
  }
  {  // BF16 copies of the thin operands of the complex BF16 products (Omega, Q, Z)
    const bool h = pl->cplx && pl->precision == HT_BF16_MIXED;
    pl->size[WS_OMH] = h ? (size_t)nZ * 2 : 0;
    pl->size[WS_YH] = h ? (size_t)nY * 2 : 0;
    pl->size[WS_ZH] = h ? (size_t)nZ * 2 : 0;
  }
  pl->size[WS_LNEW] = (size_t)pl->Ntot * es;
  pl->size[WS_XIN] = (size_t)pl->Ntot * es;
  pl->size[WS_STATE] = sizeof(AdmmState);
  // t-SVT regions first, then the solver-only regions
  const int order_[] = {WS_A,     WS_OMEGA, WS_Y,    WS_Z,    WS_K,     WS_QK,   WS_C,      WS_GP1,  WS_GP2,
                        WS_WK,    WS_CALL,  WS_WK2,  WS_WKF,  WS_SIG,   WS_KEPT, WS_ANORM,  WS_FEAT, WS_LSTATE,
                        WS_OMH,   WS_YH,    WS_ZH,   WS_STATUS, WS_LNEW, WS_XIN, WS_STATE, WS_RED, WS_GSQ};
  size_t o = 0;
  for (int r : order_) {
    pl->off[r] = o;
    o += align256(pl->size[r]);
    if (r == WS_STATUS) pl->tsvt_bytes = o;
  }
  pl->admm_bytes = o;
}

// Build a plan from tensor descriptions (one for ht_plan_create).
int build_plan(const ht_plan_desc* descs, int n, bool batch, ht_plan** out) {
  *out = nullptr;
  if (n < 1) HT_FAIL(HT_ERR_INVALID_ARG, "need at least one tensor");
  const ht_plan_desc& d0 = descs[0];
  if (d0.precision != HT_FP64 && d0.precision != HT_FP32 && d0.precision != HT_BF16_MIXED)
    HT_FAIL(HT_ERR_INVALID_ARG, "unknown precision");
  for (int t = 1; t < n; ++t)
    if (descs[t].precision != d0.precision || descs[t].q != d0.q || descs[t].seed != d0.seed ||
        descs[t].stream_id != d0.stream_id)
      HT_FAIL(HT_ERR_INVALID_ARG, "precision, q, seed and stream_id must agree across a batch");
  ht_plan* pl = new ht_plan();
  pl->batch = batch;
  pl->precision = d0.precision;
  pl->q = d0.q;
  pl->seed = d0.seed;
  pl->stream_id = d0.stream_id;
  if (hipGetDevice(&pl->device) != hipSuccess) pl->device = 0;
  std::vector<double> tab;
  std::vector<int32_t> cmap;
  pl->tens.resize(n);
  int64_t x = 0, P = 0, Atot = 0;
  int ncplx = 0;
  pl->lmax = 0;
  pl->kmax = 0;
  pl->max_n2l = 0;
  for (int t = 0; t < n; ++t) {
    int rc = add_tensor(&descs[t], tab, pl->tens[t]);
    if (rc) {
      free_plan(pl);
      return rc;
    }
    TensorHost& th = pl->tens[t];
    th.x = x;
    th.slice0 = P;
    x += batch ? (th.N + 63) / 64 * 64 : th.N;  // 256-byte aligned tensors in a packed batch
    const int f = th.cplx ? 2 : 1;                // complex slices: real embedding of twice the size
    th.nslots = th.P;
    if (th.cplx) {
      // slot map: the canonical member of every conjugate pair (partner index =
      // every transform-domain index negated modulo n_k) gets a slot
      th.cmap = (int64_t)cmap.size();
      cmap.resize(cmap.size() + 3 * th.P);  // slot per slice, then (slice, partner) per slot
      int32_t* cm = cmap.data() + th.cmap;
      int64_t slots = 0;
      for (int64_t j = 0; j < th.P; ++j) {
        int64_t rem = j, pj = 0, stride = 1;
        for (int m = 2; m < th.order; ++m) {
          const int64_t nm = th.dims[m], i = rem % nm;
          rem /= nm;
          pj += ((nm - i) % nm) * stride;
          stride *= nm;
        }
        if (pj >= j) {
          cm[th.P + 2 * slots] = (int32_t)j;
          cm[th.P + 2 * slots + 1] = pj == j ? -1 : (int32_t)pj;
          cm[j] = (int32_t)slots++;
        } else {
          cm[j] = (int32_t)(cm[pj] | (int32_t)0x80000000u);
        }
      }
      th.nslots = slots;
      cmap.resize(th.cmap + th.P + 2 * slots);
    }
    th.a = Atot;
    Atot += th.nslots * f * th.n1 * th.n2;
    Atot = (Atot + 63) / 64 * 64;
    P += th.nslots;
    pl->lmax = std::max(pl->lmax, th.l);
    pl->kmax = std::max(pl->kmax, th.k);
    pl->max_n2l = std::max<int64_t>(pl->max_n2l, (int64_t)th.n2 * th.l);  // the real Omega
    ncplx += th.cplx;
  }
  if (ncplx != 0 && ncplx != n) {
    free_plan(pl);
    HT_FAIL(HT_ERR_UNSUPPORTED, "a batch mixes DFT and real transforms");
  }
  pl->cplx = ncplx > 0;
  pl->mode_nmax = 1;
  for (const TensorHost& th : pl->tens)
    for (int m = 0; m < th.fwd.nmodes; ++m) pl->mode_nmax = std::max(pl->mode_nmax, th.fwd.n[m]);
  if (P > (int64_t)INT32_MAX / 64) {
    free_plan(pl);
    HT_FAIL(HT_ERR_UNSUPPORTED, "too many face slices in one plan");
  }
  pl->Ntot = x;
  pl->Ptot = P;
  pl->Atot = Atot;

  // slice table (complex slices: stacked real and imaginary parts, f = 2)
  pl->h_slices.resize(P);
  int64_t oY = 0, oZ = 0, oK = 0, oG1 = 0, oG2 = 0;
  for (int t = 0; t < n; ++t) {
    const TensorHost& th = pl->tens[t];
    const int f = th.cplx ? 2 : 1;
    const int64_t NT = th.n1 * th.n2, l = th.l, n1 = th.n1, n2 = th.n2;
    for (int64_t j = 0, s = 0; j < th.P; ++j) {
      if (th.cplx && cmap[th.cmap + j] < 0) continue;  // a conjugate partner: no slot
      SliceDesc& d = pl->h_slices[th.slice0 + s];
      d.a = th.a + s * f * NT;
      d.y = oY;
      d.z = oZ;
      d.kq = oK;
      d.g1 = oG1;
      d.g2 = oG2;
      d.n1 = (int32_t)n1;
      d.n2 = (int32_t)n2;
      d.l = (int32_t)l;
      d.k = th.k;
      d.tensor = t;
      d.local = (int32_t)j;  // the Philox slice word: the canonical member's index
      d.p = th.p;
      d.cplx = th.cplx;
      d.nc = (int32_t)th.n2;
      d.pad = 0;
      oY += align4(f * n1 * l);
      oZ += align4(f * n2 * l);
      oK += align4(f * l * l);
      oG1 += ceil_div(std::max(n1, n2), 64) * f * l * l;
      oG2 += ceil_div(n1, 64) * f * l * l;
      ++s;
    }
  }
  layout(pl, oY, oZ, oK, oG1, oG2);
  // the streaming nn product: FP32, real slices with 16-byte aligned columns
  pl->max_n2 = 0;
  pl->nn_stream = pl->precision == HT_FP32 && pl->lmax <= 64;
  for (const SliceDesc& d : pl->h_slices) {
    pl->max_n2 = std::max(pl->max_n2, (int)d.n2);
    // a 256-row tile of a short slice would leave most of its wavefronts idle
    if (d.cplx || d.n1 % 4 != 0 || d.n1 < 3 * kStreamRows / 4 || d.a % 4 != 0 || d.y % 4 != 0) pl->nn_stream = false;
  }
  if (pl->max_n2 > kStreamMaxK) pl->nn_stream = false;

  // item lists (the transform list is sized for the smallest LDS budget)
  std::vector<std::vector<int2>> lists;
  lists.push_back(row_items(pl, false, 64, true));   // nn, 64 rows
  lists.push_back(row_items(pl, true, 64, true));    // tn, 64 rows
  lists.push_back(row_items(pl, false, 128, true));  // nn, 128 rows
  lists.push_back(row_items(pl, true, 128, true));   // tn, 128 rows
  lists.push_back(row_items(pl, false, 64, false));  // orth Y
  lists.push_back(row_items(pl, true, 64, false));   // orth Z
  lists.push_back(row_items(pl, false, 64, false));  // recon QK
  lists.push_back(nt_items(pl));                     // recon C
  lists.push_back(row_items(pl, false, kStreamRows, true));  // nn, streaming product
  lists.push_back(row_items(pl, false, kCplxProdRows, true));  // nn, complex BF16 products
  lists.push_back(row_items(pl, true, kCplxProdRows, true));   // tn, complex BF16 products
  lists.push_back(cmul_items(pl, false));                      // complex recon QK
  lists.push_back(cmul_items(pl, true));                       // complex recon C
  lists.push_back(slice_order_tiles(pl, false));  // complex orth apply tiles, Y
  lists.push_back(slice_order_tiles(pl, true));   // complex orth apply tiles, Z
  // width classes: orthonormalization items (Y, Z) and small-SVD slices
  auto class_of = [&](int l) {
    int c = 0;
    while (c + 1 < kNumClasses && l > kClassBound[c]) ++c;
    return c;
  };
  std::vector<int2> oyc[kNumClasses], ozc[kNumClasses], svc[kNumClasses];
  {
    const std::vector<int2>& oy = lists[4];
    const std::vector<int2>& oz = lists[5];
    for (const int2& it : oy) oyc[class_of(pl->h_slices[it.x].l)].push_back(it);
    for (const int2& it : oz) ozc[class_of(pl->h_slices[it.x].l)].push_back(it);
    for (int64_t j = 0; j < P; ++j) svc[class_of(pl->h_slices[j].l)].push_back(make_int2((int)j, 0));
  }
  int nused = 0;
  for (int c = 0; c < kNumClasses; ++c) {
    nused += !svc[c].empty();
    pl->class_lmax[c] = 0;
    for (const int2& it : svc[c]) pl->class_lmax[c] = std::max(pl->class_lmax[c], (int)pl->h_slices[it.x].l);
  }
  pl->class_split = nused > 1 && !pl->cplx;
  for (int c = 0; c < kNumClasses; ++c) {
    lists.push_back(oyc[c]);
    lists.push_back(ozc[c]);
    lists.push_back(svc[c]);
  }
  lists.push_back(t16_items(pl));
  // the smallest LDS budget that fits every tensor sets the item capacity
  std::vector<int2> tfi;
  std::vector<int> tps;
  size_t lds = 0, bmin = 0;
  int rc = HT_ERR_UNSUPPORTED;
  for (size_t b : kTfBudgets) {
    if ((rc = tf_items(pl, b, tfi, tps, lds)) == HT_OK) {
      bmin = b;
      break;
    }
  }
  if (rc) {
    free_plan(pl);
    return rc;
  }
  pl->tf_capacity = (int)tfi.size();
  ItemList* dst[] = {&pl->it_nn[0], &pl->it_tn[0], &pl->it_nn[1], &pl->it_tn[1], &pl->it_oy, &pl->it_oz,
                     &pl->it_qk, &pl->it_nt, &pl->it_nns, &pl->it_cp[0], &pl->it_cp[1], &pl->it_cqk, &pl->it_cnt, &pl->it_asy, &pl->it_asz,
                     &pl->it_oyc[0], &pl->it_ozc[0], &pl->it_svc[0], &pl->it_oyc[1], &pl->it_ozc[1],
                     &pl->it_svc[1], &pl->it_oyc[2], &pl->it_ozc[2], &pl->it_svc[2], &pl->it_oyc[3],
                     &pl->it_ozc[3], &pl->it_svc[3], &pl->it_oyc[4], &pl->it_ozc[4], &pl->it_svc[4],
                     &pl->it_t16};
  static_assert(kNumClasses == 5, "item list table");
  std::vector<int2> all;
  for (size_t i = 0; i < lists.size(); ++i) {
    dst[i]->off = (int64_t)all.size();
    dst[i]->n = (int)lists[i].size();
    all.insert(all.end(), lists[i].begin(), lists[i].end());
  }
  pl->it_tf.off = (int64_t)all.size();
  pl->it_tf.n = 0;
  all.resize(all.size() + pl->tf_capacity);

  // device tables
  bool ok = hipMalloc(&pl->d_tens, n * sizeof(TensorDesc)) == hipSuccess &&
            hipMalloc(&pl->d_slices, P * sizeof(SliceDesc)) == hipSuccess &&
            hipMalloc(&pl->d_items, all.size() * sizeof(int2)) == hipSuccess;
  if (ok && !tab.empty()) {
    std::vector<float> tab32(tab.begin(), tab.end());
    ok = hipMalloc(&pl->table64, tab.size() * sizeof(double)) == hipSuccess &&
         hipMalloc(&pl->table32, tab32.size() * sizeof(float)) == hipSuccess &&
         hipMemcpy(pl->table64, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(pl->table32, tab32.data(), tab32.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) {
    free_plan(pl);
    HT_FAIL(HT_ERR_ALLOC, "could not allocate or upload the plan tables");
  }
  if (!cmap.empty() && (hipMalloc(&pl->d_cmap, cmap.size() * sizeof(int32_t)) != hipSuccess ||
                        hipMemcpy(pl->d_cmap, cmap.data(), cmap.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
                            hipSuccess)) {
    free_plan(pl);
    HT_FAIL(HT_ERR_ALLOC, "could not upload the slot map");
  }
  if (hipMemcpy(pl->d_slices, pl->h_slices.data(), P * sizeof(SliceDesc), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pl->d_items, all.data(), all.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess) {
    free_plan(pl);
    HT_FAIL(HT_ERR_HIP, "could not upload the plan tables");
  }
  pl->prod_rows = pl->precision == HT_FP64 ? 64 : 128;
  if ((rc = set_transform_budget(pl, std::max<size_t>(bmin, 64 * 1024)))) {
    free_plan(pl);
    return rc;
  }
  *out = pl;
  return HT_OK;
}

template <typename T>
T* ws_ptr(const ht_plan* pl, void* ws, int region) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + pl->off[region]);
}

template <typename T>
const T* table(const ht_plan* pl);
template <>
const double* table<double>(const ht_plan* pl) {
  return pl->table64;
}
template <>
const float* table<float>(const ht_plan* pl) {
  return pl->table32;
}

int check_ws(const void* ws, size_t bytes, size_t need) {
  if (!ws) HT_FAIL(HT_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) HT_FAIL(HT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < need)
    HT_FAIL(HT_ERR_WORKSPACE, "workspace too small: " + std::to_string(bytes) + " < " + std::to_string(need));
  return HT_OK;
}

// Run one launch; when profiling, bracket it with events on the same stream.
template <typename F>
int timed(const ht_plan* pl, int stage, hipStream_t s, F&& launch) {
  Profiler* pr = pl->prof;
  if (!pr || !pr->on) return launch();
  Profiler::Rec r{stage, nullptr, nullptr};
  HT_CHECK_HIP(hipEventCreate(&r.a));
  HT_CHECK_HIP(hipEventCreate(&r.b));
  HT_CHECK_HIP(hipEventRecord(r.a, s));
  const int rc = launch();
  HT_CHECK_HIP(hipEventRecord(r.b, s));
  pr->recs.push_back(r);
  return rc;
}

const int2* items(const ht_plan* pl, const ItemList& L) { return pl->d_items + L.off; }

// The randomized t-SVT over every slice of the plan.  tau: 1/(*mu_dev) when
// mu_dev is set (solver), else tau_dev[tensor] when tau_dev is set (batch),
// else the scalar.  The sketch call index is *call_dev when set, else call.
template <typename T>
int run_tsvt(const ht_plan* pl, const T* X, T* out, double tau, const double* tau_dev, const double* mu_dev,
             const Penalty& pen, uint32_t call, const int32_t* call_dev, void* ws, hipStream_t s, double* sigma_out,
             int* kept_out) {
  const int lmax = pl->lmax;
  const int P = (int)pl->Ptot;
  const SliceDesc* sd = pl->d_slices;
  T* A = ws_ptr<T>(pl, ws, WS_A);
  T* Om = ws_ptr<T>(pl, ws, WS_OMEGA);
  T* Y = ws_ptr<T>(pl, ws, WS_Y);
  T* Z = ws_ptr<T>(pl, ws, WS_Z);
  T* K = ws_ptr<T>(pl, ws, WS_K);
  T* QK = ws_ptr<T>(pl, ws, WS_QK);
  T* C = ws_ptr<T>(pl, ws, WS_C);
  double* gp1 = ws_ptr<double>(pl, ws, WS_GP1);
  double* gp2 = ws_ptr<double>(pl, ws, WS_GP2);
  const bool bf16 = pl->precision == HT_BF16_MIXED;
  // BF16 copies of the complex BF16 products' thin operands (null elsewhere)
  uint16_t* Omh = (bf16 && pl->cplx) ? ws_ptr<uint16_t>(pl, ws, WS_OMH) : nullptr;
  uint16_t* Yh = (bf16 && pl->cplx) ? ws_ptr<uint16_t>(pl, ws, WS_YH) : nullptr;
  uint16_t* Zh = (bf16 && pl->cplx) ? ws_ptr<uint16_t>(pl, ws, WS_ZH) : nullptr;
  const bool fp64 = pl->precision == HT_FP64;
  const uint16_t* Ah = reinterpret_cast<const uint16_t*>(A);  // BF16 view of the transformed tensor
  const int rows = fp64 ? 64 : pl->prod_rows;
  const int ri = rows == 128 ? 1 : 0;
  const int mode = pl->learn_mode;
  int2* wk1 = ws_ptr<int2>(pl, ws, WS_WK);
  int2* wk2 = ws_ptr<int2>(pl, ws, WS_WK2);
  int2* wkf = ws_ptr<int2>(pl, ws, WS_WKF);
  double* sig = ws_ptr<double>(pl, ws, WS_SIG);
  int* kept = ws_ptr<int>(pl, ws, WS_KEPT);
  double* anorm = ws_ptr<double>(pl, ws, WS_ANORM);
  int* lstate = ws_ptr<int>(pl, ws, WS_LSTATE);
  int* status = ws_ptr<int>(pl, ws, WS_STATUS);
  int rc;
  if ((rc = timed(pl, ST_TRANSFORM_FWD, s, [&] {
         if (use_t16(pl, X, A, bf16 ? 2 : 4)) {
           const int2* i16 = items(pl, pl->it_t16);
           if (bf16)
             return launch_transform16<uint16_t>((const float*)X, (uint16_t*)A, pl->d_tens, i16, pl->it_t16.n,
                                                 pl->table32, 0, s);
           return launch_transform16<float>((const float*)X, (float*)A, pl->d_tens, i16, pl->it_t16.n, pl->table32,
                                            0, s);
         }
         const int2* it = items(pl, pl->it_tf);
         if (pl->cplx) {
           const size_t lds = pl->tf_lds + pl->tf_map;
           if (bf16)
             return launch_transform_cplx<float, uint16_t>((const float*)X, (uint16_t*)A, pl->d_tens, it,
                                                           pl->it_tf.n, lds, pl->table32, pl->d_cmap, 0,
                                                           pl->mode_nmax, pl->tf_nf, s);
           return launch_transform_cplx<T, T>(X, A, pl->d_tens, it, pl->it_tf.n, lds, table<T>(pl), pl->d_cmap, 0,
                                              pl->mode_nmax, pl->tf_nf, s);
         }
         if (bf16)
           return launch_transform<float, uint16_t>((const float*)X, (uint16_t*)A, pl->d_tens, it, pl->it_tf.n,
                                                    pl->tf_lds, pl->table32, 0, s);
         return launch_transform<T, T>(X, A, pl->d_tens, it, pl->it_tf.n, pl->tf_lds, table<T>(pl), 0, s);
       })))
    return rc;
  if (mode) {  // ||A_j||^2 and this call's widths
    if ((rc = launch_anorm<T>(A, bf16 ? 1 : 0, sd, P, anorm, s))) return rc;
    if ((rc = launch_width(pl->learn_theta, mode, sd, P, lmax, sig, kept, wkf, anorm, lstate, tau, tau_dev, mu_dev,
                           call, call_dev, ws_ptr<float>(pl, ws, WS_FEAT), wk1, s)))
      return rc;
  }
  // the streaming product draws Omega itself; every other path reads it
  const OmegaKey okey{call, call_dev, pl->stream_id, pl->seed};
  const bool om_inline = !fp64 && pl->nn_stream;
  // complex BF16-mixed plans read only the BF16 copy of Omega
  if (!om_inline && (rc = timed(pl, ST_OMEGA, s, [&] {
                       return launch_omega<T>(Omh ? nullptr : Om, nullptr, Omh, sd, nullptr, P, pl->max_n2l, call,
                                              call_dev, pl->stream_id, pl->seed, 0, s);
                     })))
    return rc;
  const bool cplx = pl->cplx;
  auto sketch_nn = [&](const T* W, const int2* wk) {
    return timed(pl, ST_SKETCH_NN, s, [&] {
      if (cplx) {  // items of 64 complex rows
        const ItemList& L = pl->it_nn[0];
        if (bf16)
          return launch_bf16_cnn(Ah, W == Om ? Omh : Zh, (float*)Y, W == Om, sd, wk, items(pl, pl->it_cp[0]),
                                 pl->it_cp[0].n, lmax, gp1, s);
        if (!fp64)
          return launch_mfma_cnn((const float*)A, (const float*)W, (float*)Y, W == Om, sd, wk, items(pl, L), L.n,
                                 lmax, gp1, s);
        return launch_cgemm<T>(A, W, Y, 0, W == Om, sd, wk, items(pl, L), L.n, lmax, gp1, s);
      }
      const ItemList& L = pl->it_nn[ri];
      if (bf16)
        return launch_bf16_nn(Ah, (const float*)W, (float*)Y, sd, wk, items(pl, L), L.n, lmax, rows, gp1, s);
      if (!fp64 && pl->nn_stream)
        return launch_mfma_nn_stream((const float*)A, W == Om ? nullptr : (const float*)W, (float*)Y, sd, wk,
                                     items(pl, pl->it_nns), pl->it_nns.n, lmax, pl->max_n2, gp1, okey, s);
      if (!fp64)
        return launch_mfma_nn((const float*)A, (const float*)W, (float*)Y, sd, wk, items(pl, L), L.n, lmax, rows, gp1,
                              s);
      return launch_gemm_nn<T>(A, W, Y, sd, wk, items(pl, L), L.n, lmax, gp1, s);
    });
  };
  auto sketch_tn = [&](const int2* wk) {
    return timed(pl, ST_SKETCH_TN, s, [&] {
      if (cplx) {
        const ItemList& L = pl->it_tn[0];
        if (bf16)
          return launch_bf16_ctn(Ah, Yh, (float*)Z, sd, wk, items(pl, pl->it_cp[1]), pl->it_cp[1].n,
                                 lmax, gp1, s);
        if (!fp64)
          return launch_mfma_ctn((const float*)A, (const float*)Y, (float*)Z, sd, wk, items(pl, L), L.n, lmax, gp1,
                                 s);
        return launch_cgemm<T>(A, Y, Z, 1, 0, sd, wk, items(pl, L), L.n, lmax, gp1, s);
      }
      const ItemList& L = pl->it_tn[ri];
      if (bf16) return launch_bf16_tn(Ah, (const float*)Y, (float*)Z, sd, wk, items(pl, L), L.n, lmax, rows, gp1, s);
      if (!fp64)
        return launch_mfma_tn((const float*)A, (const float*)Y, (float*)Z, sd, wk, items(pl, L), L.n, lmax, rows, gp1,
                              s);
      return launch_gemm_tn<T>(A, Y, Z, sd, wk, items(pl, L), L.n, lmax, gp1, s);
    });
  };
  auto orth = [&](int which, double* gout, const int2* wk) {
    return timed(pl, ST_CHOLQR, s, [&] {
      if (cplx) {
        const ItemList& L = which ? pl->it_oz : pl->it_oy;
        const ItemList& S = which ? pl->it_asz : pl->it_asy;
        return launch_corth<T>(which ? Z : Y, which ? Zh : Yh, which, sd, wk, items(pl, L), L.n, items(pl, S), S.n,
                               lmax, P, gp1, gout, s);
      }
      if (wk == nullptr && pl->class_split) {  // one launch per width class
        for (int c = 0; c < kNumClasses; ++c) {
          const ItemList& L = which ? pl->it_ozc[c] : pl->it_oyc[c];
          if (L.n == 0) continue;
          const int r = launch_orth_apply<T>(which ? Z : Y, which, sd, nullptr, items(pl, L), L.n,
                                             pl->class_lmax[c], P, gp1, gout, s);
          if (r) return r;
        }
        return (int)HT_OK;
      }
      const ItemList& L = which ? pl->it_oz : pl->it_oy;
      return launch_orth_apply<T>(which ? Z : Y, which, sd, wk, items(pl, L), L.n, lmax, P, gp1, gout, s);
    });
  };
  double* sig_dst = mode ? sig : sigma_out;
  int* kept_dst = mode ? kept : kept_out;
  // One sketch of every slice at the widths wk (a width of 0 skips the slice):
  // Y = A Omega, Q1 = orth(Y); q power steps Z = orth(A^T Q1), Q1 = orth(A Z);
  // the last orthonormalization also writes the Gram partials of Q1; then
  // Bt = A^T Q1 and the small SVD with the shrinkage -> K'.
  auto sketch_all = [&](const int2* wk) -> int {
    int r;
    if ((r = sketch_nn(Om, wk))) return r;
    if ((r = orth(0, pl->q == 0 ? gp2 : nullptr, wk))) return r;
    for (int it = 0; it < pl->q; ++it) {
      if ((r = sketch_tn(wk))) return r;
      if ((r = orth(1, nullptr, wk))) return r;
      if ((r = sketch_nn(Z, wk))) return r;
      if ((r = orth(0, it == pl->q - 1 ? gp2 : nullptr, wk))) return r;
    }
    if ((r = sketch_tn(wk))) return r;
    return timed(pl, ST_SMALLSVD, s, [&] {
      if (cplx)
        return launch_csvd<T>(gp2, gp1, sd, wk, nullptr, P, lmax, lmax, tau, tau_dev, mu_dev, pen, K, sig_dst,
                              kept_dst, status, s);
      if (wk == nullptr && pl->class_split) {  // one launch per width class
        for (int c = 0; c < kNumClasses; ++c) {
          const ItemList& L = pl->it_svc[c];
          if (L.n == 0) continue;
          const int r = launch_smallsvd<T>(gp2, gp1, sd, nullptr, items(pl, L), L.n, pl->class_lmax[c], lmax, tau,
                                           tau_dev, mu_dev, pen, K, sig_dst, kept_dst, status, s);
          if (r) return r;
        }
        return (int)HT_OK;
      }
      return launch_smallsvd<T>(gp2, gp1, sd, wk, nullptr, P, lmax, lmax, tau, tau_dev, mu_dev, pen, K, sig_dst,
                                kept_dst, status, s);
    });
  };
  const int2* wk_final = nullptr;
  if (mode == 0) {
    if ((rc = sketch_all(nullptr))) return rc;
  } else {
    if ((rc = sketch_all(wk1))) return rc;
    if (mode == 2) {
      // slices whose predicted sketch could be truncated are redone at the fixed width
      if ((rc = launch_fallback(sd, P, lmax, wk1, sig, kept, anorm, tau, tau_dev, mu_dev, pen, pl->force_fallback,
                                wk2, wkf, lstate, s)))
        return rc;
      if ((rc = sketch_all(wk2))) return rc;
    } else if ((rc = launch_track_finalize(P, wk1, wkf, anorm, s))) {
      return rc;
    }
    if ((rc = launch_lstate_set(lstate, 1, 0, s))) return rc;
    wk_final = wkf;
    if (sigma_out)
      HT_CHECK_HIP(hipMemcpyAsync(sigma_out, sig, (size_t)P * lmax * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (kept_out) HT_CHECK_HIP(hipMemcpyAsync(kept_out, kept, (size_t)P * sizeof(int), hipMemcpyDeviceToDevice, s));
  }
  // C = (Q1 K') Bt^T, then the inverse transform
  if ((rc = timed(pl, ST_RECON_QK, s, [&] {
         if (cplx) {
           if (!fp64)
             return launch_mfma_cqk((const float*)Y, (const float*)K, (float*)QK, sd, wk_final, items(pl, pl->it_cqk),
                                    pl->it_cqk.n, lmax, s);
           return launch_crecon<T>(Y, K, QK, 0, sd, wk_final, items(pl, pl->it_qk), pl->it_qk.n, s);
         }
         if (!fp64 && lmax <= 64)
           return launch_mfma_qk((const float*)Y, (const float*)K, (float*)QK, sd, wk_final, items(pl, pl->it_qk),
                                 pl->it_qk.n, lmax, s);
         return launch_recon_qk<T>(Y, K, QK, sd, wk_final, items(pl, pl->it_qk), pl->it_qk.n, lmax, s);
       })))
    return rc;
  if ((rc = timed(pl, ST_RECON_NT, s, [&] {
         if (cplx) {
           if (bf16)
             return launch_bf16x3_cnt((const float*)QK, (const float*)Z, (float*)C, sd, wk_final,
                                      items(pl, pl->it_cnt), pl->it_cnt.n, lmax, s);
           if (!fp64)
             return launch_mfma_cnt((const float*)QK, (const float*)Z, (float*)C, sd, wk_final, items(pl, pl->it_cnt),
                                    pl->it_cnt.n, lmax, s);
           return launch_crecon<T>(QK, Z, C, 1, sd, wk_final, items(pl, pl->it_nt), pl->it_nt.n, s);
         }
         if (!fp64)
           return launch_mfma_nt((const float*)QK, (const float*)Z, (float*)C, sd, wk_final, items(pl, pl->it_nt),
                                 pl->it_nt.n, lmax, s);
         return launch_gemm_nt<T>(QK, Z, C, sd, wk_final, items(pl, pl->it_nt), pl->it_nt.n, s);
       })))
    return rc;
  return timed(pl, ST_TRANSFORM_INV, s, [&] {
    if (use_t16(pl, C, out, 4))
      return launch_transform16<float>((const float*)C, (float*)out, pl->d_tens, items(pl, pl->it_t16), pl->it_t16.n,
                                       pl->table32, 1, s);
    if (pl->cplx)
      return launch_transform_cplx<T, T>(C, out, pl->d_tens, items(pl, pl->it_tf), pl->it_tf.n,
                                         pl->tf_lds + pl->tf_map, table<T>(pl), pl->d_cmap, 1, pl->mode_nmax,
                                         pl->tf_nf, s);
    return launch_transform<T, T>(C, out, pl->d_tens, items(pl, pl->it_tf), pl->it_tf.n, pl->tf_lds, table<T>(pl), 1,
                                  s);
  });
}

// Eager launch, or (graph mode) replay of a recorded graph of the same
// launches whose first node writes the call index into the workspace.
int run_tsvt_any(ht_plan* pl, const void* X, void* out, double tau, const double* tau_dev, const ht_penalty* penalty,
                 uint32_t call, void* ws, hipStream_t s, double* sigma_out, int* kept_out) {
  const Penalty pen = to_dev(penalty);
  auto enqueue = [&](const int32_t* call_dev) -> int {
    if (pl->precision == HT_FP64)
      return run_tsvt<double>(pl, static_cast<const double*>(X), static_cast<double*>(out), tau, tau_dev, nullptr,
                              pen, call, call_dev, ws, s, sigma_out, kept_out);
    return run_tsvt<float>(pl, static_cast<const float*>(X), static_cast<float*>(out), tau, tau_dev, nullptr, pen,
                           call, call_dev, ws, s, sigma_out, kept_out);
  };
  if (!pl->graph_on || (pl->prof && pl->prof->on)) return enqueue(nullptr);
  if (s == nullptr) HT_FAIL(HT_ERR_INVALID_ARG, "graph replay needs a created stream (the null stream cannot be captured)");
  int32_t* slot = ws_ptr<int32_t>(pl, ws, WS_CALL);
  GraphCache& g = *pl->graph;
  const GraphKey key{X, out, ws, tau_dev, tau, penalty->kind, penalty->p0, penalty->p1, sigma_out, kept_out, s};
  int32_t callv = (int32_t)call;
  void* args[] = {&slot, &callv};
  hipKernelNodeParams np{};
  np.func = reinterpret_cast<void*>(k_set_call);
  np.gridDim = dim3(1);
  np.blockDim = dim3(64);
  np.sharedMemBytes = 0;
  np.kernelParams = args;
  np.extra = nullptr;
  if (!g.valid || !(g.key == key)) {
    g.reset();
    HT_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    const int rc = enqueue(slot);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (rc) return rc;
      HT_CHECK_HIP(e);
    }
    g.graph = graph;
    size_t nroots = 0;
    HT_CHECK_HIP(hipGraphGetRootNodes(graph, nullptr, &nroots));
    std::vector<hipGraphNode_t> roots(nroots);
    if (nroots) HT_CHECK_HIP(hipGraphGetRootNodes(graph, roots.data(), &nroots));
    HT_CHECK_HIP(hipGraphAddKernelNode(&g.call_node, graph, nullptr, 0, &np));
    for (auto& r : roots) HT_CHECK_HIP(hipGraphAddDependencies(graph, &g.call_node, &r, 1));
    HT_CHECK_HIP(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
    g.key = key;
    g.valid = true;
  } else {
    HT_CHECK_HIP(hipGraphExecKernelNodeSetParams(g.exec, g.call_node, &np));
  }
  HT_CHECK_HIP(hipGraphLaunch(g.exec, s));
  return HT_OK;
}

template <typename T>
int run_admm(const ht_plan* pl, const ht_admm_params* prm, const T* M, const uint8_t* mask, T* L, T* E, T* Yv,
             int n_iter, void* ws, hipStream_t s) {
  T* Lnew = ws_ptr<T>(pl, ws, WS_LNEW);
  T* Xin = ws_ptr<T>(pl, ws, WS_XIN);
  AdmmState* st = ws_ptr<AdmmState>(pl, ws, WS_STATE);
  const Penalty phi = to_dev(&prm->phi);
  const Penalty psi = to_dev(&prm->psi);
  int rc;
  if (n_iter <= 0) return HT_OK;
  if ((rc = launch_admm_input<T>(M, E, Yv, st, Xin, pl->Ntot, s))) return rc;
  for (int it = 0; it < n_iter; ++it) {
    if ((rc = run_tsvt<T>(pl, Xin, Lnew, 0.0, nullptr, &st->mu, phi, 0, &st->iteration, ws, s, nullptr, nullptr)))
      return rc;
    if ((rc = timed(pl, ST_ADMM_UPDATE, s, [&] {
           return launch_admm_update<T>(M, mask, Lnew, L, E, Yv, Xin, st, pl->Ntot, prm->model, psi, prm->lambda,
                                        prm->vartheta, prm->mu_max, ws_ptr<double>(pl, ws, WS_GSQ),
                                        pl->tens[0].n1 * pl->tens[0].n2, s);
         })))
      return rc;
    if ((rc = launch_admm_finalize(st, prm->vartheta, prm->mu_max, s))) return rc;
  }
  return launch_admm_rse<T>(L, static_cast<const T*>(pl->truth), pl->Ntot, ws_ptr<double>(pl, ws, WS_RED), kRseBlocks,
                            st, s);
}

// Workspace of the allocation-free t-SVT: a device array of the library, one
// copy per device.  In host code the array's name stands for a host-side
// shadow, not for a device address, so it is never passed to a kernel or a
// copy: the device address of each device's copy is looked up once, with that
// device current, and kept here.
static __device__ __align__(256) unsigned char scratch[HT_NOALLOC_SCRATCH_BYTES];

int noalloc_scratch(int device, void** ptr) {
  static std::mutex mu;
  static std::vector<void*> addr;  // per device ordinal, null until looked up
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) HT_FAIL(HT_ERR_INVALID_ARG, "bad device ordinal");
  if ((size_t)device >= addr.size()) addr.resize((size_t)device + 1, nullptr);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      HT_FAIL(HT_ERR_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    addr[device] = p;
  }
  *ptr = addr[device];
  return HT_OK;
}

// Every call on a plan runs on the device the plan was created on.
int check_device(const ht_plan* pl) {
  int dev = -1;
  HT_CHECK_HIP(hipGetDevice(&dev));
  if (dev != pl->device)
    HT_FAIL(HT_ERR_INVALID_ARG, "the current HIP device " + std::to_string(dev) + " is not the plan's device " +
                                    std::to_string(pl->device));
  return HT_OK;
}

int check_admm_params(const ht_admm_params* prm) {
  if (!prm) HT_FAIL(HT_ERR_INVALID_ARG, "admm params are NULL");
  if (prm->model < HT_COMPLETION || prm->model > HT_RPCA_SLICE) HT_FAIL(HT_ERR_INVALID_ARG, "unknown model");
  int rc;
  if ((rc = check_penalty(&prm->phi))) return rc;
  if (prm->model != HT_COMPLETION) {
    if ((rc = check_penalty(&prm->psi))) return rc;
    if (!(prm->lambda >= 0.0) || !std::isfinite(prm->lambda)) HT_FAIL(HT_ERR_INVALID_ARG, "lambda must be >= 0");
  }
  if (!(prm->mu0 > 0.0) || !std::isfinite(prm->mu0)) HT_FAIL(HT_ERR_INVALID_ARG, "mu0 must be > 0");
  if (!(prm->vartheta >= 1.0) || !std::isfinite(prm->vartheta)) HT_FAIL(HT_ERR_INVALID_ARG, "vartheta must be >= 1");
  if (!(prm->mu_max >= prm->mu0)) HT_FAIL(HT_ERR_INVALID_ARG, "mu_max must be >= mu0");
  return HT_OK;
}

}  // namespace

extern "C" {

int ht_version(void) { return 300; }

const char* ht_last_error(void) { return g_last_error.c_str(); }

int ht_plan_create(const ht_plan_desc* d, ht_plan** out) {
  if (!d || !out) HT_FAIL(HT_ERR_INVALID_ARG, "desc/out is NULL");
  return build_plan(d, 1, false, out);
}

int ht_batch_plan_create(int n_tensors, const ht_plan_desc* descs, ht_plan** out) {
  if (!descs || !out) HT_FAIL(HT_ERR_INVALID_ARG, "descs/out is NULL");
  if (n_tensors < 1) HT_FAIL(HT_ERR_INVALID_ARG, "n_tensors must be >= 1");
  return build_plan(descs, n_tensors, true, out);
}

int ht_plan_destroy(ht_plan* pl) {
  free_plan(pl);
  return HT_OK;
}

int ht_plan_device(const ht_plan* pl, int* device) {
  if (!pl || !device) HT_FAIL(HT_ERR_INVALID_ARG, "plan/device is NULL");
  *device = pl->device;
  return HT_OK;
}

int ht_plan_status(const ht_plan* pl, const void* ws, void* stream, int64_t* n_bad) {
  if (!pl || !ws) HT_FAIL(HT_ERR_INVALID_ARG, "plan/ws is NULL");
  int rc;
  if ((rc = check_device(pl))) return rc;
  std::vector<int> st((size_t)pl->Ptot);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!st.empty())
    HT_CHECK_HIP(hipMemcpyAsync(st.data(), static_cast<const char*>(ws) + pl->off[WS_STATUS], st.size() * sizeof(int),
                                hipMemcpyDeviceToHost, s));
  HT_CHECK_HIP(hipStreamSynchronize(s));
  int64_t bad = 0;
  for (int v : st) bad += v != 0;
  if (n_bad) *n_bad = bad;
  if (bad) HT_FAIL(HT_ERR_NONFINITE, std::to_string(bad) + " slice(s) of the last t-SVT met a NaN or an infinity");
  return HT_OK;
}

int ht_batch_info(const ht_plan* pl, int64_t* packed_numel, int* n_tensors) {
  if (!pl) HT_FAIL(HT_ERR_INVALID_ARG, "plan is NULL");
  if (packed_numel) *packed_numel = pl->Ntot;
  if (n_tensors) *n_tensors = (int)pl->tens.size();
  return HT_OK;
}

int ht_batch_tensor_info(const ht_plan* pl, int t, int64_t* offset, int64_t* numel, int64_t* first_slice, int* width,
                         int* kept) {
  if (!pl || t < 0 || t >= (int)pl->tens.size()) HT_FAIL(HT_ERR_INVALID_ARG, "bad plan or tensor index");
  const TensorHost& th = pl->tens[t];
  if (offset) *offset = th.x;
  if (numel) *numel = th.N;
  if (first_slice) *first_slice = th.slice0;
  if (width) *width = th.l;
  if (kept) *kept = th.k;
  return HT_OK;
}

int ht_profile_enable(ht_plan* pl, int on) {
  if (!pl) HT_FAIL(HT_ERR_INVALID_ARG, "plan is NULL");
  if (!pl->prof) pl->prof = new Profiler();
  pl->prof->on = on != 0;
  return HT_OK;
}

int ht_profile_read(ht_plan* pl, double* ms_total, int* count, int n_stages) {
  if (!pl || !ms_total || !count || n_stages < 1) HT_FAIL(HT_ERR_INVALID_ARG, "bad profile_read arguments");
  for (int i = 0; i < n_stages; ++i) {
    ms_total[i] = 0.0;
    count[i] = 0;
  }
  if (!pl->prof) return HT_OK;
  int rc = HT_OK;
  for (auto& r : pl->prof->recs) {
    if (rc == HT_OK) {
      float ms = 0.0f;
      if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
        set_error("event query failed");
        rc = HT_ERR_HIP;
      } else if (r.stage < n_stages) {
        ms_total[r.stage] += ms;
        count[r.stage] += 1;
      }
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  pl->prof->recs.clear();
  return rc;
}

int ht_plan_workspace_size(const ht_plan* pl, size_t* bytes) {
  if (!pl || !bytes) HT_FAIL(HT_ERR_INVALID_ARG, "plan/bytes is NULL");
  *bytes = pl->tsvt_bytes;
  return HT_OK;
}

int ht_plan_info(const ht_plan* pl, int64_t* n_slices, int* width, int* kept) {
  if (!pl) HT_FAIL(HT_ERR_INVALID_ARG, "plan is NULL");
  if (n_slices) *n_slices = pl->Ptot;
  if (width) *width = pl->lmax;
  if (kept) *kept = pl->kmax;
  return HT_OK;
}

int ht_plan_workspace_region(const ht_plan* pl, int region, size_t* offset, size_t* bytes) {
  if (!pl || region < 0 || region >= WS_COUNT) HT_FAIL(HT_ERR_INVALID_ARG, "bad plan or region");
  if (offset) *offset = pl->off[region];
  if (bytes) *bytes = pl->size[region];
  return HT_OK;
}

int ht_plan_set_tuning(ht_plan* pl, int prod_rows, int transform_lds_kib) {
  if (!pl) HT_FAIL(HT_ERR_INVALID_ARG, "plan is NULL");
  if (prod_rows != 0) {
    if (prod_rows != 64 && prod_rows != 128) HT_FAIL(HT_ERR_INVALID_ARG, "prod_rows must be 64 or 128");
    if (pl->precision == HT_FP64 && prod_rows != 64) HT_FAIL(HT_ERR_UNSUPPORTED, "FP64 products use 64-row tiles");
    pl->prod_rows = prod_rows;
    if (pl->graph) pl->graph->reset();
  }
  if (transform_lds_kib != 0) {
    const size_t b = (size_t)transform_lds_kib * 1024;
    bool known = false;
    for (size_t kb : kTfBudgets) known |= kb == b;
    if (!known) HT_FAIL(HT_ERR_INVALID_ARG, "transform LDS budget must be 32, 64 or 128 KiB");
    return set_transform_budget(pl, b);
  }
  return HT_OK;
}

int ht_plan_get_tuning(const ht_plan* pl, int* prod_rows, int* transform_lds_kib) {
  if (!pl) HT_FAIL(HT_ERR_INVALID_ARG, "plan is NULL");
  if (prod_rows) *prod_rows = pl->precision == HT_FP64 ? 64 : pl->prod_rows;
  if (transform_lds_kib) *transform_lds_kib = (int)(pl->tf_budget / 1024);
  return HT_OK;
}

int ht_plan_autotune(ht_plan* pl, const void* X, void* out, void* ws, size_t ws_bytes, void* stream, int repeats,
                     double* best_ms) {
  if (!pl || !X || !out) HT_FAIL(HT_ERR_INVALID_ARG, "plan/X/out is NULL");
  int rc;
  if ((rc = check_ws(ws, ws_bytes, pl->tsvt_bytes))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  repeats = std::max(1, repeats);
  const ht_penalty pen{HT_PEN_L1, 0.0, 0.0};
  std::vector<double> taus(pl->tens.size(), 0.0);
  const bool prof_on = pl->prof && pl->prof->on;
  if (pl->prof) pl->prof->on = false;
  const bool graph_on = pl->graph_on;
  pl->graph_on = false;
  hipEvent_t e0, e1;
  HT_CHECK_HIP(hipEventCreate(&e0));
  HT_CHECK_HIP(hipEventCreate(&e1));
  // time one configuration: a warm-up call, then `repeats` calls
  auto measure = [&](double& ms) -> int {
    int r = run_tsvt_any(pl, X, out, 0.0, nullptr, &pen, 0, ws, s, nullptr, nullptr);
    if (r) return r;
    HT_CHECK_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < repeats; ++i)
      if ((r = run_tsvt_any(pl, X, out, 0.0, nullptr, &pen, (uint32_t)i, ws, s, nullptr, nullptr))) return r;
    HT_CHECK_HIP(hipEventRecord(e1, s));
    HT_CHECK_HIP(hipEventSynchronize(e1));
    float f = 0.0f;
    HT_CHECK_HIP(hipEventElapsedTime(&f, e0, e1));
    ms = f / repeats;
    return HT_OK;
  };
  double best = 1e300;
  int best_rows = pl->prod_rows;
  size_t best_budget = pl->tf_budget;
  rc = HT_OK;
  const int rows_c[] = {128, 64};
  for (int rows : rows_c) {
    if (pl->precision == HT_FP64 && rows != 64) continue;
    pl->prod_rows = rows;
    double ms = 0.0;
    if ((rc = measure(ms))) break;
    if (ms < best) {
      best = ms;
      best_rows = rows;
    }
  }
  pl->prod_rows = best_rows;
  if (rc == HT_OK) {
    for (size_t b : kTfBudgets) {
      if (set_transform_budget(pl, b) != HT_OK) continue;  // a budget too small for this plan
      double ms = 0.0;
      if ((rc = measure(ms))) break;
      if (ms < best) {
        best = ms;
        best_budget = b;
      }
    }
    const int rc2 = set_transform_budget(pl, best_budget);
    if (rc == HT_OK) rc = rc2;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (pl->prof) pl->prof->on = prof_on;
  pl->graph_on = graph_on;
  if (pl->graph) pl->graph->reset();
  if (best_ms) *best_ms = best;
  return rc;
}

int ht_plan_graph_enable(ht_plan* pl, int on) {
  if (!pl) HT_FAIL(HT_ERR_INVALID_ARG, "plan is NULL");
  if (!pl->graph) pl->graph = new GraphCache();
  pl->graph->reset();
  pl->graph_on = on != 0;
  return HT_OK;
}

int ht_gnhtsvt(ht_plan* pl, const void* X, void* out, double tau, const ht_penalty* penalty, uint32_t call_index,
               void* ws, size_t ws_bytes, void* stream, double* sigma_out, int* kept_out) {
  if (!pl || !X || !out) HT_FAIL(HT_ERR_INVALID_ARG, "plan/X/out is NULL");
  if (pl->batch) HT_FAIL(HT_ERR_INVALID_ARG, "batch plans take ht_batch_gnhtsvt");
  if (!(tau >= 0.0) || !std::isfinite(tau)) HT_FAIL(HT_ERR_INVALID_ARG, "tau must be finite and >= 0");
  int rc;
  if ((rc = check_penalty(penalty))) return rc;
  if ((rc = check_device(pl))) return rc;
  if ((rc = check_ws(ws, ws_bytes, pl->tsvt_bytes))) return rc;
  return run_tsvt_any(pl, X, out, tau, nullptr, penalty, call_index, ws, static_cast<hipStream_t>(stream), sigma_out,
                      kept_out);
}

int ht_gnhtsvt_noalloc(ht_plan* pl, const void* X, void* out, double tau, const ht_penalty* penalty,
                       uint32_t call_index, void* stream, double* sigma_out, int* kept_out) {
  if (!pl || !X || !out) HT_FAIL(HT_ERR_INVALID_ARG, "plan/X/out is NULL");
  if (pl->batch) HT_FAIL(HT_ERR_UNSUPPORTED, "the allocation-free call takes a single-tensor plan");
  if (pl->learn_mode != 0 || pl->graph_on || (pl->prof && pl->prof->on))
    HT_FAIL(HT_ERR_UNSUPPORTED, "the allocation-free call needs learned widths, graph replay and profiling off");
  if (!(tau >= 0.0) || !std::isfinite(tau)) HT_FAIL(HT_ERR_INVALID_ARG, "tau must be finite and >= 0");
  int rc;
  if ((rc = check_penalty(penalty))) return rc;
  if ((rc = check_device(pl))) return rc;
  if (pl->tsvt_bytes > HT_NOALLOC_SCRATCH_BYTES)
    HT_FAIL(HT_ERR_WORKSPACE, "the plan needs " + std::to_string(pl->tsvt_bytes) +
                                  " bytes of workspace, above the library scratch of " +
                                  std::to_string((size_t)HT_NOALLOC_SCRATCH_BYTES));
  void* ws = nullptr;
  if ((rc = noalloc_scratch(pl->device, &ws))) return rc;
  return run_tsvt_any(pl, X, out, tau, nullptr, penalty, call_index, ws, static_cast<hipStream_t>(stream), sigma_out,
                      kept_out);
}

int ht_batch_gnhtsvt(ht_plan* pl, const void* X, void* out, const double* tau_dev, const ht_penalty* penalty,
                     uint32_t call_index, void* ws, size_t ws_bytes, void* stream, double* sigma_out, int* kept_out) {
  if (!pl || !X || !out || !tau_dev) HT_FAIL(HT_ERR_INVALID_ARG, "plan/X/out/tau is NULL");
  int rc;
  if ((rc = check_penalty(penalty))) return rc;
  if ((rc = check_device(pl))) return rc;
  if ((rc = check_ws(ws, ws_bytes, pl->tsvt_bytes))) return rc;
  return run_tsvt_any(pl, X, out, 0.0, tau_dev, penalty, call_index, ws, static_cast<hipStream_t>(stream), sigma_out,
                      kept_out);
}

int ht_omega_fp64(const ht_plan* pl, uint32_t call_index, double* dev_out, void* stream) {
  if (!pl || !dev_out) HT_FAIL(HT_ERR_INVALID_ARG, "plan/out is NULL");
  if (pl->batch || pl->cplx) HT_FAIL(HT_ERR_UNSUPPORTED, "ht_omega_fp64 takes a single-tensor real plan");
  const TensorHost& th = pl->tens[0];
  return launch_omega<double>(nullptr, dev_out, nullptr, pl->d_slices, nullptr, (int)pl->Ptot, pl->max_n2l, call_index,
                              nullptr, pl->stream_id, pl->seed, th.n2 * th.l, static_cast<hipStream_t>(stream));
}

int ht_transform(const ht_plan* pl, const void* X, void* out, int inverse, void* stream) {
  if (!pl || !X || !out) HT_FAIL(HT_ERR_INVALID_ARG, "plan/X/out is NULL");
  if (pl->cplx) HT_FAIL(HT_ERR_UNSUPPORTED, "ht_transform takes a real-transform plan");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int inv = inverse ? 1 : 0;
  if (pl->precision == HT_FP64)
    return launch_transform<double, double>(static_cast<const double*>(X), static_cast<double*>(out), pl->d_tens,
                                            items(pl, pl->it_tf), pl->it_tf.n, pl->tf_lds, pl->table64, inv, s);
  if (use_t16(pl, X, out, 4))
    return launch_transform16<float>(static_cast<const float*>(X), static_cast<float*>(out), pl->d_tens,
                                     items(pl, pl->it_t16), pl->it_t16.n, pl->table32, inv, s);
  return launch_transform<float, float>(static_cast<const float*>(X), static_cast<float*>(out), pl->d_tens,
                                        items(pl, pl->it_tf), pl->it_tf.n, pl->tf_lds, pl->table32, inv, s);
}

int ht_plan_learned(ht_plan* pl, int mode, const float* theta) {
  if (!pl) HT_FAIL(HT_ERR_INVALID_ARG, "plan is NULL");
  if (mode < 0 || mode > 2) HT_FAIL(HT_ERR_INVALID_ARG, "mode must be 0, 1 or 2");
  if (mode == 2 && !theta) HT_FAIL(HT_ERR_INVALID_ARG, "predicted widths need the network parameters");
  if (mode != 0 && pl->cplx) HT_FAIL(HT_ERR_UNSUPPORTED, "learned widths are not available for DFT plans");
  pl->learn_mode = mode;
  pl->learn_theta = theta;
  if (pl->graph) pl->graph->reset();
  return HT_OK;
}

int ht_plan_learned_reset(const ht_plan* pl, void* ws, size_t ws_bytes, void* stream) {
  if (!pl) HT_FAIL(HT_ERR_INVALID_ARG, "plan is NULL");
  int rc;
  if ((rc = check_ws(ws, ws_bytes, pl->tsvt_bytes))) return rc;
  return launch_lstate_set(ws_ptr<int>(pl, ws, WS_LSTATE), 0, 1, static_cast<hipStream_t>(stream));
}

int ht_plan_learned_counts(const ht_plan* pl, const void* ws, void* stream, int* valid, int* predicted,
                           int* redone) {
  if (!pl || !ws) HT_FAIL(HT_ERR_INVALID_ARG, "plan/ws is NULL");
  int st[3] = {0, 0, 0};
  hipStream_t s = static_cast<hipStream_t>(stream);
  HT_CHECK_HIP(hipMemcpyAsync(st, static_cast<const char*>(ws) + pl->off[WS_LSTATE], sizeof(st),
                              hipMemcpyDeviceToHost, s));
  HT_CHECK_HIP(hipStreamSynchronize(s));
  if (valid) *valid = st[0];
  if (predicted) *predicted = st[1];
  if (redone) *redone = st[2];
  return HT_OK;
}

int ht_plan_force_fallback(ht_plan* pl, int on) {
  if (!pl) HT_FAIL(HT_ERR_INVALID_ARG, "plan is NULL");
  pl->force_fallback = on != 0;
  if (pl->graph) pl->graph->reset();
  return HT_OK;
}

int ht_mlp_param_count(void) { return mlp_param_count(); }

int ht_mlp_workspace_size(int n, size_t* bytes) {
  if (!bytes || n < 1) HT_FAIL(HT_ERR_INVALID_ARG, "need n >= 1 and bytes");
  const size_t G = (size_t)mlp_grad_parts(n);
  *bytes = align256(G * mlp_param_count() * sizeof(float)) + align256(G * sizeof(float));
  return HT_OK;
}

int ht_mlp_forward(const float* theta, const float* X, float* z, int n, void* stream) {
  if (!theta || !X || !z || n < 0) HT_FAIL(HT_ERR_INVALID_ARG, "bad MLP forward arguments");
  return launch_mlp_forward(theta, X, z, n, static_cast<hipStream_t>(stream));
}

static int mlp_ws(int n, void* ws, size_t ws_bytes, float** part, float** lpart) {
  size_t need = 0;
  int rc;
  if ((rc = ht_mlp_workspace_size(n, &need))) return rc;
  if ((rc = check_ws(ws, ws_bytes, need))) return rc;
  const size_t G = (size_t)mlp_grad_parts(n);
  *part = static_cast<float*>(ws);
  *lpart = reinterpret_cast<float*>(static_cast<char*>(ws) + align256(G * mlp_param_count() * sizeof(float)));
  return HT_OK;
}

int ht_mlp_grad(const float* theta, const float* X, const float* y, int n, float* grad, float* loss, void* ws,
                size_t ws_bytes, void* stream) {
  if (!theta || !X || !y || !grad) HT_FAIL(HT_ERR_INVALID_ARG, "bad MLP gradient arguments");
  float *part, *lpart;
  int rc;
  if ((rc = mlp_ws(n, ws, ws_bytes, &part, &lpart))) return rc;
  return launch_mlp_grad_step(theta, X, y, n, part, lpart, grad, loss, nullptr, nullptr, nullptr, 0, 0.f, 0.f, 0.f,
                              0.f, static_cast<hipStream_t>(stream));
}

int ht_mlp_train_step(float* theta, float* m, float* v, int step, const float* X, const float* y, int n, float lr,
                      float beta1, float beta2, float eps, float* loss, void* ws, size_t ws_bytes, void* stream) {
  if (!theta || !m || !v || !X || !y) HT_FAIL(HT_ERR_INVALID_ARG, "bad MLP training arguments");
  if (step < 1) HT_FAIL(HT_ERR_INVALID_ARG, "Adam steps count from 1");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    HT_FAIL(HT_ERR_INVALID_ARG, "bad Adam hyperparameters");
  float *part, *lpart;
  int rc;
  if ((rc = mlp_ws(n, ws, ws_bytes, &part, &lpart))) return rc;
  return launch_mlp_grad_step(theta, X, y, n, part, lpart, nullptr, loss, theta, m, v, step, lr, beta1, beta2, eps,
                              static_cast<hipStream_t>(stream));
}

int ht_admm_workspace_size(const ht_plan* pl, size_t* bytes) {
  if (!pl || !bytes) HT_FAIL(HT_ERR_INVALID_ARG, "plan/bytes is NULL");
  *bytes = pl->admm_bytes;
  return HT_OK;
}

int ht_admm_init(ht_plan* pl, const ht_admm_params* prm, void* L, void* E, void* Y, void* ws, size_t ws_bytes,
                 void* stream) {
  if (!pl || !L || !E || !Y) HT_FAIL(HT_ERR_INVALID_ARG, "plan/L/E/Y is NULL");
  if (pl->batch) HT_FAIL(HT_ERR_UNSUPPORTED, "the solver takes a single-tensor plan");
  int rc;
  if ((rc = check_admm_params(prm))) return rc;
  if ((rc = check_ws(ws, ws_bytes, pl->admm_bytes))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bytes = (size_t)pl->Ntot * elem_bytes(pl->precision);
  HT_CHECK_HIP(hipMemsetAsync(L, 0, bytes, s));
  HT_CHECK_HIP(hipMemsetAsync(E, 0, bytes, s));
  HT_CHECK_HIP(hipMemsetAsync(Y, 0, bytes, s));
  if ((rc = launch_lstate_set(ws_ptr<int>(pl, ws, WS_LSTATE), 0, 1, s))) return rc;
  return launch_admm_reset(ws_ptr<AdmmState>(pl, ws, WS_STATE), prm->mu0, s);
}

int ht_admm_iterate(ht_plan* pl, const ht_admm_params* prm, const void* M, const uint8_t* mask, void* L, void* E,
                    void* Y, int n_iter, void* ws, size_t ws_bytes, void* stream) {
  if (!pl || !M || !mask || !L || !E || !Y) HT_FAIL(HT_ERR_INVALID_ARG, "plan/M/mask/L/E/Y is NULL");
  if (pl->batch) HT_FAIL(HT_ERR_UNSUPPORTED, "the solver takes a single-tensor plan");
  if (n_iter < 0) HT_FAIL(HT_ERR_INVALID_ARG, "n_iter must be >= 0");
  int rc;
  if ((rc = check_admm_params(prm))) return rc;
  if ((rc = check_device(pl))) return rc;
  if ((rc = check_ws(ws, ws_bytes, pl->admm_bytes))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->precision == HT_FP64)
    return run_admm<double>(pl, prm, static_cast<const double*>(M), mask, static_cast<double*>(L),
                            static_cast<double*>(E), static_cast<double*>(Y), n_iter, ws, s);
  return run_admm<float>(pl, prm, static_cast<const float*>(M), mask, static_cast<float*>(L), static_cast<float*>(E),
                         static_cast<float*>(Y), n_iter, ws, s);
}

int ht_admm_set_truth(ht_plan* pl, const void* truth) {
  if (!pl) HT_FAIL(HT_ERR_INVALID_ARG, "plan is NULL");
  if (pl->batch) HT_FAIL(HT_ERR_UNSUPPORTED, "the solver takes a single-tensor plan");
  pl->truth = truth;
  return HT_OK;
}

int ht_admm_get_stats(const ht_plan* pl, const void* ws, void* stream, ht_admm_stats* out) {
  if (!pl || !ws || !out) HT_FAIL(HT_ERR_INVALID_ARG, "plan/ws/out is NULL");
  int rc;
  if ((rc = check_device(pl))) return rc;
  AdmmState st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HT_CHECK_HIP(hipMemcpyAsync(&st, static_cast<const char*>(ws) + pl->off[WS_STATE], sizeof(st),
                              hipMemcpyDeviceToHost, s));
  std::vector<int> status((size_t)pl->Ptot);
  if (!status.empty())
    HT_CHECK_HIP(hipMemcpyAsync(status.data(), static_cast<const char*>(ws) + pl->off[WS_STATUS],
                                status.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  HT_CHECK_HIP(hipStreamSynchronize(s));
  out->iteration = st.iteration;
  out->mu = st.mu;
  out->dL = st.dL;
  out->dE = st.dE;
  out->resid = st.resid;
  out->rse = st.rse;
  int64_t bad = 0;
  for (int v : status) bad += v != 0;
  if (st.iteration > 0 && (!std::isfinite(st.dL) || !std::isfinite(st.dE) || !std::isfinite(st.resid) || bad))
    HT_FAIL(HT_ERR_NONFINITE, "the solver met a NaN or an infinity (stopping terms or " + std::to_string(bad) +
                                  " flagged slice(s))");
  return HT_OK;
}

}  // extern "C"
