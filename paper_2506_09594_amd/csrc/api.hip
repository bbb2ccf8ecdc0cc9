// C-ABI entry points: plans, workspace layout and the per-call orchestration
// of the randomized t-SVT and of the ADMM iteration.
#include <cmath>
#include <cstring>
#include <mutex>
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

}  // namespace ht

using namespace ht;

// Named regions of the t-SVT workspace (for introspection by the tests).
enum { WS_A = 0, WS_OMEGA, WS_Y, WS_Z, WS_K, WS_QK, WS_C, WS_LNEW, WS_XIN, WS_STATE, WS_GP1, WS_GP2, WS_COUNT };

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

struct ht_plan {
  int order;
  int64_t dims[HT_MAX_ORDER];
  int kinds[HT_MAX_ORDER];
  int64_t n1, n2, P, N;
  int r, p, q, l, k;
  int precision;
  uint64_t seed;
  uint32_t stream_id;
  int device;
  ModeTable mt_fwd, mt_inv;
  double* table64;  // device: forward then inverse matrices
  float* table32;
  size_t off[WS_COUNT];
  size_t size[WS_COUNT];
  size_t tsvt_bytes, admm_bytes;
  Profiler* prof;
  bool mfma;  // FP32 thin products on the matrix cores
};

namespace {

size_t elem_bytes(int precision) { return precision == HT_FP64 ? 8 : 4; }

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

void layout(ht_plan* pl) {
  const size_t es = elem_bytes(pl->precision);
  const size_t P = (size_t)pl->P, n1 = (size_t)pl->n1, n2 = (size_t)pl->n2, l = (size_t)pl->l;
  pl->size[WS_A] = (size_t)pl->N * (pl->precision == HT_BF16_MIXED ? 2 : es);
  pl->size[WS_OMEGA] = P * n2 * l * es;
  pl->size[WS_Y] = P * n1 * l * es;
  pl->size[WS_Z] = P * n2 * l * es;
  pl->size[WS_K] = P * l * l * es;
  pl->size[WS_QK] = P * n1 * l * es;
  pl->size[WS_C] = (size_t)pl->N * es;
  pl->size[WS_LNEW] = (size_t)pl->N * es;
  pl->size[WS_XIN] = (size_t)pl->N * es;
  pl->size[WS_STATE] = sizeof(AdmmState);
  const size_t t1 = (size_t)ceil_div(pl->n1, 64), t2 = (size_t)ceil_div(pl->n2, 64);  // >= 128-row counts
  pl->size[WS_GP1] = P * std::max(t1, t2) * l * l * sizeof(double);
  pl->size[WS_GP2] = P * t1 * l * l * sizeof(double);
  // t-SVT regions first, then the solver-only regions
  const int order_[] = {WS_A, WS_OMEGA, WS_Y, WS_Z, WS_K, WS_QK, WS_C, WS_GP1, WS_GP2, WS_LNEW, WS_XIN, WS_STATE};
  size_t o = 0;
  for (int r : order_) {
    pl->off[r] = o;
    o += align256(pl->size[r]);
    if (r == WS_GP2) pl->tsvt_bytes = o;
  }
  pl->admm_bytes = o;
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

int check_ws(const ht_plan* pl, const void* ws, size_t bytes, size_t need) {
  if (!ws) HT_FAIL(HT_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) HT_FAIL(HT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < need)
    HT_FAIL(HT_ERR_WORKSPACE, "workspace too small: " + std::to_string(bytes) + " < " + std::to_string(need));
  (void)pl;
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

// The randomized t-SVT on one plan; tau from the host, or 1/(*mu_dev) when
// mu_dev is given; sketch key from call or *call_dev.
template <typename T>
int run_tsvt(const ht_plan* pl, const T* X, T* out, double tau, const double* mu_dev, const Penalty& pen,
             uint32_t call, const int32_t* call_dev, void* ws, hipStream_t s, double* sigma_out, int* kept_out) {
  const int64_t n1 = pl->n1, n2 = pl->n2, P = pl->P, NT = n1 * n2;
  const int l = pl->l;
  T* A = ws_ptr<T>(pl, ws, WS_A);
  T* Om = ws_ptr<T>(pl, ws, WS_OMEGA);
  T* Y = ws_ptr<T>(pl, ws, WS_Y);
  T* Z = ws_ptr<T>(pl, ws, WS_Z);
  T* K = ws_ptr<T>(pl, ws, WS_K);
  T* QK = ws_ptr<T>(pl, ws, WS_QK);
  T* C = ws_ptr<T>(pl, ws, WS_C);
  const int64_t sA = NT, sY = n1 * l, sZ = n2 * l;
  const bool bf16 = pl->precision == HT_BF16_MIXED;
  const uint16_t* Ah = reinterpret_cast<const uint16_t*>(A);  // BF16 view of the transformed tensor
  int rc;
  if ((rc = timed(pl, ST_TRANSFORM_FWD, s, [&] {
         if (bf16)
           return launch_transform_bf16((const float*)X, (uint16_t*)A, NT, (int)P, pl->mt_fwd, pl->table32, s);
         return launch_transform<T>(X, A, NT, (int)P, pl->mt_fwd, table<T>(pl), s);
       })))
    return rc;
  if ((rc = timed(pl, ST_OMEGA, s, [&] {
         return launch_omega<T>(Om, nullptr, (int)P, n2 * l, call, call_dev, pl->stream_id, pl->seed, nullptr, s);
       })))
    return rc;
  double* gp1 = ws_ptr<double>(pl, ws, WS_GP1);
  double* gp2 = ws_ptr<double>(pl, ws, WS_GP2);
  const int t1 = (int)ceil_div(n1, 64);
  // FP32 slices with 16-byte aligned columns run the products on the matrix cores
  const bool mfma = pl->mfma;
  const int rt = (mfma || bf16) ? mfma_tile_rows() : 64;
  const int p1 = (int)ceil_div(n1, rt), p2 = (int)ceil_div(n2, rt);
  auto sketch_nn = [&](const T* W) {
    return timed(pl, ST_SKETCH_NN, s, [&] {
      if (bf16)
        return launch_bf16_nn(Ah, sA, (int)n1, (const float*)W, sZ, (int)n2, (float*)Y, sY, (int)n1, (int)n1,
                              (int)n2, l, (int)P, gp1, s);
      if (mfma)
        return launch_mfma_nn((const float*)A, sA, (int)n1, (const float*)W, sZ, (int)n2, (float*)Y, sY, (int)n1,
                              (int)n1, (int)n2, l, (int)P, gp1, s);
      return launch_gemm_nn<T>(A, sA, (int)n1, W, sZ, (int)n2, Y, sY, (int)n1, (int)n1, (int)n2, l, (int)P, gp1, s);
    });
  };
  auto sketch_tn = [&]() {
    return timed(pl, ST_SKETCH_TN, s, [&] {
      if (bf16)
        return launch_bf16_tn(Ah, sA, (int)n1, (const float*)Y, sY, (int)n1, (float*)Z, sZ, (int)n2, (int)n1,
                              (int)n2, l, (int)P, gp1, s);
      if (mfma)
        return launch_mfma_tn((const float*)A, sA, (int)n1, (const float*)Y, sY, (int)n1, (float*)Z, sZ, (int)n2,
                              (int)n1, (int)n2, l, (int)P, gp1, s);
      return launch_gemm_tn<T>(A, sA, (int)n1, Y, sY, (int)n1, Z, sZ, (int)n2, (int)n1, (int)n2, l, (int)P, gp1, s);
    });
  };
  auto orth = [&](T* M, int64_t sM, int m, int nparts, double* gout) {
    return timed(pl, ST_CHOLQR, s,
                 [&] { return launch_orth_apply<T>(M, sM, m, m, l, (int)P, gp1, nparts, gout, s); });
  };
  // Y = A Omega, Q1 = orth(Y); q power steps Z = orth(A^T Q1), Q1 = orth(A Z);
  // the last orthonormalization also writes the Gram partials of Q1.
  if ((rc = sketch_nn(Om))) return rc;
  if ((rc = orth(Y, sY, (int)n1, p1, pl->q == 0 ? gp2 : nullptr))) return rc;
  for (int it = 0; it < pl->q; ++it) {
    if ((rc = sketch_tn())) return rc;
    if ((rc = orth(Z, sZ, (int)n2, p2, nullptr))) return rc;
    if ((rc = sketch_nn(Z))) return rc;
    if ((rc = orth(Y, sY, (int)n1, p1, it == pl->q - 1 ? gp2 : nullptr))) return rc;
  }
  // Bt = A^T Q1 with the Gram partials of Bt
  if ((rc = sketch_tn())) return rc;
  // second CholeskyQR step in the small space, small SVD, shrink -> K'
  if ((rc = timed(pl, ST_SMALLSVD, s, [&] {
         return launch_smallsvd<T>(gp2, t1, (int)n1, gp1, p2, l, pl->k, (int)P, tau, mu_dev, pen, K, sigma_out,
                                   kept_out, s);
       })))
    return rc;
  // C = (Q1 K') Bt^T, then the inverse transform
  if ((rc = timed(pl, ST_RECON_QK, s, [&] {
         return launch_gemm_nn<T>(Y, sY, (int)n1, K, (int64_t)l * l, l, QK, sY, (int)n1, (int)n1, l, l, (int)P,
                                  nullptr, s);
       })))
    return rc;
  if ((rc = timed(pl, ST_RECON_NT, s, [&] {
         return launch_gemm_nt<T>(QK, sY, (int)n1, Z, sZ, (int)n2, C, sA, (int)n1, (int)n1, (int)n2, l, (int)P, s);
       })))
    return rc;
  return timed(pl, ST_TRANSFORM_INV, s,
               [&] { return launch_transform<T>(C, out, NT, (int)P, pl->mt_inv, table<T>(pl), s); });
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
  if ((rc = launch_admm_input<T>(M, E, Yv, st, Xin, pl->N, s))) return rc;
  for (int it = 0; it < n_iter; ++it) {
    if ((rc = run_tsvt<T>(pl, Xin, Lnew, 0.0, &st->mu, phi, 0, &st->iteration, ws, s, nullptr, nullptr))) return rc;
    if ((rc = timed(pl, ST_ADMM_UPDATE, s, [&] {
           return launch_admm_update<T>(M, mask, Lnew, L, E, Yv, Xin, st, pl->N, prm->model, psi, prm->lambda,
                                        prm->vartheta, prm->mu_max, s);
         })))
      return rc;
    if ((rc = launch_admm_finalize(st, prm->vartheta, prm->mu_max, s))) return rc;
  }
  return HT_OK;
}

int check_admm_params(const ht_admm_params* prm) {
  if (!prm) HT_FAIL(HT_ERR_INVALID_ARG, "admm params are NULL");
  if (prm->model != HT_COMPLETION && prm->model != HT_RPCA) HT_FAIL(HT_ERR_INVALID_ARG, "unknown model");
  int rc;
  if ((rc = check_penalty(&prm->phi))) return rc;
  if (prm->model == HT_RPCA) {
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

int ht_version(void) { return 100; }

const char* ht_last_error(void) { return g_last_error.c_str(); }

int ht_plan_create(const ht_plan_desc* d, ht_plan** out) {
  if (!d || !out) HT_FAIL(HT_ERR_INVALID_ARG, "desc/out is NULL");
  *out = nullptr;
  if (d->order < 2 || d->order > HT_MAX_ORDER) HT_FAIL(HT_ERR_INVALID_ARG, "order must be in [2, 8]");
  if (d->precision != HT_FP64 && d->precision != HT_FP32 && d->precision != HT_BF16_MIXED)
    HT_FAIL(HT_ERR_INVALID_ARG, "unknown precision");
  if (d->r < 1 || d->p < 0 || d->q < 0) HT_FAIL(HT_ERR_INVALID_ARG, "need r >= 1, p >= 0, q >= 0");
  ht_plan* pl = new ht_plan();
  std::memset(pl, 0, sizeof(ht_plan));
  pl->order = d->order;
  int64_t P = 1;
  for (int i = 0; i < d->order; ++i) {
    if (d->dims[i] < 1) {
      delete pl;
      HT_FAIL(HT_ERR_INVALID_ARG, "dims must be >= 1");
    }
    pl->dims[i] = d->dims[i];
    if (i >= 2) P *= d->dims[i];
  }
  pl->n1 = d->dims[0];
  pl->n2 = d->dims[1];
  pl->P = P;
  pl->N = pl->n1 * pl->n2 * P;
  if (pl->n1 > (1 << 30) || pl->n2 > (1 << 30) || P > 65535) {
    delete pl;
    HT_FAIL(HT_ERR_UNSUPPORTED, "slice count above 65535 or a spatial mode above 2^30");
  }
  pl->r = d->r;
  pl->p = d->p;
  pl->q = d->q;
  pl->l = (int)std::min<int64_t>(std::min<int64_t>(d->r + d->p, pl->n1), pl->n2);
  pl->k = std::min(d->r, pl->l);
  if (pl->l > HT_MAX_WIDTH) {
    delete pl;
    HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width min(r+p, n1, n2) above HT_MAX_WIDTH");
  }
  pl->precision = d->precision;
  pl->seed = d->seed;
  pl->stream_id = d->stream_id;
  if (hipGetDevice(&pl->device) != hipSuccess) pl->device = 0;

  // transform tables: forward U_k and inverse U_k^T / alpha_k, row-major
  std::vector<double> tab;
  pl->mt_fwd.nmodes = pl->mt_inv.nmodes = d->order - 2;
  int stride = 1;
  for (int m = 0; m < d->order - 2; ++m) {
    const int n = (int)d->dims[m + 2];
    const int kind = d->transform[m + 2];
    pl->kinds[m + 2] = kind;
    if (n > HT_MAX_MODE) {
      delete pl;
      HT_FAIL(HT_ERR_UNSUPPORTED, "transformed mode longer than HT_MAX_MODE");
    }
    std::vector<double> U;
    double alpha = 1.0;
    if (kind == HT_DCT2_ORTHO) {
      dct2_ortho(n, U);
    } else if (kind == HT_CUSTOM_REAL) {
      if (!d->custom[m + 2]) {
        delete pl;
        HT_FAIL(HT_ERR_INVALID_ARG, "CUSTOM_REAL transform needs a matrix");
      }
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
      if (!(alpha > 0.0) || err > 1e-10 * alpha) {
        delete pl;
        HT_FAIL(HT_ERR_INVALID_ARG, "CUSTOM_REAL matrix must satisfy U U^T = alpha I");
      }
    } else if (kind == HT_DFT_UNITARY) {
      delete pl;
      HT_FAIL(HT_ERR_UNSUPPORTED, "DFT_UNITARY transforms are not implemented in this build");
    } else {
      delete pl;
      HT_FAIL(HT_ERR_INVALID_ARG, "unknown transform kind");
    }
    pl->mt_fwd.n[m] = pl->mt_inv.n[m] = n;
    pl->mt_fwd.stride[m] = pl->mt_inv.stride[m] = stride;
    stride *= n;
    pl->mt_fwd.off[m] = (int)tab.size();
    tab.insert(tab.end(), U.begin(), U.end());
    pl->mt_inv.off[m] = (int)tab.size();
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) tab.push_back(U[(size_t)b * n + a] / alpha);
  }
  // the inverse applies mode d first, then d-1, ..., 3 (order does not change
  // the result since the mode products commute; kept as in the definition)
  {
    ModeTable rev = pl->mt_inv;
    const int nm = pl->mt_inv.nmodes;
    for (int m = 0; m < nm; ++m) {
      rev.n[m] = pl->mt_inv.n[nm - 1 - m];
      rev.stride[m] = pl->mt_inv.stride[nm - 1 - m];
      rev.off[m] = pl->mt_inv.off[nm - 1 - m];
    }
    pl->mt_inv = rev;
  }
  if (!tab.empty()) {
    std::vector<float> tab32(tab.begin(), tab.end());
    if (hipMalloc(&pl->table64, tab.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&pl->table32, tab32.size() * sizeof(float)) != hipSuccess) {
      (void)hipFree(pl->table64);
      delete pl;
      HT_FAIL(HT_ERR_ALLOC, "could not allocate transform tables");
    }
    if (hipMemcpy(pl->table64, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->table32, tab32.data(), tab32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(pl->table64);
      (void)hipFree(pl->table32);
      delete pl;
      HT_FAIL(HT_ERR_HIP, "could not upload transform tables");
    }
  }
  if (pl->mt_fwd.nmodes > 0 && transform_tile_width(P, elem_bytes(pl->precision)) == 0) {
    (void)hipFree(pl->table64);
    (void)hipFree(pl->table32);
    delete pl;
    HT_FAIL(HT_ERR_UNSUPPORTED, "too many face slices for the transform tile");
  }
  pl->mfma = pl->precision == HT_FP32 && pl->n1 % 4 == 0 && pl->n2 % 4 == 0;
  layout(pl);
  *out = pl;
  return HT_OK;
}

int ht_plan_destroy(ht_plan* pl) {
  if (!pl) return HT_OK;
  if (pl->prof) {
    for (auto& r : pl->prof->recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    delete pl->prof;
  }
  if (pl->table64) (void)hipFree(pl->table64);
  if (pl->table32) (void)hipFree(pl->table32);
  delete pl;
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
  if (n_slices) *n_slices = pl->P;
  if (width) *width = pl->l;
  if (kept) *kept = pl->k;
  return HT_OK;
}

int ht_plan_workspace_region(const ht_plan* pl, int region, size_t* offset, size_t* bytes) {
  if (!pl || region < 0 || region >= WS_COUNT) HT_FAIL(HT_ERR_INVALID_ARG, "bad plan or region");
  if (offset) *offset = pl->off[region];
  if (bytes) *bytes = pl->size[region];
  return HT_OK;
}

int ht_gnhtsvt(ht_plan* pl, const void* X, void* out, double tau, const ht_penalty* penalty, uint32_t call_index,
               void* ws, size_t ws_bytes, void* stream, double* sigma_out, int* kept_out) {
  if (!pl || !X || !out) HT_FAIL(HT_ERR_INVALID_ARG, "plan/X/out is NULL");
  if (!(tau >= 0.0) || !std::isfinite(tau)) HT_FAIL(HT_ERR_INVALID_ARG, "tau must be finite and >= 0");
  int rc;
  if ((rc = check_penalty(penalty))) return rc;
  if ((rc = check_ws(pl, ws, ws_bytes, pl->tsvt_bytes))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Penalty pen = to_dev(penalty);
  if (pl->precision == HT_FP64)
    return run_tsvt<double>(pl, static_cast<const double*>(X), static_cast<double*>(out), tau, nullptr, pen,
                            call_index, nullptr, ws, s, sigma_out, kept_out);
  return run_tsvt<float>(pl, static_cast<const float*>(X), static_cast<float*>(out), tau, nullptr, pen, call_index,
                         nullptr, ws, s, sigma_out, kept_out);
}

int ht_omega_fp64(const ht_plan* pl, uint32_t call_index, double* dev_out, void* stream) {
  if (!pl || !dev_out) HT_FAIL(HT_ERR_INVALID_ARG, "plan/out is NULL");
  return launch_omega<double>(nullptr, dev_out, (int)pl->P, pl->n2 * pl->l, call_index, nullptr, pl->stream_id,
                              pl->seed, nullptr, static_cast<hipStream_t>(stream));
}

int ht_transform(const ht_plan* pl, const void* X, void* out, int inverse, void* stream) {
  if (!pl || !X || !out) HT_FAIL(HT_ERR_INVALID_ARG, "plan/X/out is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ModeTable& mt = inverse ? pl->mt_inv : pl->mt_fwd;
  const int64_t NT = pl->n1 * pl->n2;
  if (pl->precision == HT_FP64)
    return launch_transform<double>(static_cast<const double*>(X), static_cast<double*>(out), NT, (int)pl->P, mt,
                                    pl->table64, s);
  return launch_transform<float>(static_cast<const float*>(X), static_cast<float*>(out), NT, (int)pl->P, mt,
                                 pl->table32, s);
}

int ht_admm_workspace_size(const ht_plan* pl, size_t* bytes) {
  if (!pl || !bytes) HT_FAIL(HT_ERR_INVALID_ARG, "plan/bytes is NULL");
  *bytes = pl->admm_bytes;
  return HT_OK;
}

int ht_admm_init(ht_plan* pl, const ht_admm_params* prm, void* L, void* E, void* Y, void* ws, size_t ws_bytes,
                 void* stream) {
  if (!pl || !L || !E || !Y) HT_FAIL(HT_ERR_INVALID_ARG, "plan/L/E/Y is NULL");
  int rc;
  if ((rc = check_admm_params(prm))) return rc;
  if ((rc = check_ws(pl, ws, ws_bytes, pl->admm_bytes))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bytes = (size_t)pl->N * elem_bytes(pl->precision);
  HT_CHECK_HIP(hipMemsetAsync(L, 0, bytes, s));
  HT_CHECK_HIP(hipMemsetAsync(E, 0, bytes, s));
  HT_CHECK_HIP(hipMemsetAsync(Y, 0, bytes, s));
  return launch_admm_reset(ws_ptr<AdmmState>(pl, ws, WS_STATE), prm->mu0, s);
}

int ht_admm_iterate(ht_plan* pl, const ht_admm_params* prm, const void* M, const uint8_t* mask, void* L, void* E,
                    void* Y, int n_iter, void* ws, size_t ws_bytes, void* stream) {
  if (!pl || !M || !mask || !L || !E || !Y) HT_FAIL(HT_ERR_INVALID_ARG, "plan/M/mask/L/E/Y is NULL");
  if (n_iter < 0) HT_FAIL(HT_ERR_INVALID_ARG, "n_iter must be >= 0");
  int rc;
  if ((rc = check_admm_params(prm))) return rc;
  if ((rc = check_ws(pl, ws, ws_bytes, pl->admm_bytes))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->precision == HT_FP64)
    return run_admm<double>(pl, prm, static_cast<const double*>(M), mask, static_cast<double*>(L),
                            static_cast<double*>(E), static_cast<double*>(Y), n_iter, ws, s);
  return run_admm<float>(pl, prm, static_cast<const float*>(M), mask, static_cast<float*>(L), static_cast<float*>(E),
                         static_cast<float*>(Y), n_iter, ws, s);
}

int ht_admm_get_stats(const ht_plan* pl, const void* ws, void* stream, ht_admm_stats* out) {
  if (!pl || !ws || !out) HT_FAIL(HT_ERR_INVALID_ARG, "plan/ws/out is NULL");
  AdmmState st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HT_CHECK_HIP(hipMemcpyAsync(&st, static_cast<const char*>(ws) + pl->off[WS_STATE], sizeof(st),
                              hipMemcpyDeviceToHost, s));
  HT_CHECK_HIP(hipStreamSynchronize(s));
  out->iteration = st.iteration;
  out->mu = st.mu;
  out->dL = st.dL;
  out->dE = st.dE;
  out->resid = st.resid;
  return HT_OK;
}

}  // extern "C"
