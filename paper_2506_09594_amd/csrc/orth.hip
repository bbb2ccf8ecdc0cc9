// Orthonormalization of the tall-skinny sketches by CholeskyQR with deflation.
//
// The product that made Y (m x l per slice) already wrote the FP64 Gram
// partials of its 64-row slabs.  Here one wavefront per (slice, 64-row tile)
// sums the partials of its slice in a fixed order (so every tile of a slice
// obtains the same G = Y^T Y bit for bit), factors G = R^T R in FP64 with
// deflation, and solves q R = y for each of its rows by forward substitution
// in registers, writing Q = Y R^{-1} in place.  The paper orthonormalizes the
// sketch blocks ("form an orthonormal basis", Alg. 1) and deflates columns
// whose pivot falls below a tolerance (defl-QR, Alg. 2): a column whose
// Schur-complement pivot is below
//   delta = 8 * m * 2^-52 * max_i G_ii
// (its residual against the previous columns is at rounding level) becomes a
// zero column of Q, which leaves the span of the kept columns intact.
//
// Slices wider than 64 factor once per slice in a workgroup of 256 threads
// (Cholesky with one barrier per column), park R^{-1} (row-major l x l) over
// the slice's first partial, and apply it per tile.
//
// One pass of this CholeskyQR gives a basis whose span is exact to rounding and
// whose orthogonality error is O(u_64 kappa(Y)^2); that suffices inside the
// power iterations, where only the span matters.  For the final basis the
// kernel also writes the Gram partials of Q, and the second CholeskyQR step is
// applied in the l x l space by the small-SVD kernel.
#include <type_traits>

#include "chol.hpp"

namespace ht {

namespace {

constexpr int TR = 64;  // rows per workgroup (matches the producing products); one lane per row

// Work item (slice, first row) of the basis `which` (0: Y, n1 rows; 1: Z, n2
// rows): its operand, row count and the number of Gram partials of the
// producing product (one per 64 rows).
struct OrthItem {
  int64_t off, g1, g2;
  int m, l, row0, nparts;
};

__device__ __forceinline__ OrthItem orth_item(const SliceDesc* sd, const int2* wk, const int2* items, int which) {
  const int2 it = items[blockIdx.x];
  const SliceDesc d = sd[it.x];
  OrthItem o;
  o.m = which ? d.n2 : d.n1;
  o.off = which ? d.z : d.y;
  o.l = slice_width(d, wk, it.x);
  o.row0 = it.y;
  o.nparts = (o.m + kGramRows - 1) / kGramRows;
  o.g1 = d.g1;
  o.g2 = d.g2;
  return o;
}

// Register path (l <= 64): lane b sums column b of G from the partials and
// the factorization runs in registers; lane i then owns row i of the tile and
// solves q R = y with the rows of R broadcast by readlane.
template <typename T, int LB>
__global__ __launch_bounds__(TR) void k_orth_fused(T* __restrict__ Yall, int which, const SliceDesc* __restrict__ sd,
                                                        const int2* __restrict__ wk, const int2* __restrict__ items,
                                                        const double* __restrict__ gin_all,
                                                        double* __restrict__ gout_all) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const OrthItem o = orth_item(sd, wk, items, which);
  const int l = o.l, m = o.m, ldy = m, nparts = o.nparts;
  if (l <= 0 || l > LB) return;  // slice not part of this pass, or on the factor-once path
  const int gp = l + 1;
  double* S = reinterpret_cast<double*>(smem_raw);  // TR x gp (Gram of the result)
  const int row0 = o.row0;
  const int rows = min(TR, m - row0);
  T* Y = Yall + o.off + row0;
  double* gout = gout_all ? gout_all + o.g2 + (int64_t)(row0 / TR) * l * l : nullptr;
  const int lane = threadIdx.x;
  const bool valid = lane < rows;
  const int ll = l * l;

  // column `lane` of G = sum of the tile partials (fixed order)
  const double* part = gin_all + o.g1;
  double g[LB];
#pragma unroll
  for (int a = 0; a < LB; ++a) g[a] = 0.0;
  const int bcol = lane < l ? lane : 0;
  for (int t = 0; t < nparts; ++t) {
    double v[LB];
#pragma unroll
    for (int a = 0; a < LB; ++a) {
      const double pv = part[(int64_t)t * ll + (a < l ? a : l - 1) * l + bcol];
      v[a] = (a < l) ? pv : 0.0;
    }
#pragma unroll
    for (int a = 0; a < LB; ++a) g[a] += v[a];
  }
  // every load unconditional (row and column clamped into the tile) so that
  // all of them are in flight at once; a guarded load compiles to a branch
  // and a wait per column
  const int lrow = valid ? lane : rows - 1;
  double y[LB];
#pragma unroll
  for (int c = 0; c < LB; ++c) {
    const T v = Y[lrow + (int64_t)(c < l ? c : l - 1) * ldy];
    y[c] = (c < l && valid) ? (double)v : 0.0;
  }

  // pivot threshold from the largest diagonal entry
  double dmax = (lane < l) ? g[0] : 0.0;
#pragma unroll
  for (int a = 1; a < LB; ++a)
    if (a == lane) dmax = g[a];
  if (lane >= l) dmax = 0.0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
  const double delta = 8.0 * (double)m * 2.220446049250313e-16 * dmax;
  chol_regs<LB>(g, l, dmax > 0.0 ? delta : 1.0);

  // 1 / R[c][c] on lane c (0 for a skipped column), all lanes at once, so no
  // reciprocal sits on the chain of the substitution below
  double rdiag = 0.0;
#pragma unroll
  for (int a = 0; a < LB; ++a)
    if (a == lane) rdiag = g[a];
  const double rinv = (rdiag != 0.0) ? fast_rcp(rdiag) : 0.0;
  // q R = y: q_c = (y_c - sum_{a<c} q_a R[a][c]) / R[c][c]; R[a][c] is g[a] on lane c
#pragma unroll
  for (int c = 0; c < LB; ++c) {
    if (c < l) {
      double t = y[c];
#pragma unroll
      for (int a = 0; a < c; ++a) t -= y[a] * readlane_d(g[a], c);
      y[c] = t * readlane_d(rinv, c);
    }
  }
#pragma unroll
  for (int c = 0; c < LB; ++c) {
    if (c < l) {
      const T v = (T)y[c];
      if (valid) Y[lane + (int64_t)c * ldy] = v;
      if (gout) S[lane * gp + c] = valid ? (double)v : 0.0;
    }
  }
  if (gout) {
    __syncthreads();
    tile_gram_mfma(S, gp, 1, rows, l, gout);
  }
}

// Widths above 64: one workgroup per slice factors G once (sum of the
// partials, Cholesky with deflation, R^{-1}) and parks R^{-1} (row-major
// l x l) in the slice's first Gram partial, which nothing reads afterwards.
template <int LB>
__global__ __launch_bounds__(256) void k_orth_factor(int which, const SliceDesc* __restrict__ sd,
                                                     const int2* __restrict__ wk, double* __restrict__ gin_all) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double s_scratch;
  const int s = blockIdx.x;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 64) return;  // not part of this pass, or on the register path
  const int m = which ? d.n2 : d.n1;
  const int nparts = (m + kGramRows - 1) / kGramRows;
  const int gp = l + 1;
  double* G = reinterpret_cast<double*>(smem_raw);  // l x gp
  double* dR = G + (size_t)l * gp;                  // gp
  double* Rinv = dR + gp;                           // l x gp
  double* part = gin_all + d.g1;
  sum_gram_partials(G, gp, part, nparts, l);
  __syncthreads();
  chol_deflate(G, dR, gp, l, 8.0 * (double)m * 2.220446049250313e-16, &s_scratch);
  tri_inverse<LB>(G, dR, gp, l, Rinv);
  for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) part[idx] = Rinv[(idx / l) * gp + (idx % l)];
}

// Apply Q = Y R^{-1} per 64-row tile with the parked R^{-1} (widths above 64):
// R^{-1} and the tile are staged in LDS (lane i owns row i; entries of R^{-1}
// are broadcast reads), q_c = sum_{a <= c} y_a Rinv[a][c] overwrites y_c from
// the last column down (a lower column never reads a higher y), with runtime
// loops so that no unrolled chain hoists thousands of loads into registers.
template <typename T>
__global__ __launch_bounds__(TR) void k_orth_apply(T* __restrict__ Yall, int which, const SliceDesc* __restrict__ sd,
                                                   const int2* __restrict__ wk, const int2* __restrict__ items,
                                                   const double* __restrict__ gin_all,
                                                   double* __restrict__ gout_all) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const OrthItem o = orth_item(sd, wk, items, which);
  const int l = o.l, m = o.m, ldy = m;
  if (l <= 64) return;  // slice not part of this pass, or on the fused path
  const int gp = l + 1, ll = l * l;
  double* Ri = reinterpret_cast<double*>(smem_raw);  // R^{-1}, row-major l x l
  double* S = Ri + ll;                               // the tile, TR x gp
  const int row0 = o.row0;
  const int rows = min(TR, m - row0);
  T* Y = Yall + o.off + row0;
  const double* Rg = gin_all + o.g1;
  double* gout = gout_all ? gout_all + o.g2 + (int64_t)(row0 / TR) * l * l : nullptr;
  const int i = threadIdx.x;
  const bool valid = i < rows;
  // loads in batches of eight with clamped indices, so that each batch is in
  // flight together (a guarded load in a runtime loop waits once per element)
  constexpr int LBT = 8;
  for (int idx0 = i; idx0 < ll; idx0 += LBT * TR) {
    double v[LBT];
#pragma unroll
    for (int u = 0; u < LBT; ++u) v[u] = Rg[min(idx0 + u * TR, ll - 1)];
#pragma unroll
    for (int u = 0; u < LBT; ++u)
      if (idx0 + u * TR < ll) Ri[idx0 + u * TR] = v[u];
  }
  double* yi = S + i * gp;
  const int lrow = valid ? i : rows - 1;
  for (int c0 = 0; c0 < l; c0 += LBT) {
    T v[LBT];
#pragma unroll
    for (int u = 0; u < LBT; ++u) v[u] = Y[lrow + (int64_t)min(c0 + u, l - 1) * ldy];
#pragma unroll
    for (int u = 0; u < LBT; ++u)
      if (c0 + u < l) yi[c0 + u] = valid ? (double)v[u] : 0.0;
  }
  __syncthreads();
  for (int c = l - 1; c >= 0; --c) {
    double t0 = 0.0, t1 = 0.0;
    int a = 0;
#pragma unroll 4
    for (; a + 1 <= c; a += 2) {
      t0 = fma(yi[a], Ri[a * l + c], t0);
      t1 = fma(yi[a + 1], Ri[(a + 1) * l + c], t1);
    }
    if (a <= c) t0 = fma(yi[a], Ri[a * l + c], t0);
    yi[c] = t0 + t1;
  }
  for (int c = 0; c < l; ++c)
    if (valid) Y[i + (int64_t)c * ldy] = (T)yi[c];
  if (gout) {
    if (!std::is_same<T, double>::value)  // the Gram of the stored (rounded) values
      for (int c = 0; c < l; ++c) yi[c] = (double)(T)yi[c];
    __syncthreads();
    tile_gram_mfma(S, gp, 1, rows, l, gout);
  }
}

size_t orth_lds_bytes(int l) {  // fused (l <= 64): TR x gp; apply (l > 64): l^2 + TR x gp
  const size_t t = (size_t)TR * (l + 1);
  if (l <= 64) return t * 8;
  return ((size_t)l * l + t) * 8;
}
size_t factor_lds_bytes(int l) { return (2 * (size_t)l * (l + 1) + (size_t)(l + 1)) * 8; }

}  // namespace

template <typename T>
int launch_orth_apply(T* Y, int which, const SliceDesc* sd, const int2* wk, const int2* items, int nitems, int lmax,
                      int nslices, double* gin, double* gout, hipStream_t s) {
  if (lmax > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  if (nitems == 0 || nslices == 0) return HT_OK;
  auto tiles = [&](auto kern, int lb) -> int {
    int rc = ensure_dynamic_lds((const void*)kern, orth_lds_bytes(lb));
    if (rc) return rc;
    hipLaunchKernelGGL(kern, dim3((unsigned)nitems), dim3(TR), orth_lds_bytes(std::min(lmax, lb)), s, Y, which, sd,
                       wk, items, gin, gout);
    HT_CHECK_LAUNCH();
    return HT_OK;
  };
  if (lmax <= 16) return tiles(k_orth_fused<T, 16>, 16);
  if (lmax <= 32) return tiles(k_orth_fused<T, 32>, 32);
  if (lmax <= 48) return tiles(k_orth_fused<T, 48>, 48);
  int rc = tiles(k_orth_fused<T, 64>, 64);
  if (rc || lmax <= 64) return rc;
  // slices wider than 64 factor once per slice, then apply per tile
  rc = ensure_dynamic_lds((const void*)k_orth_factor<80>, factor_lds_bytes(HT_MAX_WIDTH));
  if (rc) return rc;
  hipLaunchKernelGGL(k_orth_factor<80>, dim3((unsigned)nslices), dim3(256), factor_lds_bytes(lmax), s, which, sd, wk,
                     gin);
  HT_CHECK_LAUNCH();
  return tiles(k_orth_apply<T>, HT_MAX_WIDTH);
}

template int launch_orth_apply<float>(float*, int, const SliceDesc*, const int2*, const int2*, int, int, int, double*,
                                      double*, hipStream_t);
template int launch_orth_apply<double>(double*, int, const SliceDesc*, const int2*, const int2*, int, int, int,
                                       double*, double*, hipStream_t);

}  // namespace ht
