// Orthonormalization of the tall-skinny sketches by CholeskyQR with deflation.
//
// The product that made Y (m x l per slice) already wrote the FP64 Gram
// partials of its 64-row tiles.  Here one wavefront per (slice, 64-row tile)
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
// One pass of this CholeskyQR gives a basis whose span is exact to rounding and
// whose orthogonality error is O(u_64 kappa(Y)^2); that suffices inside the
// power iterations, where only the span matters.  For the final basis the
// kernel also writes the Gram partials of Q, and the second CholeskyQR step is
// applied in the l x l space by the small-SVD kernel.
#include "chol.hpp"

namespace ht {

namespace {

constexpr int TR = 64;  // rows per workgroup (matches the producing products); one lane per row

// Register path (l <= 64): lane b sums column b of G from the partials and
// the factorization runs in registers; lane i then owns row i of the tile and
// solves q R = y with the rows of R broadcast by readlane.
template <typename T, int LB>
__global__ __launch_bounds__(TR) void k_orth_apply_regs(T* __restrict__ Yall, int64_t sY, int ldy, int m, int l,
                                                        const double* __restrict__ gin, int nparts, double* __restrict__ gout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int gp = l + 1;
  double* S = reinterpret_cast<double*>(smem_raw);  // TR x gp (Gram of the result)
  const int j = blockIdx.y, tile = blockIdx.x, ntiles = gridDim.x;
  const int row0 = tile * TR;
  const int rows = min(TR, m - row0);
  T* Y = Yall + (int64_t)j * sY + row0;
  const int lane = threadIdx.x;
  const bool valid = lane < rows;
  const int ll = l * l;

  // column `lane` of G = sum of the tile partials (fixed order)
  const double* part = gin + (int64_t)j * nparts * ll;
  double g[LB];
#pragma unroll
  for (int a = 0; a < LB; ++a) g[a] = 0.0;
  const int bcol = lane < l ? lane : 0;
  for (int t = 0; t < nparts; ++t) {
    double v[LB];
#pragma unroll
    for (int a = 0; a < LB; ++a) v[a] = (a < l) ? part[(int64_t)t * ll + a * l + bcol] : 0.0;
#pragma unroll
    for (int a = 0; a < LB; ++a) g[a] += v[a];
  }
  double y[LB];
#pragma unroll
  for (int c = 0; c < LB; ++c) y[c] = (c < l && valid) ? (double)Y[lane + (int64_t)c * ldy] : 0.0;

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

  // q R = y: q_c = (y_c - sum_{a<c} q_a R[a][c]) / R[c][c]; R[a][c] is g[a] on lane c
#pragma unroll
  for (int c = 0; c < LB; ++c) {
    if (c < l) {
      double t = y[c];
#pragma unroll
      for (int a = 0; a < c; ++a) t -= y[a] * readlane_d(g[a], c);
      const double rcc = readlane_d(g[c], c);
      y[c] = (rcc != 0.0) ? t * fast_rcp(rcc) : 0.0;
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
    tile_gram_to_global(S, gp, TR, l, gout + ((int64_t)j * ntiles + tile) * (int64_t)ll);
  }
}

template <typename T, int LB>
__global__ __launch_bounds__(TR) void k_orth_apply(T* __restrict__ Yall, int64_t sY, int ldy, int m, int l,
                                                   const double* __restrict__ gin, int nparts, double* __restrict__ gout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int gp = l + 1;
  double* G = reinterpret_cast<double*>(smem_raw);  // l x gp
  double* dR = G + (size_t)l * gp;                  // gp
  double* S = dR + gp;                               // TR x gp (Gram of the result)
  __shared__ double s_scratch;
  const int j = blockIdx.y, tile = blockIdx.x, ntiles = gridDim.x;
  const int row0 = tile * TR;
  const int rows = min(TR, m - row0);
  T* Y = Yall + (int64_t)j * sY + row0;
  const int i = threadIdx.x;
  const bool valid = i < rows;

  sum_gram_partials(G, gp, gin + (int64_t)j * nparts * l * l, nparts, l);
  double y[LB];
#pragma unroll
  for (int c = 0; c < LB; ++c) y[c] = (c < l && valid) ? (double)Y[i + (int64_t)c * ldy] : 0.0;
  __syncthreads();
  chol_deflate(G, dR, gp, l, 8.0 * (double)m * 2.220446049250313e-16, &s_scratch);

  // q R = y: q_c = (y_c - sum_{a<c} q_a R[a][c]) / R[c][c]; skipped columns give q_c = 0
#pragma unroll
  for (int c = 0; c < LB; ++c) {
    if (c < l) {
      double t = y[c];
#pragma unroll
      for (int a = 0; a < c; ++a) t -= y[a] * G[c * gp + a];  // R[a][c], stored transposed
      const double r = dR[c];
      y[c] = (r != 0.0) ? t / r : 0.0;
    }
  }
#pragma unroll
  for (int c = 0; c < LB; ++c) {
    if (c < l) {
      const T v = (T)y[c];
      if (valid) Y[i + (int64_t)c * ldy] = v;
      if (gout) S[i * gp + c] = valid ? (double)v : 0.0;
    }
  }
  if (gout) {
    __syncthreads();
    tile_gram_to_global(S, gp, TR, l, gout + ((int64_t)j * ntiles + tile) * (int64_t)l * l);
  }
}

size_t orth_lds_bytes(int l) { return ((size_t)l * (l + 1) + (size_t)(l + 1) + (size_t)TR * (l + 1)) * 8; }

}  // namespace

template <typename T>
int launch_orth_apply(T* Y, int64_t sY, int ldy, int m, int l, int P, const double* gin, int nparts, double* gout,
                      hipStream_t s) {
  if (l > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  const size_t lds = orth_lds_bytes(l);
  const dim3 grid((unsigned)ceil_div(m, TR), (unsigned)P);
  auto launch = [&](auto kern) -> int {
    int rc = ensure_dynamic_lds((const void*)kern, orth_lds_bytes(HT_MAX_WIDTH));
    if (rc) return rc;
    hipLaunchKernelGGL(kern, grid, dim3(TR), lds, s, Y, sY, ldy, m, l, gin, nparts, gout);
    HT_CHECK_LAUNCH();
    return HT_OK;
  };
  if (l <= 16) return launch(k_orth_apply_regs<T, 16>);
  if (l <= 32) return launch(k_orth_apply_regs<T, 32>);
  if (l <= 48) return launch(k_orth_apply_regs<T, 48>);
  if (l <= 64) return launch(k_orth_apply_regs<T, 64>);
  return launch(k_orth_apply<T, 80>);
}

template int launch_orth_apply<float>(float*, int64_t, int, int, int, int, const double*, int, double*, hipStream_t);
template int launch_orth_apply<double>(double*, int64_t, int, int, int, int, const double*, int, double*,
                                       hipStream_t);

}  // namespace ht
