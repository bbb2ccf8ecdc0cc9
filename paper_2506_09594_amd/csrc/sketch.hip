// Thin products on the vector ALUs: the FP64 sketch products and the
// reconstruction products of every precision.
//
//   sketch nn:  Y_s (n1 x l) = A_s (n1 x n2) W_s (n2 x l)
//   sketch tn:  Z_s (n2 x l) = A_s^T Q_s
//   recon nn:   (Q1 K')_s (n1 x l) = Q1_s (n1 x l) K'_s (l x l)
//   recon nt:   C_s (n1 x n2) = (Q1 K')_s Bt_s^T
//
// Every (real) slice is a column-major block found through the slice table; one
// workgroup per work item (slice, 64-row tile) stages a K-chunk of both
// operands in LDS and accumulates in the storage precision.  One pass reads
// every slice once.  Optionally the epilogue also writes, per output tile, the
// FP64 Gram matrix of the tile's rows as stored, so that the orthonormalization
// of the thin result needs no extra pass over it.
#include "chol.hpp"

namespace ht {

namespace {

constexpr int TM = 64;  // rows (or columns of A) per workgroup
constexpr int KC = 32;  // K chunk staged in LDS

template <typename T, int LB>
constexpr size_t gemm_lds_bytes() {
  constexpr size_t main = sizeof(T) * (KC * (TM + 1) + KC * LB);
  constexpr size_t epi = sizeof(double) * TM * (LB + 1);
  return main > epi ? main : epi;
}

// Epilogue: Gram partial of the 64 x l output tile held in registers acc[i] at
// (row tr, column tc + 4 i).  Rows beyond the matrix contribute zero.
template <typename T, int LB>
__device__ inline void tile_gram_epilogue(unsigned char* smem, const T* acc, int tr, int tc, int rows, int l,
                                          double* __restrict__ out) {
  constexpr int CPT = LB / 4;
  double* S = reinterpret_cast<double*>(smem);
  const int gp = LB + 1;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int c = tc + 4 * i;
    if (c < l) S[tr * gp + c] = (tr < rows) ? (double)acc[i] : 0.0;
  }
  __syncthreads();
  tile_gram_mfma(S, gp, 1, rows < TM ? rows : TM, l, out);
}

// RECON = false: Y = A W (sketch); RECON = true: QK = Q1 K'.
template <typename T, int LB, bool RECON>
__global__ __launch_bounds__(256) void k_gemm_nn(const T* __restrict__ Aall, const T* __restrict__ Wall,
                                                 T* __restrict__ Yall, const SliceDesc* __restrict__ sd,
                                                 const int2* __restrict__ wk, const int2* __restrict__ items,
                                                 double* __restrict__ gpart) {
  constexpr int CPT = LB / 4;
  __shared__ __align__(16) unsigned char smem[gemm_lds_bytes<T, LB>()];
  T(*As)[TM + 1] = reinterpret_cast<T(*)[TM + 1]>(smem);
  T(*Ws)[LB] = reinterpret_cast<T(*)[LB]>(smem + sizeof(T) * KC * (TM + 1));
  const int2 item = items[blockIdx.x];
  const int s = item.x, row0 = item.y;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int m = d.n1, kd = RECON ? l : d.n2;
  const int lda = d.n1, ldw = RECON ? l : d.n2, ldy = d.n1;
  const T* Aj = Aall + (RECON ? d.y : d.a);
  const T* Wj = Wall + (RECON ? d.kq : d.z);
  T* Yj = Yall + d.y;
  const int tr = threadIdx.x % TM, tc = threadIdx.x / TM;
  T acc[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) acc[i] = T(0);
  for (int k0 = 0; k0 < kd; k0 += KC) {
    for (int idx = threadIdx.x; idx < KC * TM; idx += 256) {
      const int kk = idx / TM, rr = idx % TM;
      const int gr = row0 + rr, gk = k0 + kk;
      T v = T(0);
      if (gr < m && gk < kd) v = Aj[gr + (int64_t)gk * lda];
      As[kk][rr] = v;
    }
    for (int idx = threadIdx.x; idx < KC * LB; idx += 256) {
      const int c = idx / KC, kk = idx % KC;
      const int gk = k0 + kk;
      Ws[kk][c] = (c < l && gk < kd) ? Wj[gk + (int64_t)c * ldw] : T(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      const T a = As[kk][tr];
#pragma unroll
      for (int i = 0; i < CPT; ++i) acc[i] += a * Ws[kk][tc + 4 * i];
    }
    __syncthreads();
  }
  const int gr = row0 + tr;
  if (gr < m) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int c = tc + 4 * i;
      if (c < l) Yj[gr + (int64_t)c * ldy] = acc[i];
    }
  }
  if (gpart)
    tile_gram_epilogue<T, LB>(smem, acc, tr, tc, m - row0, l, gpart + d.g1 + (int64_t)(row0 / TM) * l * l);
}

template <typename T, int LB>
__global__ __launch_bounds__(256) void k_gemm_tn(const T* __restrict__ Aall, const T* __restrict__ Qall,
                                                 T* __restrict__ Zall, const SliceDesc* __restrict__ sd,
                                                 const int2* __restrict__ wk, const int2* __restrict__ items,
                                                 double* __restrict__ gpart) {
  constexpr int CPT = LB / 4;
  __shared__ __align__(16) unsigned char smem[gemm_lds_bytes<T, LB>()];
  T(*As)[TM + 1] = reinterpret_cast<T(*)[TM + 1]>(smem);
  T(*Qs)[LB] = reinterpret_cast<T(*)[LB]>(smem + sizeof(T) * KC * (TM + 1));
  const int2 item = items[blockIdx.x];
  const int s = item.x, col0 = item.y;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int m = d.n1, n = d.n2;
  const int lda = m, ldq = m, ldz = n;
  const T* Aj = Aall + d.a;
  const T* Qj = Qall + d.y;
  T* Zj = Zall + d.z;
  const int tcol = threadIdx.x % TM, tc = threadIdx.x / TM;
  T acc[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) acc[i] = T(0);
  for (int k0 = 0; k0 < m; k0 += KC) {
    for (int idx = threadIdx.x; idx < KC * TM; idx += 256) {
      const int kk = idx % KC, cc = idx / KC;
      const int gk = k0 + kk, gc = col0 + cc;
      T v = T(0);
      if (gk < m && gc < n) v = Aj[gk + (int64_t)gc * lda];
      As[kk][cc] = v;
    }
    for (int idx = threadIdx.x; idx < KC * LB; idx += 256) {
      const int kk = idx % KC, c = idx / KC;
      const int gk = k0 + kk;
      Qs[kk][c] = (c < l && gk < m) ? Qj[gk + (int64_t)c * ldq] : T(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      const T a = As[kk][tcol];
#pragma unroll
      for (int i = 0; i < CPT; ++i) acc[i] += a * Qs[kk][tc + 4 * i];
    }
    __syncthreads();
  }
  const int gc = col0 + tcol;
  if (gc < n) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int c = tc + 4 * i;
      if (c < l) Zj[gc + (int64_t)c * ldz] = acc[i];
    }
  }
  if (gpart)
    tile_gram_epilogue<T, LB>(smem, acc, tcol, tc, n - col0, l, gpart + d.g1 + (int64_t)(col0 / TM) * l * l);
}

// C_s (n1 x n2) = X_s (n1 x l) W_s^T with W_s n2 x l: 64 x 64 output tile per
// work item (slice, tile index; row tiles fastest), 4 x 4 outputs per thread,
// K = l in chunks of 16.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nt(const T* __restrict__ Xall, const T* __restrict__ Wall,
                                                 T* __restrict__ Call, const SliceDesc* __restrict__ sd,
                                                 const int2* __restrict__ wk, const int2* __restrict__ items) {
  constexpr int KN = 16;
  __shared__ T Xs[KN][64];
  __shared__ T Ws[KN][64];
  const int2 item = items[blockIdx.x];
  const int s = item.x;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int m = d.n1, n = d.nc;
  const int nrt = (m + 63) / 64;
  const int row0 = (item.y % nrt) * 64, col0 = (item.y / nrt) * 64;
  const T* Xj = Xall + d.y;
  const T* Wj = Wall + d.z;
  T* Cj = Call + d.a;
  const int ldx = m, ldw = d.n2, ldc = m;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
  for (int c0 = 0; c0 < l; c0 += KN) {
    for (int idx = threadIdx.x; idx < KN * 64; idx += 256) {
      const int kk = idx / 64, rr = idx % 64;
      const int gc = c0 + kk;
      Xs[kk][rr] = (gc < l && row0 + rr < m) ? Xj[(row0 + rr) + (int64_t)gc * ldx] : T(0);
      Ws[kk][rr] = (gc < l && col0 + rr < n) ? Wj[(col0 + rr) + (int64_t)gc * ldw] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KN; ++kk) {
      T xa[4], wb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xa[a] = Xs[kk][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) wb[b] = Ws[kk][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += xa[a] * wb[b];
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int gc = col0 + ty + 16 * b;
    if (gc >= n) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int gr = row0 + tx + 16 * a;
      if (gr < m) Cj[gr + (int64_t)gc * ldc] = acc[a][b];
    }
  }
}

}  // namespace

template <typename T>
int launch_gemm_nn(const T* A, const T* W, T* Y, const SliceDesc* sd, const int2* wk, const int2* items, int nitems,
                   int lmax, double* gpart, hipStream_t s) {
  if (lmax > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  if (nitems == 0) return HT_OK;
  const dim3 grid((unsigned)nitems);
  if (lmax <= 16)
    hipLaunchKernelGGL((k_gemm_nn<T, 16, false>), grid, dim3(256), 0, s, A, W, Y, sd, wk, items, gpart);
  else if (lmax <= 32)
    hipLaunchKernelGGL((k_gemm_nn<T, 32, false>), grid, dim3(256), 0, s, A, W, Y, sd, wk, items, gpart);
  else if (lmax <= 48)
    hipLaunchKernelGGL((k_gemm_nn<T, 48, false>), grid, dim3(256), 0, s, A, W, Y, sd, wk, items, gpart);
  else if (lmax <= 64)
    hipLaunchKernelGGL((k_gemm_nn<T, 64, false>), grid, dim3(256), 0, s, A, W, Y, sd, wk, items, gpart);
  else
    hipLaunchKernelGGL((k_gemm_nn<T, 80, false>), grid, dim3(256), 0, s, A, W, Y, sd, wk, items, gpart);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template <typename T>
int launch_recon_qk(const T* Q, const T* K, T* QK, const SliceDesc* sd, const int2* wk, const int2* items, int nitems,
                    int lmax, hipStream_t s) {
  if (lmax > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  if (nitems == 0) return HT_OK;
  const dim3 grid((unsigned)nitems);
  double* const none = nullptr;
  if (lmax <= 16)
    hipLaunchKernelGGL((k_gemm_nn<T, 16, true>), grid, dim3(256), 0, s, Q, K, QK, sd, wk, items, none);
  else if (lmax <= 32)
    hipLaunchKernelGGL((k_gemm_nn<T, 32, true>), grid, dim3(256), 0, s, Q, K, QK, sd, wk, items, none);
  else if (lmax <= 48)
    hipLaunchKernelGGL((k_gemm_nn<T, 48, true>), grid, dim3(256), 0, s, Q, K, QK, sd, wk, items, none);
  else if (lmax <= 64)
    hipLaunchKernelGGL((k_gemm_nn<T, 64, true>), grid, dim3(256), 0, s, Q, K, QK, sd, wk, items, none);
  else
    hipLaunchKernelGGL((k_gemm_nn<T, 80, true>), grid, dim3(256), 0, s, Q, K, QK, sd, wk, items, none);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template <typename T>
int launch_gemm_tn(const T* A, const T* Q, T* Z, const SliceDesc* sd, const int2* wk, const int2* items, int nitems,
                   int lmax, double* gpart, hipStream_t s) {
  if (lmax > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  if (nitems == 0) return HT_OK;
  const dim3 grid((unsigned)nitems);
  if (lmax <= 16)
    hipLaunchKernelGGL((k_gemm_tn<T, 16>), grid, dim3(256), 0, s, A, Q, Z, sd, wk, items, gpart);
  else if (lmax <= 32)
    hipLaunchKernelGGL((k_gemm_tn<T, 32>), grid, dim3(256), 0, s, A, Q, Z, sd, wk, items, gpart);
  else if (lmax <= 48)
    hipLaunchKernelGGL((k_gemm_tn<T, 48>), grid, dim3(256), 0, s, A, Q, Z, sd, wk, items, gpart);
  else if (lmax <= 64)
    hipLaunchKernelGGL((k_gemm_tn<T, 64>), grid, dim3(256), 0, s, A, Q, Z, sd, wk, items, gpart);
  else
    hipLaunchKernelGGL((k_gemm_tn<T, 80>), grid, dim3(256), 0, s, A, Q, Z, sd, wk, items, gpart);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template <typename T>
int launch_gemm_nt(const T* X, const T* W, T* C, const SliceDesc* sd, const int2* wk, const int2* items, int nitems,
                   hipStream_t s) {
  if (nitems == 0) return HT_OK;
  hipLaunchKernelGGL(k_gemm_nt<T>, dim3((unsigned)nitems), dim3(256), 0, s, X, W, C, sd, wk, items);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

#define HT_INST(T)                                                                                                  \
  template int launch_gemm_nn<T>(const T*, const T*, T*, const SliceDesc*, const int2*, const int2*, int, int,     \
                                 double*, hipStream_t);                                                             \
  template int launch_recon_qk<T>(const T*, const T*, T*, const SliceDesc*, const int2*, const int2*, int, int,    \
                                  hipStream_t);                                                                     \
  template int launch_gemm_tn<T>(const T*, const T*, T*, const SliceDesc*, const int2*, const int2*, int, int,     \
                                 double*, hipStream_t);                                                             \
  template int launch_gemm_nt<T>(const T*, const T*, T*, const SliceDesc*, const int2*, const int2*, int,          \
                                 hipStream_t);
HT_INST(float)
HT_INST(double)

}  // namespace ht
