// Thin batched products of the sketch: Y = A W, Z = A^T Q, C = X W^T.
//
// Each face slice A_j is a column-major n1 x n2 block; the thin factors are
// column-major with l <= 128 columns.  The kernels tile the long dimension in
// 64-row (or 64-column) blocks per workgroup, stage a K-chunk of both operands
// in LDS and accumulate in the storage precision (FP32 for float, FP64 for
// double).  One pass reads every slice exactly once.  Optionally the epilogue
// also writes, per output tile, the FP64 Gram matrix of the tile's rows as
// stored (rounded to the storage type), so that the orthonormalization of the
// thin result needs no extra pass over it.
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
  tile_gram_to_global(S, gp, TM, l, out);
}

template <typename T, int LB>
__global__ __launch_bounds__(256) void k_gemm_nn(const T* __restrict__ A, int64_t sA, int lda,
                                                 const T* __restrict__ W, int64_t sW, int ldw, T* __restrict__ Y,
                                                 int64_t sY, int ldy, int m, int kd, int l, double* __restrict__ gpart) {
  constexpr int CPT = LB / 4;
  __shared__ __align__(16) unsigned char smem[gemm_lds_bytes<T, LB>()];
  T(*As)[TM + 1] = reinterpret_cast<T(*)[TM + 1]>(smem);
  T(*Ws)[LB] = reinterpret_cast<T(*)[LB]>(smem + sizeof(T) * KC * (TM + 1));
  const int j = blockIdx.y;
  const int row0 = blockIdx.x * TM;
  const T* Aj = A + (int64_t)j * sA;
  const T* Wj = W + (int64_t)j * sW;
  T* Yj = Y + (int64_t)j * sY;
  const int tr = threadIdx.x % TM, tc = threadIdx.x / TM;
  T acc[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) acc[i] = T(0);
  for (int k0 = 0; k0 < kd; k0 += KC) {
    for (int idx = threadIdx.x; idx < KC * TM; idx += 256) {
      const int kk = idx / TM, rr = idx % TM;
      const int gr = row0 + rr, gk = k0 + kk;
      As[kk][rr] = (gr < m && gk < kd) ? Aj[gr + (int64_t)gk * lda] : T(0);
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
    tile_gram_epilogue<T, LB>(smem, acc, tr, tc, m - row0, l,
                              gpart + ((int64_t)j * gridDim.x + blockIdx.x) * (int64_t)l * l);
}

template <typename T, int LB>
__global__ __launch_bounds__(256) void k_gemm_tn(const T* __restrict__ A, int64_t sA, int lda,
                                                 const T* __restrict__ Q, int64_t sQ, int ldq, T* __restrict__ Z,
                                                 int64_t sZ, int ldz, int m, int n, int l, double* __restrict__ gpart) {
  constexpr int CPT = LB / 4;
  __shared__ __align__(16) unsigned char smem[gemm_lds_bytes<T, LB>()];
  T(*As)[TM + 1] = reinterpret_cast<T(*)[TM + 1]>(smem);
  T(*Qs)[LB] = reinterpret_cast<T(*)[LB]>(smem + sizeof(T) * KC * (TM + 1));
  const int j = blockIdx.y;
  const int col0 = blockIdx.x * TM;
  const T* Aj = A + (int64_t)j * sA;
  const T* Qj = Q + (int64_t)j * sQ;
  T* Zj = Z + (int64_t)j * sZ;
  const int tcol = threadIdx.x % TM, tc = threadIdx.x / TM;
  T acc[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) acc[i] = T(0);
  for (int k0 = 0; k0 < m; k0 += KC) {
    for (int idx = threadIdx.x; idx < KC * TM; idx += 256) {
      const int kk = idx % KC, cc = idx / KC;
      const int gk = k0 + kk, gc = col0 + cc;
      As[kk][cc] = (gk < m && gc < n) ? Aj[gk + (int64_t)gc * lda] : T(0);
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
    tile_gram_epilogue<T, LB>(smem, acc, tcol, tc, n - col0, l,
                              gpart + ((int64_t)j * gridDim.x + blockIdx.x) * (int64_t)l * l);
}

// C_j (m x n) = X_j (m x l) W_j^T with W_j n x l: 64 x 64 output tile per
// workgroup, 4 x 4 outputs per thread, K = l in chunks of 16.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_nt(const T* __restrict__ X, int64_t sX, int ldx,
                                                 const T* __restrict__ W, int64_t sW, int ldw, T* __restrict__ C,
                                                 int64_t sC, int ldc, int m, int n, int l) {
  constexpr int KN = 16;
  __shared__ T Xs[KN][64];
  __shared__ T Ws[KN][64];
  const int j = blockIdx.z;
  const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
  const T* Xj = X + (int64_t)j * sX;
  const T* Wj = W + (int64_t)j * sW;
  T* Cj = C + (int64_t)j * sC;
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

#define HT_WIDTH_DISPATCH(l, KERNEL, ...)                                      \
  do {                                                                         \
    if ((l) <= 16)                                                             \
      hipLaunchKernelGGL((KERNEL<T, 16>), __VA_ARGS__);                        \
    else if ((l) <= 32)                                                        \
      hipLaunchKernelGGL((KERNEL<T, 32>), __VA_ARGS__);                        \
    else if ((l) <= 48)                                                        \
      hipLaunchKernelGGL((KERNEL<T, 48>), __VA_ARGS__);                        \
    else if ((l) <= 64)                                                        \
      hipLaunchKernelGGL((KERNEL<T, 64>), __VA_ARGS__);                        \
    else                                                                       \
      hipLaunchKernelGGL((KERNEL<T, 80>), __VA_ARGS__);                        \
  } while (0)

template <typename T>
int launch_gemm_nn(const T* A, int64_t sA, int lda, const T* W, int64_t sW, int ldw, T* Y, int64_t sY, int ldy,
                   int m, int kd, int l, int P, double* gpart, hipStream_t s) {
  if (l > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  dim3 grid((unsigned)ceil_div(m, TM), (unsigned)P);
  HT_WIDTH_DISPATCH(l, k_gemm_nn, grid, dim3(256), 0, s, A, sA, lda, W, sW, ldw, Y, sY, ldy, m, kd, l, gpart);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template <typename T>
int launch_gemm_tn(const T* A, int64_t sA, int lda, const T* Q, int64_t sQ, int ldq, T* Z, int64_t sZ, int ldz,
                   int m, int n, int l, int P, double* gpart, hipStream_t s) {
  if (l > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  dim3 grid((unsigned)ceil_div(n, TM), (unsigned)P);
  HT_WIDTH_DISPATCH(l, k_gemm_tn, grid, dim3(256), 0, s, A, sA, lda, Q, sQ, ldq, Z, sZ, ldz, m, n, l, gpart);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template <typename T>
int launch_gemm_nt(const T* X, int64_t sX, int ldx, const T* W, int64_t sW, int ldw, T* C, int64_t sC, int ldc,
                   int m, int n, int l, int P, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(m, 64), (unsigned)ceil_div(n, 64), (unsigned)P);
  hipLaunchKernelGGL(k_gemm_nt<T>, grid, dim3(256), 0, s, X, sX, ldx, W, sW, ldw, C, sC, ldc, m, n, l);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

#define HT_INST(T)                                                                                              \
  template int launch_gemm_nn<T>(const T*, int64_t, int, const T*, int64_t, int, T*, int64_t, int, int, int, int, \
                                 int, double*, hipStream_t);                                                    \
  template int launch_gemm_tn<T>(const T*, int64_t, int, const T*, int64_t, int, T*, int64_t, int, int, int, int, \
                                 int, double*, hipStream_t);                                                    \
  template int launch_gemm_nt<T>(const T*, int64_t, int, const T*, int64_t, int, T*, int64_t, int, int, int, int, \
                                 int, hipStream_t);
HT_INST(float)
HT_INST(double)

}  // namespace ht
