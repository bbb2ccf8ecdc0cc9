// Orthonormalization of the tall-skinny sketches by CholeskyQR with deflation.
//
// For one slice's Y (m x l): G = Y^T Y in FP64, R = chol(G), Q = Y R^{-1}, and
// the same again on Q (CholeskyQR2).  The paper orthonormalizes the Krylov /
// power blocks ("form an orthonormal basis", Alg. 1) and deflates directions
// whose pivot falls below a tolerance (defl-QR, Alg. 2); here the Cholesky
// skips a column whose Schur-complement pivot is below
//   delta = 8 * m * 2^-52 * max_i G_ii
// (its residual against the previous columns is at rounding level), giving a
// zero column of Q and leaving the span of the kept columns intact.
//
// One workgroup per slice; G, R (upper), R^{-1} (stored transposed in the
// lower triangle) and a staging chunk of rows live in LDS in FP64.
#include "kernels.hpp"

namespace ht {

namespace {

constexpr int NT = 256;
constexpr size_t LDS_BUDGET = 160000;

__host__ __device__ inline int cholqr_chunk_rows(int l) {
  const size_t g = (size_t)l * (l + 1) * 8 + (size_t)(l + 1) * 8;
  const size_t avail = LDS_BUDGET > g ? LDS_BUDGET - g : 0;
  int ch = (int)(avail / ((size_t)(l + 1) * 8));
  if (ch > 64) ch = 64;
  return ch;
}

template <typename T, int LB>
__global__ __launch_bounds__(NT) void k_cholqr(T* __restrict__ Yall, int64_t sY, int ldy, int m, int l, int passes,
                                               int CH) {
  constexpr int NPAIR = (LB * (LB + 1) / 2 + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* G = reinterpret_cast<double*>(smem_raw);  // l x (l+1)
  const int gp = l + 1;
  double* dR = G + (size_t)l * gp;                  // l (+1)
  double* S = dR + gp;                               // CH x (l+1)
  __shared__ double s_maxdiag;
  T* Y = Yall + (int64_t)blockIdx.x * sY;
  const int tid = threadIdx.x;

  // pairs (a <= b) owned by this thread for the Gram accumulation
  int pa[NPAIR], pb[NPAIR];
  const int npairs = l * (l + 1) / 2;
#pragma unroll
  for (int s = 0; s < NPAIR; ++s) {
    int p = tid + s * NT;
    int a = 0, b = -1;
    if (p < npairs) {
      int row_len = l;
      while (p >= row_len) {
        p -= row_len;
        ++a;
        --row_len;
      }
      b = a + p;
    }
    pa[s] = a;
    pb[s] = b;
  }

  for (int pass = 0; pass < passes; ++pass) {
    // ---- Gram G = Y^T Y (FP64) --------------------------------------------
    double acc[NPAIR];
#pragma unroll
    for (int s = 0; s < NPAIR; ++s) acc[s] = 0.0;
    for (int r0 = 0; r0 < m; r0 += CH) {
      const int ch = min(CH, m - r0);
      for (int idx = tid; idx < ch * l; idx += NT) {
        const int i = idx % ch, c = idx / ch;
        S[i * gp + c] = (double)Y[(r0 + i) + (int64_t)c * ldy];
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < NPAIR; ++s) {
        if (pb[s] >= 0) {
          const double* sa = S + pa[s];
          const double* sb = S + pb[s];
          double t = 0.0;
          for (int i = 0; i < ch; ++i) t += sa[i * gp] * sb[i * gp];
          acc[s] += t;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < NPAIR; ++s)
      if (pb[s] >= 0) {
        G[pa[s] * gp + pb[s]] = acc[s];
        G[pb[s] * gp + pa[s]] = acc[s];
      }
    __syncthreads();
    if (tid == 0) {
      double md = 0.0;
      for (int a = 0; a < l; ++a) md = fmax(md, G[a * gp + a]);
      s_maxdiag = md;
    }
    __syncthreads();
    const double delta = 8.0 * (double)m * 2.220446049250313e-16 * s_maxdiag;

    // ---- Cholesky with deflation: R in the strict upper triangle, diag in dR
    for (int j = 0; j < l; ++j) {
      const double d = G[j * gp + j];
      const bool keep = d > delta && s_maxdiag > 0.0;
      const double rjj = keep ? sqrt(d) : 0.0;
      for (int c = j + 1 + tid; c < l; c += NT) G[j * gp + c] = keep ? G[j * gp + c] / rjj : 0.0;
      if (tid == 0) dR[j] = rjj;
      __syncthreads();
      if (keep) {
        const int w = l - j - 1;
        for (int idx = tid; idx < w * w; idx += NT) {
          const int a = j + 1 + idx / w, b = j + 1 + idx % w;
          if (b >= a) G[a * gp + b] -= G[j * gp + a] * G[j * gp + b];
        }
      }
      __syncthreads();
    }

    // ---- R^{-1}: column c by back substitution, stored as row c of the lower triangle
    for (int c = tid; c < l; c += NT) {
      if (dR[c] == 0.0) {
        for (int a = 0; a <= c; ++a) G[c * gp + a] = 0.0;
      } else {
        G[c * gp + c] = 1.0 / dR[c];
        for (int a = c - 1; a >= 0; --a) {
          if (dR[a] == 0.0) {
            G[c * gp + a] = 0.0;
            continue;
          }
          double s = 0.0;
          for (int b = a + 1; b <= c; ++b) s += G[a * gp + b] * G[c * gp + b];
          G[c * gp + a] = -s / dR[a];
        }
      }
    }
    __syncthreads();

    // ---- Q = Y R^{-1}, in place, chunk by chunk -----------------------------
    for (int r0 = 0; r0 < m; r0 += CH) {
      const int ch = min(CH, m - r0);
      for (int idx = tid; idx < ch * l; idx += NT) {
        const int i = idx % ch, c = idx / ch;
        S[i * gp + c] = (double)Y[(r0 + i) + (int64_t)c * ldy];
      }
      __syncthreads();
      for (int idx = tid; idx < ch * l; idx += NT) {
        const int i = idx % ch, c = idx / ch;
        const double* srow = S + i * gp;
        const double* rinv = G + c * gp;
        double t = 0.0;
        for (int a = 0; a <= c; ++a) t += srow[a] * rinv[a];
        Y[(r0 + i) + (int64_t)c * ldy] = (T)t;
      }
      __syncthreads();
    }
  }
}

}  // namespace

template <typename T>
int launch_cholqr(T* Y, int64_t sY, int ldy, int m, int l, int P, int passes, hipStream_t s) {
  if (l > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  const int CH = cholqr_chunk_rows(l);
  const size_t lds = ((size_t)l * (l + 1) + (size_t)(l + 1) + (size_t)CH * (l + 1)) * sizeof(double);
  auto launch = [&](auto kern) -> int {
    HT_CHECK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3((unsigned)P), dim3(NT), lds, s, Y, sY, ldy, m, l, passes, CH);
    HT_CHECK_LAUNCH();
    return HT_OK;
  };
  if (l <= 16) return launch(k_cholqr<T, 16>);
  if (l <= 32) return launch(k_cholqr<T, 32>);
  if (l <= 48) return launch(k_cholqr<T, 48>);
  if (l <= 64) return launch(k_cholqr<T, 64>);
  return launch(k_cholqr<T, 80>);
}

template int launch_cholqr<float>(float*, int64_t, int, int, int, int, int, hipStream_t);
template int launch_cholqr<double>(double*, int64_t, int, int, int, int, int, hipStream_t);

}  // namespace ht
