// Small projected SVD and shrinkage, one workgroup per slice, FP64.
//
// With Bt = A_j^T Q (n x l), the projected matrix is B = Bt^T = U_B diag(s) V_B^T.
// Its left singular pairs are the eigenpairs of W = B B^T = Bt^T Bt (l x l),
// which is formed in FP64 and diagonalized by the parallel cyclic Jacobi
// method (round-robin pair ordering, l/2 disjoint rotations per step).  With
// s_i = sqrt(lambda_i) in descending order and k = min(r, l) kept values, the
// shrunk reconstruction Q U_B[:, :k] diag(prox(s)) V_B[:, :k]^T equals
//   Q K B   with  K = U_B diag(w) U_B^T,  w_i = prox(s_i)/s_i (i < k), 0 otherwise,
// since V_B[:, i]^T = U_B[:, i]^T B / s_i.  The kernel writes K (l x l).
#include "kernels.hpp"

namespace ht {

namespace {

constexpr int NT = 256;

struct SvdLds {
  int pitch, CH;
  size_t bytes;
};

__host__ __device__ inline SvdLds svd_lds(int l) {
  SvdLds s;
  s.pitch = l + 1;
  const size_t mats = 2 * (size_t)l * s.pitch * 8;          // W, V
  const size_t small = (size_t)(3 * 64 + 2 * 128) * 8;       // rotations, eigen bookkeeping
  size_t avail = 150000 > mats + small ? 150000 - mats - small : 0;
  int ch = (int)(avail / ((size_t)s.pitch * 8));
  s.CH = ch > 64 ? 64 : ch;
  s.bytes = mats + small + (size_t)s.CH * s.pitch * 8;
  return s;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_smallsvd(const T* __restrict__ Btall, int64_t sB, int ldb, int n, int l,
                                                 int kkeep, double tau_host, const double* __restrict__ mu_dev,
                                                 Penalty pen, T* __restrict__ Kall, double* __restrict__ sigma_out,
                                                 int* __restrict__ kept_out, int CH) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int gp = l + 1;
  double* W = reinterpret_cast<double*>(smem_raw);
  double* V = W + (size_t)l * gp;
  double* rc = V + (size_t)l * gp;  // 64 cosines
  double* rs = rc + 64;             // 64 sines
  int* rp = reinterpret_cast<int*>(rs + 64);  // 64 p, 64 q
  int* rq = rp + 64;
  double* wv = rs + 128;                       // 128 shrink weights (after rp/rq: 64 doubles of room)
  int* perm = reinterpret_cast<int*>(wv + 128);
  double* S = reinterpret_cast<double*>(smem_raw) + 2 * (size_t)l * gp + 3 * 64 + 2 * 128;
  __shared__ int s_rotated;
  __shared__ int s_kept;

  const int j = blockIdx.x;
  const T* Bt = Btall + (int64_t)j * sB;
  const int tid = threadIdx.x;
  const double tau = mu_dev ? 1.0 / (*mu_dev) : tau_host;

  // ---- W = Bt^T Bt (FP64), V = I ------------------------------------------
  for (int idx = tid; idx < l * l; idx += NT) {
    const int a = idx % l, b = idx / l;
    V[a * gp + b] = (a == b) ? 1.0 : 0.0;
  }
  {
    // each thread owns entries (a, b), a <= b, strided over the upper triangle
    const int npairs = l * (l + 1) / 2;
    for (int p0 = 0; p0 < npairs; p0 += NT) {
      int p = p0 + tid;
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
      double acc = 0.0;
      for (int r0 = 0; r0 < n; r0 += CH) {
        const int ch = min(CH, n - r0);
        __syncthreads();
        for (int idx = tid; idx < ch * l; idx += NT) {
          const int i = idx % ch, c = idx / ch;
          S[i * gp + c] = (double)Bt[(r0 + i) + (int64_t)c * ldb];
        }
        __syncthreads();
        if (b >= 0)
          for (int i = 0; i < ch; ++i) acc += S[i * gp + a] * S[i * gp + b];
      }
      if (b >= 0) {
        W[a * gp + b] = acc;
        W[b * gp + a] = acc;
      }
    }
  }
  __syncthreads();

  // ---- parallel cyclic Jacobi ---------------------------------------------
  const int L2 = l + (l & 1);
  const int half = L2 / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) s_rotated = 0;
    __syncthreads();
    for (int step = 0; step < L2 - 1; ++step) {
      if (tid < half) {
        int p, q;
        if (tid == 0) {
          p = L2 - 1;
          q = step;
        } else {
          p = (step + tid) % (L2 - 1);
          q = (step - tid + (L2 - 1)) % (L2 - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < l) {
          const double app = W[p * gp + p], aqq = W[q * gp + q], apq = W[p * gp + q];
          if (fabs(apq) > 1e-300 && fabs(apq) > 1e-17 * sqrt(fabs(app * aqq))) {
            const double theta = (aqq - app) / (2.0 * apq);
            double t;
            if (fabs(theta) > 1e150)
              t = 0.5 / theta;
            else
              t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            s_rotated = 1;
          }
        }
        rc[tid] = c;
        rs[tid] = s;
        rp[tid] = p;
        rq[tid] = (q < l) ? q : -1;
      }
      __syncthreads();
      // rows p, q of W
      for (int idx = tid; idx < half * l; idx += NT) {
        const int t = idx / l, x = idx % l;
        const int q = rq[t];
        if (q < 0 || rs[t] == 0.0) continue;
        const int p = rp[t];
        const double c = rc[t], s = rs[t];
        const double wp = W[p * gp + x], wq = W[q * gp + x];
        W[p * gp + x] = c * wp - s * wq;
        W[q * gp + x] = s * wp + c * wq;
      }
      __syncthreads();
      // columns p, q of W and V
      for (int idx = tid; idx < half * l; idx += NT) {
        const int t = idx / l, x = idx % l;
        const int q = rq[t];
        if (q < 0 || rs[t] == 0.0) continue;
        const int p = rp[t];
        const double c = rc[t], s = rs[t];
        const double wp = W[x * gp + p], wq = W[x * gp + q];
        W[x * gp + p] = c * wp - s * wq;
        W[x * gp + q] = s * wp + c * wq;
        const double vp = V[x * gp + p], vq = V[x * gp + q];
        V[x * gp + p] = c * vp - s * vq;
        V[x * gp + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    if (!s_rotated) break;
    __syncthreads();
  }

  // ---- order eigenvalues, shrink, K = U diag(w) U^T -------------------------
  for (int a = tid; a < l; a += NT) {
    const double la = W[a * gp + a];
    int rank = 0;
    for (int b = 0; b < l; ++b) {
      const double lb = W[b * gp + b];
      rank += (lb > la) || (lb == la && b < a);
    }
    perm[rank] = a;
  }
  if (tid == 0) s_kept = 0;
  __syncthreads();
  for (int i = tid; i < l; i += NT) {
    const double lam = W[perm[i] * gp + perm[i]];
    const double sig = lam > 0.0 ? sqrt(lam) : 0.0;
    double w = 0.0;
    if (i < kkeep && sig > 0.0) {
      const double sh = prox_pos(pen, sig, tau);
      w = sh / sig;
      if (sh > 0.0) atomicAdd(&s_kept, 1);
    }
    wv[i] = w;
    if (sigma_out) sigma_out[(int64_t)j * l + i] = sig;
  }
  __syncthreads();
  T* K = Kall + (int64_t)j * l * l;
  for (int idx = tid; idx < l * l; idx += NT) {
    const int a = idx % l, b = idx / l;
    double t = 0.0;
    for (int i = 0; i < kkeep; ++i) {
      const int e = perm[i];
      t += V[a * gp + e] * wv[i] * V[b * gp + e];
    }
    K[a + (int64_t)b * l] = (T)t;
  }
  if (kept_out && tid == 0) kept_out[j] = s_kept;
}

}  // namespace

template <typename T>
int launch_smallsvd(const T* Bt, int64_t sB, int ldb, int n, int l, int k, int P, double tau, const double* mu_dev,
                    Penalty pen, T* K, double* sigma_out, int* kept_out, hipStream_t s) {
  if (l > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  const SvdLds L = svd_lds(l);
  HT_CHECK_HIP(hipFuncSetAttribute((const void*)k_smallsvd<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)L.bytes));
  hipLaunchKernelGGL(k_smallsvd<T>, dim3((unsigned)P), dim3(NT), L.bytes, s, Bt, sB, ldb, n, l, k, tau, mu_dev, pen,
                     K, sigma_out, kept_out, L.CH);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template int launch_smallsvd<float>(const float*, int64_t, int, int, int, int, int, double, const double*, Penalty,
                                    float*, double*, int*, hipStream_t);
template int launch_smallsvd<double>(const double*, int64_t, int, int, int, int, int, double, const double*, Penalty,
                                     double*, double*, int*, hipStream_t);

}  // namespace ht
