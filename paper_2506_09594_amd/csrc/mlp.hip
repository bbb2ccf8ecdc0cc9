// Learned sketch widths: the rank-predicting MLP (forward, backward, Adam) and
// the per-slice kernels around it.
//
// Network: z = W3 relu(W2 relu(W1 x + b1) + b2) + b3 with x in R^32, two hidden
// layers of 128 units, FP32; z predicts log(1 + s), s the number of singular
// values of a slice that survive the shrinkage.  Parameters are one flat FP32
// vector: W1 (128 x 32, row-major), b1, W2 (128 x 128), b2, W3 (128), b3.
//
// A workgroup of 128 threads (thread j = hidden unit j) takes 32 samples: the
// inputs and both activation layers live in LDS, each thread computes its unit
// for all 32 samples, and the backward pass runs the chain rule through the two
// ReLU layers with every gradient entry owned by one thread.  Gradients of a
// workgroup are accumulated into its own row of a partial buffer (no atomics),
// and a second kernel sums the rows in a fixed order and applies Adam, so a
// training step is deterministic.
//
// Width rule: s = exp(z) - 1, l = clamp(ceil(s) + p, p + 1, l_fix),
// k = min(k_fix, l).  Fallback: a slice sketched at l < l_fix is redone at the
// fixed width when every kept value survived (kept >= k) or when the residual
// certainly holds a value above tau: its energy ||A_j||^2 - ||B_j||^2 (the
// energy identity behind the adaptive stopping test of Alg. 3) exceeds
// (min(n1, n2) - l) tau^2, the most that many values <= tau can hold.
#include "kernels.hpp"

namespace ht {

namespace {

constexpr int NIN = 32, NH = 128, S = 32;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;

struct MlpLds {
  float xs[S][NIN];
  float h1[S][NH + 1];
  float h2[S][NH + 1];
  float z[S];
  float dz[S];
  float lossp[S];
};

// Forward pass of the workgroup's samples (xs filled, ns valid).  Leaves the
// ReLU outputs in h1, h2 and z in L.z.  blockDim.x == NH.
__device__ void mlp_forward_block(const float* __restrict__ th, MlpLds& L) {
  const int j = threadIdx.x;
  {
    float w[NIN];
#pragma unroll
    for (int c = 0; c < NIN; ++c) w[c] = th[OFF_W1 + j * NIN + c];
    const float b = th[OFF_B1 + j];
    for (int s = 0; s < S; ++s) {
      float a = b;
#pragma unroll
      for (int c = 0; c < NIN; ++c) a = fmaf(w[c], L.xs[s][c], a);
      L.h1[s][j] = a > 0.0f ? a : 0.0f;
    }
  }
  __syncthreads();
  {
    float acc[S];
    const float b = th[OFF_B2 + j];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = b;
    for (int i = 0; i < NH; ++i) {
      const float w = th[OFF_W2 + j * NH + i];
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] = fmaf(w, L.h1[s][i], acc[s]);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) L.h2[s][j] = acc[s] > 0.0f ? acc[s] : 0.0f;
  }
  __syncthreads();
  if (j < S) {
    float z = th[OFF_B3];
    for (int i = 0; i < NH; ++i) z = fmaf(th[OFF_W3 + i], L.h2[j][i], z);
    L.z[j] = z;
  }
  __syncthreads();
}

__device__ void load_samples(const float* __restrict__ X, int s0, int ns, MlpLds& L) {
  for (int idx = threadIdx.x; idx < S * NIN; idx += NH) {
    const int s = idx / NIN, c = idx % NIN;
    L.xs[s][c] = s < ns ? X[(int64_t)(s0 + s) * NIN + c] : 0.0f;
  }
  __syncthreads();
}

__global__ __launch_bounds__(NH) void k_mlp_forward(const float* __restrict__ th, const float* __restrict__ X,
                                                    float* __restrict__ z, int n) {
  __shared__ MlpLds L;
  const int s0 = blockIdx.x * S;
  const int ns = min(S, n - s0);
  load_samples(X, s0, ns, L);
  mlp_forward_block(th, L);
  if (threadIdx.x < ns) z[s0 + threadIdx.x] = L.z[threadIdx.x];
}

// Gradient partials: workgroup b walks chunks b, b + G, ... of 32 samples and
// accumulates its gradient of the mean squared error into part[b][:] and its
// summed squared error into lpart[b].
__global__ __launch_bounds__(NH) void k_mlp_grad(const float* __restrict__ th, const float* __restrict__ X,
                                                 const float* __restrict__ y, int n, float* __restrict__ part,
                                                 float* __restrict__ lpart) {
  __shared__ MlpLds L;
  const int j = threadIdx.x;
  float* g = part + (int64_t)blockIdx.x * NPARAM;
  const float inv_n = 1.0f / (float)n;
  // zero this workgroup's row
  for (int p = j; p < NPARAM; p += NH) g[p] = 0.0f;
  float lsum = 0.0f;
  const int nchunks = (n + S - 1) / S;
  for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int s0 = ch * S;
    const int ns = min(S, n - s0);
    __syncthreads();
    load_samples(X, s0, ns, L);
    mlp_forward_block(th, L);
    if (j < S) {
      const float e = j < ns ? L.z[j] - y[s0 + j] : 0.0f;
      L.dz[j] = 2.0f * e * inv_n;
      L.lossp[j] = e * e;
    }
    __syncthreads();
    // layer 3 and dh2 (in place of h2, column j owned by thread j)
    {
      const float w3 = th[OFF_W3 + j];
      float gw3 = 0.0f;
      for (int s = 0; s < S; ++s) {
        const float h = L.h2[s][j];
        gw3 = fmaf(L.dz[s], h, gw3);
        L.h2[s][j] = h > 0.0f ? L.dz[s] * w3 : 0.0f;
      }
      g[OFF_W3 + j] += gw3;
      if (j == 0) {
        float gb3 = 0.0f, ls = 0.0f;
        for (int s = 0; s < S; ++s) {
          gb3 += L.dz[s];
          ls += L.lossp[s];
        }
        g[OFF_B3] += gb3;
        lsum += ls;
      }
    }
    __syncthreads();
    // gW2[r][j] = sum_s dh2[s][r] h1[s][j]  (thread j: column j, coalesced rows);
    // gb2[j] = sum_s dh2[s][j]
    {
      float h1c[S];
#pragma unroll
      for (int s = 0; s < S; ++s) h1c[s] = L.h1[s][j];
      for (int r = 0; r < NH; ++r) {
        float a = 0.0f;
#pragma unroll
        for (int s = 0; s < S; ++s) a = fmaf(L.h2[s][r], h1c[s], a);
        g[OFF_W2 + r * NH + j] += a;
      }
      float gb2 = 0.0f;
      for (int s = 0; s < S; ++s) gb2 += L.h2[s][j];
      g[OFF_B2 + j] += gb2;
      // dh1[s][j] = (sum_r W2[r][j] dh2[s][r]) * (h1[s][j] > 0), in place of column j of h1
      float acc[S];
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] = 0.0f;
      for (int r = 0; r < NH; ++r) {
        const float w = th[OFF_W2 + r * NH + j];
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] = fmaf(w, L.h2[s][r], acc[s]);
      }
#pragma unroll
      for (int s = 0; s < S; ++s) L.h1[s][j] = h1c[s] > 0.0f ? acc[s] : 0.0f;
    }
    // gW1[j][c] = sum_s dh1[s][j] x[s][c];  gb1[j] = sum_s dh1[s][j]  (own column of h1)
    {
      float gb1 = 0.0f;
      for (int s = 0; s < S; ++s) gb1 += L.h1[s][j];
      g[OFF_B1 + j] += gb1;
      for (int c = 0; c < NIN; ++c) {
        float a = 0.0f;
#pragma unroll
        for (int s = 0; s < S; ++s) a = fmaf(L.h1[s][j], L.xs[s][c], a);
        g[OFF_W1 + j * NIN + c] += a;
      }
    }
  }
  if (j == 0) lpart[blockIdx.x] = lsum;
}

// Sum the partial rows in order; optionally one Adam step (bias-corrected).
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, const float* __restrict__ lpart,
                                                    int nparts, int n, float* __restrict__ grad,
                                                    float* __restrict__ loss, float* __restrict__ th,
                                                    float* __restrict__ m, float* __restrict__ v, int step, float lr,
                                                    float beta1, float beta2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0 && loss) {
    float l = 0.0f;
    for (int b = 0; b < nparts; ++b) l += lpart[b];
    *loss = l / (float)n;
  }
  if (p >= NPARAM) return;
  float gs = 0.0f;
  for (int b = 0; b < nparts; ++b) gs += part[(int64_t)b * NPARAM + p];
  if (grad) grad[p] = gs;
  if (th) {
    const float mn = beta1 * m[p] + (1.0f - beta1) * gs;
    const float vn = beta2 * v[p] + (1.0f - beta2) * gs * gs;
    m[p] = mn;
    v[p] = vn;
    const float mh = mn / (1.0f - powf(beta1, (float)step));
    const float vh = vn / (1.0f - powf(beta2, (float)step));
    th[p] -= lr * mh / (sqrtf(vh) + eps);
  }
}

// ---------------------------------------------------------------------------
// Per-slice kernels of the learned-width t-SVT
// ---------------------------------------------------------------------------

// ||A_s||_F^2 in FP64 (A in T, or BF16 bits when bf16).
template <typename T>
__global__ __launch_bounds__(256) void k_anorm(const T* __restrict__ A, int bf16, const SliceDesc* __restrict__ sd,
                                               double* __restrict__ anorm) {
  const int s = blockIdx.x;
  const SliceDesc d = sd[s];
  const int64_t n = (int64_t)d.n1 * d.n2;
  double acc = 0.0;
  if (bf16) {
    const uint16_t* a = reinterpret_cast<const uint16_t*>(A) + d.a;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const float f = __uint_as_float((uint32_t)a[i] << 16);
      acc += (double)f * (double)f;
    }
  } else {
    const T* a = A + d.a;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const double f = (double)a[i];
      acc += f * f;
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) anorm[2 * s + 1] = red[0];
}

__device__ inline double clipd(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }

// Features of slice s from the previous call's statistics (sigma row of lmax
// values, kept count, width used, previous ||A||^2) and the current tau.
__device__ void slice_features(const double* __restrict__ sig, int kept, int lp, double anorm2, double tau,
                               int iteration, int n1, int n2, float* f) {
  const double s1 = sig[0];
  for (int i = 0; i < 16; ++i) f[i] = (s1 > 0.0 && i < lp) ? (float)(sig[i] / s1) : 0.0f;
  double b2 = 0.0;
  int above = 0;
  for (int i = 0; i < lp; ++i) {
    b2 += sig[i] * sig[i];
    above += sig[i] > tau;
  }
  f[16] = (float)(log10(anorm2 + 1e-30) / 10.0);
  f[17] = anorm2 > 0.0 ? (float)clipd((anorm2 - b2) / anorm2, 0.0, 1.0) : 0.0f;
  f[18] = s1 > 0.0 ? (float)clipd(tau / s1, 0.0, 10.0) : 10.0f;
  f[19] = (float)((double)above / lp);
  f[20] = (float)((double)kept / lp);
  const int ks[4] = {2, 4, 8, 16};
  for (int c = 0; c < 4; ++c) {
    const int k = ks[c];
    double v = 0.0;
    if (k < lp) {
      const double a = sig[k - 1], b = sig[k];
      v = b > 0.0 ? clipd(log(a / b), 0.0, 10.0) : (a > 0.0 ? 10.0 : 0.0);
    }
    f[21 + c] = (float)v;
  }
  f[25] = tau > 0.0 ? (float)(log10(1.0 / tau) / 10.0) : 1.0f;
  f[26] = (float)((double)min(iteration, 200) / 100.0);
  f[27] = (float)log((double)n1 / (double)n2);
  f[28] = (float)(log2((double)min(n1, n2)) / 10.0);
  f[29] = (float)(lp / 64.0);
  f[30] = (float)(above / 64.0);
  f[31] = 0.0f;
}

__device__ inline double current_tau(double tau_host, const double* tau_dev, const double* mu_dev, int tensor) {
  return mu_dev ? 1.0 / (*mu_dev) : (tau_dev ? tau_dev[tensor] : tau_host);
}

// Features and widths of 32 slices per workgroup.  mode 1: fixed widths
// (features recorded for tracing); mode 2: widths from the network when the
// previous call's statistics are valid.
__global__ __launch_bounds__(NH) void k_width(const float* __restrict__ th, int mode, const SliceDesc* __restrict__ sd,
                                              int nslices, int lmax, const double* __restrict__ sig,
                                              const int* __restrict__ kept, const int2* __restrict__ wk_prev,
                                              const double* __restrict__ anorm, const int* __restrict__ lstate,
                                              double tau_host, const double* __restrict__ tau_dev,
                                              const double* __restrict__ mu_dev, uint32_t call,
                                              const int32_t* __restrict__ call_dev, float* __restrict__ feat,
                                              int2* __restrict__ wk) {
  __shared__ MlpLds L;
  const int s0 = blockIdx.x * S;
  const int ns = min(S, nslices - s0);
  const int valid = lstate[0];
  const int it = call_dev ? *call_dev : (int)call;
  const int t = threadIdx.x;
  if (t < S) {
    float f[NIN];
    for (int c = 0; c < NIN; ++c) f[c] = 0.0f;
    if (t < ns && valid) {
      const int s = s0 + t;
      const SliceDesc d = sd[s];
      const int lp = min(max(wk_prev[s].x, 1), d.l);  // the width this slice used last time
      const int kp = min(max(kept[s], 0), lp);
      slice_features(sig + (int64_t)s * lmax, kp, lp, anorm[2 * s], current_tau(tau_host, tau_dev, mu_dev, d.tensor),
                     it, d.n1, d.n2, f);
    }
    for (int c = 0; c < NIN; ++c) L.xs[t][c] = f[c];
    if (t < ns)
      for (int c = 0; c < NIN; ++c) feat[(int64_t)(s0 + t) * NIN + c] = f[c];
  }
  __syncthreads();
  if (mode == 2 && valid) mlp_forward_block(th, L);
  if (t < ns) {
    const int s = s0 + t;
    const SliceDesc d = sd[s];
    int l = d.l, k = d.k;
    if (mode == 2 && valid) {
      const double z = (double)L.z[t];
      const double sp = z < 700.0 ? expm1(z) : INFINITY;
      if (isfinite(sp)) {
        const double c = ceil(sp) + d.p;
        l = (int)fmin(fmax(c, (double)(d.p + 1)), (double)d.l);
      }
      k = min(d.k, l);
    }
    wk[s] = make_int2(l, k);
  }
}

// After the predicted pass: decide the redo set (wk2: fixed width or 0 = skip),
// the final widths (wkf), keep ||A||^2 for the next call's features and count.
__global__ __launch_bounds__(256) void k_fallback(const SliceDesc* __restrict__ sd, int nslices, int lmax,
                                                  const int2* __restrict__ wk1, const double* __restrict__ sig,
                                                  const int* __restrict__ kept, double* __restrict__ anorm,
                                                  double tau_host, const double* __restrict__ tau_dev,
                                                  const double* __restrict__ mu_dev, Penalty pen, int force,
                                                  int2* __restrict__ wk2, int2* __restrict__ wkf,
                                                  int* __restrict__ lstate) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslices) return;
  const SliceDesc d = sd[s];
  const int2 w = wk1[s];
  bool redo = false;
  if (w.x < d.l) {
    // the residual certainly holds a value that would survive when its energy
    // exceeds (number of residual values) x (zero threshold of the prox)^2
    const double t0 = prox_zero_threshold(pen, current_tau(tau_host, tau_dev, mu_dev, d.tensor));
    double b2 = 0.0;
    for (int i = 0; i < w.x; ++i) b2 += sig[(int64_t)s * lmax + i] * sig[(int64_t)s * lmax + i];
    const double tail = anorm[2 * s + 1] - b2;
    redo = force || kept[s] >= w.y || tail > (double)(min(d.n1, d.n2) - w.x) * t0 * t0;
    atomicAdd(&lstate[1], 1);
    if (redo) atomicAdd(&lstate[2], 1);
  }
  wk2[s] = redo ? make_int2(d.l, d.k) : make_int2(0, 0);
  wkf[s] = redo ? make_int2(d.l, d.k) : w;
  anorm[2 * s] = anorm[2 * s + 1];
}

// Tracking without prediction: the widths used are the fixed ones.
__global__ __launch_bounds__(256) void k_track_finalize(int nslices, const int2* __restrict__ wk1,
                                                        int2* __restrict__ wkf, double* __restrict__ anorm) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslices) return;
  wkf[s] = wk1[s];
  anorm[2 * s] = anorm[2 * s + 1];
}

__global__ void k_lstate_set(int* __restrict__ lstate, int valid, int clear_counts) {
  if (threadIdx.x == 0) {
    lstate[0] = valid;
    if (clear_counts) {
      lstate[1] = 0;
      lstate[2] = 0;
    }
  }
}

}  // namespace

int mlp_param_count() { return NPARAM; }
int mlp_samples_per_block() { return S; }

int launch_mlp_forward(const float* th, const float* X, float* z, int n, hipStream_t s) {
  if (n <= 0) return HT_OK;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)ceil_div(n, S)), dim3(NH), 0, s, th, X, z, n);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

int mlp_grad_parts(int n) { return (int)std::min<int64_t>(ceil_div(n, S), 256); }

int launch_mlp_grad_step(const float* th_in, const float* X, const float* y, int n, float* part, float* lpart,
                         float* grad, float* loss, float* th, float* m, float* v, int step, float lr, float beta1,
                         float beta2, float eps, hipStream_t s) {
  if (n <= 0) HT_FAIL(HT_ERR_INVALID_ARG, "need at least one sample");
  const int G = mlp_grad_parts(n);
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)G), dim3(NH), 0, s, th_in, X, y, n, part, lpart);
  HT_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)ceil_div(NPARAM, 256)), dim3(256), 0, s, part, lpart, G, n, grad,
                     loss, th, m, v, step, lr, beta1, beta2, eps);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template <typename T>
int launch_anorm(const T* A, int bf16, const SliceDesc* sd, int nslices, double* anorm, hipStream_t s) {
  if (nslices == 0) return HT_OK;
  hipLaunchKernelGGL(k_anorm<T>, dim3((unsigned)nslices), dim3(256), 0, s, A, bf16, sd, anorm);
  HT_CHECK_LAUNCH();
  return HT_OK;
}
template int launch_anorm<float>(const float*, int, const SliceDesc*, int, double*, hipStream_t);
template int launch_anorm<double>(const double*, int, const SliceDesc*, int, double*, hipStream_t);

int launch_width(const float* th, int mode, const SliceDesc* sd, int nslices, int lmax, const double* sig,
                 const int* kept, const int2* wk_prev, const double* anorm, const int* lstate, double tau,
                 const double* tau_dev, const double* mu_dev, uint32_t call, const int32_t* call_dev, float* feat,
                 int2* wk, hipStream_t s) {
  if (nslices == 0) return HT_OK;
  hipLaunchKernelGGL(k_width, dim3((unsigned)ceil_div(nslices, S)), dim3(NH), 0, s, th, mode, sd, nslices, lmax, sig,
                     kept, wk_prev, anorm, lstate, tau, tau_dev, mu_dev, call, call_dev, feat, wk);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

int launch_fallback(const SliceDesc* sd, int nslices, int lmax, const int2* wk1, const double* sig, const int* kept,
                    double* anorm, double tau, const double* tau_dev, const double* mu_dev, Penalty pen, int force,
                    int2* wk2, int2* wkf, int* lstate, hipStream_t s) {
  if (nslices == 0) return HT_OK;
  hipLaunchKernelGGL(k_fallback, dim3((unsigned)ceil_div(nslices, 256)), dim3(256), 0, s, sd, nslices, lmax, wk1, sig,
                     kept, anorm, tau, tau_dev, mu_dev, pen, force, wk2, wkf, lstate);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

int launch_track_finalize(int nslices, const int2* wk1, int2* wkf, double* anorm, hipStream_t s) {
  if (nslices == 0) return HT_OK;
  hipLaunchKernelGGL(k_track_finalize, dim3((unsigned)ceil_div(nslices, 256)), dim3(256), 0, s, nslices, wk1, wkf,
                     anorm);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

int launch_lstate_set(int* lstate, int valid, int clear_counts, hipStream_t s) {
  hipLaunchKernelGGL(k_lstate_set, dim3(1), dim3(64), 0, s, lstate, valid, clear_counts);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

}  // namespace ht
