// Recovery update of the pure-L ADMM (Sec. V updates of E, the multiplier and
// mu), fused with the stopping-term reductions and with the formation of the
// next iteration's t-SVT input M - E + Y/mu.  The sparse part is shrunk
// element-wise, or tube-wise / slice-wise (GNHTT, Sec. IV-B): then the squared
// norm of every group of P_Omega(H) is formed first (FP64, fixed order) and
// the update scales the group's observed entries by Prox(||g||) / ||g||.
#include "kernels.hpp"

namespace ht {

namespace {

__device__ __forceinline__ unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }

// Maximum that keeps a NaN (fmax drops it): a NaN iterate must show in the
// stopping terms instead of letting a stopping rule converge on it.
__device__ __forceinline__ double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_xor(v, off, 64));
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_admm_input(const T* __restrict__ M, const T* __restrict__ E,
                                                    const T* __restrict__ Y, const AdmmState* __restrict__ st,
                                                    T* __restrict__ Xin, int64_t N) {
  const double inv_mu = 1.0 / st->mu;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    Xin[i] = (T)((double)M[i] - (double)E[i] + (double)Y[i] * inv_mu);
}

// Squared norms of the groups of P_Omega(H), H = M - L_new + Y/mu: tube t
// (tube-wise: one thread per tube position, the P entries at stride NT) or
// slice j (slice-wise: one workgroup per slice, fixed-order tree reduction).
template <typename T>
__global__ __launch_bounds__(256) void k_group_sq(const T* __restrict__ M, const uint8_t* __restrict__ mask,
                                                  const T* __restrict__ Lnew, const T* __restrict__ Y,
                                                  const AdmmState* __restrict__ st, int64_t NT, int64_t P, int tube,
                                                  double* __restrict__ gsq) {
  const double inv_mu = 1.0 / st->mu;
  auto hsq = [&](int64_t i) -> double {
    if (!mask[i]) return 0.0;
    const double h = (double)M[i] - (double)Lnew[i] + (double)Y[i] * inv_mu;
    return h * h;
  };
  if (tube) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < NT; t += (int64_t)gridDim.x * blockDim.x) {
      double acc = 0.0;
      for (int64_t j = 0; j < P; ++j) acc += hsq(j * NT + t);
      gsq[t] = acc;
    }
    return;
  }
  __shared__ double red[256];
  for (int64_t j = blockIdx.x; j < P; j += gridDim.x) {
    double acc = 0.0;
    for (int64_t t = threadIdx.x; t < NT; t += blockDim.x) acc += hsq(j * NT + t);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) gsq[j] = red[0];
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_admm_update(const T* __restrict__ M, const uint8_t* __restrict__ mask,
                                                     const T* __restrict__ Lnew, T* __restrict__ L,
                                                     T* __restrict__ E, T* __restrict__ Y, T* __restrict__ Xin,
                                                     AdmmState* __restrict__ st, int64_t N, int model, Penalty psi,
                                                     double lambda, double vartheta, double mu_max,
                                                     const double* __restrict__ gsq, int64_t NT) {
  const double mu = st->mu;
  const double inv_mu = 1.0 / mu;
  const double mu_next = fmin(mu_max, vartheta * mu);
  const double inv_mu_next = 1.0 / mu_next;
  const double thr = lambda * inv_mu;
  double mdl = 0.0, mde = 0.0, mres = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const double m = (double)M[i], ln = (double)Lnew[i], lo = (double)L[i];
    const double e = (double)E[i], y = (double)Y[i];
    const double h = m - ln + y * inv_mu;
    double en;
    if (mask[i]) {
      if (model == HT_RPCA) {
        en = prox_signed(psi, h, thr);
      } else if (model == HT_RPCA_TUBE || model == HT_RPCA_SLICE) {
        const double nrm = sqrt(gsq[model == HT_RPCA_TUBE ? i % NT : i / NT]);
        en = nrm > 0.0 ? h * (prox_pos(psi, nrm, thr) / nrm) : 0.0;
      } else {
        en = 0.0;
      }
    } else {
      en = h;
    }
    const double r = m - ln - en;
    const double yn = y + mu * r;
    mdl = nan_max(mdl, fabs(ln - lo));
    mde = nan_max(mde, fabs(en - e));
    mres = nan_max(mres, fabs(r));
    L[i] = (T)ln;
    E[i] = (T)en;
    Y[i] = (T)yn;
    Xin[i] = (T)(m - en + yn * inv_mu_next);
  }
  __shared__ double red[3][4];
  mdl = wave_max(mdl);
  mde = wave_max(mde);
  mres = wave_max(mres);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    red[0][wave] = mdl;
    red[1][wave] = mde;
    red[2][wave] = mres;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = red[0][0], b = red[1][0], c = red[2][0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) {
      a = nan_max(a, red[0][w]);
      b = nan_max(b, red[1][w]);
      c = nan_max(c, red[2][w]);
    }
    // the values are >= 0 or a NaN with the sign bit clear (fabs), so the bit
    // patterns order like the values with NaN above +inf
    atomicMax(&st->red_dL, dbits(fabs(a)));
    atomicMax(&st->red_dE, dbits(fabs(b)));
    atomicMax(&st->red_res, dbits(fabs(c)));
  }
}

__global__ void k_admm_finalize(AdmmState* st, double vartheta, double mu_max) {
  st->dL = __longlong_as_double((long long)st->red_dL);
  st->dE = __longlong_as_double((long long)st->red_dE);
  st->resid = __longlong_as_double((long long)st->red_res);
  st->red_dL = 0ull;
  st->red_dE = 0ull;
  st->red_res = 0ull;
  st->mu = fmin(mu_max, vartheta * st->mu);
  st->iteration += 1;
}

__global__ void k_admm_reset(AdmmState* st, double mu0) {
  st->mu = mu0;
  st->iteration = 0;
  st->pad0 = 0;
  st->dL = st->dE = st->resid = 0.0;
  st->red_dL = st->red_dE = st->red_res = 0ull;
  st->rse = __longlong_as_double(0x7ff8000000000000ll);
}

// RSE against the ground truth: block b sums (L - L*)^2 and L*^2 over its
// grid-stride share in FP64 (fixed order within the block), the last kernel
// adds the block partials in index order.
template <typename T>
__global__ __launch_bounds__(256) void k_rse_part(const T* __restrict__ L, const T* __restrict__ truth, int64_t N,
                                                  double* __restrict__ part) {
  double e2 = 0.0, t2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const double t = (double)truth[i], d = (double)L[i] - t;
    e2 = fma(d, d, e2);
    t2 = fma(t, t, t2);
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = e2;
  red[1][threadIdx.x] = t2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void k_rse_final(const double* __restrict__ part, int nblocks, AdmmState* st) {
  if (threadIdx.x != 0) return;
  double e2 = 0.0, t2 = 0.0;
  for (int b = 0; b < nblocks; ++b) {
    e2 += part[2 * b];
    t2 += part[2 * b + 1];
  }
  st->rse = sqrt(e2) / sqrt(t2);
}

__global__ void k_rse_none(AdmmState* st) {
  if (threadIdx.x == 0) st->rse = __longlong_as_double(0x7ff8000000000000ll);
}

unsigned elementwise_blocks(int64_t N) {
  int64_t b = ceil_div(N, 256);
  return (unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 8192);
}

}  // namespace

template <typename T>
int launch_admm_input(const T* M, const T* E, const T* Y, const AdmmState* st, T* Xin, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_admm_input<T>, dim3(elementwise_blocks(N)), dim3(256), 0, s, M, E, Y, st, Xin, N);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template <typename T>
int launch_admm_update(const T* M, const uint8_t* mask, const T* Lnew, T* L, T* E, T* Y, T* Xin, AdmmState* st,
                       int64_t N, int model, Penalty psi, double lambda, double vartheta, double mu_max, double* gsq,
                       int64_t NT, hipStream_t s) {
  if (model == HT_RPCA_TUBE || model == HT_RPCA_SLICE) {
    const int64_t P = N / NT;
    const bool tube = model == HT_RPCA_TUBE;
    const unsigned nb = tube ? elementwise_blocks(NT) : (unsigned)std::min<int64_t>(P, 4096);
    hipLaunchKernelGGL(k_group_sq<T>, dim3(nb), dim3(256), 0, s, M, mask, Lnew, Y, st, NT, P, tube ? 1 : 0, gsq);
    HT_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_admm_update<T>, dim3(elementwise_blocks(N)), dim3(256), 0, s, M, mask, Lnew, L, E, Y, Xin, st,
                     N, model, psi, lambda, vartheta, mu_max, gsq, NT);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

int launch_admm_finalize(AdmmState* st, double vartheta, double mu_max, hipStream_t s) {
  hipLaunchKernelGGL(k_admm_finalize, dim3(1), dim3(1), 0, s, st, vartheta, mu_max);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

int launch_admm_reset(AdmmState* st, double mu0, hipStream_t s) {
  hipLaunchKernelGGL(k_admm_reset, dim3(1), dim3(1), 0, s, st, mu0);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template <typename T>
int launch_admm_rse(const T* L, const T* truth, int64_t N, double* part, int nblocks, AdmmState* st, hipStream_t s) {
  if (!truth) {
    hipLaunchKernelGGL(k_rse_none, dim3(1), dim3(64), 0, s, st);
    HT_CHECK_LAUNCH();
    return HT_OK;
  }
  const int nb = (int)std::min<int64_t>(std::max<int64_t>(ceil_div(N, 256), 1), nblocks);
  hipLaunchKernelGGL(k_rse_part<T>, dim3(nb), dim3(256), 0, s, L, truth, N, part);
  HT_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_rse_final, dim3(1), dim3(64), 0, s, part, nb, st);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template int launch_admm_rse<float>(const float*, const float*, int64_t, double*, int, AdmmState*, hipStream_t);
template int launch_admm_rse<double>(const double*, const double*, int64_t, double*, int, AdmmState*, hipStream_t);

template int launch_admm_input<float>(const float*, const float*, const float*, const AdmmState*, float*, int64_t,
                                      hipStream_t);
template int launch_admm_input<double>(const double*, const double*, const double*, const AdmmState*, double*,
                                       int64_t, hipStream_t);
template int launch_admm_update<float>(const float*, const uint8_t*, const float*, float*, float*, float*, float*,
                                       AdmmState*, int64_t, int, Penalty, double, double, double, double*, int64_t,
                                       hipStream_t);
template int launch_admm_update<double>(const double*, const uint8_t*, const double*, double*, double*, double*,
                                        double*, AdmmState*, int64_t, int, Penalty, double, double, double, double*,
                                        int64_t, hipStream_t);

}  // namespace ht
