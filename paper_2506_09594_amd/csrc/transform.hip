// Transforms along modes 3..d and the Gaussian sketch generator.
//
// Forward transform (the transform L of Sec. II): A = X x_3 U_3 ... x_d U_d.
// With the tensor stored in Fortran order, a "tube position" t = i1 + n1*i2
// owns the n3*...*nd values X(t, j) = X[j*n1*n2 + t] across all face slices j,
// and the transform acts on the slice index only.  One workgroup takes TP
// consecutive tube positions for all P slices into LDS (TP*P values, loaded as
// P coalesced runs of TP elements), applies every mode's n_k x n_k matrix to
// the fibers of that mode with the fiber held in registers, and writes the tile
// back.  HBM traffic is one read and one write of the tensor; the mode
// matrices are broadcast from the scalar cache.
#include "kernels.hpp"

namespace ht {

template <typename T, int NMAX>
__device__ __forceinline__ void apply_fiber(T* tile, int base, int stride, int n, const T* __restrict__ U) {
  T v[NMAX];
#pragma unroll
  for (int b = 0; b < NMAX; ++b) v[b] = (b < n) ? tile[base + b * stride] : T(0);
#pragma unroll
  for (int a = 0; a < NMAX; ++a) {
    if (a < n) {
      T s = T(0);
#pragma unroll
      for (int b = 0; b < NMAX; ++b)
        if (b < n) s += U[a * n + b] * v[b];
      tile[base + a * stride] = s;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_transform(const T* __restrict__ in, T* __restrict__ out, int64_t NT,
                                                   int P, int TP, ModeTable mt, const T* __restrict__ table) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  const int64_t t0 = (int64_t)blockIdx.x * TP;
  const int64_t rem = NT - t0;
  const int tp = rem < TP ? (int)rem : TP;
  const int total = TP * P;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int j = idx / TP, t = idx - j * TP;
    tile[idx] = (t < tp) ? in[(int64_t)j * NT + t0 + t] : T(0);
  }
  __syncthreads();
  for (int m = 0; m < mt.nmodes; ++m) {
    const int n = mt.n[m];
    const int s = mt.stride[m];
    const T* U = table + mt.off[m];
    const int nfib = total / n;
    for (int f = threadIdx.x; f < nfib; f += blockDim.x) {
      const int t = f % TP;
      const int rest = f / TP;
      const int lo = rest % s, hi = rest / s;
      const int base = (lo + hi * s * n) * TP + t;
      const int stride = s * TP;
      if (n <= 4)
        apply_fiber<T, 4>(tile, base, stride, n, U);
      else if (n <= 8)
        apply_fiber<T, 8>(tile, base, stride, n, U);
      else if (n <= 16)
        apply_fiber<T, 16>(tile, base, stride, n, U);
      else if (n <= 32)
        apply_fiber<T, 32>(tile, base, stride, n, U);
      else
        apply_fiber<T, 64>(tile, base, stride, n, U);
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int j = idx / TP, t = idx - j * TP;
    if (t < tp) out[(int64_t)j * NT + t0 + t] = tile[idx];
  }
}

int transform_tile_width(int64_t P, size_t elem_bytes) {
  const size_t budget = 64 * 1024;
  int64_t tp = 256;
  while (tp > 1 && (size_t)(tp * P) * elem_bytes > budget) tp >>= 1;
  if ((size_t)(tp * P) * elem_bytes > budget) return 0;
  return (int)tp;
}

template <typename T>
int launch_transform(const T* in, T* out, int64_t NT, int P, const ModeTable& mt, const T* table,
                     hipStream_t stream) {
  if (mt.nmodes == 0) {
    if (in != out) HT_CHECK_HIP(hipMemcpyAsync(out, in, sizeof(T) * NT * P, hipMemcpyDeviceToDevice, stream));
    return HT_OK;
  }
  const int TP = transform_tile_width(P, sizeof(T));
  if (TP == 0) HT_FAIL(HT_ERR_UNSUPPORTED, "too many face slices for the LDS transform tile");
  const size_t lds = sizeof(T) * (size_t)TP * P;
  const int64_t blocks = ceil_div(NT, TP);
  hipLaunchKernelGGL(k_transform<T>, dim3((unsigned)blocks), dim3(256), lds, stream, in, out, NT, P, TP, mt, table);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template int launch_transform<float>(const float*, float*, int64_t, int, const ModeTable&, const float*, hipStream_t);
template int launch_transform<double>(const double*, double*, int64_t, int, const ModeTable&, const double*,
                                      hipStream_t);

// ---------------------------------------------------------------------------
// Gaussian sketch matrices Omega_j (n2 x l, column-major), one per slice,
// keyed by the canonical slice index (identity for real transforms).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_omega(T* __restrict__ om, double* __restrict__ om64, int64_t per_slice,
                                               uint32_t call, const int32_t* __restrict__ call_dev, uint32_t stream_id,
                                               uint64_t seed, const int32_t* __restrict__ canon) {
  const int j = blockIdx.y;
  const uint32_t key = canon ? (uint32_t)canon[j] : (uint32_t)j;
  const uint32_t c = call_dev ? (uint32_t)(*call_dev) : call;
  const int64_t ngroups = (per_slice + 3) / 4;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups; g += (int64_t)gridDim.x * blockDim.x) {
    double z[4];
    gaussian4((uint64_t)g, key, c, stream_id, seed, z);
#pragma unroll
    for (int lane = 0; lane < 4; ++lane) {
      const int64_t e = 4 * g + lane;
      if (e < per_slice) {
        if (om) om[(int64_t)j * per_slice + e] = (T)z[lane];
        if (om64) om64[(int64_t)j * per_slice + e] = z[lane];
      }
    }
  }
}

template <typename T>
int launch_omega(T* om, double* om64, int P, int64_t per_slice, uint32_t call, const int32_t* call_dev,
                 uint32_t stream_id, uint64_t seed, const int32_t* canon, hipStream_t stream) {
  const int64_t ngroups = (per_slice + 3) / 4;
  const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(ngroups, 256), 64);
  hipLaunchKernelGGL(k_omega<T>, dim3(gx, (unsigned)P), dim3(256), 0, stream, om, om64, per_slice, call, call_dev,
                     stream_id, seed, canon);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template int launch_omega<float>(float*, double*, int, int64_t, uint32_t, const int32_t*, uint32_t, uint64_t,
                                 const int32_t*, hipStream_t);
template int launch_omega<double>(double*, double*, int, int64_t, uint32_t, const int32_t*, uint32_t, uint64_t,
                                  const int32_t*, hipStream_t);

}  // namespace ht
