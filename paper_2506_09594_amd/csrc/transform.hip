// Transforms along modes 3..d and the Gaussian sketch generator.
//
// Forward transform (the transform L of Sec. II): A = X x_3 U_3 ... x_d U_d.
// With the tensor stored in Fortran order, a "tube position" t = i1 + n1*i2
// owns the n3*...*nd values X(t, j) = X[j*n1*n2 + t] across all face slices j,
// and the transform acts on the slice index only.  One workgroup takes TP
// consecutive tube positions for all P slices into LDS (TP*P values, loaded as
// P coalesced runs of TP elements, 16-byte accesses batched in registers so
// that many loads are in flight), applies every mode's n_k x n_k matrix to the
// fibers of that mode with several fibers held in registers per thread, and
// writes the tile back.  HBM traffic is one read and one write of the tensor;
// the mode matrices are scalar operands.
#include <type_traits>

#include "kernels.hpp"

namespace ht {

// Apply U (n x n, row-major) to F fibers at once: fiber k of this thread starts
// at tile[base[k]] with element stride `stride`.  N is the exact mode length
// (compile-time) so U's entries are fixed scalar operands.
template <typename T, int N, int F>
__device__ __forceinline__ void apply_fibers_exact(T* tile, const int* base, int stride, int nvalid,
                                                   const T* __restrict__ U) {
  T v[F][N];
#pragma unroll
  for (int k = 0; k < F; ++k)
#pragma unroll
    for (int b = 0; b < N; ++b) v[k][b] = (k < nvalid) ? tile[base[k] + b * stride] : T(0);
#pragma unroll
  for (int a = 0; a < N; ++a) {
    T acc[F];
#pragma unroll
    for (int k = 0; k < F; ++k) acc[k] = T(0);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const T u = U[a * N + b];
#pragma unroll
      for (int k = 0; k < F; ++k) acc[k] += u * v[k][b];
    }
#pragma unroll
    for (int k = 0; k < F; ++k)
      if (k < nvalid) tile[base[k] + a * stride] = acc[k];
  }
}

// Generic mode length n <= NMAX (predicated).
template <typename T, int NMAX>
__device__ __forceinline__ void apply_fiber_generic(T* tile, int base, int stride, int n, const T* __restrict__ U) {
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

// Fiber f of a mode with slice stride s and length n: tube position t = f % TP,
// remaining multi-index rest = f / TP split around the mode.
__device__ __forceinline__ int fiber_base(int f, int TP, int lgTP, int s, int n) {
  const int t = f & (TP - 1);
  const int rest = f >> lgTP;
  const int lo = rest % s, hi = rest / s;
  return (lo + hi * s * n) * TP + t;
}

template <typename T, int N>
__device__ __forceinline__ void mode_exact(T* tile, int TP, int lgTP, int s, int nfib, const T* __restrict__ U) {
  constexpr int F = (N <= 8) ? 4 : (N <= 16 ? 4 : 2);
  for (int f0 = threadIdx.x; f0 < nfib; f0 += F * blockDim.x) {
    int base[F];
    int nvalid = 0;
#pragma unroll
    for (int k = 0; k < F; ++k) {
      const int f = f0 + k * blockDim.x;
      base[k] = (f < nfib) ? fiber_base(f, TP, lgTP, s, N) : 0;
      nvalid += (f < nfib);
    }
    apply_fibers_exact<T, N, F>(tile, base, s * TP, nvalid, U);
  }
}

// Mode product on the matrix cores (FP32, n in {4, 8, 16}; used for n = 16):
// for 16 tube positions t0..t0+15 and NB = 16 / n fibers of the mode at
// consecutive "rest" indices, the fibers stacked along k form a 16 x 16
// operand X and the new values are blockdiag(U, ..., U) X, four
// v_mfma_f32_16x16x4f32 steps.
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] at each k step and
// receives D[4 (l / 16) + v][l % 16].  A group is read and written back in
// place by one wavefront; groups are disjoint.  Requires TP % 16 == 0 and
// (P / n) % NB == 0 (checked by the caller).
typedef float tf_f32x4 __attribute__((ext_vector_type(4)));
template <int N>
__device__ __forceinline__ void mode_mfma(float* tile, int TP, int s, int P, const float* __restrict__ U) {
  constexpr int NB = 16 / N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  float ua[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 4 * kk + lk;
    ua[kk] = (li / N == k / N) ? U[(li % N) * N + (k % N)] : 0.0f;
  }
  const int ngt = TP >> 4, ngr = P / (N * NB);
  for (int gidx = wave; gidx < ngt * ngr; gidx += nwv) {
    const int tg = gidx % ngt, gr = gidx / ngt;
    const int col = (tg << 4) + li;
    // row (slice index) of element k' of the fiber at rest index r
    auto jrow = [&](int r, int kp) { return (r % s) + s * (kp + N * (r / s)); };
    float b[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * kk + lk;
      b[kk] = tile[jrow(gr * NB + k / N, k % N) * TP + col];
    }
    tf_f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) d = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[kk], b[kk], d, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * lk + v;
      tile[jrow(gr * NB + i / N, i % N) * TP + col] = d[v];
    }
  }
}

// One workgroup per work item (tensor, first tube position).  TO = T, or
// uint16_t for BF16 output (rounded to nearest even).
template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_transform(const T* __restrict__ in_all, TO* __restrict__ out_all,
                                                   const TensorDesc* __restrict__ tds, const int2* __restrict__ items,
                                                   const T* __restrict__ table, int inverse, int aligned) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  constexpr int V = 16 / sizeof(T);  // elements per 16-byte access
  constexpr int UNR = 8;
  const int2 item = items[blockIdx.x];
  const TensorDesc* td = tds + item.x;
  const int64_t NT = td->NT;
  const int P = td->P, TP = td->TP, lgTP = td->lgTP;
  const ModeTable* mt = inverse ? &td->inv : &td->fwd;
  // forward: X (packed, offset x) -> A (offset a); inverse: C (offset a) -> out (offset x)
  const T* in = in_all + (inverse ? td->a : td->x);
  TO* out = out_all + (inverse ? td->x : td->a);
  const int vec = aligned && (NT % V == 0) && (TP % V == 0) && (td->x % V == 0) && (td->a % V == 0);
  const int64_t t0 = item.y;
  const int64_t rem = NT - t0;
  const int tp = rem < TP ? (int)rem : TP;
  const int total = TP * P;
  const int tid = threadIdx.x, nt = blockDim.x;

  // ---- load the TP x P tile: P runs of TP contiguous elements --------------
  if (vec) {
    using VT = __attribute__((ext_vector_type(V))) T;
    const int nv = total / V;
    for (int v0 = tid; v0 < nv; v0 += UNR * nt) {
      VT r[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int vi = v0 + u * nt;
        const int idx = vi * V;
        const int j = idx >> lgTP, t = idx & (TP - 1);
        if (vi < nv && t < tp)
          r[u] = *reinterpret_cast<const VT*>(in + (int64_t)j * NT + t0 + t);
        else
          r[u] = VT{};
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int vi = v0 + u * nt;
        if (vi < nv) *reinterpret_cast<VT*>(tile + vi * V) = r[u];
      }
    }
  } else {
    for (int i0 = tid; i0 < total; i0 += UNR * nt) {
      T r[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int idx = i0 + u * nt;
        const int j = idx >> lgTP, t = idx & (TP - 1);
        r[u] = (idx < total && t < tp) ? in[(int64_t)j * NT + t0 + t] : T(0);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int idx = i0 + u * nt;
        if (idx < total) tile[idx] = r[u];
      }
    }
  }
  __syncthreads();

  // ---- modes ---------------------------------------------------------------
  const int nmodes = mt->nmodes;
  for (int m = 0; m < nmodes; ++m) {
    const int n = mt->n[m];
    const int s = mt->stride[m];
    const T* U = table + mt->off[m];
    const int nfib = total / n;
    if constexpr (std::is_same<T, float>::value) {
      // length-16 modes on the matrix cores; shorter ones stay on the vector
      // units (block-diagonal packing would double their multiply-adds)
      if (n == 16 && (TP & 15) == 0) {
        mode_mfma<16>(tile, TP, s, P, U);
        __syncthreads();
        continue;
      }
    }
    switch (n) {
      case 2: mode_exact<T, 2>(tile, TP, lgTP, s, nfib, U); break;
      case 3: mode_exact<T, 3>(tile, TP, lgTP, s, nfib, U); break;
      case 4: mode_exact<T, 4>(tile, TP, lgTP, s, nfib, U); break;
      case 8: mode_exact<T, 8>(tile, TP, lgTP, s, nfib, U); break;
      case 16: mode_exact<T, 16>(tile, TP, lgTP, s, nfib, U); break;
      case 32: mode_exact<T, 32>(tile, TP, lgTP, s, nfib, U); break;
      default:
        for (int f = tid; f < nfib; f += nt) {
          const int base = fiber_base(f, TP, lgTP, s, n);
          if (n <= 8)
            apply_fiber_generic<T, 8>(tile, base, s * TP, n, U);
          else if (n <= 16)
            apply_fiber_generic<T, 16>(tile, base, s * TP, n, U);
          else if (n <= 32)
            apply_fiber_generic<T, 32>(tile, base, s * TP, n, U);
          else
            apply_fiber_generic<T, 64>(tile, base, s * TP, n, U);
        }
    }
    __syncthreads();
  }

  // ---- store ---------------------------------------------------------------
  if constexpr (!std::is_same<TO, T>::value) {
    if (vec) {  // four BF16 values (8 bytes) per store
      typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
      const int nq = total / 4;
      for (int q = tid; q < nq; q += nt) {
        const int idx = 4 * q;
        const int j = idx >> lgTP, t = idx & (TP - 1);
        if (t < tp) {
          u16x4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = f32_to_bf16_rne((float)tile[idx + e]);
          *reinterpret_cast<u16x4*>(out + (int64_t)j * NT + t0 + t) = v;
        }
      }
    } else {
      for (int idx = tid; idx < total; idx += nt) {
        const int j = idx >> lgTP, t = idx & (TP - 1);
        if (t < tp) out[(int64_t)j * NT + t0 + t] = f32_to_bf16_rne((float)tile[idx]);
      }
    }
  } else if (vec) {
    using VT = __attribute__((ext_vector_type(V))) T;
    const int nv = total / V;
    for (int v0 = tid; v0 < nv; v0 += UNR * nt) {
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int vi = v0 + u * nt;
        const int idx = vi * V;
        const int j = idx >> lgTP, t = idx & (TP - 1);
        if (vi < nv && t < tp)
          *reinterpret_cast<VT*>(out + (int64_t)j * NT + t0 + t) = *reinterpret_cast<const VT*>(tile + idx);
      }
    }
  } else {
    for (int idx = tid; idx < total; idx += nt) {
      const int j = idx >> lgTP, t = idx & (TP - 1);
      if (t < tp) out[(int64_t)j * NT + t0 + t] = tile[idx];
    }
  }
}

// ---------------------------------------------------------------------------
// Two transformed modes of length 16 (P = 256, slice j = i3 + 16 i4), FP32.
// Every wavefront works alone (no workgroup barrier) on an item of 32
// consecutive tube positions t0 .. t0 + 31, as two blocks of 16: lane (g, c)
// with g = lane / 16, c = lane % 16 reads the pair t0 + 2c, t0 + 2c + 1 with
// one 8-byte load (16 lanes cover a 128-byte line) for slice rows
// i3 = 4 g + kk (kk < 4) and all 16 values of i4: element 0 of the pair
// belongs to block 0, element 1 to block 1.  Per block, mode 3 is sixteen
// 16 x 16 x 16 products on the matrix cores (one per i4, four
// v_mfma_f32_16x16x4f32 steps), contracting i3 in the order 4 g + kk so that
// every lane already holds its B operand; lane (g, c) receives
// Y(i3' = 4 g + v, i4).  One pass through a private LDS region of the
// wavefront (pitch kT16Pitch floats per tube position, 16-byte accesses)
// hands lane (g, c) the four values i4 = 4 g + kk of every i3'; mode 4 is
// another sixteen products with the same contraction order and gives
// A(i3' + 16 (4 g + v)).  Block 0's results wait in registers until block 1's
// are ready, and each pair leaves with one 8-byte store.  HBM traffic is one
// read and one write of the tensor.  A last item of 16 positions masks the
// lanes whose pair lies past the end (their columns stay zero and are not
// stored; columns of the products never mix).
// ---------------------------------------------------------------------------
constexpr int kT16Pitch = 16 * 16 + 4;
constexpr int kT16Waves = 2;

template <typename TO>
struct T16Pair;
template <>
struct T16Pair<float> {
  typedef float __attribute__((ext_vector_type(2))) type;
  static __device__ __forceinline__ type make(float a, float b) { return type{a, b}; }
};
template <>
struct T16Pair<uint16_t> {
  typedef unsigned short __attribute__((ext_vector_type(2))) type;
  static __device__ __forceinline__ type make(float a, float b) { return type{f32_to_bf16_rne(a), f32_to_bf16_rne(b)}; }
};

// Mode 3 of one block (x: the lane's 64 values) into the exchange region.
__device__ __forceinline__ void t16_mode3(const float (&x)[16][4], const float (&ua)[4], float* xw, int g) {
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    tf_f32x4 d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      d[q] = tf_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) d[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[kk], x[4 * w + q][kk], d[q], 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
      *reinterpret_cast<tf_f32x4*>(xw + (4 * g + v) * 16 + 4 * w) = tf_f32x4{d[0][v], d[1][v], d[2][v], d[3][v]};
  }
  // the stores above reach the LDS before the loads that follow (same wavefront)
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Mode 4 of chain i3' from the exchange region.
__device__ __forceinline__ tf_f32x4 t16_mode4(const float (&ub)[4], const float* xw, int i3, int g) {
  const tf_f32x4 y = *reinterpret_cast<const tf_f32x4*>(xw + i3 * 16 + 4 * g);
  tf_f32x4 e = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) e = __builtin_amdgcn_mfma_f32_16x16x4f32(ub[kk], y[kk], e, 0, 0, 0);
  return e;
}

template <typename TO>
__global__ __launch_bounds__(64 * kT16Waves) __attribute__((amdgpu_waves_per_eu(2))) void k_transform16(
    const float* __restrict__ in_all, TO* __restrict__ out_all, const TensorDesc* __restrict__ tds,
    const int2* __restrict__ items, int nitems, const float* __restrict__ table, int inverse) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  typedef typename T16Pair<TO>::type PT;
  typedef float __attribute__((ext_vector_type(2))) f32x2;
  // the wavefront index as a scalar, so that item, tensor and every row base
  // below live in scalar registers and a lane keeps only 32-bit offsets
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int it = blockIdx.x * kT16Waves + wave;
  if (it >= nitems) return;
  const int2 item = items[it];
  const TensorDesc* td = tds + item.x;
  const int64_t NT = td->NT;
  const ModeTable* mt = inverse ? &td->inv : &td->fwd;
  const float* in = in_all + (inverse ? td->a : td->x);
  TO* out = out_all + (inverse ? td->x : td->a);
  const int m3 = mt->stride[0] == 1 ? 0 : 1;  // table entry of mode 3 (the inverse lists mode 4 first)
  const float* U3 = table + mt->off[m3];
  const float* U4 = table + mt->off[1 - m3];
  const int g = lane >> 4, c = lane & 15;
  const int64_t t0 = item.y;
  const bool live = t0 + 2 * c < NT;  // false only in a last item of 16 positions
  float ua[4], ub[4];  // A operands: U[c][4 g + kk]
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    ua[kk] = U3[c * 16 + 4 * g + kk];
    ub[kk] = U4[c * 16 + 4 * g + kk];
  }
  float* xw = reinterpret_cast<float*>(smem_raw) + wave * 16 * kT16Pitch + c * kT16Pitch;
  float x0[16][4], x1[16][4];
#pragma unroll
  for (int i4 = 0; i4 < 16; ++i4) {
    const float* src = in + t0 + (int64_t)(16 * i4) * NT;  // uniform
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      f32x2 v = {0.0f, 0.0f};
      if (live) v = *reinterpret_cast<const f32x2*>(src + (uint32_t)((4 * g + kk) * (uint32_t)NT + 2 * c));
      x0[i4][kk] = v[0];
      x1[i4][kk] = v[1];
    }
  }
  float e0[16][4];
  t16_mode3(x0, ua, xw, g);
#pragma unroll
  for (int i3 = 0; i3 < 16; ++i3) {
    const tf_f32x4 e = t16_mode4(ub, xw, i3, g);
#pragma unroll
    for (int v = 0; v < 4; ++v) e0[i3][v] = e[v];
  }
  // block 1's LDS stores follow block 0's LDS loads
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  t16_mode3(x1, ua, xw, g);
  const uint32_t so = (uint32_t)(64 * g) * (uint32_t)NT + 2 * c;
#pragma unroll
  for (int i3 = 0; i3 < 16; ++i3) {
    const tf_f32x4 e = t16_mode4(ub, xw, i3, g);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (live) *reinterpret_cast<PT*>(out + t0 + (int64_t)(i3 + 16 * v) * NT + so) = T16Pair<TO>::make(e0[i3][v], e[v]);
  }
}

size_t transform16_lds_bytes() { return (size_t)kT16Waves * 16 * kT16Pitch * sizeof(float); }

template <typename TO>
int launch_transform16(const float* in, TO* out, const TensorDesc* tds, const int2* items, int nitems,
                       const float* table, int inverse, hipStream_t stream) {
  if (nitems == 0) return HT_OK;
  if (reinterpret_cast<uintptr_t>(in) % 8 != 0 || reinterpret_cast<uintptr_t>(out) % (2 * sizeof(TO)) != 0)
    HT_FAIL(HT_ERR_UNSUPPORTED, "two-modes-of-16 transform: unaligned buffers");
  const size_t lds = transform16_lds_bytes();
  int rc = ensure_dynamic_lds((const void*)k_transform16<TO>, lds);
  if (rc) return rc;
  const unsigned grid = (unsigned)((nitems + kT16Waves - 1) / kT16Waves);
  hipLaunchKernelGGL((k_transform16<TO>), dim3(grid), dim3(64 * kT16Waves), lds, stream, in, out, tds, items, nitems,
                     table, inverse);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template int launch_transform16<float>(const float*, float*, const TensorDesc*, const int2*, int, const float*, int,
                                       hipStream_t);
template int launch_transform16<uint16_t>(const float*, uint16_t*, const TensorDesc*, const int2*, int, const float*,
                                          int, hipStream_t);

// ---------------------------------------------------------------------------
// Unitary DFT on every mode 3..d (complex slices).  The tile holds TP tube
// positions of all P slices as two planes (real, imaginary).  Forward: the
// real X tile is transformed mode by mode with the complex matrices and the
// canonical slice of every conjugate pair is stored as its stacked block
// [Re; Im]; the partner (the conjugate, for real X) is not stored.  Inverse:
// every slice is filled from its slot (conjugated for partners), the inverse
// matrices are applied and the real part is stored (the imaginary part is
// zero up to rounding for conjugate-symmetric data).
// ---------------------------------------------------------------------------
template <typename T, int NMAX>
__device__ __forceinline__ void cplx_fiber(T* re, T* im, int base, int stride, int n, const T* __restrict__ M) {
  T vr[NMAX], vi[NMAX];
#pragma unroll
  for (int b = 0; b < NMAX; ++b) {
    vr[b] = (b < n) ? re[base + b * stride] : T(0);
    vi[b] = (b < n) ? im[base + b * stride] : T(0);
  }
#pragma unroll
  for (int a = 0; a < NMAX; ++a) {
    if (a < n) {
      T sr = T(0), si = T(0);
#pragma unroll
      for (int b = 0; b < NMAX; ++b) {
        if (b < n) {
          const T mr = M[2 * (a * n + b)], mi = M[2 * (a * n + b) + 1];
          sr += mr * vr[b] - mi * vi[b];
          si += mr * vi[b] + mi * vr[b];
        }
      }
      re[base + a * stride] = sr;
      im[base + a * stride] = si;
    }
  }
}

// The same product for a DFT mode of power-of-two length N, as an in-register
// radix-2 fast Fourier transform (decimation in time, bit-reversed load,
// natural-order result) of the unscaled sums: the mode's matrix is
// s exp(-+ 2 pi i a b / N) (minus forward, plus inverse), and its real scale s
// (the first entry) is left to the caller, which applies the product of the
// scales of all such modes once.  The twiddles exp(-+ 2 pi i k / N) are
// compile-time constants: k = 0 and k = N / 4 (a multiply by -+ i) cost no
// multiplications; N log2 N / 2 butterflies instead of N^2 multiply-adds.
template <int N>
struct Log2 {
  static constexpr int value = 1 + Log2<N / 2>::value;
};
template <>
struct Log2<1> {
  static constexpr int value = 0;
};

// cos(2 pi k / n) and sin(2 pi k / n) by their Taylor series (evaluated by the
// compiler; |angle| <= pi, 40 terms leave an error far below FP64 rounding)
constexpr double ce_trig(int k, int n, bool want_sin) {
  const double pi = 3.14159265358979323846264338327950288;
  double x = 2.0 * pi * (double)k / (double)n;
  if (x > pi) x -= 2.0 * pi;
  double term = want_sin ? x : 1.0, sum = term;
  for (int i = 0; i < 40; ++i) {
    const double d1 = 2.0 * i + (want_sin ? 2.0 : 1.0), d2 = 2.0 * i + (want_sin ? 3.0 : 2.0);
    term *= -x * x / (d1 * d2);
    sum += term;
  }
  return sum;
}

template <typename T, int N, bool INV>
struct Twiddles {
  T re[N / 2 > 0 ? N / 2 : 1], im[N / 2 > 0 ? N / 2 : 1];
  constexpr Twiddles() : re(), im() {
    for (int k = 0; k < N / 2; ++k) {
      re[k] = (T)ce_trig(k, N, false);
      im[k] = (T)((INV ? 1.0 : -1.0) * ce_trig(k, N, true));
    }
  }
};

// In-register form: xr, xi hold the N values in natural order on entry and
// their transform in natural order on return (the bit-reversed placement is
// resolved at compile time).  E is T, or a vector of T holding independent
// transforms in its lanes.
template <typename T, int N, bool INV, typename E = T>
__device__ __forceinline__ void fft_regs(E (&xr)[N], E (&xi)[N]) {
  constexpr int LG = Log2<N>::value;
  constexpr Twiddles<T, N, INV> W{};
  E yr[N], yi[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    int r = 0;
#pragma unroll
    for (int b = 0; b < LG; ++b) r |= ((m >> b) & 1) << (LG - 1 - b);
    yr[r] = xr[m];
    yi[r] = xi[m];
  }
#pragma unroll
  for (int len = 2; len <= N; len <<= 1) {
    const int half = len / 2, step = N / len;
#pragma unroll
    for (int s0 = 0; s0 < N; s0 += len)
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const int a = s0 + j, b = s0 + j + half, k = j * step;
        E tr, ti;
        if (k == 0) {
          tr = yr[b];
          ti = yi[b];
        } else if (4 * k == N) {  // exp(-+ i pi / 2) = -+ i
          tr = INV ? -yi[b] : yi[b];
          ti = INV ? yr[b] : -yr[b];
        } else {
          tr = W.re[k] * yr[b] - W.im[k] * yi[b];
          ti = W.re[k] * yi[b] + W.im[k] * yr[b];
        }
        yr[b] = yr[a] - tr;
        yi[b] = yi[a] - ti;
        yr[a] += tr;
        yi[a] += ti;
      }
  }
#pragma unroll
  for (int m = 0; m < N; ++m) {
    xr[m] = yr[m];
    xi[m] = yi[m];
  }
}

template <typename T, int N, bool INV>
__device__ __forceinline__ void fft_fiber(T* re, T* im, int base, int stride) {
  T xr[N], xi[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    xr[m] = re[base + m * stride];
    xi[m] = im[base + m * stride];
  }
  fft_regs<T, N, INV>(xr, xi);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    re[base + k * stride] = xr[k];
    im[base + k * stride] = xi[k];
  }
}

template <typename T, typename TO, bool inverse, int NMAX>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) void k_transform_cplx(const T* __restrict__ in_all, TO* __restrict__ out_all,
                                                        const TensorDesc* __restrict__ tds,
                                                        const int2* __restrict__ items, int nitems,
                                                        const T* __restrict__ table,
                                                        const int32_t* __restrict__ cmap_all, int aligned) {
  constexpr int V = 16 / sizeof(T);  // elements per 16-byte access
  constexpr int UNR = (inverse || NMAX > 32) ? 4 : 8;  // accesses in flight per thread (two per access when inverse)
  using VT = __attribute__((ext_vector_type(V))) T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* re = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  // The workgroup walks the items blockIdx.x, blockIdx.x + gridDim.x, ...; the
  // first batch of loads of the next item is in flight while the current one
  // is transformed and stored.
  struct Tile {
    const TensorDesc* td;
    int64_t NT, t0;
    int64_t sbase;  // offset in a stacked slot of the first tube position
    int P, TP, lgTP, n1, tp, total, nv;
    int nvl;           // vector accesses of the loads (inverse: over the stored slots)
    bool vec, onecol;  // onecol: the tile's tube positions share one slice column
  };
  // offset in a stacked slot [Re; Im] (2 n1 x n2) of tube position t0 + t
  auto slot_off = [](const Tile& c, int t) -> int64_t {
    if (c.onecol) return c.sbase + t;
    const int64_t tt = c.t0 + t;
    return tt % c.n1 + (tt / c.n1) * 2 * c.n1;
  };
  auto tile_of = [&](int it) -> Tile {
    const int2 item = items[it];
    Tile c;
    c.td = tds + item.x;
    c.NT = c.td->NT;
    c.P = c.td->P;
    c.TP = c.td->TP;
    c.lgTP = c.td->lgTP;
    c.n1 = c.td->n1;
    c.t0 = item.y;
    const int64_t rem = c.NT - c.t0;
    c.tp = rem < c.TP ? (int)rem : c.TP;
    c.total = c.TP * c.P;
    c.nv = c.total / V;
    c.nvl = (inverse ? c.TP * c.td->nslots : c.total) / V;
    // V consecutive tube positions of one slice are V consecutive rows of one
    // column of the slice (and of its slot) when these hold
    c.vec = aligned && c.TP % V == 0 && c.NT % V == 0 && c.n1 % V == 0 && c.td->x % V == 0 && c.td->a % V == 0;
    const int64_t i1 = c.t0 % c.n1;
    c.sbase = i1 + (c.t0 / c.n1) * 2 * c.n1;
    c.onecol = i1 + c.TP <= c.n1;
    return c;
  };
  VT rr[UNR], ri[inverse ? UNR : 1];
  // one batch of vector loads (vector tiles only): the UNR accesses from v0;
  // inverse: access vi covers V tube positions of stored slot vi V / TP, read
  // once and placed in the tile for both members of its conjugate pair
  auto issue = [&](const Tile& c, int v0) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int vi = v0 + u * nt, idx = vi * V;
      const int j = idx >> c.lgTP, t = idx & (c.TP - 1);
      const bool ok = vi < c.nvl && t < c.tp;
      if constexpr (!inverse) {
        const T* in = in_all + c.td->x;
        rr[u] = ok ? *reinterpret_cast<const VT*>(in + (int64_t)j * c.NT + c.t0 + t) : VT{};
      } else {
        const T* S = in_all + c.td->a + (int64_t)(ok ? j : 0) * 2 * c.NT + slot_off(c, t);  // slots [Re; Im]
        rr[u] = ok ? *reinterpret_cast<const VT*>(S) : VT{};
        ri[u] = ok ? *reinterpret_cast<const VT*>(S + c.n1) : VT{};
      }
    }
  };
  auto stash = [&](const Tile& c, int v0) {
    T* im = re + c.total;
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int vi = v0 + u * nt;
      if (vi < c.nvl) {
        if constexpr (inverse) {
          const int idx = vi * V, slot = idx >> c.lgTP, t = idx & (c.TP - 1);
          const int32_t* smap = cmap_all + c.td->cmap + c.P + 2 * slot;
          const int j = smap[0], jp = smap[1];
          *reinterpret_cast<VT*>(re + j * c.TP + t) = rr[u];
          *reinterpret_cast<VT*>(im + j * c.TP + t) = ri[u];
          if (jp >= 0) {  // the conjugate partner
            *reinterpret_cast<VT*>(re + jp * c.TP + t) = rr[u];
            *reinterpret_cast<VT*>(im + jp * c.TP + t) = -ri[u];
          }
        } else {
          *reinterpret_cast<VT*>(re + vi * V) = rr[u];
          *reinterpret_cast<VT*>(im + vi * V) = VT{};
        }
      }
    }
  };
  int it = blockIdx.x;
  if (it >= nitems) return;
  Tile cur = tile_of(it);
  if (cur.vec) issue(cur, tid);
  for (;;) {
    T* im = re + cur.total;
    const int32_t* cmap = cmap_all + cur.td->cmap;
    // ---- load: the batch in flight, then any further batches ------------------
    if (cur.vec) {
      stash(cur, tid);
      for (int v0 = tid + UNR * nt; v0 < cur.nvl; v0 += UNR * nt) {
        issue(cur, v0);
        stash(cur, v0);
      }
    } else if constexpr (!inverse) {
      const T* in = in_all + cur.td->x;
      for (int idx = tid; idx < cur.total; idx += nt) {
        const int j = idx >> cur.lgTP, t = idx & (cur.TP - 1);
        re[idx] = (t < cur.tp) ? in[(int64_t)j * cur.NT + cur.t0 + t] : T(0);
        im[idx] = T(0);
      }
    } else {
      const T* C = in_all + cur.td->a;
      for (int idx = tid; idx < cur.total; idx += nt) {
        const int j = idx >> cur.lgTP, t = idx & (cur.TP - 1);
        T vr = T(0), vi = T(0);
        if (t < cur.tp) {
          const int32_t code = cmap[j];
          const int slot = code & 0x7fffffff;
          const T* S = C + (int64_t)slot * 2 * cur.NT + slot_off(cur, t);
          vr = S[0];
          vi = S[cur.n1];
          if (code < 0) vi = -vi;  // conjugate partner
        }
        re[idx] = vr;
        im[idx] = vi;
      }
    }
    __syncthreads();
    const int nxt = it + gridDim.x;
    Tile nc{};
    if (nxt < nitems) {
      nc = tile_of(nxt);
      if (nc.vec) issue(nc, tid);
    }
    // ---- modes ---------------------------------------------------------------------
    const ModeTable* mt = inverse ? &cur.td->inv : &cur.td->fwd;
    T post = T(1);  // product of the scales the FFT modes leave out
    for (int m = 0; m < mt->nmodes; ++m) {
      const int n = mt->n[m];
      const int s = mt->stride[m];
      const T* M = table + mt->off[m];
      const int nfib = cur.total / n;
      if (n == 2 || n == 4 || n == 8 || (NMAX >= 16 && n == 16) || (NMAX >= 32 && n == 32)) post *= M[0];
      for (int f = tid; f < nfib; f += nt) {
        const int base = fiber_base(f, cur.TP, cur.lgTP, s, n);
        const int st = s * cur.TP;
        if (n == 2) {
          fft_fiber<T, 2, inverse>(re, im, base, st);
        } else if (n == 4) {
          fft_fiber<T, 4, inverse>(re, im, base, st);
        } else if (n == 8) {
          fft_fiber<T, 8, inverse>(re, im, base, st);
        } else if (n <= 8) {
          cplx_fiber<T, 8>(re, im, base, st, n, M);
        } else if constexpr (NMAX >= 16) {
          if (n == 16) {
            fft_fiber<T, 16, inverse>(re, im, base, st);
          } else if (n <= 16) {
            cplx_fiber<T, 16>(re, im, base, st, n, M);
          } else if constexpr (NMAX >= 32) {
            if (n == 32) {
              fft_fiber<T, 32, inverse>(re, im, base, st);
            } else if (n <= 32) {
              cplx_fiber<T, 32>(re, im, base, st, n, M);
            } else if constexpr (NMAX >= 64) {
              cplx_fiber<T, 64>(re, im, base, st, n, M);
            }
          }
        }
      }
      __syncthreads();
    }
    // ---- store ---------------------------------------------------------------------
    const int64_t NT = cur.NT;
    const int n1 = cur.n1, TP = cur.TP, lgTP = cur.lgTP, tp = cur.tp;
    if (!inverse) {
      TO* A = out_all + cur.td->a;
      if (cur.vec) {
        for (int vi = tid; vi < cur.nv; vi += nt) {
          const int idx = vi * V;
          const int j = idx >> lgTP, t = idx & (TP - 1);
          const int32_t code = cmap[j];
          if (t < tp && code >= 0) {  // canonical member of its pair
            TO* S = A + (int64_t)code * 2 * NT + slot_off(cur, t);
            const VT vr = *reinterpret_cast<const VT*>(re + idx) * post;
            const VT vi2 = *reinterpret_cast<const VT*>(im + idx) * post;
            if constexpr (std::is_same<TO, T>::value) {
              *reinterpret_cast<VT*>(S) = vr;
              *reinterpret_cast<VT*>(S + n1) = vi2;
            } else {
              typedef unsigned int u2 __attribute__((ext_vector_type(2)));
              *reinterpret_cast<u2*>(S) = u2{f32x2_to_bf16x2(vr[0], vr[1]), f32x2_to_bf16x2(vr[2], vr[3])};
              *reinterpret_cast<u2*>(S + n1) = u2{f32x2_to_bf16x2(vi2[0], vi2[1]), f32x2_to_bf16x2(vi2[2], vi2[3])};
            }
          }
        }
      } else {
        for (int idx = tid; idx < cur.total; idx += nt) {
          const int j = idx >> lgTP, t = idx & (TP - 1);
          const int32_t code = cmap[j];
          if (t < tp && code >= 0) {  // canonical member of its pair
            TO* S = A + (int64_t)code * 2 * NT + slot_off(cur, t);
            if constexpr (std::is_same<TO, T>::value) {
              S[0] = re[idx] * post;
              S[n1] = im[idx] * post;
            } else {
              S[0] = f32_to_bf16_rne((float)(re[idx] * post));
              S[n1] = f32_to_bf16_rne((float)(im[idx] * post));
            }
          }
        }
      }
    } else {
      TO* out = out_all + cur.td->x;
      if (cur.vec && std::is_same<TO, T>::value) {
        for (int vi = tid; vi < cur.nv; vi += nt) {
          const int idx = vi * V;
          const int j = idx >> lgTP, t = idx & (TP - 1);
          if (t < tp)
            *reinterpret_cast<VT*>(out + (int64_t)j * NT + cur.t0 + t) = *reinterpret_cast<const VT*>(re + idx) * post;
        }
      } else {
        for (int idx = tid; idx < cur.total; idx += nt) {
          const int j = idx >> lgTP, t = idx & (TP - 1);
          if (t < tp) out[(int64_t)j * NT + cur.t0 + t] = (TO)(re[idx] * post);
        }
      }
    }
    if (nxt >= nitems) break;
    __syncthreads();  // the tile's LDS is read by the stores above before the next stash
    it = nxt;
    cur = nc;
  }
}

// ---------------------------------------------------------------------------
// Fused form of the same transform, for tensors with at least two transformed
// modes, all of power-of-two length <= 32, whose tiles take 16-byte accesses
// (ModeTable::first names the shortest mode).  The first mode (length
// NF <= 8, slice stride sf) is applied in registers while the tile is loaded:
// a thread takes V consecutive tube positions of the NF slices j0 + k sf of
// one fiber of that mode (one 16-byte load per slice and plane; the inverse
// reads each slice's slot, conjugated for a partner), transforms the V fibers
// and writes them to the LDS tile.  The other modes run in place in LDS; the
// forward tile leaves with 16-byte stores (8 BF16 or V values of a canonical
// slot); the inverse applies its last mode (ModeTable::last) in registers as
// it stores the real parts (dft_last_inverse), which measured faster than a
// further LDS pass with 16-byte stores.  The slot map of the tile's tensor is copied next to
// the tile so that no global load of the map waits behind the next tile's
// loads, which are in flight while the current tile is transformed and
// stored.
// ---------------------------------------------------------------------------
// Last mode of the inverse in registers: fiber (tube position t, slices
// j0 + k sl) from the LDS tile, transformed, and the real parts stored
// straight to the output slices (consecutive lanes hold consecutive
// positions, so each store covers runs of the slice's row).
template <typename T, int N>
__device__ __forceinline__ void dft_last_inverse(const T* re, const T* im, int base, int stride, int j0, int sl,
                                                 int t, bool live, T post, T* __restrict__ out, int64_t NT,
                                                 int64_t t0) {
  T xr[N], xi[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    xr[k] = re[base + k * stride];
    xi[k] = im[base + k * stride];
  }
  fft_regs<T, N, true>(xr, xi);
  if (!live) return;
#pragma unroll
  for (int k = 0; k < N; ++k) __builtin_nontemporal_store(xr[k] * post, out + (int64_t)(j0 + k * sl) * NT + t0 + t);
}

template <typename T, typename TO, bool inverse, int NF>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) void k_transform_dft(
    const T* __restrict__ in_all, TO* __restrict__ out_all, const TensorDesc* __restrict__ tds,
    const int2* __restrict__ items, int nitems, const T* __restrict__ table, const int32_t* __restrict__ cmap_all) {
  constexpr int V = 16 / sizeof(T);  // elements per 16-byte access
  using VT = __attribute__((ext_vector_type(V))) T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* re = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  struct Tile {
    const TensorDesc* td;
    const ModeTable* mt;
    int64_t NT, t0;
    int P, TP, lgTP, n1, tp, total;
    int nu;    // load units: TP / V tube vectors x P / NF fibers of the first mode
    int lgTV;  // log2(TP / V)
    int sf;    // slice stride of the first mode
  };
  auto tile_of = [&](int it) -> Tile {
    const int2 item = items[it];
    Tile c;
    c.td = tds + item.x;
    c.mt = inverse ? &c.td->inv : &c.td->fwd;
    c.NT = c.td->NT;
    c.P = c.td->P;
    c.TP = c.td->TP;
    c.lgTP = c.td->lgTP;
    c.n1 = c.td->n1;
    c.t0 = item.y;
    const int64_t rem = c.NT - c.t0;
    c.tp = rem < c.TP ? (int)rem : c.TP;
    c.total = c.TP * c.P;
    c.lgTV = c.lgTP - Log2<V>::value;
    c.nu = c.total / (V * NF);
    c.sf = c.mt->stride[c.mt->first];
    return c;
  };
  // offset in a stacked slot [Re; Im] (2 n1 x n2) of tube position t0 + t
  auto slot_off = [](const Tile& c, int t) -> int64_t {
    const int64_t tt = c.t0 + t;
    return tt % c.n1 + (tt / c.n1) * 2 * c.n1;
  };
  // LDS copy of the slot map of tile c's tensor
  auto lds_map = [&](const Tile& c) { return reinterpret_cast<int32_t*>(re + 2 * c.total); };
  // unit u: tube positions t .. t + V - 1 (t = V (u mod TP / V)) of the slices
  // j0 + k sf, k < NF, of fiber u / (TP / V) of the first mode
  auto unit = [](const Tile& c, int u, int& t, int& j0) {
    const int f = u >> c.lgTV;
    t = (u & ((1 << c.lgTV) - 1)) * V;
    j0 = f % c.sf + (f / c.sf) * c.sf * NF;
  };
  VT lr[NF], li[inverse ? NF : 1];
  unsigned neg = 0;  // inverse: slices read conjugated (partners), one bit per k
  // the loads of unit u, with the slot map of its tensor from LDS (FROM_LDS) or global memory
  auto issue = [&](const Tile& c, int u, auto from_lds) {
    constexpr bool L = decltype(from_lds)::value;
    int t, j0;
    unit(c, u, t, j0);
    const bool ok = u < c.nu && t < c.tp;
    neg = 0;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int j = j0 + k * c.sf;
      if constexpr (!inverse) {
        const T* src = in_all + c.td->x + (ok ? (int64_t)j * c.NT + c.t0 + t : 0);
        lr[k] = ok ? *reinterpret_cast<const VT*>(src) : VT{};
      } else {
        const int32_t* mp = L ? lds_map(c) : cmap_all + c.td->cmap;
        const int32_t code = ok ? mp[j] : 0;
        const T* S = in_all + c.td->a + (int64_t)(code & 0x7fffffff) * 2 * c.NT + (ok ? slot_off(c, t) : 0);
        lr[k] = ok ? *reinterpret_cast<const VT*>(S) : VT{};
        li[k] = ok ? *reinterpret_cast<const VT*>(S + c.n1) : VT{};
        neg |= (code < 0 ? 1u : 0u) << k;
      }
    }
  };
  // the first mode of unit u (loads in lr / li) into the LDS tile
  auto first_mode = [&](const Tile& c, int u) {
    if (u >= c.nu) return;
    int t, j0;
    unit(c, u, t, j0);
    T* im = re + c.total;
    VT orr[NF], oii[NF];  // V transforms at once, one per vector lane
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      orr[k] = lr[k];
      if constexpr (inverse)
        oii[k] = ((neg >> k) & 1u) ? -li[k] : li[k];
      else
        oii[k] = VT{};
    }
    fft_regs<T, NF, inverse, VT>(orr, oii);
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int o = (j0 + k * c.sf) * c.TP + t;
      *reinterpret_cast<VT*>(re + o) = orr[k];
      *reinterpret_cast<VT*>(im + o) = oii[k];
    }
  };
  int it = blockIdx.x;
  if (it >= nitems) return;
  Tile cur = tile_of(it);
  issue(cur, tid, std::false_type{});
  for (;;) {
    T* im = re + cur.total;
    int32_t* smap = lds_map(cur);
    // ---- load with the first mode ------------------------------------------------
    {
      const int32_t* gmap = cmap_all + cur.td->cmap;
      for (int j = tid; j < cur.P; j += nt) smap[j] = gmap[j];
    }
    first_mode(cur, tid);
    for (int u = tid + nt; u < cur.nu; u += nt) {
      issue(cur, u, std::false_type{});
      first_mode(cur, u);
    }
    __syncthreads();
    const int nxt = it + gridDim.x;
    Tile nc{};
    if (nxt < nitems) {
      nc = tile_of(nxt);
      if (nc.td == cur.td)
        issue(nc, tid, std::true_type{});
      else
        issue(nc, tid, std::false_type{});
    }
    // ---- the other modes -----------------------------------------------------------
    const ModeTable* mt = cur.mt;
    T post = table[mt->off[mt->first]];  // scales the FFTs leave out
    for (int m = 0; m < mt->nmodes; ++m) {
      if (m == mt->first || (inverse && m == mt->last)) continue;  // inverse: last mode with the store
      const int n = mt->n[m];  // a power of two <= 32 (ModeTable::first)
      const int s = mt->stride[m];
      post *= table[mt->off[m]];
      const int nfib = cur.total / n, st = s * cur.TP;
      for (int f = tid; f < nfib; f += nt) {
        const int base = fiber_base(f, cur.TP, cur.lgTP, s, n);
        if (n == 2)
          fft_fiber<T, 2, inverse>(re, im, base, st);
        else if (n == 4)
          fft_fiber<T, 4, inverse>(re, im, base, st);
        else if (n == 8)
          fft_fiber<T, 8, inverse>(re, im, base, st);
        else if (n == 16)
          fft_fiber<T, 16, inverse>(re, im, base, st);
        else if (n == 32)
          fft_fiber<T, 32, inverse>(re, im, base, st);
      }
      __syncthreads();
    }
    // ---- store ---------------------------------------------------------------------
    const int64_t NT = cur.NT;
    const int n1 = cur.n1, TP = cur.TP, lgTP = cur.lgTP, tp = cur.tp;
    if constexpr (!inverse) {
      TO* A = out_all + cur.td->a;
      bool wide = false;  // 8 BF16 (16 bytes) per store
      if constexpr (!std::is_same<TO, T>::value)
        wide = n1 % 8 == 0 && NT % 8 == 0 && cur.td->a % 8 == 0 && TP % 8 == 0;
      if constexpr (!std::is_same<TO, T>::value) {
        if (wide) {
          typedef unsigned int u4 __attribute__((ext_vector_type(4)));
          auto pack = [&](const T* p) {
            const VT a = *reinterpret_cast<const VT*>(p) * post, b = *reinterpret_cast<const VT*>(p + 4) * post;
            return u4{f32x2_to_bf16x2(a[0], a[1]), f32x2_to_bf16x2(a[2], a[3]), f32x2_to_bf16x2(b[0], b[1]),
                      f32x2_to_bf16x2(b[2], b[3])};
          };
          for (int vi = tid; vi < cur.total / 8; vi += nt) {
            const int idx = vi * 8, j = idx >> lgTP, t = idx & (TP - 1);
            const int32_t code = smap[j];
            if (t < tp && code >= 0) {  // canonical member of its pair
              TO* S = A + (int64_t)code * 2 * NT + slot_off(cur, t);
              *reinterpret_cast<u4*>(S) = pack(re + idx);
              *reinterpret_cast<u4*>(S + n1) = pack(im + idx);
            }
          }
        }
      }
      if (!wide) {
        for (int vi = tid; vi < cur.total / V; vi += nt) {
          const int idx = vi * V, j = idx >> lgTP, t = idx & (TP - 1);
          const int32_t code = smap[j];
          if (t < tp && code >= 0) {
            TO* S = A + (int64_t)code * 2 * NT + slot_off(cur, t);
            const VT vr = *reinterpret_cast<const VT*>(re + idx) * post;
            const VT vi2 = *reinterpret_cast<const VT*>(im + idx) * post;
            if constexpr (std::is_same<TO, T>::value) {
              *reinterpret_cast<VT*>(S) = vr;
              *reinterpret_cast<VT*>(S + n1) = vi2;
            } else {
              typedef unsigned int u2 __attribute__((ext_vector_type(2)));
              *reinterpret_cast<u2*>(S) = u2{f32x2_to_bf16x2(vr[0], vr[1]), f32x2_to_bf16x2(vr[2], vr[3])};
              *reinterpret_cast<u2*>(S + n1) = u2{f32x2_to_bf16x2(vi2[0], vi2[1]), f32x2_to_bf16x2(vi2[2], vi2[3])};
            }
          }
        }
      }
    } else {
      post *= table[mt->off[mt->last]];
      const int nl = mt->n[mt->last], sl = mt->stride[mt->last], nfib = cur.total / nl, st = sl * TP;
      T* out = reinterpret_cast<T*>(out_all) + cur.td->x;
      for (int f = tid; f < nfib; f += nt) {
        const int base = fiber_base(f, TP, lgTP, sl, nl);
        const int t = f & (TP - 1), j0 = base >> lgTP;
        const bool live = t < tp;
        if (nl == 2)
          dft_last_inverse<T, 2>(re, im, base, st, j0, sl, t, live, post, out, NT, cur.t0);
        else if (nl == 4)
          dft_last_inverse<T, 4>(re, im, base, st, j0, sl, t, live, post, out, NT, cur.t0);
        else if (nl == 8)
          dft_last_inverse<T, 8>(re, im, base, st, j0, sl, t, live, post, out, NT, cur.t0);
        else if (nl == 16)
          dft_last_inverse<T, 16>(re, im, base, st, j0, sl, t, live, post, out, NT, cur.t0);
        else if (nl == 32)
          dft_last_inverse<T, 32>(re, im, base, st, j0, sl, t, live, post, out, NT, cur.t0);
      }
    }
    if (nxt >= nitems) break;
    __syncthreads();  // the tile and its map are read above before the next tile replaces them
    it = nxt;
    cur = nc;
  }
}

// workgroups that stay resident for the whole launch, each walking its items
int resident_grid(const void* kern, size_t lds, int nitems) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds) != hipSuccess) return -1;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  return std::max(1, std::min(nitems, std::max(per_cu, 1) * ncu));
}

template <typename T, typename TO, int NF>
int launch_transform_dft(const T* in, TO* out, const TensorDesc* tds, const int2* items, int nitems, size_t lds,
                         const T* table, const int32_t* cmap, int inverse, hipStream_t stream) {
  const void* kern = inverse ? (const void*)k_transform_dft<T, TO, true, NF>
                             : (const void*)k_transform_dft<T, TO, false, NF>;
  int rc = ensure_dynamic_lds(kern, 160 * 1024);
  if (rc) return rc;
  const int grid = resident_grid(kern, lds, nitems);
  if (grid < 0) HT_FAIL(HT_ERR_HIP, "occupancy query failed");
  if (inverse)
    hipLaunchKernelGGL((k_transform_dft<T, TO, true, NF>), dim3((unsigned)grid), dim3(256), lds, stream, in,
                       out, tds, items, nitems, table, cmap);
  else
    hipLaunchKernelGGL((k_transform_dft<T, TO, false, NF>), dim3((unsigned)grid), dim3(256), lds, stream, in,
                       out, tds, items, nitems, table, cmap);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template <typename T, typename TO, int NMAX>
int launch_transform_cplx_n(const T* in, TO* out, const TensorDesc* tds, const int2* items, int nitems, size_t lds,
                            const T* table, const int32_t* cmap, int inverse, hipStream_t stream) {
  const int aligned = (reinterpret_cast<uintptr_t>(in) % 16 == 0) && (reinterpret_cast<uintptr_t>(out) % 16 == 0);
  const void* kern = inverse ? (const void*)k_transform_cplx<T, TO, true, NMAX>
                             : (const void*)k_transform_cplx<T, TO, false, NMAX>;
  int rc = ensure_dynamic_lds(kern, 160 * 1024);
  if (rc) return rc;
  const int grid = resident_grid(kern, lds, nitems);
  if (grid < 0) HT_FAIL(HT_ERR_HIP, "occupancy query failed");
  if (inverse)
    hipLaunchKernelGGL((k_transform_cplx<T, TO, true, NMAX>), dim3((unsigned)grid), dim3(256), lds, stream, in, out,
                       tds, items, nitems, table, cmap, aligned);
  else
    hipLaunchKernelGGL((k_transform_cplx<T, TO, false, NMAX>), dim3((unsigned)grid), dim3(256), lds, stream, in, out,
                       tds, items, nitems, table, cmap, aligned);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

// nmax: the longest transformed mode (selects the fiber kernels compiled in)
template <typename T, typename TO>
int launch_transform_cplx(const T* in, TO* out, const TensorDesc* tds, const int2* items, int nitems, size_t lds,
                          const T* table, const int32_t* cmap, int inverse, int nmax, int nf, hipStream_t stream) {
  if (nitems == 0) return HT_OK;
  if (lds > 160 * 1024) HT_FAIL(HT_ERR_UNSUPPORTED, "transform tile above the LDS size");
  if (nmax > 64) HT_FAIL(HT_ERR_UNSUPPORTED, "DFT mode longer than 64");
  const bool aligned = reinterpret_cast<uintptr_t>(in) % 16 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0;
  if (nf > 0 && aligned) {
    if (nf == 2) return launch_transform_dft<T, TO, 2>(in, out, tds, items, nitems, lds, table, cmap, inverse, stream);
    if (nf == 4) return launch_transform_dft<T, TO, 4>(in, out, tds, items, nitems, lds, table, cmap, inverse, stream);
    if (nf == 8) return launch_transform_dft<T, TO, 8>(in, out, tds, items, nitems, lds, table, cmap, inverse, stream);
    HT_FAIL(HT_ERR_UNSUPPORTED, "fused DFT transform: first mode longer than 8");
  }
  if (nmax <= 8)
    return launch_transform_cplx_n<T, TO, 8>(in, out, tds, items, nitems, lds, table, cmap, inverse, stream);
  if (nmax <= 16)
    return launch_transform_cplx_n<T, TO, 16>(in, out, tds, items, nitems, lds, table, cmap, inverse, stream);
  if (nmax <= 32)
    return launch_transform_cplx_n<T, TO, 32>(in, out, tds, items, nitems, lds, table, cmap, inverse, stream);
  return launch_transform_cplx_n<T, TO, 64>(in, out, tds, items, nitems, lds, table, cmap, inverse, stream);
}

template int launch_transform_cplx<float, float>(const float*, float*, const TensorDesc*, const int2*, int, size_t,
                                                 const float*, const int32_t*, int, int, int, hipStream_t);
template int launch_transform_cplx<double, double>(const double*, double*, const TensorDesc*, const int2*, int,
                                                   size_t, const double*, const int32_t*, int, int, int, hipStream_t);
template int launch_transform_cplx<float, uint16_t>(const float*, uint16_t*, const TensorDesc*, const int2*, int,
                                                    size_t, const float*, const int32_t*, int, int, int,
                                                    hipStream_t);

int transform_tile_width(int64_t P, size_t elem_bytes, size_t budget) {
  int64_t tp = 256;
  while (tp > 1 && (size_t)(tp * P) * elem_bytes > budget) tp >>= 1;
  if ((size_t)(tp * P) * elem_bytes > budget) return 0;
  return (int)tp;
}

template <typename T, typename TO>
int launch_transform(const T* in, TO* out, const TensorDesc* tds, const int2* items, int nitems, size_t lds,
                     const T* table, int inverse, hipStream_t stream) {
  if (nitems == 0) return HT_OK;
  if (lds > 160 * 1024) HT_FAIL(HT_ERR_UNSUPPORTED, "transform tile above the LDS size");
  int rc = ensure_dynamic_lds((const void*)k_transform<T, TO>, 160 * 1024);
  if (rc) return rc;
  const int aligned = (reinterpret_cast<uintptr_t>(in) % 16 == 0) && (reinterpret_cast<uintptr_t>(out) % 16 == 0);
  hipLaunchKernelGGL((k_transform<T, TO>), dim3((unsigned)nitems), dim3(256), lds, stream, in, out, tds, items, table,
                     inverse, aligned);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template int launch_transform<float, float>(const float*, float*, const TensorDesc*, const int2*, int, size_t,
                                            const float*, int, hipStream_t);
template int launch_transform<double, double>(const double*, double*, const TensorDesc*, const int2*, int, size_t,
                                              const double*, int, hipStream_t);
template int launch_transform<float, uint16_t>(const float*, uint16_t*, const TensorDesc*, const int2*, int, size_t,
                                               const float*, int, hipStream_t);

// ---------------------------------------------------------------------------
// Gaussian sketch matrices Omega_s (n2 x l, column-major), one per slice,
// keyed by (seed; group, slice index within the tensor, call, stream).  The
// n2 * l entries of slice s go to its table offset, or to s * dense_stride when
// dense_stride > 0; the draw of a narrower width is the prefix of a wider one.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_omega(T* __restrict__ om, double* __restrict__ om64,
                                               uint16_t* __restrict__ omh, const SliceDesc* __restrict__ sd,
                                               const int2* __restrict__ wk, uint32_t call,
                                               const int32_t* __restrict__ call_dev, uint32_t stream_base,
                                               uint64_t seed, int64_t dense_stride) {
  const int s = blockIdx.x;
  const SliceDesc d = sd[s];
  const int64_t base = dense_stride > 0 ? (int64_t)s * dense_stride : d.z;
  // complex slices draw the same real Omega (n2 x l) as real ones
  const int64_t per_slice = (int64_t)d.n2 * slice_width(d, wk, s);
  const uint32_t c = call_dev ? (uint32_t)(*call_dev) : call;
  const int64_t ngroups = (per_slice + 3) / 4;
  for (int64_t g = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; g < ngroups; g += (int64_t)gridDim.y * blockDim.x) {
    double z[4];
    gaussian4((uint64_t)g, (uint32_t)d.local, c, stream_base + (uint32_t)d.tensor, seed, z);
#pragma unroll
    for (int lane = 0; lane < 4; ++lane) {
      const int64_t e = 4 * g + lane;
      if (e < per_slice) {
        if (om) om[base + e] = (T)z[lane];
        if (om64) om64[base + e] = z[lane];
        if (omh) omh[base + e] = (uint16_t)(f32x2_to_bf16x2((float)(T)z[lane], 0.0f) & 0xffffu);
      }
    }
  }
}

template <typename T>
int launch_omega(T* om, double* om64, uint16_t* omh, const SliceDesc* sd, const int2* wk, int nslices, int64_t max_per_slice,
                 uint32_t call, const int32_t* call_dev, uint32_t stream_base, uint64_t seed, int64_t dense_stride,
                 hipStream_t stream) {
  if (nslices == 0) return HT_OK;
  const int64_t ngroups = (max_per_slice + 3) / 4;
  const unsigned gy = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(ngroups, 256), 64));
  hipLaunchKernelGGL(k_omega<T>, dim3((unsigned)nslices, gy), dim3(256), 0, stream, om, om64, omh, sd, wk, call,
                     call_dev, stream_base, seed, dense_stride);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template int launch_omega<float>(float*, double*, uint16_t*, const SliceDesc*, const int2*, int, int64_t, uint32_t,
                                 const int32_t*, uint32_t, uint64_t, int64_t, hipStream_t);
template int launch_omega<double>(double*, double*, uint16_t*, const SliceDesc*, const int2*, int, int64_t, uint32_t,
                                  const int32_t*, uint32_t, uint64_t, int64_t, hipStream_t);

}  // namespace ht
