// BF16 sketch products on the matrix cores (v_mfma_f32_32x32x16_bf16), FP32
// accumulation.  The transformed tensor A is stored in BF16; the thin operand
// (sketch matrix or basis, FP32 in memory) is rounded to BF16 while it is
// staged; the result and its FP64 Gram partials are written as in the FP32
// kernel.
//
//   nn:  Y_s (n1 x l) = A_s (n1 x n2) W_s (n2 x l)
//   tn:  Z_s (n2 x l) = A_s^T (n2 x n1) Q_s (n1 x l)
//
// One workgroup per work item (slice, first output row): MT = 32 NW output
// rows x l (<= 32 NB) columns, wavefront w owns rows 32w..32w+31.  K chunks of
// 32 are double-buffered in LDS, both operands stored with k contiguous so that each lane fetches its 8 consecutive k values with
// one 16-byte LDS read.  MFMA operand layout (32x32x16 bf16): lane t supplies
// A[t % 32][8 (t / 32) .. 8 (t / 32) + 7] and B[8 (t / 32) ..][t % 32]; the
// accumulator layout is that of the FP32 32x32 instruction.
#include "chol.hpp"

namespace ht {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int KC = 32;
constexpr int KP = KC + 8;  // LDS pitch (bf16 elements) of a k-contiguous row: 80 bytes
// Pitch of the complex kernel's rows: 88 bytes (22 banks), so that the four
// row groups of a wavefront's transposing stores fall in disjoint bank ranges
// and 32 consecutive rows read at one k cover every bank once; rows are 8-byte
// aligned, read as two 8-byte halves.
constexpr int KPC = KC + 12;

__device__ __forceinline__ u16x8 lds_u16x8(const uint16_t* p) {
  const uint2* q = reinterpret_cast<const uint2*>(p);
  const uint2 lo = q[0], hi = q[1];
  return __builtin_bit_cast(u16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
}

template <int NB, int NW>
struct Bf16Lds {
  static constexpr int MT = 32 * NW;
  static constexpr int A_ELEMS = MT * KP;
  static constexpr int B_ELEMS = 32 * NB * KP;
  static constexpr int MAIN_BYTES = 2 * (A_ELEMS + B_ELEMS) * 2;
  static constexpr int EPI_BYTES = MT * (32 * NB + 1) * 4;  // FP32 tile (the values the products store)
  static constexpr int BYTES = MAIN_BYTES > EPI_BYTES ? MAIN_BYTES : EPI_BYTES;
};

// CPLX: complex slices in the stacked layout, as the FP32 kernel (NW = 4;
// 64 complex rows per tile; wreal: the real Omega against the stored block).
template <int NB, int NW, bool TRANS, bool CPLX>
__global__ __launch_bounds__(64 * NW) void k_mfma_thin_bf16(const uint16_t* __restrict__ Aall,
                                                            const float* __restrict__ Wall, float* __restrict__ Yall,
                                                            const SliceDesc* __restrict__ sd,
                                                            const int2* __restrict__ wk, const int2* __restrict__ items,
                                                            double* __restrict__ gpart, int aligned, int wreal) {
  using L = Bf16Lds<NB, NW>;
  constexpr int MT = L::MT;
  constexpr int HM = MT / 2;
  static_assert(!CPLX || MT == 128, "complex tiles hold 64 complex rows");
  constexpr int NTH = 64 * NW;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint16_t* const lds_h = reinterpret_cast<uint16_t*>(smem_raw);
  const int2 item = items[blockIdx.x];
  const int s = item.x, r0 = item.y;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int mo = TRANS ? d.n2 : d.n1;
  const int lda = CPLX ? 2 * d.n1 : d.n1;
  const int M_out = CPLX ? 2 * mo : mo;
  const int K = CPLX ? (TRANS ? 2 * d.n1 : (wreal ? d.n2 : 2 * d.n2)) : (TRANS ? d.n1 : d.n2);
  const int ldw = K, ldy = M_out;
  const int64_t woff = TRANS ? d.y : d.z, yoff = TRANS ? d.z : d.y;
  const uint16_t* Aj = Aall + d.a;
  const float* Wj = Wall + woff;
  float* Yj = Yall + yoff;
  const bool vecA = aligned && (lda % 8 == 0) && (d.a % 8 == 0) && (!CPLX || d.n1 % 8 == 0);
  const bool vecW = aligned && (ldw % 4 == 0) && (woff % 4 == 0);
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int LW = 32 * NB;
  auto orow = [&](int i) -> int { return CPLX ? (i >= HM ? mo + r0 + i - HM : r0 + i) : r0 + i; };
  auto ovalid = [&](int i) -> bool { return CPLX ? r0 + (i >= HM ? i - HM : i) < mo : r0 + i < M_out; };
  // element (r, k) of the slice operand as BF16 bits (complex slices: the real
  // embedding; a negation flips the sign bit)
  auto aval = [&](int r, int k) -> uint16_t {
    bool neg;
    const uint16_t v = Aj[embed_index(r, k, lda, CPLX, d.n1, d.n2, neg)];
    return neg ? (uint16_t)(v ^ 0x8000u) : v;
  };
  auto avec = [&](int r, int k) -> u16x8 {  // rows r..r+7 of column k (no straddle when vecA)
    bool neg;
    u16x8 v = *reinterpret_cast<const u16x8*>(Aj + embed_index(r, k, lda, CPLX, d.n1, d.n2, neg));
    if (neg) v ^= (unsigned short)0x8000u;
    return v;
  };

  // A chunk: MT x 32 bf16 = 4 MT 16-byte groups of 8, two per thread.
  // nn: group = 8 consecutive rows of one column k;  tn: 8 consecutive k of one column.
  constexpr int NRA = MT * KC / 8 / NTH;
  constexpr int NWB = (32 * NB * KC / 4 + NTH - 1) / NTH;  // float4 groups of the thin chunk per thread
  u16x8 ra0[NRA], ra1[NRA];  // two chunks of loads in flight
  f32x4 rw0[NWB], rw1[NWB];
  auto fetch = [&](u16x8 (&ra)[NRA], f32x4 (&rw)[NWB], int k0) {
#pragma unroll
    for (int u = 0; u < NRA; ++u) {
      const int g = tid + u * NTH;
      u16x8 v;
      if (!TRANS) {
        const int kk = g / (MT / 8), row = (g % (MT / 8)) * 8;  // eight rows within one half of a complex tile
        const int gr = orow(row), gk = k0 + kk;
        if (vecA && gk < K && ovalid(row + 7)) {
          v = avec(gr, gk);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (gk < K && ovalid(row + e)) ? aval(gr + e, gk) : 0;
        }
      } else {
        const int row = g / (KC / 8), kk = (g % (KC / 8)) * 8;
        const int gc = orow(row), gk = k0 + kk;
        if (vecA && ovalid(row) && gk + 7 < K) {
          v = avec(gk, gc);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (ovalid(row) && gk + e < K) ? aval(gk + e, gc) : 0;
        }
      }
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < NWB; ++u) {
      const int f = tid + u * NTH;
      const int c = f / (KC / 4), k4 = (f % (KC / 4)) * 4;
      const int gk = k0 + k4;
      f32x4 v;
      if (vecW && f < LW * KC / 4 && c < l && gk + 3 < K) {
        v = *reinterpret_cast<const f32x4*>(Wj + gk + (int64_t)c * ldw);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (f < LW * KC / 4 && c < l && gk + e < K) ? Wj[gk + e + (int64_t)c * ldw] : 0.0f;
      }
      rw[u] = v;
    }
  };
  auto stash = [&](const u16x8 (&ra)[NRA], const f32x4 (&rw)[NWB], int buf) {
    uint16_t* As = lds_h + buf * L::A_ELEMS;
    uint16_t* Ws = lds_h + 2 * L::A_ELEMS + buf * L::B_ELEMS;
#pragma unroll
    for (int u = 0; u < NRA; ++u) {
      const int g = tid + u * NTH;
      if (!TRANS) {
        const int kk = g / (MT / 8), row = (g % (MT / 8)) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) As[(row + e) * KP + kk] = ra[u][e];
      } else {
        const int row = g / (KC / 8), kk = (g % (KC / 8)) * 8;
        *reinterpret_cast<u16x8*>(As + row * KP + kk) = ra[u];
      }
    }
#pragma unroll
    for (int u = 0; u < NWB; ++u) {
      const int f = tid + u * NTH;
      if (f < LW * KC / 4) {
        const int c = f / (KC / 4), k4 = (f % (KC / 4)) * 4;
        *reinterpret_cast<uint2*>(Ws + c * KP + k4) =
            make_uint2(f32x2_to_bf16x2(rw[u][0], rw[u][1]), f32x2_to_bf16x2(rw[u][2], rw[u][3]));
      }
    }
  };

  f32x16 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[b][r] = 0.0f;

  const int nchunks = (K + KC - 1) / KC;
  const int nbl = (l + 31) / 32;
  const int mrow = 32 * wave + (lane % 32);
  const int koff = 8 * (lane / 32);
  auto compute = [&](int buf) {
    const uint16_t* As = lds_h + buf * L::A_ELEMS;
    const uint16_t* Ws = lds_h + 2 * L::A_ELEMS + buf * L::B_ELEMS;
#pragma unroll
    for (int kh = 0; kh < KC / 16; ++kh) {
      const bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(As + mrow * KP + 16 * kh + koff));
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b < nbl) {
          const bf16x8 bv = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const u16x8*>(Ws + (32 * b + (lane % 32)) * KP + 16 * kh + koff));
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc[b], 0, 0, 0);
        }
      }
    }
  };
  // chunk c sits in LDS buffer c & 1 while chunks c + 1 and c + 2 load into
  // the register sets (unrolled by two so that the sets are fixed)
  fetch(ra0, rw0, 0);
  if (nchunks > 1) fetch(ra1, rw1, KC);
  stash(ra0, rw0, 0);
  __syncthreads();
  for (int ch = 0; ch < nchunks; ch += 2) {
    if (ch + 2 < nchunks) fetch(ra0, rw0, (ch + 2) * KC);
    compute(0);
    if (ch + 1 < nchunks) stash(ra1, rw1, 1);
    __syncthreads();
    if (ch + 1 >= nchunks) break;
    if (ch + 3 < nchunks) fetch(ra1, rw1, (ch + 3) * KC);
    compute(1);
    if (ch + 2 < nchunks) stash(ra0, rw0, 0);
    __syncthreads();
  }

  float* S = reinterpret_cast<float*>(smem_raw);
  const int sp = LW + 1;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 32 * wave + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
      const int c = 32 * b + (lane % 32);
      S[i * sp + c] = (ovalid(i) && c < l) ? acc[b][r] : 0.0f;
    }
  __syncthreads();
  for (int idx = tid; idx < MT * l; idx += NTH) {
    const int i = idx % MT, c = idx / MT;
    if (ovalid(i)) Yj[orow(i) + (int64_t)c * ldy] = S[i * sp + c];
  }
  if (gpart) {
    if (CPLX)
      tile_cgram_mfma(S, sp, 1, l, gpart + d.g1 + (int64_t)(r0 / kGramRows) * 2 * l * l);
    else
      tile_gram_mfma(S, sp, 1, min(MT, M_out - r0), l, gpart + d.g1 + (int64_t)(r0 / kGramRows) * l * l);
  }
}

// Complex slices (stacked [Ar; Ai] blocks) in BF16: Y = A W (nn; W = [Wr; Wi]
// stacked, or with wreal the real Omega) and Z = A^H Q (tn), each stored
// element of A read once.  A work item is MT / 2 complex rows of the result
// (MT / 64 groups of 64 complex rows, each held as 128 tile rows: its real
// parts, then its imaginary parts) and all l <= 32 NB columns; wavefront w
// owns tile rows 32 w .. 32 w + 31.  The reduction runs over the stored
// columns (nn) or rows (tn) of A in chunks of 32: the chunk of Ar and Ai (MT x
// 32 in LDS, k contiguous, rows in the tile's order) and the chunks of the
// real and imaginary parts of the thin operand (the BF16 copy its producer
// wrote) feed two passes of the MFMA loop,
//   nn:  Yr = Ar Wr - Ai Wi,   Yi = Ai Wr + Ar Wi
//   tn:  Zr = Ar^T Qr + Ai^T Qi,   Zi = -Ai^T Qr + Ar^T Qi
// where the second pass takes the other half of the row's group (tile row
// r ^ 64) and a sign flip is an XOR of the BF16 sign bits.  Two chunks of loads
// are in flight in registers (three when every chunk of the tile is interior);
// the epilogue writes the tile and one complex Gram partial per 64 complex rows.
template <int NB, int MT, bool TRANS>
__global__ __launch_bounds__(2 * MT) void k_cthin_bf16(const uint16_t* __restrict__ Aall,
                                                       const uint16_t* __restrict__ Wall, float* __restrict__ Yall,
                                                       const SliceDesc* __restrict__ sd, const int2* __restrict__ wk,
                                                       const int2* __restrict__ items, double* __restrict__ gpart,
                                                       int aligned, int wreal) {
  constexpr int NTH = 2 * MT, LW = 32 * NB;
  constexpr int A_ELEMS = MT * KPC, B_ELEMS = LW * KPC;  // one buffer: A chunk, then the two thin chunks
  constexpr int BUF = A_ELEMS + 2 * B_ELEMS;
  static_assert(MT % 128 == 0, "groups of 64 complex rows");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint16_t* const lds_h = reinterpret_cast<uint16_t*>(smem_raw);
  const int2 item = items[blockIdx.x];
  const int s = item.x, r0 = item.y;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int n1 = d.n1, n2 = d.n2, lda = 2 * n1;
  const int mo = TRANS ? n2 : n1;           // complex output rows
  const int K = TRANS ? n1 : n2;            // stored reduction length
  const int ldw = TRANS ? 2 * n1 : (wreal ? n2 : 2 * n2), wim = TRANS ? n1 : n2;
  const bool two = TRANS || !wreal;         // the thin operand has an imaginary part
  const int64_t woff = TRANS ? d.y : d.z, yoff = TRANS ? d.z : d.y;
  const uint16_t* Aj = Aall + d.a;
  const uint16_t* Wj = Wall + woff;  // the thin operand as BF16 (rounded by its producer)
  float* Yj = Yall + yoff;
  const bool vecA = aligned && (d.a % 8 == 0) && (n1 % 8 == 0);
  const bool vecW = aligned && (ldw % 8 == 0) && (woff % 8 == 0) && (wim % 8 == 0);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  // complex row of tile row i, whether it holds an imaginary part, validity, stacked output row
  auto crow = [&](int i) -> int { return r0 + 64 * (i >> 7) + (i & 63); };
  auto ovalid = [&](int i) -> bool { return crow(i) < mo; };
  auto orow = [&](int i) -> int { return ((i & 64) ? mo : 0) + crow(i); };

  // A chunk: MT x 32 bf16, two groups of 8 per thread.
  //   nn: thread t holds tile rows 8 (t / 16) .. + 7 of stored columns 2 (t % 16)
  //       and 2 (t % 16) + 1 (stored to LDS as pairs: rows of a wavefront's
  //       four row groups land in disjoint bank ranges with the pitch KPC)
  //   tn: group = 8 consecutive k (stored rows of Ar or Ai) of one column
  constexpr int NRA = MT * KC / 8 / NTH;
  static_assert(NRA == 2, "two groups of eight per thread");
  constexpr int NWB = (LW * KC / 8 + NTH - 1) / NTH;  // groups of 8 BF16 of one thin chunk per thread
  u16x8 ra0[NRA], ra1[NRA];
  u16x8 rw0[2][NWB], rw1[2][NWB];
  // interior chunks of a tile whose rows are all valid take plain loads
  const bool rowsA = vecA && vecW && r0 + 64 <= mo;
  // the loads of an interior chunk (rowsA, k0 + KC <= K): a fixed set of 16-byte loads
  auto fetch_fast = [&](u16x8 (&ra)[NRA], u16x8 (&rw)[2][NWB], int k0) {
#pragma unroll
      for (int u = 0; u < NRA; ++u) {
        const uint16_t* src;
        if (!TRANS) {
          const int row = (tid / 16) * 8;
          src = Aj + ((row & 64) ? n1 : 0) + crow(row) + (int64_t)(k0 + 2 * (tid % 16) + u) * lda;
        } else {
          const int g = tid + u * NTH;
          const int row = g / (KC / 8), kk = (g % (KC / 8)) * 8;
          src = Aj + ((row & 64) ? n1 : 0) + k0 + kk + (int64_t)crow(row) * lda;
        }
        ra[u] = *reinterpret_cast<const u16x8*>(src);
      }
#pragma unroll
      for (int part = 0; part < 2; ++part)
#pragma unroll
        for (int u = 0; u < NWB; ++u) {
          const int f = tid + u * NTH;
          const int c = f / (KC / 8), k8 = (f % (KC / 8)) * 8;
          const bool live = (part == 0 || two) && f < LW * KC / 8 && c < l;
          // a lane with nothing to load reads column 0 of the real part (always valid)
          const uint16_t* src = Wj + (live && part ? wim : 0) + k0 + k8 + (int64_t)(live ? c : 0) * ldw;
          const u16x8 v = *reinterpret_cast<const u16x8*>(src);
          rw[part][u] = live ? v : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        }
  };
  auto fetch = [&](u16x8 (&ra)[NRA], u16x8 (&rw)[2][NWB], int k0) {
    if (rowsA && k0 + KC <= K) {
      fetch_fast(ra, rw, k0);
      return;
    }
#pragma unroll
    for (int u = 0; u < NRA; ++u) {
      u16x8 v;
      if (!TRANS) {
        const int row = (tid / 16) * 8, gk = k0 + 2 * (tid % 16) + u, rr = crow(row);
        const uint16_t* src = Aj + ((row & 64) ? n1 : 0) + rr + (int64_t)gk * lda;
        if (vecA && gk < K && rr + 7 < n1) {
          v = *reinterpret_cast<const u16x8*>(src);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (gk < K && rr + e < n1) ? src[e] : 0;
        }
      } else {
        const int g = tid + u * NTH;
        const int row = g / (KC / 8), kk = (g % (KC / 8)) * 8;
        const int c = crow(row), gk = k0 + kk;
        const uint16_t* src = Aj + ((row & 64) ? n1 : 0) + gk + (int64_t)c * lda;
        if (vecA && c < n2 && gk + 7 < K) {
          v = *reinterpret_cast<const u16x8*>(src);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (c < n2 && gk + e < K) ? src[e] : 0;
        }
      }
      ra[u] = v;
    }
#pragma unroll
    for (int part = 0; part < 2; ++part)
#pragma unroll
      for (int u = 0; u < NWB; ++u) {
        const int f = tid + u * NTH;
        const int c = f / (KC / 8), k8 = (f % (KC / 8)) * 8;
        const int gk = k0 + k8;
        const uint16_t* src = Wj + (part ? wim : 0) + gk + (int64_t)c * ldw;
        const bool live = (part == 0 || two) && f < LW * KC / 8 && c < l;
        u16x8 v;
        if (vecW && live && gk + 7 < K) {
          v = *reinterpret_cast<const u16x8*>(src);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (live && gk + e < K) ? src[e] : (unsigned short)0;
        }
        rw[part][u] = v;
      }
  };
  auto stash = [&](const u16x8 (&ra)[NRA], const u16x8 (&rw)[2][NWB], int buf) {
    uint16_t* As = lds_h + buf * BUF;
    if (!TRANS) {
      const int row = (tid / 16) * 8, kk = 2 * (tid % 16);
#pragma unroll
      for (int e = 0; e < 8; ++e)
        *reinterpret_cast<uint32_t*>(As + (row + e) * KPC + kk) = (uint32_t)ra[0][e] | ((uint32_t)ra[1][e] << 16);
    } else {
#pragma unroll
      for (int u = 0; u < NRA; ++u) {
        const int g = tid + u * NTH;
        const int row = g / (KC / 8), kk = (g % (KC / 8)) * 8;
        uint2* dst = reinterpret_cast<uint2*>(As + row * KPC + kk);
        const uint4 w = __builtin_bit_cast(uint4, ra[u]);
        dst[0] = make_uint2(w.x, w.y);
        dst[1] = make_uint2(w.z, w.w);
      }
    }
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      uint16_t* Ws = As + A_ELEMS + part * B_ELEMS;
#pragma unroll
      for (int u = 0; u < NWB; ++u) {
        const int f = tid + u * NTH;
        if ((LW * KC / 8) % NTH == 0 || f < LW * KC / 8) {  // every thread has a group when the count divides
          const int c = f / (KC / 8), k8 = (f % (KC / 8)) * 8;
          uint2* dst = reinterpret_cast<uint2*>(Ws + c * KPC + k8);
          const uint4 w = __builtin_bit_cast(uint4, rw[part][u]);
          dst[0] = make_uint2(w.x, w.y);
          dst[1] = make_uint2(w.z, w.w);
        }
      }
    }
  };

  f32x16 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[b][r] = 0.0f;
  const int nchunks = (K + KC - 1) / KC;
  const int nbl = (l + 31) / 32;
  const int mrow = 32 * wave + (lane % 32), koff = 8 * (lane / 32);
  const bool top = (mrow & 64) == 0;  // this wavefront's rows are real parts
  // sign flips of the two passes (see above)
  const unsigned short flip1 = (TRANS && !top) ? 0x8000u : 0u;
  const unsigned short flip2 = (!TRANS && top) ? 0x8000u : 0u;
  auto compute = [&](int buf) {
    const uint16_t* As = lds_h + buf * BUF;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      if (part == 1 && !two) break;
      const uint16_t* Ws = As + A_ELEMS + part * B_ELEMS;
      const int arow = part ? (mrow ^ 64) : mrow;
      const unsigned short flip = part ? flip2 : flip1;
#pragma unroll
      for (int kh = 0; kh < KC / 16; ++kh) {
        u16x8 av = lds_u16x8(As + arow * KPC + 16 * kh + koff);
        av ^= flip;
        const bf16x8 a = __builtin_bit_cast(bf16x8, av);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          if (b < nbl) {
            const bf16x8 bv =
                __builtin_bit_cast(bf16x8, lds_u16x8(Ws + (32 * b + (lane % 32)) * KPC + 16 * kh + koff));
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc[b], 0, 0, 0);
          }
        }
      }
    }
  };
  if (rowsA && K % KC == 0) {
    // Every chunk interior: unconditional fetches with the prefetch past the
    // end clamped to the last chunk (loaded, never used), so that every path
    // through the loop issues the same loads and each stash waits only for its
    // own chunk while the next one stays in flight.
    // Three register slots: step c refills the slot of chunk c (already in
    // LDS) with chunk c + 3, multiplies chunk c and stashes chunk c + 1.
    u16x8 ra2[NRA], rw2[2][NWB];
    fetch_fast(ra0, rw0, 0);
    fetch_fast(ra1, rw1, min(1, nchunks - 1) * KC);
    fetch_fast(ra2, rw2, min(2, nchunks - 1) * KC);
    stash(ra0, rw0, 0);
    __syncthreads();
    for (int ch = 0; ch < nchunks; ch += 3) {
      fetch_fast(ra0, rw0, min(ch + 3, nchunks - 1) * KC);
      compute(ch & 1);
      stash(ra1, rw1, (ch + 1) & 1);
      __syncthreads();
      if (ch + 1 >= nchunks) break;
      fetch_fast(ra1, rw1, min(ch + 4, nchunks - 1) * KC);
      compute((ch + 1) & 1);
      stash(ra2, rw2, (ch + 2) & 1);
      __syncthreads();
      if (ch + 2 >= nchunks) break;
      fetch_fast(ra2, rw2, min(ch + 5, nchunks - 1) * KC);
      compute((ch + 2) & 1);
      stash(ra0, rw0, (ch + 3) & 1);
      __syncthreads();
    }
  } else {
    fetch(ra0, rw0, 0);
    if (nchunks > 1) fetch(ra1, rw1, KC);
    stash(ra0, rw0, 0);
    __syncthreads();
    for (int ch = 0; ch < nchunks; ch += 2) {
      if (ch + 2 < nchunks) fetch(ra0, rw0, (ch + 2) * KC);
      compute(0);
      if (ch + 1 < nchunks) stash(ra1, rw1, 1);
      __syncthreads();
      if (ch + 1 >= nchunks) break;
      if (ch + 3 < nchunks) fetch(ra1, rw1, (ch + 3) * KC);
      compute(1);
      if (ch + 2 < nchunks) stash(ra0, rw0, 0);
      __syncthreads();
    }
  }

  float* S = reinterpret_cast<float*>(smem_raw);
  const int sp = LW + 1;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 32 * wave + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
      const int c = 32 * b + (lane % 32);
      S[i * sp + c] = (ovalid(i) && c < l) ? acc[b][r] : 0.0f;
    }
  __syncthreads();
  const int ldy = 2 * mo;
  for (int idx = tid; idx < MT * l; idx += NTH) {
    const int i = idx % MT, c = idx / MT;
    if (ovalid(i)) Yj[orow(i) + (int64_t)c * ldy] = S[i * sp + c];
  }
  if (gpart)
    for (int g = 0; g < MT / 128; ++g)
      if (r0 + 64 * g < mo)
        tile_cgram_mfma(S + 128 * g * sp, sp, 1, l, gpart + d.g1 + (int64_t)((r0 + 64 * g) / kGramRows) * 2 * l * l);
}

template <int NB, bool TRANS>
int launch_cthin_bf16(const uint16_t* A, const uint16_t* W, float* Y, const SliceDesc* sd, const int2* wk,
                      const int2* items, int nitems, double* gpart, hipStream_t s, int wreal) {
  constexpr int MT = 2 * kCplxProdRows;
  constexpr size_t main = 2 * (size_t)(MT * KPC + 2 * 32 * NB * KPC) * 2, epi = MT * (size_t)(32 * NB + 1) * 4;
  constexpr size_t bytes = main > epi ? main : epi;
  if (nitems == 0) return HT_OK;
  int rc = ensure_dynamic_lds((const void*)k_cthin_bf16<NB, MT, TRANS>, bytes);
  if (rc) return rc;
  const int aligned = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (reinterpret_cast<uintptr_t>(W) % 16 == 0);
  hipLaunchKernelGGL((k_cthin_bf16<NB, MT, TRANS>), dim3((unsigned)nitems), dim3(2 * MT), bytes, s, A, W, Y, sd, wk,
                     items, gpart, aligned, wreal);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

// Complex reconstruction C = X B, B = Bt^H (X = Q1 K', n1 x l; Bt, n2 x l;
// both FP32 in the stacked layout), for BF16-mixed plans, on the BF16 matrix
// cores with every operand split in two BF16 terms, x = xh + xl (xh = bf16(x),
// xl = bf16(x - xh)): X B ~ Xh Bh + Xh Bl + Xl Bh, a relative error of a few
// 2^-17 per product (the dropped Xl Bl and the split remainders).
// Real form over K = 2 q (q = l rounded up to 8): Cr = [Xr, Xi] E1 and
// Ci = [Xr, Xi] E2 with E1 = [Btr^T; Bti^T] and E2 = [-Bti^T; Btr^T], so E2 is
// E1 with its halves exchanged and the first negated: one staged operand.
// Work items as k_cmul_strip (strips of 128 complex rows, groups of up to four
// 64-column tiles); wavefront w keeps rows 32 w .. 32 w + 31 of [Xr, Xi] as
// split A operands (lane t: row t % 32, k = 16 s + 8 (t / 32) .. + 7); per
// column tile E1 (split) goes to LDS column by column with k contiguous;
// results are stored from the accumulators.
constexpr int kXPitch = 136;  // bf16 per LDS column of E1: 2 q <= 128, 272 bytes
constexpr size_t kX3Lds = 2 * 64 * kXPitch * sizeof(uint16_t);

// Two FP32 values -> packed BF16 leading terms and packed BF16 remainders.
__device__ __forceinline__ void split_bf16x2(float a, float b, uint32_t& hi, uint32_t& lo) {
  hi = f32x2_to_bf16x2(a, b);
  lo = f32x2_to_bf16x2(a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xffff0000u));
}

__global__ __launch_bounds__(256, 1) void k_cmul_bf16x3(const float* __restrict__ Xall, const float* __restrict__ Wall,
                                                        float* __restrict__ Call, const SliceDesc* __restrict__ sd,
                                                        const int2* __restrict__ wk, const int2* __restrict__ items,
                                                        int aligned) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint16_t* Eh = reinterpret_cast<uint16_t*>(smem_raw);  // [column][k]
  uint16_t* El = Eh + 64 * kXPitch;
  const int2 item = items[blockIdx.x];
  const int s = item.x;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int n1 = d.n1, n2 = d.n2, ldx = 2 * n1;
  const int nct = (n2 + 63) / 64, ncg = (nct + kCmulGroup - 1) / kCmulGroup;
  const int row0 = (item.y / ncg) * kCmulRows, cg = item.y % ncg;
  const int ct_begin = cg * kCmulGroup, ct_end = min(nct, ct_begin + kCmulGroup);
  const int q = (l + 7) & ~7, nsteps = q / 8;  // K = 2 q in steps of 16
  const float* X = Xall + d.y;
  const float* W = Wall + d.z;
  float* C = Call + d.a;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, li = lane % 32, h = lane / 32;
  // ---- A operands: [Xr, Xi] rows of this wavefront, split ----
  const int xrow = row0 + 32 * wave + li;
  uint4 ah[8], al[8];  // eight BF16 per step, packed
#pragma unroll
  for (int st = 0; st < 8; ++st) {
    float x[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 16 * st + 8 * h + e;  // < 2 q
      const int part = k >= q, kk = part ? k - q : k;
      const bool ok = st < nsteps && kk < l && xrow < n1;
      x[e] = ok ? X[(part ? n1 : 0) + xrow + (int64_t)kk * ldx] : 0.0f;
    }
    split_bf16x2(x[0], x[1], ah[st].x, al[st].x);
    split_bf16x2(x[2], x[3], ah[st].y, al[st].y);
    split_bf16x2(x[4], x[5], ah[st].z, al[st].z);
    split_bf16x2(x[6], x[7], ah[st].w, al[st].w);
  }
  // ---- staging of E1 for one column tile: unit = (column c, k group of 8) ----
  // E1[k][c] = Btr(c, k) for k < q, Bti(c, k - q) after (zero past l).  The
  // next tile's loads (stage_load) are issued before the current tile's
  // products and split (stage_split) after them, before its stores: their
  // wait then covers only the previous tile's stores, which drained during
  // the products; the split terms go to LDS (stage_store) after a barrier.
  float pv[4][8];
  uint4 sh[4], sl[4];
  // loads from clamped (always valid) addresses, unconditionally, so that no
  // path leaves a load pending; entries past the operand are zeroed at the split
  auto stage_load = [&](int ct) {
    const int col0 = 64 * ct;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = tid + 256 * u;
      const int c = f % 64, g = f / 64;  // g < 16: k = 8 g .. 8 g + 7
      const int gc = min(col0 + c, n2 - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 8 * g + e, part = k >= q, kk = min(part ? k - q : k, l - 1);
        pv[u][e] = W[(part ? n2 : 0) + gc + (int64_t)kk * 2 * n2];
      }
    }
  };
  auto stage_split = [&](int ct) {
    const int col0 = 64 * ct;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = tid + 256 * u;
      const int c = f % 64, g = f / 64;
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 8 * g + e, part = k >= q, kk = part ? k - q : k;
        v[e] = (8 * g < 2 * q && kk < l && col0 + c < n2) ? pv[u][e] : 0.0f;
      }
      split_bf16x2(v[0], v[1], sh[u].x, sl[u].x);
      split_bf16x2(v[2], v[3], sh[u].y, sl[u].y);
      split_bf16x2(v[4], v[5], sh[u].z, sl[u].z);
      split_bf16x2(v[6], v[7], sh[u].w, sl[u].w);
      // the split happens here, before the stores that follow (not sunk to its LDS store)
      asm volatile("" ::"v"(sh[u].x), "v"(sh[u].y), "v"(sh[u].z), "v"(sh[u].w), "v"(sl[u].x), "v"(sl[u].y),
                   "v"(sl[u].z), "v"(sl[u].w)
                   : "memory");
    }
  };
  auto stage_store = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = tid + 256 * u;
      const int c = f % 64, g = f / 64;
      *reinterpret_cast<uint4*>(Eh + c * kXPitch + 8 * g) = sh[u];
      *reinterpret_cast<uint4*>(El + c * kXPitch + 8 * g) = sl[u];
    }
  };
  // every row of the strip in range and 16-byte aligned column segments: vector stores only
  const bool full = aligned && d.a % 4 == 0 && n1 % 4 == 0 && row0 + kCmulRows <= n1;
  stage_load(ct_begin);
  stage_split(ct_begin);
  stage_store();
  __syncthreads();
  for (int ct = ct_begin; ct < ct_end; ++ct) {
    const int col0 = 64 * ct;
    const bool more = ct + 1 < ct_end;  // uniform
    const int cn = more ? ct + 1 : ct;  // the last tile reloads itself (cached, unused)
    stage_load(cn);
    f32x16 acr[2], aci[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acr[cb][r] = aci[cb][r] = 0.0f;
    const bool two = col0 + 32 < n2;
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      if (st >= nsteps) break;
      const int k1 = 16 * st + 8 * h;  // this lane's k (E1), and its E2 source in the other half
      const bool first = k1 < q;
      const int k2 = first ? k1 + q : k1 - q;
      const unsigned short flip = first ? 0x8000u : 0u;
      const bf16x8 xa = __builtin_bit_cast(bf16x8, ah[st]), xb = __builtin_bit_cast(bf16x8, al[st]);
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        if (cb == 1 && !two) break;
        const int c = 32 * cb + li;
        const bf16x8 e1h = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(Eh + c * kXPitch + k1));
        const bf16x8 e1l = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(El + c * kXPitch + k1));
        const bf16x8 e2h =
            __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(Eh + c * kXPitch + k2) ^ flip);
        const bf16x8 e2l =
            __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(El + c * kXPitch + k2) ^ flip);
        acr[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, e1h, acr[cb], 0, 0, 0);
        aci[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, e2h, aci[cb], 0, 0, 0);
        acr[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, e1l, acr[cb], 0, 0, 0);
        aci[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, e2l, aci[cb], 0, 0, 0);
        acr[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xb, e1h, acr[cb], 0, 0, 0);
        aci[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xb, e2h, aci[cb], 0, 0, 0);
      }
    }
    stage_split(cn);
    // ---- store: 16-byte column segments straight from the accumulators ----
    auto put = [&](const f32x16& acc, int cb, int part) {
      const int col = col0 + 32 * cb + li;
      if (col >= n2) return;
      float* dst = C + (part ? n1 : 0) + (int64_t)col * ldx;
      if (full) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rb = row0 + 32 * wave + 8 * j + 4 * h;
          *reinterpret_cast<f32x4*>(dst + rb) = f32x4{acc[4 * j], acc[4 * j + 1], acc[4 * j + 2], acc[4 * j + 3]};
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rb = row0 + 32 * wave + 8 * j + 4 * h;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (rb + e < n1) dst[rb + e] = acc[4 * j + e];
        }
      }
    };
    put(acr[0], 0, 0);
    put(aci[0], 0, 1);
    if (two) {
      put(acr[1], 1, 0);
      put(aci[1], 1, 1);
    }
    if (more) {
      __syncthreads();  // every wavefront is done reading this tile's operands
      stage_store();
      __syncthreads();
    }
  }
}

template <int NB, int NW, bool TRANS, bool CPLX = false>
int launch_thin_bf16(const uint16_t* A, const float* W, float* Y, const SliceDesc* sd, const int2* wk,
                     const int2* items, int nitems, double* gpart, hipStream_t s, int wreal = 0) {
  using L = Bf16Lds<NB, NW>;
  if (nitems == 0) return HT_OK;
  int rc = ensure_dynamic_lds((const void*)k_mfma_thin_bf16<NB, NW, TRANS, CPLX>, L::BYTES);
  if (rc) return rc;
  const int aligned = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (reinterpret_cast<uintptr_t>(W) % 16 == 0);
  hipLaunchKernelGGL((k_mfma_thin_bf16<NB, NW, TRANS, CPLX>), dim3((unsigned)nitems), dim3(64 * NW), L::BYTES, s, A,
                     W, Y, sd, wk, items, gpart, aligned, wreal);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template <bool TRANS>
int dispatch_bf16(const uint16_t* A, const float* W, float* Y, const SliceDesc* sd, const int2* wk,
                  const int2* items, int nitems, int lmax, int rows, double* gpart, hipStream_t s) {
  if (lmax > 96 || (rows != 64 && rows != 128)) HT_FAIL(HT_ERR_UNSUPPORTED, "matrix-core product: bad width or tile");
  if (rows == 64) {
    if (lmax <= 32) return launch_thin_bf16<1, 2, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
    if (lmax <= 64) return launch_thin_bf16<2, 2, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
    return launch_thin_bf16<3, 2, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
  }
  if (lmax <= 32) return launch_thin_bf16<1, 4, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
  if (lmax <= 64) return launch_thin_bf16<2, 4, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
  return launch_thin_bf16<3, 4, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
}

}  // namespace

int launch_bf16_nn(const uint16_t* A, const float* W, float* Y, const SliceDesc* sd, const int2* wk,
                   const int2* items, int nitems, int lmax, int rows, double* gpart, hipStream_t s) {
  return dispatch_bf16<false>(A, W, Y, sd, wk, items, nitems, lmax, rows, gpart, s);
}

int launch_bf16_cnn(const uint16_t* A, const uint16_t* W, float* Y, int wreal, const SliceDesc* sd, const int2* wk,
                    const int2* items, int nitems, int lmax, double* gpart, hipStream_t s) {
  if (lmax > kMaxComplexWidth) HT_FAIL(HT_ERR_UNSUPPORTED, "complex sketch width above 64");
  if (lmax <= 32) return launch_cthin_bf16<1, false>(A, W, Y, sd, wk, items, nitems, gpart, s, wreal);
  return launch_cthin_bf16<2, false>(A, W, Y, sd, wk, items, nitems, gpart, s, wreal);
}

int launch_bf16_ctn(const uint16_t* A, const uint16_t* Q, float* Z, const SliceDesc* sd, const int2* wk,
                    const int2* items, int nitems, int lmax, double* gpart, hipStream_t s) {
  if (lmax > kMaxComplexWidth) HT_FAIL(HT_ERR_UNSUPPORTED, "complex sketch width above 64");
  if (lmax <= 32) return launch_cthin_bf16<1, true>(A, Q, Z, sd, wk, items, nitems, gpart, s, 0);
  return launch_cthin_bf16<2, true>(A, Q, Z, sd, wk, items, nitems, gpart, s, 0);
}

int launch_bf16x3_cnt(const float* X, const float* W, float* C, const SliceDesc* sd, const int2* wk,
                      const int2* items, int nitems, int lmax, hipStream_t s) {
  if (lmax > kMaxComplexWidth) HT_FAIL(HT_ERR_UNSUPPORTED, "complex sketch width above 64");
  if (nitems == 0) return HT_OK;
  int rc = ensure_dynamic_lds((const void*)k_cmul_bf16x3, kX3Lds);
  if (rc) return rc;
  const int aligned = reinterpret_cast<uintptr_t>(C) % 16 == 0;
  hipLaunchKernelGGL(k_cmul_bf16x3, dim3((unsigned)nitems), dim3(256), kX3Lds, s, X, W, C, sd, wk, items, aligned);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

int launch_bf16_tn(const uint16_t* A, const float* Q, float* Z, const SliceDesc* sd, const int2* wk,
                   const int2* items, int nitems, int lmax, int rows, double* gpart, hipStream_t s) {
  return dispatch_bf16<true>(A, Q, Z, sd, wk, items, nitems, lmax, rows, gpart, s);
}

}  // namespace ht
