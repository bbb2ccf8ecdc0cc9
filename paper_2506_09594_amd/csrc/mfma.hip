// FP32 sketch products on the matrix cores (v_mfma_f32_32x32x2_f32).
//
//   nn:  Y_s (n1 x l) = A_s (n1 x n2) W_s (n2 x l)    (range sketch, power step)
//   tn:  Z_s (n2 x l) = A_s^T (n2 x n1) Q_s (n1 x l)  (adjoint step, projection)
//
// One workgroup per work item (slice s, first output row): NW wavefronts own
// MT = 32 NW output rows and all l (<= 32 NB) columns, wavefront w computing
// rows 32w..32w+31 as NB 32 x 32 MFMA blocks.  The reduction dimension is
// walked in chunks of 32: the A chunk (MT x 32) and the thin-operand chunk
// (32 x l) are fetched into registers (16-byte loads where the slice's columns
// allow it) two chunks ahead, while the matrix cores work on the current chunk
// in LDS (two LDS buffers, two register sets).  MFMA operand layout (32x32x2, one block): lane t supplies
// A[t % 32][t / 32] and B[t / 32][t % 32]; accumulator r of lane t is
// D[8 (r / 4) + 4 (t / 32) + r % 4][t % 32].
//
// Epilogue: the tile goes through LDS so that the column-major store is
// coalesced, and (optionally) the FP64 Gram matrix of the stored tile rows is
// written for the orthonormalization that follows.
#include "chol.hpp"

namespace ht {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;  // K chunk

template <int NB, int NW>
struct MfmaLds {
  static constexpr int MT = 32 * NW;
  // A chunk stored as [k][row] (nn) or [row][k] (tn); thin chunk as [k][col]
  static constexpr int AP_NN = MT + 4;    // pitch of [k][row]
  static constexpr int AP_TN = KC + 1;    // pitch of [row][k]
  static constexpr int BP = 32 * NB + 1;  // pitch of [k][col]
  static constexpr int A_WORDS = (KC * AP_NN > MT * AP_TN) ? KC * AP_NN : MT * AP_TN;
  static constexpr int B_WORDS = KC * BP;
  static constexpr int MAIN_BYTES = 2 * (A_WORDS + B_WORDS) * 4;
  static constexpr int EPI_BYTES = MT * (32 * NB + 1) * 4;  // FP32 tile (the values the products store)
  static constexpr int BYTES = MAIN_BYTES > EPI_BYTES ? MAIN_BYTES : EPI_BYTES;
};

// TRANS = false: nn (A rows are output rows); TRANS = true: tn (A columns are
// output rows).  CPLX: complex slices in the stacked layout (NW = 4): A enters
// through its real embedding, so that the product with a stacked thin operand
// is the stacked complex product (nn: Y = A W, or with wreal the real Omega
// against the stored block; tn: Z = A^H Q), and the tile's 128 rows are 64
// complex rows, their real parts then their imaginary parts, whose complex
// Gram partial the epilogue writes.
template <int NB, int NW, bool TRANS, bool CPLX>
__global__ __launch_bounds__(64 * NW) void k_mfma_thin(const float* __restrict__ Aall, const float* __restrict__ Wall,
                                                       float* __restrict__ Yall, const SliceDesc* __restrict__ sd,
                                                       const int2* __restrict__ wk, const int2* __restrict__ items,
                                                       double* __restrict__ gpart, int aligned, int wreal) {
  using L = MfmaLds<NB, NW>;
  constexpr int MT = L::MT;
  constexpr int HM = MT / 2;  // complex rows of a tile
  static_assert(!CPLX || MT == 128, "complex tiles hold 64 complex rows");
  constexpr int NTH = 64 * NW;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* const lds_f = reinterpret_cast<float*>(smem_raw);
  // buffer b: A chunk at lds_f + b * A_WORDS, thin chunk at lds_f + 2 * A_WORDS + b * B_WORDS
  const int2 item = items[blockIdx.x];
  const int s = item.x, r0 = item.y;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int mo = TRANS ? d.n2 : d.n1;  // output rows (complex rows when CPLX)
  const int lda = CPLX ? 2 * d.n1 : d.n1;
  const int M_out = CPLX ? 2 * mo : mo;
  const int K = CPLX ? (TRANS ? 2 * d.n1 : (wreal ? d.n2 : 2 * d.n2)) : (TRANS ? d.n1 : d.n2);
  const int ldw = K, ldy = M_out;
  const int64_t woff = TRANS ? d.y : d.z, yoff = TRANS ? d.z : d.y;
  const float* Aj = Aall + d.a;
  const float* Wj = Wall + woff;
  float* Yj = Yall + yoff;
  const bool vecA = aligned && (lda % 4 == 0) && (d.a % 4 == 0) && (!CPLX || d.n1 % 4 == 0);
  const bool vecW = aligned && (ldw % 4 == 0) && (woff % 4 == 0);
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int LW = 32 * NB;
  // stacked output row of tile row i, and whether it exists
  auto orow = [&](int i) -> int { return CPLX ? (i >= HM ? mo + r0 + i - HM : r0 + i) : r0 + i; };
  auto ovalid = [&](int i) -> bool { return CPLX ? r0 + (i >= HM ? i - HM : i) < mo : r0 + i < M_out; };
  // element (r, k) of the slice operand (complex slices: the real embedding)
  auto aval = [&](int r, int k) -> float {
    bool neg;
    const float v = Aj[embed_index(r, k, lda, CPLX, d.n1, d.n2, neg)];
    return neg ? -v : v;
  };
  auto avec = [&](int r, int k) -> f32x4 {  // rows r..r+3 of column k (no straddle when vecA)
    bool neg;
    const f32x4 v = *reinterpret_cast<const f32x4*>(Aj + embed_index(r, k, lda, CPLX, d.n1, d.n2, neg));
    return neg ? -v : v;
  };

  // ---- global -> register staging of one K chunk --------------------------
  // A chunk: MT x KC values = 8 MT float4 groups; 4 per thread.
  // nn: column-major A, rows r0.. (contiguous) for columns k0..k0+31
  // tn: column-major A, rows k0..k0+31 (contiguous) for columns r0..r0+MT-1
  constexpr int NRA = MT * KC / 4 / NTH;
  constexpr int NRB = (KC * 32 * NB / 4 + NTH - 1) / NTH;
  f32x4 ra0[NRA], rb0[NRB], ra1[NRA], rb1[NRB];  // two chunks of loads in flight
  auto fetch = [&](f32x4 (&ra)[NRA], f32x4 (&rb)[NRB], int k0) {
#pragma unroll
    for (int u = 0; u < NRA; ++u) {
      const int f = tid + u * NTH;
      if (!TRANS) {
        const int kk = f / (MT / 4), row = (f % (MT / 4)) * 4;  // four rows within one half of a complex tile
        const int gr = orow(row), gk = k0 + kk;
        if (vecA && gk < K && ovalid(row + 3)) {
          ra[u] = avec(gr, gk);
        } else {
          f32x4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (gk < K && ovalid(row + e)) ? aval(gr + e, gk) : 0.0f;
          ra[u] = v;
        }
      } else {
        const int row = f / (KC / 4), kk = (f % (KC / 4)) * 4;
        const int gc = orow(row), gk = k0 + kk;
        if (vecA && ovalid(row) && gk + 3 < K) {
          ra[u] = avec(gk, gc);
        } else {
          f32x4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (ovalid(row) && gk + e < K) ? aval(gk + e, gc) : 0.0f;
          ra[u] = v;
        }
      }
    }
    // thin chunk: rows k0..k0+31 of W (column-major, ldw), LW columns
#pragma unroll
    for (int u = 0; u < NRB; ++u) {
      const int f = tid + u * NTH;
      const int c = f / (KC / 4), k4 = (f % (KC / 4)) * 4;
      f32x4 v;
      const int gk = k0 + k4;
      if (vecW && f < KC * LW / 4 && c < l && gk + 3 < K) {
        v = *reinterpret_cast<const f32x4*>(Wj + gk + (int64_t)c * ldw);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          v[e] = (f < KC * LW / 4 && c < l && gk + e < K) ? Wj[gk + e + (int64_t)c * ldw] : 0.0f;
      }
      rb[u] = v;
    }
  };
  auto stash = [&](const f32x4 (&ra)[NRA], const f32x4 (&rb)[NRB], int buf) {
    float* As = lds_f + buf * L::A_WORDS;
    float* Bs = lds_f + 2 * L::A_WORDS + buf * L::B_WORDS;
#pragma unroll
    for (int u = 0; u < NRA; ++u) {
      const int f = tid + u * NTH;
      if (!TRANS) {
        const int kk = f / (MT / 4), row = (f % (MT / 4)) * 4;
        *reinterpret_cast<f32x4*>(As + kk * L::AP_NN + row) = ra[u];
      } else {
        const int row = f / (KC / 4), kk = (f % (KC / 4)) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) As[row * L::AP_TN + kk + e] = ra[u][e];
      }
    }
#pragma unroll
    for (int u = 0; u < NRB; ++u) {
      const int f = tid + u * NTH;
      if (f < KC * LW / 4) {
        const int c = f / (KC / 4), k4 = (f % (KC / 4)) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) Bs[(k4 + e) * L::BP + c] = rb[u][e];
      }
    }
  };

  f32x16 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[b][r] = 0.0f;

  const int nchunks = (K + KC - 1) / KC;
  const int nbl = (l + 31) / 32;  // column blocks in use (uniform)
  const int mrow = 32 * wave + (lane % 32);  // A-operand row of this lane within the tile
  const int khalf = lane / 32;
  auto compute = [&](int buf) {
    const float* As = lds_f + buf * L::A_WORDS;
    const float* Bs = lds_f + 2 * L::A_WORDS + buf * L::B_WORDS;
#pragma unroll
    for (int kp = 0; kp < KC / 2; ++kp) {
      const int k = 2 * kp + khalf;
      const float a = TRANS ? As[mrow * L::AP_TN + k] : As[k * L::AP_NN + mrow];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b < nbl) {
          const float bv = Bs[k * L::BP + 32 * b + (lane % 32)];
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc[b], 0, 0, 0);
        }
      }
    }
  };
  // chunk c sits in LDS buffer c & 1 while chunks c + 1 and c + 2 load into
  // the register sets (unrolled by two so that the sets are fixed)
  fetch(ra0, rb0, 0);
  if (nchunks > 1) fetch(ra1, rb1, KC);
  stash(ra0, rb0, 0);
  __syncthreads();
  for (int ch = 0; ch < nchunks; ch += 2) {
    if (ch + 2 < nchunks) fetch(ra0, rb0, (ch + 2) * KC);
    compute(0);
    if (ch + 1 < nchunks) stash(ra1, rb1, 1);
    __syncthreads();
    if (ch + 1 >= nchunks) break;
    if (ch + 3 < nchunks) fetch(ra1, rb1, (ch + 3) * KC);
    compute(1);
    if (ch + 2 < nchunks) stash(ra0, rb0, 0);
    __syncthreads();
  }

  // ---- epilogue: tile to LDS (as double), coalesced store, Gram partial ----
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

// Streaming nn product for real FP32 slices (n1 % 4 == 0, n2 <= kStreamMaxK):
// a workgroup of 8 wavefronts owns 256 output rows; wavefront (rw, ks) computes
// rows 128 rw .. 128 rw + 127 over the ks-th quarter of the reduction.  A is
// read straight from HBM into the MFMA operand registers: lane t loads rows
// 4 (t % 32) .. +3 of column k (one 16-byte load), and element e of that
// load feeds MFMA block e, whose row i stands for tile row 4 i + e.  Two
// register buffers of U loads per lane are in flight at all times (the next
// buffer is issued before the current one is consumed; loads past the end are
// clamped to a valid address and their values zeroed), so each CU keeps about
// 128 KB of reads outstanding.  The thin operand is staged in LDS whole; with
// W null it is the Gaussian sketch, drawn here while the first loads of A are
// in flight (element e = k + c n2 of Omega_s is draw e % 4 of group e / 4 of
// the slice's key, as the sketch generator writes it).  The
// four partial tiles are summed through one LDS tile, which then feeds the
// coalesced store of Y and the Gram partials.
template <int NB, int U>
__global__ __launch_bounds__(512) void k_mfma_nn_stream(const float* __restrict__ Aall, const float* __restrict__ Wall,
                                                       float* __restrict__ Yall, const SliceDesc* __restrict__ sd,
                                                       const int2* __restrict__ wk, const int2* __restrict__ items,
                                                       double* __restrict__ gpart, OmegaKey key) {
  constexpr int RW = 2, KS = 4, VR = 4, NTH = 64 * RW * KS;
  constexpr int ROWS = 32 * VR * RW, LW = 32 * NB, RP = ROWS + 4;
  static_assert(ROWS == kStreamRows, "tile rows");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* const Ws = reinterpret_cast<float*>(smem_raw);  // [K][LW], then the tile [LW][RP]
  float* const Ts = Ws;
  const int2 item = items[blockIdx.x];
  const int s = item.x, r0 = item.y;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int M = d.n1, K = d.n2;
  const float* A = Aall + d.a;
  const float* W = Wall + d.z;
  float* Y = Yall + d.y;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int rw = wave % RW, ks = wave / RW;
  const int half = lane / 32, li = lane % 32;
  const int kper = ((K + KS - 1) / KS + 1) & ~1;
  const int kb = min(K, ks * kper), ke = min(K, kb + kper);
  const int rowl = r0 + 32 * VR * rw + VR * li;  // first of this lane's four rows
  const bool rowok = rowl + VR - 1 < M;
  const float* Arow = A + (rowok ? rowl : 0);
  f32x4 bufA[U], bufB[U];
  auto load = [&](f32x4* buf, int k0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int k = k0 + 2 * u + half;
      k = k < ke ? k : ke - 1;
      buf[u] = *reinterpret_cast<const f32x4*>(Arow + (int64_t)k * M);
    }
  };
  if (kb < ke) {
    load(bufA, kb);
    load(bufB, kb + 2 * U);
  }
  if (W) {
    for (int f = tid; f < K * LW; f += NTH) {
      const int k = f % K, c = f / K;
      Ws[k * LW + c] = (c < l) ? W[k + (int64_t)c * K] : 0.0f;
    }
  } else {
    const uint32_t call = key.call_dev ? (uint32_t)(*key.call_dev) : key.call;
    const int ne = K * l;
    for (int gi = tid; gi < (ne + 3) / 4; gi += NTH) {
      double z[4];
      gaussian4((uint64_t)gi, (uint32_t)d.local, call, key.stream_base + (uint32_t)d.tensor, key.seed, z);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = 4 * gi + u;
        if (e < ne) Ws[(e % K) * LW + e / K] = (float)z[u];
      }
    }
    for (int f = tid; f < K * (LW - l); f += NTH) Ws[(f % K) * LW + l + f / K] = 0.0f;
  }
  __syncthreads();
  f32x16 acc[VR][NB];
#pragma unroll
  for (int e = 0; e < VR; ++e)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[e][b][r] = 0.0f;
  const int nbl = (l + 31) / 32;
  auto compute = [&](const f32x4* buf, int k0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + 2 * u + half;
      const bool ok = k < ke && rowok;
      const int kr = k < ke ? k : 0;
      float bv[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = Ws[kr * LW + 32 * b + li];
#pragma unroll
      for (int e = 0; e < VR; ++e) {
        const float av = ok ? buf[u][e] : 0.0f;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (b < nbl) acc[e][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[b], acc[e][b], 0, 0, 0);
      }
    }
  };
  for (int k0 = kb; k0 < ke; k0 += 4 * U) {
    compute(bufA, k0);
    if (k0 + 4 * U < ke) load(bufA, k0 + 4 * U);
    compute(bufB, k0 + 2 * U);
    if (k0 + 6 * U < ke) load(bufB, k0 + 6 * U);
  }
  // ---- sum the KS partial tiles through one LDS tile [LW][RP] -------------
  auto tile_index = [&](int e, int b, int r) {
    const int i = 8 * (r / 4) + 4 * half + (r % 4);
    return (32 * b + li) * RP + 32 * VR * rw + VR * i + e;
  };
  __syncthreads();  // the thin operand is no longer read
  for (int q = 1; q < KS; ++q) {
    if (ks == q) {
#pragma unroll
      for (int e = 0; e < VR; ++e)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int r = 0; r < 16; ++r) Ts[tile_index(e, b, r)] = acc[e][b][r];
    }
    __syncthreads();
    if (ks == 0) {
#pragma unroll
      for (int e = 0; e < VR; ++e)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[e][b][r] += Ts[tile_index(e, b, r)];
    }
    __syncthreads();
  }
  if (ks == 0) {
#pragma unroll
    for (int e = 0; e < VR; ++e)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) Ts[tile_index(e, b, r)] = acc[e][b][r];
  }
  __syncthreads();
  const int rows = min(ROWS, M - r0);
  for (int f = tid; f < l * (ROWS / 4); f += NTH) {
    const int c = f / (ROWS / 4), q = (f % (ROWS / 4)) * 4;
    if (q + 3 < rows)
      *reinterpret_cast<f32x4*>(Y + r0 + q + (int64_t)c * M) = *reinterpret_cast<const f32x4*>(Ts + c * RP + q);
    else
      for (int e = 0; e < 4; ++e)
        if (q + e < rows) Y[r0 + q + e + (int64_t)c * M] = Ts[c * RP + q + e];
  }
  if (gpart) tile_gram_mfma(Ts, 1, RP, rows, l, gpart + d.g1 + (int64_t)(r0 / kGramRows) * l * l);
}

template <int NB>
size_t stream_lds_bytes(int kmax) {
  const size_t w = (size_t)kmax * 32 * NB * 4, t = (size_t)32 * NB * (kStreamRows + 4) * 4;
  return w > t ? w : t;
}

// Reconstruction C_s (n1 x nc) = X_s (n1 x l) W_s^T (W_s n2 x l, first nc
// rows) on the matrix cores: a 64 x 64 tile per work item (slice, tile index,
// row tiles fastest), wavefront w computing the 32 x 32 block (w % 2, w / 2).
// Operands load straight into the MFMA registers (lane t: rows / columns
// t % 32 of the block at k = 2 s + t / 32, coalesced along the column-major
// blocks), every load of the tile before the first step; the result goes
// through LDS so that the column-major store is 16-byte and coalesced.
template <int KMAX>
__global__ __launch_bounds__(256) void k_mfma_nt(const float* __restrict__ Xall, const float* __restrict__ Wall,
                                                 float* __restrict__ Call, const SliceDesc* __restrict__ sd,
                                                 const int2* __restrict__ wk, const int2* __restrict__ items) {
  constexpr int TP = 68;  // pitch of the [column][row] staging tile
  __shared__ __align__(16) float Ts[64 * TP];
  const int2 item = items[blockIdx.x];
  const int s = item.x;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int m = d.n1, n = d.nc;
  const int nrt = (m + 63) / 64;
  const int row0 = (item.y % nrt) * 64, col0 = (item.y / nrt) * 64;
  const float* X = Xall + d.y;
  const float* W = Wall + d.z;
  float* C = Call + d.a;
  const int ldx = m, ldw = d.n2, ldc = m;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int li = lane % 32, h = lane / 32;
  const int br = 32 * (wave % 2), bc = 32 * (wave / 2);
  const int gr = row0 + br + li, gc = col0 + bc + li;
  const bool rok = gr < m, cok = gc < n;
  constexpr int NS = (KMAX + 1) / 2;
  float av[NS], bv[NS];
#pragma unroll
  for (int st = 0; st < NS; ++st) {
    const int k = 2 * st + h;
    av[st] = (k < l && rok) ? X[gr + (int64_t)k * ldx] : 0.0f;
    bv[st] = (k < l && cok) ? W[gc + (int64_t)k * ldw] : 0.0f;
  }
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
  for (int st = 0; st < NS; ++st)
    if (2 * st < l) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[st], bv[st], acc, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r / 4) + 4 * h + (r % 4);
    Ts[(bc + li) * TP + br + i] = acc[r];
  }
  __syncthreads();
  const int rows = min(64, m - row0), cols = min(64, n - col0);
  const bool vec = (ldc % 4 == 0) && (d.a % 4 == 0);
  for (int f = threadIdx.x; f < 64 * 16; f += 256) {
    const int c = f / 16, q = (f % 16) * 4;
    if (c >= cols) continue;
    float* dst = C + row0 + q + (int64_t)(col0 + c) * ldc;
    if (vec && q + 3 < rows)
      *reinterpret_cast<f32x4*>(dst) = *reinterpret_cast<const f32x4*>(Ts + c * TP + q);
    else
      for (int e = 0; e < 4; ++e)
        if (q + e < rows) dst[e] = Ts[c * TP + q + e];
  }
}

// Q1 K' (n1 x l per slice) on the matrix cores, FP32, l <= KMAX <= 64: one
// 64-row tile per work item (slice, first row), wavefront w computing the
// 32 x 32 block (rows 32 (w % 2), columns 32 (w / 2)); lane t supplies
// Q1[row t % 32][k] and K'[k][column t % 32] at k = 2 s + t / 32, and the
// block goes through LDS for coalesced 16-byte column stores.
template <int KMAX>
__global__ __launch_bounds__(4 * KMAX) void k_mfma_qk(const float* __restrict__ Qall, const float* __restrict__ Kall,
                                                      float* __restrict__ QKall, const SliceDesc* __restrict__ sd,
                                                      const int2* __restrict__ wk, const int2* __restrict__ items) {
  constexpr int NT = 4 * KMAX, TP = 68, NS = KMAX / 2;
  __shared__ __align__(16) float Ts[KMAX * TP];  // [column][row]
  const int2 item = items[blockIdx.x];
  const int s = item.x, row0 = item.y;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int m = d.n1;
  const float* Q = Qall + d.y;
  const float* Kq = Kall + d.kq;  // K' column-major, l x l
  float* QK = QKall + d.y;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int li = lane % 32, h = lane / 32;
  const int br = 32 * (wave % 2), bc = 32 * (wave / 2);
  const int gr = row0 + br + li, gc = bc + li;
  const bool rok = gr < m, cok = gc < l;
  float av[NS], bv[NS];
#pragma unroll
  for (int st = 0; st < NS; ++st) {
    const int k = 2 * st + h;
    av[st] = (k < l && rok) ? Q[gr + (int64_t)k * m] : 0.0f;
    bv[st] = (k < l && cok) ? Kq[k + gc * l] : 0.0f;
  }
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
  for (int st = 0; st < NS; ++st)
    if (2 * st < l) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[st], bv[st], acc, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r / 4) + 4 * h + (r % 4);
    Ts[(bc + li) * TP + br + i] = acc[r];
  }
  __syncthreads();
  const int rows = min(64, m - row0);
  const bool vec = (m % 4 == 0) && (d.y % 4 == 0);
  for (int f = threadIdx.x; f < l * 16; f += NT) {
    const int c = f / 16, q = (f % 16) * 4;
    float* dst = QK + row0 + q + (int64_t)c * m;
    if (vec && q + 3 < rows)
      *reinterpret_cast<f32x4*>(dst) = *reinterpret_cast<const f32x4*>(Ts + c * TP + q);
    else
      for (int e = 0; e < 4; ++e)
        if (q + e < rows) dst[e] = Ts[c * TP + q + e];
  }
}

template <int NB, int NW, bool TRANS, bool CPLX = false>
int launch_thin(const float* A, const float* W, float* Y, const SliceDesc* sd, const int2* wk, const int2* items,
                int nitems, double* gpart, hipStream_t s, int wreal = 0) {
  using L = MfmaLds<NB, NW>;
  if (nitems == 0) return HT_OK;
  int rc = ensure_dynamic_lds((const void*)k_mfma_thin<NB, NW, TRANS, CPLX>, L::BYTES);
  if (rc) return rc;
  const int aligned = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (reinterpret_cast<uintptr_t>(W) % 16 == 0);
  hipLaunchKernelGGL((k_mfma_thin<NB, NW, TRANS, CPLX>), dim3((unsigned)nitems), dim3(64 * NW), L::BYTES, s, A, W, Y,
                     sd, wk, items, gpart, aligned, wreal);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

// Complex reconstruction on the matrix cores (FP32, complex slices in the
// stacked layout, l <= 64):
//   MODE 0: QK = Q1 K'   (n1 x l),  B = K' (l x l, stored as 2 l x l);
//   MODE 1: C = QK Bt^H  (n1 x n2), B = Bt^H with Bt (n2 x l, stored as 2 n2 x l).
// With X = Xr + i Xi:  Cr = Xr Br - Xi Bi,  Ci = Xi Br + Xr Bi.
// A work item is a strip of 128 complex rows and a group of up to kCmulGroup
// column tiles of 64 columns (item.y = strip * groups + group).  Wavefront w
// keeps rows 32 w .. 32 w + 31 of Xr and Xi in registers for the whole item,
// as the A operands of v_mfma_f32_32x32x2_f32 (lane t: row t % 32, k = 2 st +
// t / 32; k past l reads zero).  Per column tile, Br and Bi (k x 64) go to LDS
// with the two k of a step interleaved, so that the 64 lanes of a step read 64
// consecutive floats; the next tile's loads are in flight in registers while
// the matrix cores work on the current one.  The wavefront's 32 x 64 block of
// both parts (2 column blocks x real / imaginary accumulators) is stored
// straight from the accumulators: accumulators 4 j .. 4 j + 3 of lane t are
// rows 8 j + 4 (t / 32) .. + 3 of column t % 32, one 16-byte segment.
constexpr size_t kCmulLds = 2 * 32 * 64 * 2 * sizeof(float);  // [part][step][column][k parity]

template <int MODE>
__global__ __launch_bounds__(256, 2) void k_cmul_strip(const float* __restrict__ Xall, const float* __restrict__ Wall,
                                                    float* __restrict__ Call, const SliceDesc* __restrict__ sd,
                                                    const int2* __restrict__ wk, const int2* __restrict__ items,
                                                    int aligned) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* Es = reinterpret_cast<float*>(smem_raw);
  const int2 item = items[blockIdx.x];
  const int s = item.x;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int n1 = d.n1, n2 = d.n2, ldx = 2 * n1;
  const int ncols = MODE == 0 ? l : n2;
  const int nct = (ncols + 63) / 64, ncg = (nct + kCmulGroup - 1) / kCmulGroup;
  const int row0 = (item.y / ncg) * kCmulRows, cg = item.y % ncg;
  const int ct_begin = cg * kCmulGroup, ct_end = min(nct, ct_begin + kCmulGroup);
  const int half = (l + 1) / 2;  // steps: k = 2 st + parity < 2 half
  const float* X = Xall + d.y;                       // Q1 (MODE 0) or Q1 K' (MODE 1)
  const float* W = Wall + (MODE == 0 ? d.kq : d.z);  // K' or Bt
  const int64_t cbase = MODE == 0 ? d.y : d.a;
  float* C = Call + cbase;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, li = lane % 32, h = lane / 32;
  // ---- the strip's rows of X, in registers for every column tile ----
  const int xrow = row0 + 32 * wave + li;
  float xr[32], xi[32];
#pragma unroll
  for (int st = 0; st < 32; ++st) {
    const int kk = 2 * st + h;
    const bool ok = st < half && kk < l && xrow < n1;
    const float* src = X + (ok ? xrow + (int64_t)kk * ldx : 0);
    xr[st] = ok ? src[0] : 0.0f;
    xi[st] = ok ? src[n1] : 0.0f;
  }
  // ---- staging of Br, Bi for one column tile: unit f = (part, step, column pair) ----
  const bool vecw = MODE == 1 && aligned && n2 % 2 == 0 && d.z % 2 == 0;
  f32x4 pre[8];
  auto fetch = [&](int ct) {
    const int col0 = 64 * ct;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int f = tid + 256 * u;
      const int cp = f % 32, st = (f / 32) % 32, part = f / 1024;
      const int k0 = 2 * st, c0 = col0 + 2 * cp;
      float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // (k0, c0), (k0 + 1, c0), (k0, c0 + 1), (k0 + 1, c0 + 1)
      if (st < half) {
        if (MODE == 1) {
          const float sg = part ? -1.0f : 1.0f;  // Bi = -Im Bt^T
          const float* src = W + (part ? n2 : 0) + c0;
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int kk = k0 + e;
            if (kk < l) {
              const float* p = src + (int64_t)kk * 2 * n2;
              if (vecw && c0 + 1 < ncols) {
                const float2 t = *reinterpret_cast<const float2*>(p);
                v[e] = sg * t.x;
                v[2 + e] = sg * t.y;
              } else {
                if (c0 < ncols) v[e] = sg * p[0];
                if (c0 + 1 < ncols) v[2 + e] = sg * p[1];
              }
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int kk = k0 + e;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const int c = c0 + q;
              if (kk < l && c < ncols) v[2 * q + e] = W[(part ? l : 0) + kk + (int64_t)c * 2 * l];
            }
          }
        }
      }
      pre[u] = f32x4{v[0], v[1], v[2], v[3]};
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int f = tid + 256 * u;
      const int cp = f % 32, st = (f / 32) % 32, part = f / 1024;
      if (st < half) *reinterpret_cast<f32x4*>(Es + ((part * 32 + st) * 64 + 2 * cp) * 2) = pre[u];
    }
  };
  const bool vecc = aligned && cbase % 4 == 0 && n1 % 4 == 0;
  fetch(ct_begin);
  for (int ct = ct_begin; ct < ct_end; ++ct) {
    const int col0 = 64 * ct;
    if (ct > ct_begin) __syncthreads();  // the previous tile's operands are no longer read
    stash();
    __syncthreads();
    if (ct + 1 < ct_end) fetch(ct + 1);
    const bool two = col0 + 32 < ncols;  // second column block
    f32x16 ar0, ai0, ar1, ai1;
#pragma unroll
    for (int r = 0; r < 16; ++r) ar0[r] = ai0[r] = ar1[r] = ai1[r] = 0.0f;
#pragma unroll
    for (int st = 0; st < 32; ++st) {
      if (st < half) {
        const float* e0 = Es + ((st * 64) + li) * 2 + h;
        const float br0 = e0[0], bi0 = e0[32 * 64 * 2];
        ar0 = __builtin_amdgcn_mfma_f32_32x32x2f32(xr[st], br0, ar0, 0, 0, 0);
        ai0 = __builtin_amdgcn_mfma_f32_32x32x2f32(xi[st], br0, ai0, 0, 0, 0);
        ar0 = __builtin_amdgcn_mfma_f32_32x32x2f32(xi[st], -bi0, ar0, 0, 0, 0);
        ai0 = __builtin_amdgcn_mfma_f32_32x32x2f32(xr[st], bi0, ai0, 0, 0, 0);
        if (two) {
          const float br1 = e0[64], bi1 = e0[64 + 32 * 64 * 2];
          ar1 = __builtin_amdgcn_mfma_f32_32x32x2f32(xr[st], br1, ar1, 0, 0, 0);
          ai1 = __builtin_amdgcn_mfma_f32_32x32x2f32(xi[st], br1, ai1, 0, 0, 0);
          ar1 = __builtin_amdgcn_mfma_f32_32x32x2f32(xi[st], -bi1, ar1, 0, 0, 0);
          ai1 = __builtin_amdgcn_mfma_f32_32x32x2f32(xr[st], bi1, ai1, 0, 0, 0);
        }
      }
    }
    // ---- store: 16-byte column segments straight from the accumulators ----
    auto put = [&](const f32x16& acc, int cb, int part) {
      const int col = col0 + 32 * cb + li;
      if (col >= ncols) return;
      float* dst = C + (part ? n1 : 0) + (int64_t)col * ldx;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rb = row0 + 32 * wave + 8 * j + 4 * h;
        if (vecc && rb + 3 < n1) {
          *reinterpret_cast<f32x4*>(dst + rb) = f32x4{acc[4 * j], acc[4 * j + 1], acc[4 * j + 2], acc[4 * j + 3]};
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (rb + e < n1) dst[rb + e] = acc[4 * j + e];
        }
      }
    };
    put(ar0, 0, 0);
    put(ai0, 0, 1);
    if (two) {
      put(ar1, 1, 0);
      put(ai1, 1, 1);
    }
  }
}

template <bool TRANS>
int dispatch(const float* A, const float* W, float* Y, const SliceDesc* sd, const int2* wk, const int2* items,
             int nitems, int lmax, int rows, double* gpart, hipStream_t s) {
  if (rows == 64) {
    if (lmax <= 32) return launch_thin<1, 2, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
    if (lmax <= 64) return launch_thin<2, 2, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
    return launch_thin<3, 2, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
  }
  if (lmax <= 32) return launch_thin<1, 4, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
  if (lmax <= 64) return launch_thin<2, 4, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
  return launch_thin<3, 4, TRANS>(A, W, Y, sd, wk, items, nitems, gpart, s);
}

}  // namespace

int launch_mfma_nn(const float* A, const float* W, float* Y, const SliceDesc* sd, const int2* wk, const int2* items,
                   int nitems, int lmax, int rows, double* gpart, hipStream_t s) {
  if (lmax > 96 || (rows != 64 && rows != 128)) HT_FAIL(HT_ERR_UNSUPPORTED, "matrix-core product: bad width or tile");
  return dispatch<false>(A, W, Y, sd, wk, items, nitems, lmax, rows, gpart, s);
}

int launch_mfma_nn_stream(const float* A, const float* W, float* Y, const SliceDesc* sd, const int2* wk,
                          const int2* items, int nitems, int lmax, int kmax, double* gpart, const OmegaKey& key,
                          hipStream_t s) {
  if (lmax > 64 || kmax > kStreamMaxK || kmax < 1) HT_FAIL(HT_ERR_UNSUPPORTED, "streaming product: bad width or n2");
  if (reinterpret_cast<uintptr_t>(A) % 16 != 0 || reinterpret_cast<uintptr_t>(Y) % 16 != 0)
    HT_FAIL(HT_ERR_UNSUPPORTED, "streaming product: unaligned operands");
  if (nitems == 0) return HT_OK;
  auto launch = [&](auto kern, size_t lds, size_t lds_max) -> int {
    int rc = ensure_dynamic_lds((const void*)kern, lds_max);
    if (rc) return rc;
    hipLaunchKernelGGL(kern, dim3((unsigned)nitems), dim3(512), lds, s, A, W, Y, sd, wk, items, gpart, key);
    HT_CHECK_LAUNCH();
    return HT_OK;
  };
  if (lmax <= 32) return launch(k_mfma_nn_stream<1, 8>, stream_lds_bytes<1>(kmax), stream_lds_bytes<1>(kStreamMaxK));
  return launch(k_mfma_nn_stream<2, 8>, stream_lds_bytes<2>(kmax), stream_lds_bytes<2>(kStreamMaxK));
}

int launch_mfma_nt(const float* X, const float* W, float* C, const SliceDesc* sd, const int2* wk, const int2* items,
                   int nitems, int lmax, hipStream_t s) {
  if (lmax > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  if (nitems == 0) return HT_OK;
  const dim3 grid((unsigned)nitems);
  if (lmax <= 32)
    hipLaunchKernelGGL(k_mfma_nt<32>, grid, dim3(256), 0, s, X, W, C, sd, wk, items);
  else if (lmax <= 64)
    hipLaunchKernelGGL(k_mfma_nt<64>, grid, dim3(256), 0, s, X, W, C, sd, wk, items);
  else
    hipLaunchKernelGGL(k_mfma_nt<HT_MAX_WIDTH>, grid, dim3(256), 0, s, X, W, C, sd, wk, items);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

int launch_mfma_qk(const float* Q, const float* K, float* QK, const SliceDesc* sd, const int2* wk, const int2* items,
                   int nitems, int lmax, hipStream_t s) {
  if (lmax > 64) HT_FAIL(HT_ERR_UNSUPPORTED, "matrix-core Q1 K': width above 64");
  if (nitems == 0) return HT_OK;
  const dim3 grid((unsigned)nitems);
  if (lmax <= 32)
    hipLaunchKernelGGL(k_mfma_qk<32>, grid, dim3(128), 0, s, Q, K, QK, sd, wk, items);
  else
    hipLaunchKernelGGL(k_mfma_qk<64>, grid, dim3(256), 0, s, Q, K, QK, sd, wk, items);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

int launch_mfma_cnn(const float* A, const float* W, float* Y, int wreal, const SliceDesc* sd, const int2* wk,
                    const int2* items, int nitems, int lmax, double* gpart, hipStream_t s) {
  if (lmax > kMaxComplexWidth) HT_FAIL(HT_ERR_UNSUPPORTED, "complex sketch width above 64");
  if (lmax <= 32) return launch_thin<1, 4, false, true>(A, W, Y, sd, wk, items, nitems, gpart, s, wreal);
  return launch_thin<2, 4, false, true>(A, W, Y, sd, wk, items, nitems, gpart, s, wreal);
}

int launch_mfma_ctn(const float* A, const float* Q, float* Z, const SliceDesc* sd, const int2* wk, const int2* items,
                    int nitems, int lmax, double* gpart, hipStream_t s) {
  if (lmax > kMaxComplexWidth) HT_FAIL(HT_ERR_UNSUPPORTED, "complex sketch width above 64");
  if (lmax <= 32) return launch_thin<1, 4, true, true>(A, Q, Z, sd, wk, items, nitems, gpart, s);
  return launch_thin<2, 4, true, true>(A, Q, Z, sd, wk, items, nitems, gpart, s);
}

template <int MODE>
int launch_cmul(const float* X, const float* W, float* C, const SliceDesc* sd, const int2* wk, const int2* items,
                int nitems, int lmax, hipStream_t s) {
  if (lmax > kMaxComplexWidth) HT_FAIL(HT_ERR_UNSUPPORTED, "complex sketch width above 64");
  if (nitems == 0) return HT_OK;
  int rc = ensure_dynamic_lds((const void*)k_cmul_strip<MODE>, kCmulLds);
  if (rc) return rc;
  const int aligned = (reinterpret_cast<uintptr_t>(W) % 8 == 0) && (reinterpret_cast<uintptr_t>(C) % 16 == 0);
  hipLaunchKernelGGL(k_cmul_strip<MODE>, dim3((unsigned)nitems), dim3(256), kCmulLds, s, X, W, C, sd, wk, items,
                     aligned);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

int launch_mfma_cqk(const float* Q, const float* K, float* QK, const SliceDesc* sd, const int2* wk, const int2* items,
                    int nitems, int lmax, hipStream_t s) {
  return launch_cmul<0>(Q, K, QK, sd, wk, items, nitems, lmax, s);
}

int launch_mfma_cnt(const float* X, const float* W, float* C, const SliceDesc* sd, const int2* wk, const int2* items,
                    int nitems, int lmax, hipStream_t s) {
  return launch_cmul<1>(X, W, C, sd, wk, items, nitems, lmax, s);
}

int launch_mfma_tn(const float* A, const float* Q, float* Z, const SliceDesc* sd, const int2* wk, const int2* items,
                   int nitems, int lmax, int rows, double* gpart, hipStream_t s) {
  if (lmax > 96 || (rows != 64 && rows != 128)) HT_FAIL(HT_ERR_UNSUPPORTED, "matrix-core product: bad width or tile");
  return dispatch<true>(A, Q, Z, sd, wk, items, nitems, lmax, rows, gpart, s);
}

}  // namespace ht
