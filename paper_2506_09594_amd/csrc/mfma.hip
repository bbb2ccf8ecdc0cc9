// FP32 sketch products on the matrix cores (v_mfma_f32_32x32x2_f32).
//
//   nn:  Y_j (m x l) = A_j (m x kd) W_j (kd x l)      (range sketch, power step)
//   tn:  Z_j (n x l) = A_j^T (n x m) Q_j (m x l)      (adjoint step, projection)
//
// A workgroup of four wavefronts owns a 128-row output tile of one slice and
// all l (<= 32 * NB) columns; wavefront w computes rows 32w..32w+31 as NB
// 32 x 32 MFMA blocks.  K is walked in chunks of 32: the A chunk (128 x 32) and
// the thin-operand chunk (32 x l) are fetched with 16-byte coalesced loads
// into registers while the matrix cores work on the previous chunk in LDS
// (double buffering).  MFMA operand layout (32x32x2, one block): lane t
// supplies A[t % 32][t / 32] and B[t / 32][t % 32]; accumulator r of lane t is
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

constexpr int MT = 128;  // output rows per workgroup
constexpr int KC = 32;   // K chunk
constexpr int NTH = 256;

template <int NB>
struct MfmaLds {
  // A chunk stored as [k][row] (nn) or [row][k] (tn); thin chunk as [k][col]
  static constexpr int AP_NN = MT + 4;   // pitch of [k][row]
  static constexpr int AP_TN = KC + 1;   // pitch of [row][k]
  static constexpr int BP = 32 * NB + 1; // pitch of [k][col]
  static constexpr int A_WORDS = (KC * AP_NN > MT * AP_TN) ? KC * AP_NN : MT * AP_TN;
  static constexpr int B_WORDS = KC * BP;
  static constexpr int MAIN_BYTES = 2 * (A_WORDS + B_WORDS) * 4;
  static constexpr int EPI_BYTES = MT * (32 * NB + 1) * 8;
  static constexpr int BYTES = MAIN_BYTES > EPI_BYTES ? MAIN_BYTES : EPI_BYTES;
};

// TRANS = false: nn (A rows are output rows); TRANS = true: tn (A columns are
// output rows).  M_out: output rows, K: reduction length, lda: column stride of A.
template <int NB, bool TRANS>
__global__ __launch_bounds__(NTH) void k_mfma_thin(const float* __restrict__ A, int64_t sA, int lda,
                                                   const float* __restrict__ W, int64_t sW, int ldw,
                                                   float* __restrict__ Y, int64_t sY, int ldy, int M_out, int K,
                                                   int l, double* __restrict__ gpart) {
  using L = MfmaLds<NB>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* const lds_f = reinterpret_cast<float*>(smem_raw);
  // buffer b: A chunk at lds_f + b * A_WORDS, thin chunk at lds_f + 2 * A_WORDS + b * B_WORDS
  const int j = blockIdx.y;
  const int r0 = blockIdx.x * MT;
  const float* Aj = A + (int64_t)j * sA;
  const float* Wj = W + (int64_t)j * sW;
  float* Yj = Y + (int64_t)j * sY;
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int LW = 32 * NB;

  // ---- global -> register staging of one K chunk --------------------------
  // A chunk: MT x KC values = 1024 float4; 4 per thread.
  // nn: column-major A, rows r0.. (contiguous) for columns k0..k0+31
  // tn: column-major A, rows k0..k0+31 (contiguous) for columns r0..r0+127
  f32x4 ra[4];
  f32x4 rb[(KC * 32 * NB / 4 + NTH - 1) / NTH];
  constexpr int NRB = (KC * 32 * NB / 4 + NTH - 1) / NTH;
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = tid + u * NTH;
      int row, kk;
      if (!TRANS) {
        kk = f / (MT / 4);
        row = (f % (MT / 4)) * 4;
        const int gr = r0 + row, gk = k0 + kk;
        if (gk < K && gr + 3 < M_out) {
          ra[u] = *reinterpret_cast<const f32x4*>(Aj + gr + (int64_t)gk * lda);
        } else {
          f32x4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (gk < K && gr + e < M_out) ? Aj[gr + e + (int64_t)gk * lda] : 0.0f;
          ra[u] = v;
        }
      } else {
        row = f / (KC / 4);
        kk = (f % (KC / 4)) * 4;
        const int gc = r0 + row, gk = k0 + kk;
        if (gc < M_out && gk + 3 < K) {
          ra[u] = *reinterpret_cast<const f32x4*>(Aj + gk + (int64_t)gc * lda);
        } else {
          f32x4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (gc < M_out && gk + e < K) ? Aj[gk + e + (int64_t)gc * lda] : 0.0f;
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
      if (f < KC * LW / 4 && c < l && gk + 3 < K) {
        v = *reinterpret_cast<const f32x4*>(Wj + gk + (int64_t)c * ldw);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          v[e] = (f < KC * LW / 4 && c < l && gk + e < K) ? Wj[gk + e + (int64_t)c * ldw] : 0.0f;
      }
      rb[u] = v;
    }
  };
  auto stash = [&](int buf) {
    float* As = lds_f + buf * L::A_WORDS;
    float* Bs = lds_f + 2 * L::A_WORDS + buf * L::B_WORDS;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
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
  fetch(0);
  stash(0);
  __syncthreads();
  const int mrow = 32 * wave + (lane % 32);  // A-operand row of this lane within the tile
  const int khalf = lane / 32;
  for (int ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunks) fetch((ch + 1) * KC);
    const float* As = lds_f + buf * L::A_WORDS;
    const float* Bs = lds_f + 2 * L::A_WORDS + buf * L::B_WORDS;
#pragma unroll
    for (int kp = 0; kp < KC / 2; ++kp) {
      const int k = 2 * kp + khalf;
      const float a = TRANS ? As[mrow * L::AP_TN + k] : As[k * L::AP_NN + mrow];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float bv = Bs[k * L::BP + 32 * b + (lane % 32)];
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc[b], 0, 0, 0);
      }
    }
    if (ch + 1 < nchunks) stash(buf ^ 1);
    __syncthreads();
  }

  // ---- epilogue: tile to LDS (as double), coalesced store, Gram partial ----
  double* S = reinterpret_cast<double*>(smem_raw);
  const int sp = LW + 1;
  const int rows = min(MT, M_out - r0);
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 32 * wave + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
      const int c = 32 * b + (lane % 32);
      S[i * sp + c] = (i < rows && c < l) ? (double)acc[b][r] : 0.0;
    }
  __syncthreads();
  for (int idx = tid; idx < MT * l; idx += NTH) {
    const int i = idx % MT, c = idx / MT;
    if (i < rows) Yj[(r0 + i) + (int64_t)c * ldy] = (float)S[i * sp + c];
  }
  if (gpart) tile_gram_to_global(S, sp, MT, l, gpart + ((int64_t)j * gridDim.x + blockIdx.x) * (int64_t)l * l);
}

template <int NB, bool TRANS>
int launch_thin(const float* A, int64_t sA, int lda, const float* W, int64_t sW, int ldw, float* Y, int64_t sY,
                int ldy, int M_out, int K, int l, int P, double* gpart, hipStream_t s) {
  using L = MfmaLds<NB>;
  int rc = ensure_dynamic_lds((const void*)k_mfma_thin<NB, TRANS>, L::BYTES);
  if (rc) return rc;
  dim3 grid((unsigned)ceil_div(M_out, MT), (unsigned)P);
  hipLaunchKernelGGL((k_mfma_thin<NB, TRANS>), grid, dim3(NTH), L::BYTES, s, A, sA, lda, W, sW, ldw, Y, sY, ldy,
                     M_out, K, l, gpart);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

}  // namespace

int mfma_tile_rows() { return MT; }

int launch_mfma_nn(const float* A, int64_t sA, int lda, const float* W, int64_t sW, int ldw, float* Y, int64_t sY,
                   int ldy, int m, int kd, int l, int P, double* gpart, hipStream_t s) {
  if (l <= 32) return launch_thin<1, false>(A, sA, lda, W, sW, ldw, Y, sY, ldy, m, kd, l, P, gpart, s);
  if (l <= 64) return launch_thin<2, false>(A, sA, lda, W, sW, ldw, Y, sY, ldy, m, kd, l, P, gpart, s);
  return launch_thin<3, false>(A, sA, lda, W, sW, ldw, Y, sY, ldy, m, kd, l, P, gpart, s);
}

int launch_mfma_tn(const float* A, int64_t sA, int lda, const float* Q, int64_t sQ, int ldq, float* Z, int64_t sZ,
                   int ldz, int m, int n, int l, int P, double* gpart, hipStream_t s) {
  if (l <= 32) return launch_thin<1, true>(A, sA, lda, Q, sQ, ldq, Z, sZ, ldz, n, m, l, P, gpart, s);
  if (l <= 64) return launch_thin<2, true>(A, sA, lda, Q, sQ, ldq, Z, sZ, ldz, n, m, l, P, gpart, s);
  return launch_thin<3, true>(A, sA, lda, Q, sQ, ldq, Z, sZ, ldz, n, m, l, P, gpart, s);
}

}  // namespace ht
