// Block-level FP64 helpers shared by the orthonormalization and small-SVD
// kernels: summation of per-tile Gram partials, Cholesky with deflation and
// triangular solves.  All routines are called by every thread of the workgroup
// (uniform control flow, __syncthreads inside).  They are latency-bound, so
// every phase first issues all of a thread's independent loads and only then
// computes and stores.
#pragma once

#include "kernels.hpp"

namespace ht {

// 1/x for x != 0 (finite, not denormal) from the hardware estimate refined by
// two Newton steps (relative error at the level of the FP64 rounding unit).
__device__ __forceinline__ double fast_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * (2.0 - x * y);
  y = y * (2.0 - x * y);
  return y;
}

// 1/sqrt(x) for x > 0, estimate refined by two Newton steps.
__device__ __forceinline__ double fast_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// Broadcast lane `lane` (a compile-time or wave-uniform index) of a double.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cholesky with deflation held in registers of one wavefront: lane b owns
// column b of G (g[a] = G[a][b], a < LB, LB <= 64).  On return g[a] holds
// R[a][b] for a < b and g[b] = R[b][b] (0 for a skipped column); entries below
// the diagonal are meaningless.  Rows of R are broadcast with readlane, so the
// factorization needs no shared memory and no barriers.  delta: absolute pivot
// threshold (uniform).
template <int LB>
__device__ __forceinline__ void chol_regs(double (&g)[LB], int l, double delta) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < LB; ++j) {
    if (j < l) {
      const double d = readlane_d(g[j], j);
      if (d > delta) {
        const double inv_r = fast_rsqrt(d);
        const double rjb = g[j] * inv_r;  // R[j][b] on lane b >= j (R[j][j] on lane j)
        if (lane >= j) g[j] = rjb;
        // every a up to LB, without a test against l: a guard here becomes a
        // branch per entry and serializes the broadcasts.  Rows a >= l are
        // never read afterwards; their entries stay finite (the column lanes
        // past l hold copies of column 0).
        // up to 32 columns: eight broadcasts, then their updates (no wait
        // states between a broadcast and its use); wider kernels already run
        // short of scalar registers and update one entry at a time
        constexpr int NB = LB <= 32 ? 8 : 1;
#pragma unroll
        for (int a0 = j + 1; a0 < LB; a0 += NB) {
          double r[NB];
#pragma unroll
          for (int u = 0; u < NB; ++u)
            if (a0 + u < LB) r[u] = readlane_d(rjb, a0 + u);
#pragma unroll
          for (int u = 0; u < NB; ++u)
            if (a0 + u < LB) g[a0 + u] -= r[u] * rjb;
        }
      } else {
        if (lane >= j) g[j] = 0.0;
      }
    }
  }
}

// One wavefront: load column `lane` of the symmetric G (LDS, pitch gp), factor
// G = R^T R with deflation in registers, and write R^{-1} (upper, strict lower
// triangle zero) to Rinv (LDS, pitch gp).  Lane c forms column c of R^{-1} by
// column-oriented back substitution with the entries R[a][b] broadcast from
// lane b.  delta_rel: relative pivot threshold.
template <int LB>
__device__ inline void chol_inverse_regs(const double* G, int gp, int l, double delta_rel, double* Rinv) {
  const int lane = threadIdx.x & 63;
  const int col = lane < l ? lane : 0;
  double g[LB];
#pragma unroll
  for (int a = 0; a < LB; ++a) g[a] = (a < l) ? G[a * gp + col] : 0.0;
  double dmax = 0.0;
#pragma unroll
  for (int a = 0; a < LB; ++a)
    if (a == lane && a < l) dmax = g[a];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
  chol_regs<LB>(g, l, dmax > 0.0 ? delta_rel * dmax : 1.0);
  // back substitution: s[a] accumulates -sum_b R[a][b] x[b]
  double s[LB];
#pragma unroll
  for (int a = 0; a < LB; ++a) s[a] = (a == lane) ? 1.0 : 0.0;
#pragma unroll
  for (int b = LB - 1; b >= 0; --b) {
    if (b < l) {
      const double rbb = readlane_d(g[b], b);
      const double xb = (b <= lane && rbb != 0.0) ? s[b] * fast_rcp(rbb) : 0.0;
      s[b] = xb;
#pragma unroll
      for (int a = 0; a < b; ++a) s[a] -= readlane_d(g[a], b) * xb;  // R[a][b]
    }
  }
  if (lane < l) {
#pragma unroll
    for (int a = 0; a < LB; ++a)
      if (a < l) Rinv[a * gp + lane] = (a <= lane) ? s[a] : 0.0;
  }
}

// G (l x l, pitch gp) = sum over tiles t of part[t*l*l + a*l + b], in tile order.
__device__ inline void sum_gram_partials(double* G, int gp, const double* __restrict__ part, int ntiles, int l) {
  const int ll = l * l;
  constexpr int E = 4;  // entries per batch
  for (int e0 = threadIdx.x; e0 < ll; e0 += E * blockDim.x) {
    double s[E];
#pragma unroll
    for (int e = 0; e < E; ++e) s[e] = 0.0;
    for (int t0 = 0; t0 < ntiles; t0 += 4) {
      double v[E][4];
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int idx = e0 + e * blockDim.x;
          v[e][t] = (idx < ll && t0 + t < ntiles) ? part[(int64_t)(t0 + t) * ll + idx] : 0.0;
        }
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int t = 0; t < 4; ++t) s[e] += v[e][t];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = e0 + e * blockDim.x;
      if (idx < ll) G[(idx / l) * gp + (idx % l)] = s[e];
    }
  }
}

// Right-looking Cholesky with deflation of the upper triangle of G (l x l,
// pitch gp): on return the lower triangle holds R transposed,
// G[b*gp + j] = R[j][b] for j < b, and dR[j] = R[j][j], with G = R^T R on the
// kept columns.  A column whose Schur-complement pivot is <= delta_rel *
// max_i G_ii is skipped (row of R = 0, dR = 0).  One barrier per column: the
// trailing update reads the unscaled pivot row, which this column never
// writes, and R goes to the (unused) lower triangle.  s_scratch: one shared
// double.
__device__ inline void chol_deflate(double* G, double* dR, int gp, int l, double delta_rel, double* s_scratch) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) {
    double md = 0.0;
    for (int a = 0; a < l; ++a) md = fmax(md, G[a * gp + a]);
    *s_scratch = md;
  }
  __syncthreads();
  const double maxdiag = *s_scratch;
  const double delta = delta_rel * maxdiag;
  constexpr int RB = 16;  // rows per batch of the trailing update
  for (int j = 0; j < l; ++j) {
    const double d = G[j * gp + j];
    const bool keep = d > delta && maxdiag > 0.0;
    const double inv_r = keep ? fast_rsqrt(d) : 0.0;  // 1 / R[j][j]
    const double inv_d = inv_r * inv_r;
    // branch-free: the loads below do not wait for the pivot arithmetic
    for (int b = j + 1 + tid; b < l; b += nt) {
      const double gjb = G[j * gp + b];
      for (int a0 = j + 1; a0 <= b; a0 += RB) {
        double gja[RB], gab[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const int a = min(a0 + u, b);
          gja[u] = G[j * gp + a];
          gab[u] = G[a * gp + b];
        }
        const double f = gjb * inv_d;
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const int a = a0 + u;
          if (a <= b) G[a * gp + b] = gab[u] - gja[u] * f;
        }
      }
      G[b * gp + j] = gjb * inv_r;
    }
    if (tid == 0) dR[j] = keep ? d * inv_r : 0.0;
    __syncthreads();
  }
}

// After chol_deflate: R^{-1} (zero rows and columns at skipped indices) into
// Rinv (l x l, pitch gp, upper triangle; the strict lower triangle is zeroed).
// Column c of R^{-1} by column-oriented back substitution in registers
// (LB >= l): once x[b] is known it is removed from every pending row at once,
// so the dependent chain is one multiply-add per row.
template <int LB>
__device__ inline void tri_inverse(const double* G, const double* dR, int gp, int l, double* Rinv) {
  for (int c = threadIdx.x; c < l; c += blockDim.x) {
    double s[LB];
#pragma unroll
    for (int a = 0; a < LB; ++a) s[a] = (a == c) ? 1.0 : 0.0;
#pragma unroll
    for (int b = LB - 1; b >= 0; --b) {
      if (b <= c) {
        const double d = dR[b];
        const double xb = (d != 0.0) ? s[b] * fast_rcp(d) : 0.0;
        s[b] = xb;
#pragma unroll
        for (int a = 0; a < b; ++a) s[a] -= G[b * gp + a] * xb;  // R[a][b]
      }
    }
#pragma unroll
    for (int a = 0; a < LB; ++a)
      if (a < l) Rinv[a * gp + c] = (a <= c) ? s[a] : 0.0;
  }
  __syncthreads();
}

// FP64 Gram partials of an LDS tile on the matrix cores: element (i, c) of the
// tile is S[i * rs + c * cs] (rows i >= rows and columns c >= l read as zero),
// and each slab of kGramRows = 64 rows gets its own l x l partial,
//   out[h l l + a l + b] = sum_{i in slab h} S[i][a] S[i][b].
// Consumers sum ceil(m / 64) partials per slice whatever tile the producer
// used.  A wavefront takes (slab, 16 x 16 block of the upper triangle) units:
// 16 steps of v_mfma_f64_16x16x4f64 (the FP32 products are exact in FP64),
// operands loaded before the first step, and the block stored with its
// mirror.  No barrier: S is only read.  Operand layout of the instruction:
// lane t supplies A[t % 16][t / 16] and B[t / 16][t % 16]; accumulator v of
// lane t is D[4 v + t / 16][t % 16].
typedef double gram_d4 __attribute__((ext_vector_type(4)));
template <typename TS>
__device__ inline void tile_gram_mfma(const TS* S, int rs, int cs, int rows, int l, double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwv = (blockDim.x + 63) >> 6;
  const int nb = (l + 15) / 16, nblk = nb * (nb + 1) / 2;
  const int nslab = (rows + kGramRows - 1) / kGramRows;
  const int ll = l * l;
  for (int unit = wave; unit < nslab * nblk; unit += nwv) {
    const int h = unit / nblk;
    int blk = unit % nblk, bi = 0, len = nb;
    while (blk >= len) {
      blk -= len;
      ++bi;
      --len;
    }
    const int bj = bi + blk;
    const int ci = 16 * bi + (lane & 15), cj = 16 * bj + (lane & 15), kq = lane >> 4;
    double a[16], b[16];
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int row = h * kGramRows + 4 * st + kq;
      const bool ok = row < rows;
      a[st] = (ok && ci < l) ? (double)S[row * rs + ci * cs] : 0.0;
      b[st] = (ok && cj < l) ? (double)S[row * rs + cj * cs] : 0.0;
    }
    gram_d4 g = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < 16; ++st) g = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b[st], g, 0, 0, 0);
    double* o = out + (int64_t)h * ll;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * bi + 4 * v + kq, j = 16 * bj + (lane & 15);
      if (i < l && j < l) {
        o[i * l + j] = g[v];
        o[j * l + i] = g[v];
      }
    }
  }
}

// Complex Gram partial of an LDS tile of 64 complex rows kept as 128 real
// rows: row i < 64 is the real part of complex row i, row 64 + i its
// imaginary part (element (i, c) at S[i * rs + c * cs]; rows past the slice
// and columns c >= l hold zeros).  With Y = Yr + i Yi the tile's rows,
//   out[a l + b]       = (Yr^T Yr + Yi^T Yi)[a][b] = Re (Y^H Y)  (both triangles)
//   out[l^2 + a l + b] = (Yr^T Yi)[a][b] = M,  and Im (Y^H Y) = M - M^T.
// Units: 16 x 16 blocks of the upper triangle of the real part (32 steps of
// v_mfma_f64_16x16x4f64 over the 128 rows) and every 16 x 16 block of M (16
// steps over the 64 row pairs); operand layout as tile_gram_mfma.
template <typename TS>
__device__ inline void tile_cgram_mfma(const TS* S, int rs, int cs, int l, double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwv = (blockDim.x + 63) >> 6;
  const int nb = (l + 15) / 16, nsym = nb * (nb + 1) / 2;
  const int ll = l * l;
  for (int unit = wave; unit < nsym + nb * nb; unit += nwv) {
    const bool cross = unit >= nsym;
    int bi = 0, bj = 0;
    if (!cross) {
      int blk = unit, len = nb;
      while (blk >= len) {
        blk -= len;
        ++bi;
        --len;
      }
      bj = bi + blk;
    } else {
      bi = (unit - nsym) / nb;
      bj = (unit - nsym) % nb;
    }
    const int ci = 16 * bi + (lane & 15), cj = 16 * bj + (lane & 15), kq = lane >> 4;
    gram_d4 g = {0.0, 0.0, 0.0, 0.0};
    for (int part = 0; part < (cross ? 1 : 2); ++part) {
      double a[16], b[16];
#pragma unroll
      for (int st = 0; st < 16; ++st) {
        const int row = 64 * part + 4 * st + kq;
        const int rowb = cross ? 64 + row : row;
        a[st] = (ci < l) ? (double)S[row * rs + ci * cs] : 0.0;
        b[st] = (cj < l) ? (double)S[rowb * rs + cj * cs] : 0.0;
      }
#pragma unroll
      for (int st = 0; st < 16; ++st) g = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b[st], g, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * bi + 4 * v + kq, j = 16 * bj + (lane & 15);
      if (i < l && j < l) {
        if (cross) {
          out[ll + i * l + j] = g[v];
        } else {
          out[i * l + j] = g[v];
          out[j * l + i] = g[v];
        }
      }
    }
  }
}

}  // namespace ht
