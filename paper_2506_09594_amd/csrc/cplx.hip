// Complex face slices: the unitary or plain DFT on every mode 3..d turns the
// real tensor into complex transformed slices (one kept per conjugate pair).
//
// Storage.  A complex slice of n1 x n2 entries is the stacked real block
// [Re; Im] (2 n1 x n2, column-major, leading dimension 2 n1).  Its thin blocks
// are stacked the same way: Y and Q1 (2 n1 x l), Z and Bt (2 n2 x l), Q1 K'
// (2 n1 x l), K' (2 l x l).  The sketch Omega is real (n2 x l): the draws of
// the canonical slice, as for real slices.  Every product of the method is the
// complex one, with the conjugate transpose where the method transposes:
//   Y = A W,  Z = A^H Q,  Bt = A^H Q1,  C = (Q1 K') Bt^H.
// Gram partials come one per 64 complex rows, 2 l^2 doubles each: Re(Y^H Y)
// of the rows and M = Yr^T Yi, with Im(Y^H Y) = M - M^T (tile_cgram_mfma).
//
// This file holds the FP64 l x l stages of complex slices (CholeskyQR with
// deflation, the Hermitian eigensolver with the shrinkage), the FP64 matrix-core
// CholeskyQR apply and the vector-unit products that FP64 plans use; the FP32
// and BF16 sketch products run on the matrix cores (mfma.hip, mfma_bf16.hip).
#include <algorithm>
#include <type_traits>

#include "chol.hpp"

namespace ht {

namespace {

constexpr double kEps = 2.220446049250313e-16;

// Sum of the complex Gram partials of a thin block (ntiles tiles, fixed
// order): G = Gr + i Gi with Gr the summed real parts and Gi = M - M^T of the
// summed M.  Every thread takes up to NE entries and issues the loads of four
// tiles for all of them before adding, so that many loads are in flight; M is
// summed into Gi and made antisymmetric after a barrier (each pair of entries
// by one thread).  Ends with a barrier.
template <int NE>
__device__ inline void sum_cgram_partials(double* Gr, double* Gi, int gp, const double* __restrict__ part,
                                          int ntiles, int l) {
  const int ll = l * l, nt = blockDim.x;
  double sr[NE], sm[NE];
  int o[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    sr[e] = sm[e] = 0.0;
    o[e] = min((int)threadIdx.x + e * nt, ll - 1);
  }
  for (int t0 = 0; t0 < ntiles; t0 += 4) {
    double vr[4][NE], vm[4][NE];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double* p = part + (int64_t)min(t0 + u, ntiles - 1) * 2 * ll;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        vr[u][e] = p[o[e]];
        vm[u][e] = p[ll + o[e]];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (t0 + u < ntiles)
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          sr[e] += vr[u][e];
          sm[e] += vm[u][e];
        }
  }
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int idx = (int)threadIdx.x + e * nt;
    if (idx < ll) {
      Gr[(idx / l) * gp + idx % l] = sr[e];
      Gi[(idx / l) * gp + idx % l] = sm[e];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < ll; idx += nt) {
    const int a = idx / l, b = idx % l;
    if (a < b) {
      const double x = Gi[a * gp + b], y = Gi[b * gp + a];
      Gi[a * gp + b] = x - y;
      Gi[b * gp + a] = y - x;
    } else if (a == b) {
      Gi[a * gp + a] = 0.0;
    }
  }
  __syncthreads();
}

// Complex Cholesky with deflation: on entry the upper triangle of the
// Hermitian G = Gr + i Gi (pitch gp); G = R^H R with R upper triangular and a
// real positive diagonal.  On return dR[j] = R[j][j] (0 for a skipped column,
// whose row of R is zero) and R[j][b] for b > j sits in the strict lower
// triangle at (b, j).  A column is skipped when its Schur-complement pivot is
// at most delta_rel * max_a G[a][a].  Each thread holds up to NE entries
// (a <= b) of the triangle in registers for the whole factorization (entry
// e = b (b + 1) / 2 + a, dealt out once).  Column j: the owners of row j
// publish it to a row buffer (two, alternating, so that one barrier per column
// suffices), then every thread updates its trailing entries,
// G[a][b] -= conj(G[j][a]) G[j][b] / G[j][j] for j < a <= b, and the owners of
// row j store it scaled by 1 / sqrt(G[j][j]).
template <int NE>
__device__ inline void cchol_deflate(double* Gr, double* Gi, double* dR, int gp, int l, double delta_rel,
                                     double* s_scr) {
  __shared__ double rowr[2][kMaxComplexWidth], rowi[2][kMaxComplexWidth];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ntri = l * (l + 1) / 2;
  int ea[NE], eb[NE];
  double vr[NE], vi[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + u * nt;
    int bb = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while ((bb + 1) * (bb + 2) / 2 <= e) ++bb;
    while (bb * (bb + 1) / 2 > e) --bb;
    const bool ok = e < ntri;
    ea[u] = ok ? e - bb * (bb + 1) / 2 : l;  // a = l: no entry
    eb[u] = ok ? bb : l;
    vr[u] = ok ? Gr[ea[u] * gp + eb[u]] : 0.0;
    vi[u] = ok ? Gi[ea[u] * gp + eb[u]] : 0.0;
  }
  if (tid == 0) {
    double md = 0.0;
    for (int a = 0; a < l; ++a) md = fmax(md, Gr[a * gp + a]);
    *s_scr = md;
  }
  __syncthreads();
  const double maxdiag = *s_scr;
  const double delta = delta_rel * maxdiag;
  for (int j = 0; j < l; ++j) {
    const int buf = j & 1;
#pragma unroll
    for (int u = 0; u < NE; ++u)
      if (ea[u] == j) {
        rowr[buf][eb[u]] = vr[u];
        rowi[buf][eb[u]] = vi[u];
      }
    __syncthreads();
    const double d = rowr[buf][j];
    const bool keep = d > delta && maxdiag > 0.0;
    const double inv_r = keep ? fast_rsqrt(d) : 0.0;
    const double inv_d = inv_r * inv_r;
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int a = ea[u], b = eb[u];
      if (a < l && a > j) {
        const double jar = rowr[buf][a], jai = rowi[buf][a];
        const double fr = rowr[buf][b] * inv_d, fi = rowi[buf][b] * inv_d;
        vr[u] -= fma(jar, fr, jai * fi);
        vi[u] -= fma(jar, fi, -(jai * fr));
      } else if (a == j) {
        if (b > j) {
          Gr[b * gp + j] = vr[u] * inv_r;
          Gi[b * gp + j] = vi[u] * inv_r;
        } else {
          dR[j] = keep ? d * inv_r : 0.0;
        }
      }
    }
  }
  __syncthreads();
}

// X = R^{-1} (upper triangular, zero below the diagonal and at skipped
// indices) from the factor left by cchol_deflate (l <= 64).  Column c is
// formed by one wavefront: lane a holds x[a]; for b = c down to 0 lane b
// finishes x[b] = s[b] / R[b][b], which is broadcast to the lanes a < b that
// subtract R[a][b] x[b].  Columns are dealt to the wavefronts in turn.  X may
// be global or shared memory other than G's strict lower triangle.
__device__ inline void ctri_inverse_waves(const double* Gr, const double* Gi, const double* dR, int gp, int l,
                                          double* Xr, double* Xi, int xp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const double inv = (lane < l && dR[lane] != 0.0) ? fast_rcp(dR[lane]) : 0.0;
  for (int c = wave; c < l; c += nwv) {
    double sr = (lane == c) ? 1.0 : 0.0, si = 0.0;
    for (int b = c; b >= 0; --b) {
      const double xr = readlane_d(sr * inv, b), xi = readlane_d(si * inv, b);
      if (lane == b) {
        sr = xr;
        si = xi;
      } else if (lane < b) {
        const double rr = Gr[b * gp + lane], ri = Gi[b * gp + lane];  // R[lane][b]
        sr -= fma(rr, xr, -(ri * xi));
        si -= fma(rr, xi, ri * xr);
      }
    }
    if (lane < l) {
      Xr[lane * xp + c] = lane <= c ? sr : 0.0;
      Xi[lane * xp + c] = lane <= c ? si : 0.0;
    }
  }
}

// Products of l x l complex matrices held as planes (pitch gp) by a workgroup
// of at least ceil(l/2) ceil(l/4) threads, each forming a 2 x 4 block of the
// result in registers:
//   MODE 0: B <- B A       MODE 1: B <- A^H B      MODE 2: B <- B A^H
//   MODE 3: out <- A B, written to global memory as the stacked [Re; Im]
//           (2 l x l, column-major) in the storage type T.
// In-place modes read everything before a barrier and write after it.
template <int MODE, typename T>
__device__ inline void cmat_product(double* Br, double* Bi, const double* Ar, const double* Ai, int gp, int l,
                                    T* out) {
  const int nbc = (l + 3) / 4, nblk = ((l + 1) / 2) * nbc;
  const int blk = threadIdx.x;
  const bool act = blk < nblk;
  const int a0 = act ? 2 * (blk / nbc) : 0, b0 = act ? 4 * (blk % nbc) : 0;
  double accr[2][4], acci[2][4];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) accr[u][v] = acci[u][v] = 0.0;
  int ra[2], cb[4];
#pragma unroll
  for (int u = 0; u < 2; ++u) ra[u] = min(a0 + u, l - 1);
#pragma unroll
  for (int v = 0; v < 4; ++v) cb[v] = min(b0 + v, l - 1);
  if (act) {
    for (int c = 0; c < l; ++c) {
      double xr[2], xi[2], yr[4], yi[4];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (MODE == 0 || MODE == 2) {  // B[a][c]
          xr[u] = Br[ra[u] * gp + c];
          xi[u] = Bi[ra[u] * gp + c];
        } else if (MODE == 1) {  // conj(A[c][a])
          xr[u] = Ar[c * gp + ra[u]];
          xi[u] = -Ai[c * gp + ra[u]];
        } else {  // A[a][c]
          xr[u] = Ar[ra[u] * gp + c];
          xi[u] = Ai[ra[u] * gp + c];
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (MODE == 0) {  // A[c][b]
          yr[v] = Ar[c * gp + cb[v]];
          yi[v] = Ai[c * gp + cb[v]];
        } else if (MODE == 2) {  // conj(A[b][c])
          yr[v] = Ar[cb[v] * gp + c];
          yi[v] = -Ai[cb[v] * gp + c];
        } else {  // B[c][b]
          yr[v] = Br[c * gp + cb[v]];
          yi[v] = Bi[c * gp + cb[v]];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          accr[u][v] = fma(xr[u], yr[v], fma(-xi[u], yi[v], accr[u][v]));
          acci[u][v] = fma(xr[u], yi[v], fma(xi[u], yr[v], acci[u][v]));
        }
    }
  }
  if (MODE == 3) {
    if (act)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = a0 + u, b = b0 + v;
          if (a < l && b < l) {
            out[a + (int64_t)b * 2 * l] = (T)accr[u][v];
            out[l + a + (int64_t)b * 2 * l] = (T)acci[u][v];
          }
        }
    return;
  }
  __syncthreads();
  if (act)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = a0 + u, b = b0 + v;
        if (a < l && b < l) {
          Br[a * gp + b] = accr[u][v];
          Bi[a * gp + b] = acci[u][v];
        }
      }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// CholeskyQR of complex thin blocks: one workgroup per slice factors the
// summed Gram matrix and parks R^{-1} (real rows, then imaginary rows, l x l
// each, row-major) over the slice's first Gram partial; the apply kernel then
// forms Q = Y R^{-1} per 64 complex rows.
// ---------------------------------------------------------------------------
constexpr int kFactorThreads = 512;

__global__ __launch_bounds__(kFactorThreads) void k_corth_factor(int which, const SliceDesc* __restrict__ sd,
                                                                 const int2* __restrict__ wk,
                                                                 double* __restrict__ gin_all) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double s_scr;
  const int s = blockIdx.x;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int m = which ? d.n2 : d.n1;
  const int nparts = (m + kGramRows - 1) / kGramRows;
  const int gp = l + 1, ll = l * l;
  double* Gr = reinterpret_cast<double*>(smem_raw);
  double* Gi = Gr + (size_t)l * gp;
  double* dR = Gi + (size_t)l * gp;
  double* part = gin_all + d.g1;
  sum_cgram_partials<(kMaxComplexWidth * kMaxComplexWidth + kFactorThreads - 1) / kFactorThreads>(Gr, Gi, gp, part,
                                                                                                 nparts, l);
  cchol_deflate<(kMaxComplexWidth * (kMaxComplexWidth + 1) / 2 + kFactorThreads - 1) / kFactorThreads>(
      Gr, Gi, dR, gp, l, 8.0 * (double)m * kEps, &s_scr);
  ctri_inverse_waves(Gr, Gi, dR, gp, l, part, part + ll, l);
}

size_t cfactor_lds_bytes(int l) { return (2 * (size_t)l * (l + 1) + (size_t)l + 1) * 8; }

// Q = Y R^{-1} for 64 complex rows of one slice on the FP64 matrix cores, in
// real form: [Qr, Qi] (64 x 2l) = [Yr, Yi] (64 x 2l) E with
// E = [[Rr, Ri], [-Ri, Rr]] (2l x 2l) for R^{-1} = Rr + i Ri, whose four
// quadrants are upper triangular.  Wavefront w owns rows 16w .. 16w + 15 and
// every 16-column block of the result on v_mfma_f64_16x16x4f64 (lane t
// supplies A[t % 16][t / 16] and B[t / 16][t % 16]; accumulator v of lane t
// is D[4 v + t / 16][t % 16]); a (4-step, 16-column) pair whose entries of E
// all lie below the diagonal of their quadrant is skipped.  R^{-1} sits in LDS
// as two planes; the result goes through an LDS tile (real parts of the 64
// rows, then their imaginary parts, FP32 as stored) for coalesced column
// stores and, optionally, the complex Gram partial of the stored rows.
template <typename T, int LB>
__global__ __launch_bounds__(256) void k_corth_apply(T* __restrict__ Yall, uint16_t* __restrict__ Yhall, int which,
                                                     const SliceDesc* __restrict__ sd, const int2* __restrict__ wk,
                                                     const int2* __restrict__ items,
                                                     const double* __restrict__ gin_all,
                                                     double* __restrict__ gout_all) {
  constexpr int NCB = LB / 8;     // 16-column blocks of the 2 l <= 2 LB result columns
  constexpr int NST = LB / 2;     // 4-deep steps over the 2 l <= 2 LB reduction
  constexpr int SP = LB + 1;      // pitch of the staging tile (storage type: the values as stored)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int2 it = items[blockIdx.x];
  const int s = it.x, r0 = it.y;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int m = which ? d.n2 : d.n1, ld = 2 * m, ll = l * l, l2 = 2 * l;
  T* Y = Yall + (which ? d.z : d.y);
  const double* Rg = gin_all + d.g1;
  double* Rr = reinterpret_cast<double*>(smem_raw);  // R^{-1}, row-major l x l (pitch l)
  double* Ri = Rr + ll;
  {  // both planes are contiguous in the parked area: every load issued at once
    constexpr int NL = (2 * LB * LB + 255) / 256;
    double v[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) v[u] = Rg[min((int)threadIdx.x + u * 256, 2 * ll - 1)];
#pragma unroll
    for (int u = 0; u < NL; ++u)
      if ((int)threadIdx.x + u * 256 < 2 * ll) Rr[threadIdx.x + u * 256] = v[u];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  // A operand: row 16 w + li of the tile at k = 4 st + lq (k < l: Yr, k < 2l: Yi)
  const int arow = r0 + 16 * w + li;
  const int lrow = arow < m ? arow : m - 1;
  double a[NST];
#pragma unroll
  for (int st = 0; st < NST; ++st) {
    const int k = 4 * st + lq;
    const int kk = k < l ? k : (k < l2 ? k - l : 0);
    const T v = Y[(k < l ? 0 : m) + lrow + (int64_t)kk * ld];
    a[st] = (k < l2 && arow < m) ? (double)v : 0.0;
  }
  __syncthreads();
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
  // entry (k, c) of E: quadrant (k >= l, c >= l), position (k mod l, c mod l)
  auto eval = [&](int k, int c) -> double {
    if (k >= l2 || c >= l2) return 0.0;
    const bool kh = k >= l, ch = c >= l;
    const int kq = kh ? k - l : k, cq = ch ? c - l : c;
    const int o = kq * l + cq;
    return kh == ch ? Rr[o] : (ch ? Ri[o] : -Ri[o]);
  };
#pragma unroll
  for (int st = 0; st < NST; ++st) {
    if (4 * st >= l2) break;
    const int k0 = 4 * st, k0q = k0 >= l ? k0 - l : k0;
    const bool kstraddle = k0 < l && k0 + 3 >= l;
    double b[NCB];
    bool use[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      // skip when every k of the step is past every c of the block within its quadrant;
      // blocks and steps that straddle a quadrant boundary are always computed
      const int c0 = 16 * cb, c1 = min(c0 + 15, l2 - 1);
      const bool cstraddle = c0 < l && c1 >= l;
      const int c1q = c1 >= l ? c1 - l : c1;
      use[cb] = c0 < l2 && (cstraddle || kstraddle || k0q <= c1q);
      b[cb] = use[cb] ? eval(k0 + lq, c0 + li) : 0.0;
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
      if (use[cb]) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b[cb], acc[cb], 0, 0, 0);
  }
  __syncthreads();  // R^{-1} is no longer read: its LDS holds the result tile
  T* S = reinterpret_cast<T*>(smem_raw);  // [part * 64 + row][column]
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * w + 4 * v + lq, c = 16 * cb + li;
      if (c < l2) {
        const bool part = c >= l;
        S[((part ? 64 : 0) + row) * SP + (part ? c - l : c)] = (r0 + row < m) ? (T)acc[cb][v] : T(0);
      }
    }
  __syncthreads();
  const int rows = min(64, m - r0);
  for (int idx = threadIdx.x; idx < 2 * 64 * l; idx += 256) {
    const int row = idx % 64, pc = idx / 64, part = pc / l, c = pc % l;
    if (row < rows) {
      const int64_t o = (part ? m : 0) + r0 + row + (int64_t)c * ld;
      Y[o] = S[(part * 64 + row) * SP + c];
      if (Yhall)
        Yhall[(which ? d.z : d.y) + o] = (uint16_t)(f32x2_to_bf16x2((float)S[(part * 64 + row) * SP + c], 0.0f) & 0xffffu);
    }
  }
  if (gout_all) tile_cgram_mfma(S, SP, 1, l, gout_all + d.g2 + (int64_t)(r0 / kGramRows) * 2 * ll);
}

// The same product for FP32 blocks without Gram partials.  The 64-row tiles
// of every slice, in slice order, are split into one contiguous range per
// resident workgroup; R^{-1} is staged in LDS when the range enters a slice,
// as two 64 x 64 planes with the quadrants padded to 64, so that every
// (4-deep step, 16-column block) pair lies in one quadrant of E: its plane,
// sign and triangular skip are uniform across the wavefront.  Wavefront w owns
// rows 16 w .. 16 w + 15 of each tile and holds them as the A operands
// (k = 4 st + t / 16: real parts for st < 16, imaginary parts after); the next
// tile's rows load while the current one is multiplied.  The product is
// taken transposed (E block as the A operand, the rows as the B operand), so
// accumulator v of lane t holds row t % 16 of column 4 v + t / 16 of its
// block: the result goes straight from the accumulators to Y as runs of 16
// consecutive rows per column, and an optional BF16 copy as pairs of rows
// joined across neighbouring lanes.  Each wavefront reads and then overwrites
// only its own rows.
constexpr int kApplyPitch = 72;  // doubles per LDS row of a plane
constexpr size_t kApplyLds = 2 * 64 * kApplyPitch * sizeof(double);

__global__ __launch_bounds__(256, 2) void k_corth_apply_tiles(float* __restrict__ Yall, uint16_t* __restrict__ Yhall,
                                                              int which, const SliceDesc* __restrict__ sd,
                                                              const int2* __restrict__ wk,
                                                              const int2* __restrict__ tiles, int ntiles,
                                                              const double* __restrict__ gin_all) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Er = reinterpret_cast<double*>(smem_raw);  // Re R^{-1}, padded 64 x 64
  double* Ei = Er + 64 * kApplyPitch;                // Im R^{-1}
  const int t_begin = (int)((int64_t)blockIdx.x * ntiles / gridDim.x);
  const int t_end = (int)((int64_t)(blockIdx.x + 1) * ntiles / gridDim.x);
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, li = lane & 15, lq = lane >> 4;
  // B operands of tile t: rows 16 w + li, k = 4 (st mod 16) + t / 16 of part st / 16
  auto fetch = [&](int t, float (&dst)[32]) {
    const int2 it = tiles[t];
    const SliceDesc d = sd[it.x];
    const int l = slice_width(d, wk, it.x);
    const int m = which ? d.n2 : d.n1, ld = 2 * m;
    const int row = it.y + 16 * w + li;
    const bool okr = row < m && l > 0;
    const float* src = Yall + (which ? d.z : d.y) + (okr ? row : 0);
#pragma unroll
    for (int st = 0; st < 32; ++st) {
      const int kk = 4 * (st & 15) + lq;
      const bool ok = okr && kk < l;
      dst[st] = ok ? src[(st >= 16 ? m : 0) + (int64_t)kk * ld] : 0.0f;
    }
  };
  float a[32], an[32];
  if (t_begin < t_end) fetch(t_begin, a);
  int cur = -1;
  typedef double d4 __attribute__((ext_vector_type(4)));
  for (int t = t_begin; t < t_end; ++t) {
    const int2 it = tiles[t];
    const int s = it.x, r0 = it.y;
    const SliceDesc d = sd[s];
    const int l = slice_width(d, wk, s);
    if (s != cur) {  // stage this slice's R^{-1} (uniform branch)
      if (cur >= 0) __syncthreads();
      cur = s;
      if (l > 0) {
        const int ll = l * l;
        const double* Rg = gin_all + d.g1;
        double vr[16], vi[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int idx = tid + 256 * u, a0 = idx / 64, b0 = idx % 64;
          const bool ok = a0 < l && b0 < l;
          const int o = ok ? a0 * l + b0 : 0;
          vr[u] = Rg[o];
          vi[u] = Rg[ll + o];
          vr[u] = ok ? vr[u] : 0.0;
          vi[u] = ok ? vi[u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int idx = tid + 256 * u, a0 = idx / 64, b0 = idx % 64;
          Er[a0 * kApplyPitch + b0] = vr[u];
          Ei[a0 * kApplyPitch + b0] = vi[u];
        }
      }
      __syncthreads();
    }
    if (t + 1 < t_end) fetch(t + 1, an);
    if (l > 0) {
      const int m = which ? d.n2 : d.n1, ld = 2 * m;
      d4 acc[8];
#pragma unroll
      for (int cb = 0; cb < 8; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < 32; ++st) {
        const int kp = st >> 4, kq0 = 4 * (st & 15);
        if (kq0 >= l) continue;
        const double av = (double)a[st];
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) {
          const int cp = cb >> 2, cq0 = 16 * (cb & 3);
          if (kq0 > cq0 + 15 || cq0 >= l) continue;  // zero block of the quadrant
          // E = [[Rr, Ri], [-Ri, Rr]] by quadrant (k part, c part)
          const double* P = kp == cp ? Er : Ei;
          double b = P[(kq0 + lq) * kApplyPitch + cq0 + li];
          if (kp == 1 && cp == 0) b = -b;
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(b, av, acc[cb], 0, 0, 0);
        }
      }
      const int row = r0 + 16 * w + li;
      const bool pairs = (m & 1) == 0;  // row pairs (2 j, 2 j + 1) are 4-byte aligned in the BF16 copy
#pragma unroll
      for (int cb = 0; cb < 8; ++cb) {
        const int cp = cb >> 2, cq0 = 16 * (cb & 3);
        if (cq0 >= l) continue;  // uniform
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cq = cq0 + 4 * v + lq;
          const int64_t o = (which ? d.z : d.y) + (cp ? m : 0) + (int64_t)cq * ld + row;
          const float q = (float)acc[cb][v];
          const bool ok = cq < l && row < m;
          if (ok) Yall[o] = q;
          if (Yhall) {
            // every lane takes part in the exchange; even lanes store the pair
            const float qn = __int_as_float(
                __builtin_amdgcn_mov_dpp(__float_as_int(q), 0xb1, 0xf, 0xf, false));
            if (pairs) {
              if (ok && (li & 1) == 0)
                *reinterpret_cast<uint32_t*>(Yhall + o) = f32x2_to_bf16x2(q, qn);
            } else if (ok) {
              Yhall[o] = (uint16_t)(f32x2_to_bf16x2(q, 0.0f) & 0xffffu);
            }
          }
        }
      }
    }
    if (t + 1 < t_end)
#pragma unroll
      for (int st = 0; st < 32; ++st) a[st] = an[st];
  }
}

// Complex Gram partials of a stored basis, one workgroup per 64-row tile
// (the items of the apply): the tile's values as stored go to LDS as 128 real
// rows (real parts of the 64 rows, then their imaginary parts; zeros past the
// slice and past l) and tile_cgram_mfma forms the partial.  Follows the
// resident tile apply for the final basis, which then needs no per-tile
// restaging of R^-1.
template <typename T, int LB>
__global__ __launch_bounds__(256) void k_cgram_tiles(const T* __restrict__ Yall, int which,
                                                     const SliceDesc* __restrict__ sd, const int2* __restrict__ wk,
                                                     const int2* __restrict__ items, double* __restrict__ gout_all) {
  constexpr int SP = LB + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* S = reinterpret_cast<T*>(smem_raw);  // [part * 64 + row][column]
  const int2 it = items[blockIdx.x];
  const int s = it.x, r0 = it.y;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int m = which ? d.n2 : d.n1, ld = 2 * m, rows = min(64, m - r0);
  const T* Y = Yall + (which ? d.z : d.y);
  constexpr int NL = 2 * 64 * LB / 256;  // loads per thread, all issued before the first LDS store
  T v[NL];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int idx = threadIdx.x + 256 * u, row = idx % 64, pc = idx / 64, part = pc / LB, c = pc % LB;
    const bool ok = row < rows && c < l;
    v[u] = Y[ok ? (part ? m : 0) + r0 + row + (int64_t)c * ld : 0];
  }
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int idx = threadIdx.x + 256 * u, row = idx % 64, pc = idx / 64, part = pc / LB, c = pc % LB;
    S[(part * 64 + row) * SP + c] = (row < rows && c < l) ? v[u] : T(0);
  }
  __syncthreads();
  tile_cgram_mfma(S, SP, 1, l, gout_all + d.g2 + (int64_t)(r0 / kGramRows) * 2 * l * l);
}

template <typename T, int LB>
constexpr size_t capply_lds_bytes() {
  constexpr size_t r = 2 * (size_t)LB * LB * 8, t = 128 * (size_t)(LB + 1) * sizeof(T);
  return r > t ? r : t;
}

// ---------------------------------------------------------------------------
// Small SVD and shrinkage of complex slices, FP64, one workgroup per slice.
// With R2 = chol(Q1^H Q1) (from the Gram partials of Q1) and Wt = Bt^H Bt
// (from those of Bt = A^H Q1): W = R2^{-H} Wt R2^{-1} = B B^H for
// B = Q^H A, Q = Q1 R2^{-1}.  W = U diag(s^2) U^H (heev_tridiag); with
// the k = min(r, l) largest s shrunk,
//   K' = R2^{-1} U diag(w) U^H R2^{-H},  w_i = prox(s_i) / s_i,
// so that the reconstruction is C = Q1 K' Bt^H.
// ---------------------------------------------------------------------------
constexpr int kSvdThreads = 512;

// Data-parallel move of a double across lanes (DPP control CTRL, every lane
// active).
template <int CTRL>
__device__ __forceinline__ double mov_dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wavefront (every lane active), the same value in
// every lane: butterflies within quads (quad_perm [1,0,3,2], [2,3,0,1]), then
// rotations by 4 and 8 within rows of 16, then the four row sums.
__device__ __forceinline__ double wave_sum(double v) {
  v += mov_dpp_d<0xb1>(v);
  v += mov_dpp_d<0x4e>(v);
  v += mov_dpp_d<0x124>(v);
  v += mov_dpp_d<0x128>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Eigen-decomposition of a Hermitian W = Wr + i Wi (n x n, n <= 64, pitch gp,
// full matrix) by a workgroup of 512 threads:
//  1. Householder reduction W = Q T Q^H (T Hermitian tridiagonal), Q
//     accumulated in (Vr, Vi), which hold the identity on entry.  Step k
//     reflects x = W[k+1:n][k] to beta e1, beta = -(x0 / |x0|) |x|, with
//     H = I - tau v v^H, v = x - beta e1, tau = 1 / (|x| (|x| + |x0|)); the
//     trailing block becomes H W2 H = W2 - v w^H - w v^H with p = tau W2 v,
//     w = p - (tau / 2)(v^H p) v, and Q2 <- Q2 - tau (Q2 v) v^H.  Every
//     wavefront forms v itself (lane i holds v_i); the products W2 v and Q2 v
//     are split over the wavefronts by columns (lane = row) and summed after a
//     barrier; the rank-two update follows the same split.  Two barriers a step.
//  2. The diagonal unitary D = diag(phi), phi_{k+1} = phi_k e_k / |e_k|, makes
//     T' = D^H T D real with subdiagonal |e_k|.
//  3. Eigenvalues of T' by bisection on Sturm counts (the number of negative
//     pivots of T' - x I), nine-way: eight lanes per eigenvalue test eight
//     points of its interval per round.
//  4. Eigenvectors of T' from the twisted factorization of T' - lambda I: the
//     forward and backward pivots d+ and d-, the twist r minimizing
//     |d+_r + d-_r - (d_r - lambda)|, z_r = 1 and the two recurrences away
//     from r; then the members of each cluster of eigenvalues closer than
//     1e-3 ||T'|| are made orthogonal (below).  Only eigenpairs the caller
//     uses need this: those with an eigenvalue above `thr` among the `keep`
//     largest (the others may come out of a cluster non-orthogonal).
//  5. U = Q D Z into (Vr, Vi); lam[i] ascending.
// The planes (Wr, Wi) are scratch from step 3 on (they hold Z).
__device__ __forceinline__ void heev_tridiag(double* Wr, double* Wi, double* Vr, double* Vi, int gp, int n, double* lam,
                                    double thr, int keep) {
  __shared__ double s_part[8][4][64];  // per-wavefront partial sums: Re p, Im p, Re y, Im y
  __shared__ double s_d[64], s_er[64], s_ei[64], s_eh[64], s_e2[64], s_phr[64], s_phi[64];
  __shared__ int s_twist[64];
  __shared__ double s_solve[5][64];  // elimination of T' - lambda I: multipliers, diagonals, right side
  __shared__ double s_nrm;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = kSvdThreads / 64;
  // ---- 1. Householder tridiagonalization ----
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1, c0 = k + 1;
    const bool li = lane < m;
    const double xr = li ? Wr[(c0 + lane) * gp + k] : 0.0, xi = li ? Wi[(c0 + lane) * gp + k] : 0.0;
    const double alpha = sqrt(wave_sum(xr * xr + xi * xi));
    const double x0r = readlane_d(xr, 0), x0i = readlane_d(xi, 0);
    const double ax0 = sqrt(x0r * x0r + x0i * x0i);
    const double phr = ax0 > 0.0 ? x0r / ax0 : 1.0, phi = ax0 > 0.0 ? x0i / ax0 : 0.0;
    if (tid == 0) {
      s_d[k] = Wr[k * gp + k];
      s_er[k] = -phr * alpha;
      s_ei[k] = -phi * alpha;
    }
    if (!(alpha > 0.0)) continue;  // nothing to reflect (uniform: every wavefront sums the same column)
    const double tau = 1.0 / (alpha * (alpha + ax0));
    const double vr = lane == 0 ? x0r + phr * alpha : xr, vi = lane == 0 ? x0i + phi * alpha : xi;
    // partial products over this wavefront's columns j = wv, wv + 8, ...
    double ppr = 0.0, ppi = 0.0, pyr = 0.0, pyi = 0.0;
    for (int j = wv; j < m; j += NW) {
      const double bjr = readlane_d(vr, j), bji = readlane_d(vi, j);
      if (li) {
        const double ar = Wr[(c0 + lane) * gp + c0 + j], ai = Wi[(c0 + lane) * gp + c0 + j];
        ppr = fma(ar, bjr, fma(-ai, bji, ppr));
        ppi = fma(ar, bji, fma(ai, bjr, ppi));
      }
      if (lane < n) {
        const double qr = Vr[lane * gp + c0 + j], qi = Vi[lane * gp + c0 + j];
        pyr = fma(qr, bjr, fma(-qi, bji, pyr));
        pyi = fma(qr, bji, fma(qi, bjr, pyi));
      }
    }
    s_part[wv][0][lane] = ppr;
    s_part[wv][1][lane] = ppi;
    s_part[wv][2][lane] = pyr;
    s_part[wv][3][lane] = pyi;
    __syncthreads();
    double pr = 0.0, pi = 0.0, yr = 0.0, yi = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      pr += s_part[w][0][lane];
      pi += s_part[w][1][lane];
      yr += s_part[w][2][lane];
      yi += s_part[w][3][lane];
    }
    pr *= tau;
    pi *= tau;
    // K = (tau / 2) v^H p (real), w = p - K v
    const double K = 0.5 * tau * wave_sum(li ? vr * pr + vi * pi : 0.0);
    const double wr = pr - K * vr, wi = pi - K * vi;
    for (int j = wv; j < m; j += NW) {
      const double bvr = readlane_d(vr, j), bvi = readlane_d(vi, j);
      const double bwr = readlane_d(wr, j), bwi = readlane_d(wi, j);
      if (li) {  // W2[i][j] -= v_i conj(w_j) + w_i conj(v_j)
        const int o = (c0 + lane) * gp + c0 + j;
        Wr[o] -= (vr * bwr + vi * bwi) + (wr * bvr + wi * bvi);
        Wi[o] -= (vi * bwr - vr * bwi) + (wi * bvr - wr * bvi);
      }
      if (lane < n) {  // Q2[a][j] -= tau y_a conj(v_j)
        const int o = lane * gp + c0 + j;
        Vr[o] -= tau * (yr * bvr + yi * bvi);
        Vi[o] -= tau * (yi * bvr - yr * bvi);
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int k = (n >= 2 ? n - 2 : 0); k < n; ++k) s_d[k] = Wr[k * gp + k];
    if (n >= 2) {
      s_er[n - 2] = Wr[(n - 1) * gp + n - 2];
      s_ei[n - 2] = Wi[(n - 1) * gp + n - 2];
    }
    // ---- 2. phases: T' = D^H T D real ----
    double fr = 1.0, fi = 0.0;
    s_phr[0] = 1.0;
    s_phi[0] = 0.0;
    for (int k = 0; k + 1 < n; ++k) {
      const double er = s_er[k], ei = s_ei[k], ae = sqrt(er * er + ei * ei);
      s_eh[k] = ae;
      s_e2[k] = ae * ae;
      if (ae > 0.0) {
        const double ur = er / ae, ui = ei / ae;
        const double nr = fr * ur - fi * ui, ni = fr * ui + fi * ur;
        fr = nr;
        fi = ni;
      }
      s_phr[k + 1] = fr;
      s_phi[k + 1] = fi;
    }
    double nrm = 0.0;  // ||T'||_1
    for (int k = 0; k < n; ++k)
      nrm = fmax(nrm, fabs(s_d[k]) + (k > 0 ? s_eh[k - 1] : 0.0) + (k + 1 < n ? s_eh[k] : 0.0));
    s_nrm = nrm;
  }
  __syncthreads();
  const double tnorm = s_nrm;
  double e2max = 0.0;
  for (int k = 0; k + 1 < n; ++k) e2max = fmax(e2max, s_eh[k] * s_eh[k]);
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, e2max);
  // ---- 3. bisection: eigenvalue i = tid / 8, sub-point tid % 8 ----
  {
    const int i = tid >> 3, sub = tid & 7;
    double lo = -tnorm - pivmin, hi = tnorm + pivmin;
    for (int round = 0; round < 19; ++round) {
      const double x = lo + (hi - lo) * (double)(sub + 1) / 9.0;
      int cnt = 0;
      if (i < n) {  // negative pivots of T' - x I (reciprocal refined to the FP64 rounding level)
        double q = s_d[0] - x;
        if (q <= pivmin) {
          ++cnt;
          q = fmin(q, -pivmin);
        }
#pragma unroll 4
        for (int k = 1; k < n; ++k) {
          q = (s_d[k] - x) - s_e2[k - 1] * fast_rcp(q);
          if (q <= pivmin) {
            ++cnt;
            q = fmin(q, -pivmin);
          }
        }
      }
      // points with at most i eigenvalues below them form a prefix of the eight
      const unsigned long long below = __ballot(cnt <= i);
      const int t = __popcll((below >> (lane & ~7)) & 0xffull);
      const double xlo = lo + (hi - lo) * (double)t / 9.0, xhi = lo + (hi - lo) * (double)(t + 1) / 9.0;
      lo = t > 0 ? xlo : lo;
      hi = t < 8 ? xhi : hi;
    }
    if (i < n && sub == 0) lam[i] = 0.5 * (lo + hi);
  }
  __syncthreads();
  // ---- 4. eigenvectors of T' (thread e < n): Z row e at Wr + e * n ----
  double* Z = Wr;
  double* Dm = Wr + n * n;  // backward pivots
  if (tid < n) {
    const int e = tid;
    const double lm = lam[e];
    double* zp = Z + e * n;
    double* dm = Dm + e * n;
    auto guard = [&](double q) { return fabs(q) < pivmin ? (q < 0.0 ? -pivmin : pivmin) : q; };
    double q = guard(s_d[n - 1] - lm);
    dm[n - 1] = q;
    for (int k = n - 2; k >= 0; --k) {
      q = guard((s_d[k] - lm) - s_eh[k] * s_eh[k] / q);
      dm[k] = q;
    }
    int r = 0;
    double best = 0.0, qp = 0.0;
    for (int k = 0; k < n; ++k) {
      qp = guard(k == 0 ? s_d[0] - lm : (s_d[k] - lm) - s_eh[k - 1] * s_eh[k - 1] / qp);
      zp[k] = qp;  // forward pivot d+_k
      const double g = fabs(qp + dm[k] - (s_d[k] - lm));
      if (k == 0 || g < best) {
        best = g;
        r = k;
      }
    }
    double nz = 1.0, z = 1.0;
    for (int k = r - 1; k >= 0; --k) {
      z = -(s_eh[k] / zp[k]) * z;
      zp[k] = z;
      nz += z * z;
    }
    z = 1.0;
    for (int k = r + 1; k < n; ++k) {
      z = -(s_eh[k - 1] / dm[k]) * z;
      zp[k] = z;
      nz += z * z;
    }
    zp[r] = 1.0;
    const double inv = 1.0 / sqrt(nz);
    for (int k = 0; k < n; ++k) zp[k] *= inv;
    s_twist[e] = r;
  }
  __syncthreads();
  // Clusters of eigenvalues closer than 1e-3 ||T'|| (wavefront 0, lane =
  // component): every member after the first is refined by three steps of
  // inverse iteration, each preceded by Gram-Schmidt (twice) against the
  // members before it, and orthogonalized once more at the end.  A vector
  // that Gram-Schmidt annihilates restarts from a fixed dense vector.  The
  // solves of T' - lambda I use Gaussian elimination with partial pivoting
  // (lane 0; a zero pivot becomes eps ||T'||).
  if (wv == 0) {
    double* sdl = s_solve[0];  // subdiagonal multipliers, diagonal, first and second superdiagonals, right side
    double* sdd = s_solve[1];
    double* sdu = s_solve[2];
    double* sdu2 = s_solve[3];
    double* sx = s_solve[4];
    const double ortol = 1e-3 * tnorm, tiny = 2.220446049250313e-16 * tnorm;
    auto gs = [&](double x, int a, int e) {  // against members a + 1 .. e - 1
      for (int pass = 0; pass < 2; ++pass)
        for (int b = a + 1; b < e; ++b) {
          const double zb = lane < n ? Z[b * n + lane] : 0.0;
          x -= wave_sum(x * zb) * zb;
        }
      return x;
    };
    // first eigenpair the caller uses (eigenvalues ascend)
    int i0 = max(0, n - keep);
    while (i0 < n && !(lam[i0] > thr)) ++i0;
    int c0 = 0;
    for (int e = 1; e <= n; ++e) {
      if (e < n && lam[e] - lam[e - 1] <= ortol) continue;
      // cluster c0 .. e - 1: its largest member stays, the others (from the
      // top) are refined against the members above them
      for (int a = e - 2; a >= max(c0, i0); --a) {
        double x = lane < n ? Z[a * n + lane] : 0.0;
        for (int it = 0; it < 3; ++it) {
          x = gs(x, a, e);
          double nn = wave_sum(x * x);
          if (!(nn > 1e-20)) {
            x = lane < n ? 1.0 + 0.5 * sin(0.7 * lane + 1.3 * a) : 0.0;
            x = gs(x, a, e);
            nn = wave_sum(x * x);
          }
          x *= 1.0 / sqrt(nn);
          if (lane < n) sx[lane] = x;
          __threadfence_block();
          if (lane == 0) {
            const double lm = lam[a];
            for (int k = 0; k < n; ++k) {
              sdd[k] = s_d[k] - lm;
              if (k + 1 < n) sdl[k] = sdu[k] = s_eh[k];
              sdu2[k] = 0.0;
            }
            for (int i = 0; i + 1 < n; ++i) {
              if (fabs(sdd[i]) >= fabs(sdl[i])) {  // no interchange
                if (sdd[i] == 0.0) sdd[i] = tiny;
                const double f = sdl[i] / sdd[i];
                sdl[i] = f;
                sdd[i + 1] -= f * sdu[i];
                s_twist[i] = 0;
              } else {  // rows i and i + 1 interchanged
                const double f = sdd[i] / sdl[i];
                sdd[i] = sdl[i];
                sdl[i] = f;
                const double t = sdu[i];
                sdu[i] = sdd[i + 1];
                sdd[i + 1] = t - f * sdd[i + 1];
                if (i + 2 < n) {
                  sdu2[i] = sdu[i + 1];
                  sdu[i + 1] = -f * sdu[i + 1];
                }
                s_twist[i] = 1;
              }
            }
            if (sdd[n - 1] == 0.0) sdd[n - 1] = tiny;
            for (int i = 0; i + 1 < n; ++i) {
              if (s_twist[i] == 0) {
                sx[i + 1] -= sdl[i] * sx[i];
              } else {
                const double t = sx[i];
                sx[i] = sx[i + 1];
                sx[i + 1] = t - sdl[i] * sx[i];
              }
            }
            sx[n - 1] /= sdd[n - 1];
            if (n > 1) sx[n - 2] = (sx[n - 2] - sdu[n - 2] * sx[n - 1]) / sdd[n - 2];
            for (int i = n - 3; i >= 0; --i) sx[i] = (sx[i] - sdu[i] * sx[i + 1] - sdu2[i] * sx[i + 2]) / sdd[i];
          }
          __threadfence_block();
          x = lane < n ? sx[lane] : 0.0;
          x *= 1.0 / sqrt(wave_sum(x * x));
        }
        x = gs(x, a, e);
        x *= 1.0 / sqrt(wave_sum(x * x));
        if (lane < n) Z[a * n + lane] = x;
        __threadfence_block();
      }
      c0 = e;
    }
  }
  __syncthreads();
  // ---- 5. U = Q D Z into (Vr, Vi): 2 x 4 blocks per thread ----
  {
    const int nbc = (n + 3) / 4, nblk = ((n + 1) / 2) * nbc;
    const bool act = tid < nblk;
    const int a0 = act ? 2 * (tid / nbc) : 0, b0 = act ? 4 * (tid % nbc) : 0;
    double ur[2][4], ui[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) ur[u][v] = ui[u][v] = 0.0;
    if (act) {
      const int ra[2] = {min(a0, n - 1), min(a0 + 1, n - 1)};
      const int cb[4] = {min(b0, n - 1), min(b0 + 1, n - 1), min(b0 + 2, n - 1), min(b0 + 3, n - 1)};
      for (int k = 0; k < n; ++k) {
        const double fr = s_phr[k], fi = s_phi[k];
        double qr[2], qi[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {  // (Q D)[a][k]
          const double xr = Vr[ra[u] * gp + k], xi = Vi[ra[u] * gp + k];
          qr[u] = xr * fr - xi * fi;
          qi[u] = xr * fi + xi * fr;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double z = Z[cb[v] * n + k];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            ur[u][v] = fma(qr[u], z, ur[u][v]);
            ui[u][v] = fma(qi[u], z, ui[u][v]);
          }
        }
      }
    }
    __syncthreads();
    if (act)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (a0 + u < n && b0 + v < n) {
            Vr[(a0 + u) * gp + b0 + v] = ur[u][v];
            Vi[(a0 + u) * gp + b0 + v] = ui[u][v];
          }
    __syncthreads();
  }
}


template <int LB>
size_t csvd_lds_bytes(int l) {
  const size_t L2 = (size_t)l + (l & 1), gp = L2 + 1;
  return (4 * L2 * gp + gp + 2 * (size_t)LB) * 8 + (size_t)LB * 4;
}

template <typename T, int LB>
__global__ __launch_bounds__(kSvdThreads) void k_csvd(double* __restrict__ g2_all, const double* __restrict__ gw_all,
                                                      const SliceDesc* __restrict__ sd, const int2* __restrict__ wk,
                                                      const int2* __restrict__ slices, double tau_host,
                                                      const double* __restrict__ tau_dev,
                                                      const double* __restrict__ mu_dev, Penalty pen,
                                                      T* __restrict__ Kall, double* __restrict__ sigma_out,
                                                      int sigma_ld, int* __restrict__ kept_out,
                                                      int* __restrict__ status) {
  constexpr int NT = kSvdThreads;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double s_scr;
  __shared__ int s_kept;
  const int j = slices ? slices[blockIdx.x].x : (int)blockIdx.x;
  const int tid = threadIdx.x;
  const SliceDesc d = sd[j];
  const int l = slice_width(d, wk, j), kkeep = slice_kept(d, wk, j);
  if (l <= 0) return;  // slice not part of this pass
  const int L2 = l + (l & 1), gp = L2 + 1, ll = l * l;
  const int nt_q = (d.n1 + kGramRows - 1) / kGramRows, nt_b = (d.n2 + kGramRows - 1) / kGramRows;
  const double tau = mu_dev ? 1.0 / (*mu_dev) : (tau_dev ? tau_dev[d.tensor] : tau_host);
  double* Ar = reinterpret_cast<double*>(smem_raw);  // G2, R2^{-1}, eigenvectors V, R2^{-1}
  double* Ai = Ar + (size_t)L2 * gp;
  double* Br = Ai + (size_t)L2 * gp;  // Wt, W, K, K R2^{-H}
  double* Bi = Br + (size_t)L2 * gp;
  double* dR = Bi + (size_t)L2 * gp;
  double* lam = dR + gp;
  double* wv = lam + LB;
  int* perm = reinterpret_cast<int*>(wv + LB);
  double* gq = g2_all + d.g2;  // partials of Q1; the first 2 l^2 doubles park R2^{-1}

  constexpr int NE = (LB * LB + NT - 1) / NT;
  sum_cgram_partials<NE>(Ar, Ai, gp, gq, nt_q, l);
  sum_cgram_partials<NE>(Br, Bi, gp, gw_all + d.g1, nt_b, l);
  if (status && tid < 64) {  // a non-finite entry of the slice reaches a diagonal entry of the sums
    bool bad = false;
    for (int a = tid; a < l; a += 64) bad |= !isfinite(Ar[a * gp + a]) || !isfinite(Br[a * gp + a]);
    const bool any_bad = __ballot(bad) != 0;
    if (tid == 0) status[j] = any_bad ? 1 : 0;
  }
  cchol_deflate<(kMaxComplexWidth * (kMaxComplexWidth + 1) / 2 + NT - 1) / NT>(Ar, Ai, dR, gp, l,
                                                                          8.0 * (double)d.n1 * kEps, &s_scr);
  ctri_inverse_waves(Ar, Ai, dR, gp, l, gq, gq + ll, l);
  __syncthreads();
  for (int idx = tid; idx < ll; idx += NT) {
    Ar[(idx / l) * gp + idx % l] = gq[idx];
    Ai[(idx / l) * gp + idx % l] = gq[ll + idx];
  }
  __syncthreads();
  cmat_product<0, T>(Br, Bi, Ar, Ai, gp, l, nullptr);  // Wt R2^{-1}
  cmat_product<1, T>(Br, Bi, Ar, Ai, gp, l, nullptr);  // W = R2^{-H} Wt R2^{-1}
  // Hermitian part, zero padding row and column, V = I
  for (int idx = tid; idx < L2 * L2; idx += NT) {
    const int a = idx / L2, b = idx % L2;
    if (a < l && b < l) {
      if (a < b) {
        const double mr = 0.5 * (Br[a * gp + b] + Br[b * gp + a]);
        const double mi = 0.5 * (Bi[a * gp + b] - Bi[b * gp + a]);
        Br[a * gp + b] = mr;
        Br[b * gp + a] = mr;
        Bi[a * gp + b] = mi;
        Bi[b * gp + a] = -mi;
      } else if (a == b) {
        Bi[a * gp + a] = 0.0;
      }
    } else {
      Br[a * gp + b] = 0.0;
      Bi[a * gp + b] = 0.0;
    }
    Ar[a * gp + b] = (a == b) ? 1.0 : 0.0;
    Ai[a * gp + b] = 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    double md = 0.0;
    for (int a = tid; a < l; a += 64) md = fmax(md, fabs(Br[a * gp + a]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) md = fmax(md, __shfl_xor(md, off, 64));
    if (tid == 0) s_scr = md;
  }
  __syncthreads();
  const double scale = s_scr > 0.0 ? s_scr : 1.0;  // W <- W / max diag
  const double inv_scale = 1.0 / scale;
  for (int idx = tid; idx < L2 * L2; idx += NT) {
    const int a = idx / L2, b = idx % L2;
    Br[a * gp + b] *= inv_scale;
    Bi[a * gp + b] *= inv_scale;
  }
  __syncthreads();
  // ---- eigenvectors V and eigenvalues of W (tridiagonal route) ----
  // eigenpairs whose singular value the shrinkage zeroes (or past the kept
  // count) carry no weight in K': their refinement within clusters is skipped
  const double t0 = prox_zero_threshold(pen, tau);
  heev_tridiag(Br, Bi, Ar, Ai, gp, l, lam, 0.99 * t0 * t0 * inv_scale, kkeep);
  for (int a = tid; a < l; a += NT) Br[a * gp + a] = lam[a];
  __syncthreads();

  // ---- order, shrink, K = U diag(w) U^H, K' = R2^{-1} K R2^{-H} ------------
  for (int a = tid; a < l; a += NT) lam[a] = Br[a * gp + a] * scale;
  __syncthreads();
  for (int a = tid; a < l; a += NT) {
    const double la = lam[a];
    int rank = 0;
    for (int b = 0; b < l; ++b) {
      const double lb = lam[b];
      rank += (lb > la) || (lb == la && b < a);
    }
    perm[rank] = a;
  }
  if (tid == 0) s_kept = 0;
  __syncthreads();
  for (int i = tid; i < l; i += NT) {
    const double lv = lam[perm[i]];
    const double sv = lv > 0.0 ? sqrt(lv) : 0.0;
    double w = 0.0;
    if (i < kkeep && sv > 0.0) {
      const double sh = prox_pos(pen, sv, tau);
      w = sh / sv;
      if (sh > 0.0) atomicAdd(&s_kept, 1);
    }
    wv[i] = w;
    if (sigma_out) sigma_out[(int64_t)j * sigma_ld + i] = sv;
  }
  if (sigma_out)
    for (int i = l + tid; i < sigma_ld; i += NT) sigma_out[(int64_t)j * sigma_ld + i] = 0.0;
  __syncthreads();
  // K[a][b] = sum_i V[a][e_i] w_i conj(V[b][e_i]) into the B planes
  for (int idx = tid; idx < ll; idx += NT) {
    const int a = idx / l, b = idx % l;
    double kr = 0.0, ki = 0.0;
    for (int i = 0; i < kkeep; ++i) {
      const int e = perm[i];
      const double w = wv[i];
      if (w == 0.0) continue;
      const double xr = Ar[a * gp + e], xi = Ai[a * gp + e];
      const double yr = Ar[b * gp + e], yi = Ai[b * gp + e];
      kr = fma(w, fma(xr, yr, xi * yi), kr);
      ki = fma(w, fma(xi, yr, -(xr * yi)), ki);
    }
    Br[a * gp + b] = kr;
    Bi[a * gp + b] = ki;
  }
  __syncthreads();
  for (int idx = tid; idx < ll; idx += NT) {
    Ar[(idx / l) * gp + idx % l] = gq[idx];
    Ai[(idx / l) * gp + idx % l] = gq[ll + idx];
  }
  __syncthreads();
  cmat_product<2, T>(Br, Bi, Ar, Ai, gp, l, nullptr);    // K R2^{-H}
  cmat_product<3, T>(Br, Bi, Ar, Ai, gp, l, Kall + d.kq);  // K' = R2^{-1} K R2^{-H}
  if (kept_out && tid == 0) kept_out[j] = s_kept;
}

// ---------------------------------------------------------------------------
// Vector-unit complex products (FP64 plans).  Work items are (slice, first
// complex row of a 64-row tile); 256 threads, thread (r, g) computes complex
// row r of the tile for the columns g, g + 4, ...
// ---------------------------------------------------------------------------
constexpr int CKC = 32;

template <typename T, int LB>
constexpr size_t cgemm_lds_bytes() {
  constexpr size_t main = sizeof(T) * 2 * (CKC * 65 + CKC * LB);
  constexpr size_t epi = sizeof(double) * 128 * (LB + 1);
  return main > epi ? main : epi;
}

// Gram partial of the tile: thread (r, g) holds row r's real and imaginary
// values for its columns.
template <typename T, int LB>
__device__ inline void cgram_epilogue(unsigned char* smem, const double* accr, const double* acci, int r, int g,
                                      bool valid, int l, double* __restrict__ out) {
  constexpr int CPT = LB / 4, SP = LB + 1;
  double* S = reinterpret_cast<double*>(smem);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int c = g + 4 * i;
    if (c < l) {
      S[r * SP + c] = valid ? (double)(T)accr[i] : 0.0;
      S[(64 + r) * SP + c] = valid ? (double)(T)acci[i] : 0.0;
    }
  }
  __syncthreads();
  tile_cgram_mfma(S, SP, 1, l, out);
}

// TRANS = false: Y = A W (W the stacked Z, or with wreal the real Omega);
// TRANS = true:  Z = A^H Q.
template <typename T, int LB, bool TRANS>
__global__ __launch_bounds__(256) void k_cgemm(const T* __restrict__ Aall, const T* __restrict__ Wall,
                                               T* __restrict__ Yall, const SliceDesc* __restrict__ sd,
                                               const int2* __restrict__ wk, const int2* __restrict__ items,
                                               double* __restrict__ gpart, int wreal) {
  constexpr int CPT = LB / 4;
  extern __shared__ __align__(16) unsigned char smem[];
  T* Asr = reinterpret_cast<T*>(smem);  // [CKC][65]
  T* Asi = Asr + CKC * 65;
  T* Wsr = Asi + CKC * 65;  // [CKC][LB]
  T* Wsi = Wsr + CKC * LB;
  const int2 item = items[blockIdx.x];
  const int s = item.x, r0 = item.y;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int n1 = d.n1, n2 = d.n2, lda = 2 * n1;
  const int mo = TRANS ? n2 : n1, K = TRANS ? n1 : n2;
  const int ldw = TRANS ? 2 * n1 : (wreal ? n2 : 2 * n2), ldy = 2 * mo;
  const T* Aj = Aall + d.a;
  const T* Wj = Wall + (TRANS ? d.y : d.z);
  T* Yj = Yall + (TRANS ? d.z : d.y);
  const int r = threadIdx.x % 64, g = threadIdx.x / 64;
  double accr[CPT], acci[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) accr[i] = acci[i] = 0.0;
  for (int k0 = 0; k0 < K; k0 += CKC) {
    for (int idx = threadIdx.x; idx < CKC * 64; idx += 256) {
      int kk, rr;
      if (TRANS) {
        kk = idx % CKC;
        rr = idx / CKC;
      } else {
        kk = idx / 64;
        rr = idx % 64;
      }
      const int gk = k0 + kk, gr = r0 + rr;
      T vr = T(0), vi = T(0);
      if (gk < K && gr < mo) {
        const int64_t o = TRANS ? (gk + (int64_t)gr * lda) : (gr + (int64_t)gk * lda);  // A[gr][gk] or A[gk][gr]
        vr = Aj[o];
        vi = Aj[o + n1];
      }
      Asr[kk * 65 + rr] = vr;
      Asi[kk * 65 + rr] = vi;
    }
    for (int idx = threadIdx.x; idx < CKC * LB; idx += 256) {
      const int c = idx / CKC, kk = idx % CKC;
      const int gk = k0 + kk;
      const bool ok = c < l && gk < K;
      const int64_t o = gk + (int64_t)c * ldw;
      Wsr[kk * LB + c] = ok ? Wj[o] : T(0);
      Wsi[kk * LB + c] = (ok && !(wreal && !TRANS)) ? Wj[o + (TRANS ? n1 : n2)] : T(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < CKC; ++kk) {
      const double ar = (double)Asr[kk * 65 + r], ai = (double)Asi[kk * 65 + r];
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        const double wr = (double)Wsr[kk * LB + g + 4 * i], wi = (double)Wsi[kk * LB + g + 4 * i];
        if (TRANS) {  // conj(a) w
          accr[i] = fma(ar, wr, fma(ai, wi, accr[i]));
          acci[i] = fma(ar, wi, fma(-ai, wr, acci[i]));
        } else {
          accr[i] = fma(ar, wr, fma(-ai, wi, accr[i]));
          acci[i] = fma(ar, wi, fma(ai, wr, acci[i]));
        }
      }
    }
    __syncthreads();
  }
  const int gr = r0 + r;
  const bool valid = gr < mo;
  if (valid) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int c = g + 4 * i;
      if (c < l) {
        Yj[gr + (int64_t)c * ldy] = (T)accr[i];
        Yj[mo + gr + (int64_t)c * ldy] = (T)acci[i];
      }
    }
  }
  if (gpart)
    cgram_epilogue<T, LB>(smem, accr, acci, r, g, valid, l, gpart + d.g1 + (int64_t)(r0 / kGramRows) * 2 * l * l);
}

// Reconstruction on the vector units:
//   QK (MODE 0): (Q1 K') rows r0.. of the slice, all l columns
//   C  (MODE 1): C = (Q1 K') Bt^H, 64 x 64 tile (slice, tile index, row tiles fastest)
// Thread (r, g): complex row r of the tile, columns g, g + 4, ... (MODE 0) or
// g * 16 .. g * 16 + 15 (MODE 1).
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_crecon(const T* __restrict__ Xall, const T* __restrict__ Wall,
                                                T* __restrict__ Call, const SliceDesc* __restrict__ sd,
                                                const int2* __restrict__ wk, const int2* __restrict__ items) {
  constexpr int NC = 16;
  __shared__ double Wr_s[64], Wi_s[64];
  const int2 item = items[blockIdx.x];
  const int s = item.x;
  const SliceDesc d = sd[s];
  const int l = slice_width(d, wk, s);
  if (l <= 0) return;  // slice not part of this pass
  const int n1 = d.n1, n2 = d.n2, ldx = 2 * n1;
  const int nrt = (n1 + 63) / 64;
  const int row0 = MODE == 0 ? item.y : (item.y % nrt) * 64;
  const int col0 = MODE == 0 ? 0 : (item.y / nrt) * 64;
  const int ncols = MODE == 0 ? l : n2;
  const T* X = Xall + d.y;                       // Q1 (MODE 0) or Q1 K' (MODE 1), stacked 2 n1 x l
  const T* W = Wall + (MODE == 0 ? d.kq : d.z);  // K' (2 l x l) or Bt (2 n2 x l)
  T* C = Call + (MODE == 0 ? d.y : d.a);
  const int r = threadIdx.x % 64, g = threadIdx.x / 64;
  const int gr = row0 + r;
  const bool valid = gr < n1;
  const int lr = valid ? gr : n1 - 1;
  // 64 columns of the result per pass, 16 per thread group
  for (int cb = col0; cb < (MODE == 0 ? ncols : min(ncols, col0 + 64)); cb += 64) {
    double accr[NC], acci[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) accr[i] = acci[i] = 0.0;
    for (int a = 0; a < l; ++a) {
      __syncthreads();
      // column block of the right operand for this a: Wc[c] = K'[a][c] (MODE 0) or conj(Bt[c][a]) (MODE 1)
      for (int idx = threadIdx.x; idx < 64; idx += 256) {
        const int c = cb + idx;
        double wr = 0.0, wi = 0.0;
        if (c < ncols) {
          if (MODE == 0) {
            wr = (double)W[a + (int64_t)c * 2 * l];
            wi = (double)W[l + a + (int64_t)c * 2 * l];
          } else {
            wr = (double)W[c + (int64_t)a * 2 * n2];
            wi = -(double)W[n2 + c + (int64_t)a * 2 * n2];
          }
        }
        Wr_s[idx] = wr;
        Wi_s[idx] = wi;
      }
      __syncthreads();
      const double xr = (double)X[lr + (int64_t)a * ldx], xi = (double)X[n1 + lr + (int64_t)a * ldx];
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        const int cl = g * NC + i;
        const double wr = Wr_s[cl], wi = Wi_s[cl];
        accr[i] = fma(xr, wr, fma(-xi, wi, accr[i]));
        acci[i] = fma(xr, wi, fma(xi, wr, acci[i]));
      }
    }
    if (valid) {
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        const int c = cb + g * NC + i;
        if (c < ncols) {
          C[gr + (int64_t)c * ldx] = (T)accr[i];
          C[n1 + gr + (int64_t)c * ldx] = (T)acci[i];
        }
      }
    }
  }
}

}  // namespace

template <typename T>
int launch_corth(T* Y, uint16_t* Yh, int which, const SliceDesc* sd, const int2* wk, const int2* items, int nitems,
                 const int2* tiles, int ntiles, int lmax, int nslices, double* gin, double* gout, hipStream_t s) {
  if (lmax > kMaxComplexWidth) HT_FAIL(HT_ERR_UNSUPPORTED, "complex sketch width above 64");
  if (nitems == 0 || nslices == 0) return HT_OK;
  int rc = ensure_dynamic_lds((const void*)k_corth_factor, cfactor_lds_bytes(kMaxComplexWidth));
  if (rc) return rc;
  hipLaunchKernelGGL(k_corth_factor, dim3((unsigned)nslices), dim3(kFactorThreads), cfactor_lds_bytes(lmax), s,
                     which, sd, wk, gin);
  HT_CHECK_LAUNCH();
  if (std::is_same<T, float>::value && tiles != nullptr && ntiles > 0) {
    if ((rc = ensure_dynamic_lds((const void*)k_corth_apply_tiles, kApplyLds))) return rc;
    int per_cu = 0, dev = 0, ncu = 0;
    HT_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_corth_apply_tiles, 256, kApplyLds));
    HT_CHECK_HIP(hipGetDevice(&dev));
    HT_CHECK_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int grid = std::max(1, std::min(ntiles, std::max(per_cu, 1) * ncu));
    hipLaunchKernelGGL(k_corth_apply_tiles, dim3((unsigned)grid), dim3(256), kApplyLds, s, reinterpret_cast<float*>(Y),
                       Yh, which, sd, wk, tiles, ntiles, gin);
    HT_CHECK_LAUNCH();
    if (gout == nullptr) return HT_OK;
    // the final basis: Gram partials of the stored tiles
    auto gram = [&](auto kern, size_t lds) -> int {
      int r = ensure_dynamic_lds((const void*)kern, lds);
      if (r) return r;
      hipLaunchKernelGGL(kern, dim3((unsigned)nitems), dim3(256), lds, s, Y, which, sd, wk, items, gout);
      HT_CHECK_LAUNCH();
      return HT_OK;
    };
    if (lmax <= 32) return gram(k_cgram_tiles<T, 32>, 128 * 33 * sizeof(T));
    return gram(k_cgram_tiles<T, 64>, 128 * 65 * sizeof(T));
  }
  auto apply = [&](auto kern, size_t lds) -> int {
    int r = ensure_dynamic_lds((const void*)kern, lds);
    if (r) return r;
    hipLaunchKernelGGL(kern, dim3((unsigned)nitems), dim3(256), lds, s, Y, Yh, which, sd, wk, items, gin, gout);
    HT_CHECK_LAUNCH();
    return HT_OK;
  };
  if (lmax <= 32) return apply(k_corth_apply<T, 32>, capply_lds_bytes<T, 32>());
  return apply(k_corth_apply<T, 64>, capply_lds_bytes<T, 64>());
}

template <typename T>
int launch_csvd(double* g2, const double* gw, const SliceDesc* sd, const int2* wk, const int2* slices, int nslices,
                int lmax, int sigma_ld, double tau, const double* tau_dev, const double* mu_dev, Penalty pen, T* K,
                double* sigma_out, int* kept_out, int* status, hipStream_t s) {
  if (lmax > kMaxComplexWidth) HT_FAIL(HT_ERR_UNSUPPORTED, "complex sketch width above 64");
  if (nslices == 0) return HT_OK;
  auto launch = [&](auto kern, size_t lds_max, size_t lds) -> int {
    int rc = ensure_dynamic_lds((const void*)kern, lds_max);
    if (rc) return rc;
    hipLaunchKernelGGL(kern, dim3((unsigned)nslices), dim3(kSvdThreads), lds, s, g2, gw, sd, wk, slices, tau,
                       tau_dev, mu_dev, pen, K, sigma_out, sigma_ld, kept_out, status);
    HT_CHECK_LAUNCH();
    return HT_OK;
  };
  if (lmax <= 32) return launch(k_csvd<T, 32>, csvd_lds_bytes<32>(32), csvd_lds_bytes<32>(lmax));
  return launch(k_csvd<T, 64>, csvd_lds_bytes<64>(64), csvd_lds_bytes<64>(lmax));
}

template <typename T>
int launch_cgemm(const T* A, const T* W, T* Y, int trans, int wreal, const SliceDesc* sd, const int2* wk,
                 const int2* items, int nitems, int lmax, double* gpart, hipStream_t s) {
  if (lmax > kMaxComplexWidth) HT_FAIL(HT_ERR_UNSUPPORTED, "complex sketch width above 64");
  if (nitems == 0) return HT_OK;
  auto launch = [&](auto kern, size_t lds) -> int {
    int rc = ensure_dynamic_lds((const void*)kern, lds);
    if (rc) return rc;
    hipLaunchKernelGGL(kern, dim3((unsigned)nitems), dim3(256), lds, s, A, W, Y, sd, wk, items, gpart, wreal);
    HT_CHECK_LAUNCH();
    return HT_OK;
  };
  if (trans) {
    if (lmax <= 32) return launch(k_cgemm<T, 32, true>, cgemm_lds_bytes<T, 32>());
    return launch(k_cgemm<T, 64, true>, cgemm_lds_bytes<T, 64>());
  }
  if (lmax <= 32) return launch(k_cgemm<T, 32, false>, cgemm_lds_bytes<T, 32>());
  return launch(k_cgemm<T, 64, false>, cgemm_lds_bytes<T, 64>());
}

template <typename T>
int launch_crecon(const T* X, const T* W, T* C, int mode, const SliceDesc* sd, const int2* wk, const int2* items,
                  int nitems, hipStream_t s) {
  if (nitems == 0) return HT_OK;
  if (mode == 0)
    hipLaunchKernelGGL((k_crecon<T, 0>), dim3((unsigned)nitems), dim3(256), 0, s, X, W, C, sd, wk, items);
  else
    hipLaunchKernelGGL((k_crecon<T, 1>), dim3((unsigned)nitems), dim3(256), 0, s, X, W, C, sd, wk, items);
  HT_CHECK_LAUNCH();
  return HT_OK;
}

template int launch_corth<float>(float*, uint16_t*, int, const SliceDesc*, const int2*, const int2*, int, const int2*,
                                 int, int, int, double*, double*, hipStream_t);
template int launch_corth<double>(double*, uint16_t*, int, const SliceDesc*, const int2*, const int2*, int,
                                  const int2*, int, int, int, double*, double*, hipStream_t);
template int launch_csvd<float>(double*, const double*, const SliceDesc*, const int2*, const int2*, int, int, int,
                                double, const double*, const double*, Penalty, float*, double*, int*, int*,
                                hipStream_t);
template int launch_csvd<double>(double*, const double*, const SliceDesc*, const int2*, const int2*, int, int, int,
                                 double, const double*, const double*, Penalty, double*, double*, int*, int*,
                                 hipStream_t);
template int launch_cgemm<float>(const float*, const float*, float*, int, int, const SliceDesc*, const int2*,
                                 const int2*, int, int, double*, hipStream_t);
template int launch_cgemm<double>(const double*, const double*, double*, int, int, const SliceDesc*, const int2*,
                                  const int2*, int, int, double*, hipStream_t);
template int launch_crecon<float>(const float*, const float*, float*, int, const SliceDesc*, const int2*, const int2*,
                                  int, hipStream_t);
template int launch_crecon<double>(const double*, const double*, double*, int, const SliceDesc*, const int2*,
                                   const int2*, int, hipStream_t);

}  // namespace ht
