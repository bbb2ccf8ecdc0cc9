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
// deflation, the Hermitian Jacobi eigensolver with the shrinkage) and the
// vector-unit products that FP64 plans use; the FP32 and BF16 products run on
// the matrix cores (mfma.hip, mfma_bf16.hip).
//
// Hermitian Jacobi.  For a pair (p, q) with W[p][q] = b = |b| e, the rotation
// J = [[c, s e], [-s conj(e), c]] makes J^H W J diagonal on (p, q) when (c, s)
// is the real rotation of [[W[p][p], |b|], [|b|, W[q][q]]]: the phase e turns
// the block into that real symmetric one.  Steps apply l/2 disjoint rotations
// (round-robin ordering) in place: one barrier after the rotations of the step
// are computed from W, one after they are applied.
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

// Complex Cholesky with deflation, in place: on entry the upper triangle of
// the Hermitian G = Gr + i Gi (pitch gp); G = R^H R with R upper triangular
// and a real positive diagonal.  On return dR[j] = R[j][j] (0 for a skipped
// column, whose row of R is zero) and R[j][b] for b > j sits in the strict
// lower triangle at (b, j).  A column is skipped when its Schur-complement
// pivot is at most delta_rel * max_a G[a][a].  One barrier per column: the
// trailing update reads only the unscaled pivot row, which the column never
// writes, and its entries (a, b), j < a <= b, are spread over every thread of
// the workgroup (entry e of the column-packed triangle is (a, b) with
// e = b'(b' + 1)/2 + a', a' = a - j - 1, b' = b - j - 1).
__device__ inline void cchol_deflate(double* Gr, double* Gi, double* dR, int gp, int l, double delta_rel,
                                     double* s_scr) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) {
    double md = 0.0;
    for (int a = 0; a < l; ++a) md = fmax(md, Gr[a * gp + a]);
    *s_scr = md;
  }
  __syncthreads();
  const double maxdiag = *s_scr;
  const double delta = delta_rel * maxdiag;
  constexpr int UE = 4;  // entries per thread per batch of loads
  for (int j = 0; j < l; ++j) {
    const double d = Gr[j * gp + j];
    const bool keep = d > delta && maxdiag > 0.0;
    const double inv_r = keep ? fast_rsqrt(d) : 0.0;
    const double inv_d = inv_r * inv_r;
    const int mrem = l - j - 1, ntri = mrem * (mrem + 1) / 2;
    const double* pr = Gr + j * gp + j + 1;  // pivot row past the diagonal
    const double* pi = Gi + j * gp + j + 1;
    for (int e0 = tid; e0 < ntri; e0 += UE * nt) {
      int ia[UE], ib[UE];
      double jar[UE], jai[UE], jbr[UE], jbi[UE], xr[UE], xi[UE];
#pragma unroll
      for (int u = 0; u < UE; ++u) {
        const int e = min(e0 + u * nt, ntri - 1);
        int bb = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
        while ((bb + 1) * (bb + 2) / 2 <= e) ++bb;
        while (bb * (bb + 1) / 2 > e) --bb;
        const int aa = e - bb * (bb + 1) / 2;
        ia[u] = aa;
        ib[u] = bb;
        jar[u] = pr[aa];
        jai[u] = pi[aa];
        jbr[u] = pr[bb];
        jbi[u] = pi[bb];
        xr[u] = Gr[(j + 1 + aa) * gp + j + 1 + bb];
        xi[u] = Gi[(j + 1 + aa) * gp + j + 1 + bb];
      }
#pragma unroll
      for (int u = 0; u < UE; ++u) {
        if (e0 + u * nt < ntri) {  // G[a][b] -= conj(G[j][a]) G[j][b] / d
          const double fr = jbr[u] * inv_d, fi = jbi[u] * inv_d;
          const int o = (j + 1 + ia[u]) * gp + j + 1 + ib[u];
          Gr[o] = xr[u] - fma(jar[u], fr, jai[u] * fi);
          Gi[o] = xi[u] - fma(jar[u], fi, -(jai[u] * fr));
        }
      }
    }
    for (int b = j + 1 + tid; b < l; b += nt) {
      Gr[b * gp + j] = Gr[j * gp + b] * inv_r;
      Gi[b * gp + j] = Gi[j * gp + b] * inv_r;
    }
    if (tid == 0) dR[j] = keep ? d * inv_r : 0.0;
    __syncthreads();
  }
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
  cchol_deflate(Gr, Gi, dR, gp, l, 8.0 * (double)m * kEps, &s_scr);
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
__global__ __launch_bounds__(256) void k_corth_apply(T* __restrict__ Yall, int which, const SliceDesc* __restrict__ sd,
                                                     const int2* __restrict__ wk, const int2* __restrict__ items,
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
    if (row < rows) Y[(part ? m : 0) + r0 + row + (int64_t)c * ld] = S[(part * 64 + row) * SP + c];
  }
  if (gout_all) tile_cgram_mfma(S, SP, 1, l, gout_all + d.g2 + (int64_t)(r0 / kGramRows) * 2 * ll);
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
// B = Q^H A, Q = Q1 R2^{-1}.  W = U diag(s^2) U^H by Hermitian Jacobi; with
// the k = min(r, l) largest s shrunk,
//   K' = R2^{-1} U diag(w) U^H R2^{-H},  w_i = prox(s_i) / s_i,
// so that the reconstruction is C = Q1 K' Bt^H.
// ---------------------------------------------------------------------------
struct CRot {
  double c, sr, si;  // rotation [[c, s], [-conj(s), c]] of pair (p, q)
  int p, q;
};

__device__ __forceinline__ void rr_pair_c(int step, int t, int m, int& p, int& q) {
  int a, b;
  if (t == 0) {
    a = m;
    b = step;
  } else {
    a = step + t;
    a = a >= m ? a - m : a;
    b = step - t + m;
    b = b >= m ? b - m : b;
  }
  p = min(a, b);
  q = max(a, b);
}

// Real symmetric Schur rotation of [[app, apq], [apq, aqq]] (apq >= 0): the
// identity when apq is at most tol or tol sqrt(app aqq).
__device__ __forceinline__ bool schur_c(double app, double aqq, double apq, double tol, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (apq > tol && apq * apq > tol * tol * fabs(app * aqq)) {
    const double dd = aqq - app;
    const double h = sqrt(dd * dd + 4.0 * apq * apq);
    const double t = 2.0 * apq * (dd >= 0.0 ? 1.0 : -1.0) * fast_rcp(fabs(dd) + h);
    c = fast_rsqrt(1.0 + t * t);
    s = t * c;
    return true;
  }
  return false;
}

constexpr int kSvdThreads = 512;

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
  __shared__ int s_kept, s_cnt[3], s_open;
  __shared__ CRot s_rot[2][LB / 2];
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
  cchol_deflate(Ar, Ai, dR, gp, l, 8.0 * (double)d.n1 * kEps, &s_scr);
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
  if (tid < 3) s_cnt[tid] = 0;
  __syncthreads();
  // A pair rotates only when |W[p][q]| is above tol and tol sqrt(W[p][p] W[q][q]):
  // FP64 output 1e-15, FP32 output 1e-10 (as for real slices).
  const double tol = std::is_same<T, double>::value ? 1e-15 : 1e-10;

  // ---- parallel cyclic Jacobi, in place on W (B planes) and V (A planes) ----
  const int half = L2 / 2, m = L2 - 1;
  const int nblk = half * half, nvit = half * l;
  constexpr int NBI = ((LB / 2) * (LB / 2) + NT - 1) / NT;
  constexpr int NVI = ((LB / 2) * LB + NT - 1) / NT;
  int step = 0, still = 0;
  for (int g = 0; g < 30 * m; ++g) {
    CRot* rot = s_rot[g & 1];
    if (tid < half) {
      int p, q;
      rr_pair_c(step, tid, m, p, q);
      const double br = Br[p * gp + q], bi = Bi[p * gp + q];
      const double ab = sqrt(br * br + bi * bi);
      double c, sn;
      CRot r{1.0, 0.0, 0.0, p, q};
      if (schur_c(Br[p * gp + p], Br[q * gp + q], ab, tol, c, sn)) {
        const double inv_ab = 1.0 / ab;
        r.c = c;
        r.sr = sn * br * inv_ab;
        r.si = sn * bi * inv_ab;
        s_cnt[g % 3] = 1;
      }
      rot[tid] = r;
    }
    if (tid == 0) {
      s_cnt[(g + 2) % 3] = 0;
      s_open = 0;
    }
    __syncthreads();
    if (s_cnt[g % 3] != 0) {
      CRot ra[NBI], rb[NBI], rv[NVI];
      int vx[NVI];
      bool bok[NBI], vok[NVI];
#pragma unroll
      for (int u = 0; u < NBI; ++u) {
        const int item = tid + u * NT;
        bok[u] = item < nblk;
        const int it2 = bok[u] ? item : 0;
        ra[u] = rot[it2 / half];
        rb[u] = rot[it2 % half];
      }
#pragma unroll
      for (int u = 0; u < NVI; ++u) {
        const int item = tid + u * NT;
        vok[u] = item < nvit;
        const int it2 = vok[u] ? item : 0;
        rv[u] = rot[it2 / l];
        vx[u] = it2 % l;
      }
      double wr[NBI][4], wi[NBI][4], vr[NVI][2], vi[NVI][2];
#pragma unroll
      for (int u = 0; u < NBI; ++u) {
        const int o[4] = {ra[u].p * gp + rb[u].p, ra[u].p * gp + rb[u].q, ra[u].q * gp + rb[u].p,
                          ra[u].q * gp + rb[u].q};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          wr[u][e] = Br[o[e]];
          wi[u][e] = Bi[o[e]];
        }
      }
#pragma unroll
      for (int u = 0; u < NVI; ++u) {
        vr[u][0] = Ar[vx[u] * gp + rv[u].p];
        vi[u][0] = Ai[vx[u] * gp + rv[u].p];
        vr[u][1] = Ar[vx[u] * gp + rv[u].q];
        vi[u][1] = Ai[vx[u] * gp + rv[u].q];
      }
#pragma unroll
      for (int u = 0; u < NBI; ++u) {
        // rows: J_s^H = [[c, -s], [conj(s), c]];  columns: J_t = [[c, s], [-conj(s), c]]
        const double cs = ra[u].c, ssr = ra[u].sr, ssi = ra[u].si;
        const double ct = rb[u].c, str = rb[u].sr, sti = rb[u].si;
        double rr[4], ri[4];
        // r0x = c w0x - s w1x ; r1x = conj(s) w0x + c w1x   (x = column 0, 1)
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const double w0r = wr[u][x], w0i = wi[u][x], w1r = wr[u][2 + x], w1i = wi[u][2 + x];
          rr[x] = cs * w0r - (ssr * w1r - ssi * w1i);
          ri[x] = cs * w0i - (ssr * w1i + ssi * w1r);
          rr[2 + x] = (ssr * w0r + ssi * w0i) + cs * w1r;
          ri[2 + x] = (ssr * w0i - ssi * w0r) + cs * w1i;
        }
        double nr[4], ni[4];
        // ny0 = c ry0 - conj(s) ry1 ; ny1 = s ry0 + c ry1   (y = row 0, 1)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const double a0r = rr[2 * y], a0i = ri[2 * y], a1r = rr[2 * y + 1], a1i = ri[2 * y + 1];
          nr[2 * y] = ct * a0r - (str * a1r + sti * a1i);
          ni[2 * y] = ct * a0i - (str * a1i - sti * a1r);
          nr[2 * y + 1] = (str * a0r - sti * a0i) + ct * a1r;
          ni[2 * y + 1] = (str * a0i + sti * a0r) + ct * a1i;
        }
        if (bok[u]) {
          const bool diag = ra[u].p == rb[u].p;
          if (diag) {  // the diagonal stays real; the annihilated pair is zero
            ni[0] = 0.0;
            ni[3] = 0.0;
            if (ra[u].sr != 0.0 || ra[u].si != 0.0) nr[1] = ni[1] = nr[2] = ni[2] = 0.0;
          }
          const int o[4] = {ra[u].p * gp + rb[u].p, ra[u].p * gp + rb[u].q, ra[u].q * gp + rb[u].p,
                            ra[u].q * gp + rb[u].q};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            Br[o[e]] = nr[e];
            Bi[o[e]] = ni[e];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < NVI; ++u) {
        // V <- V J: col p = c Vp - conj(s) Vq ; col q = s Vp + c Vq
        const double c = rv[u].c, sr = rv[u].sr, si = rv[u].si;
        const double pr = vr[u][0], pi = vi[u][0], qr = vr[u][1], qi = vi[u][1];
        const double npr = c * pr - (sr * qr + si * qi), npi = c * pi - (sr * qi - si * qr);
        const double nqr = (sr * pr - si * pi) + c * qr, nqi = (sr * pi + si * pr) + c * qi;
        if (vok[u]) {
          Ar[vx[u] * gp + rv[u].p] = npr;
          Ai[vx[u] * gp + rv[u].p] = npi;
          Ar[vx[u] * gp + rv[u].q] = nqr;
          Ai[vx[u] * gp + rv[u].q] = nqi;
        }
      }
      __syncthreads();
      still = 0;
    } else if (++still >= m) {
      break;
    } else if (still == 1) {
      // first quiet step: W changes from here on only if some pair passes the
      // test, so testing every pair now decides the rest of the check
      for (int idx = tid; idx < ll; idx += NT) {
        const int p = idx / l, q = idx % l;
        if (p < q) {
          const double br = Br[p * gp + q], bi = Bi[p * gp + q];
          const double ab = sqrt(br * br + bi * bi);
          if (ab > tol && ab * ab > tol * tol * fabs(Br[p * gp + p] * Br[q * gp + q])) s_open = 1;
        }
      }
      __syncthreads();
      const bool open = s_open != 0;
      __syncthreads();
      if (!open) break;
    }
    step = (step + 1 == m) ? 0 : step + 1;
  }
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
int launch_corth(T* Y, int which, const SliceDesc* sd, const int2* wk, const int2* items, int nitems, int lmax,
                 int nslices, double* gin, double* gout, hipStream_t s) {
  if (lmax > kMaxComplexWidth) HT_FAIL(HT_ERR_UNSUPPORTED, "complex sketch width above 64");
  if (nitems == 0 || nslices == 0) return HT_OK;
  int rc = ensure_dynamic_lds((const void*)k_corth_factor, cfactor_lds_bytes(kMaxComplexWidth));
  if (rc) return rc;
  hipLaunchKernelGGL(k_corth_factor, dim3((unsigned)nslices), dim3(kFactorThreads), cfactor_lds_bytes(lmax), s,
                     which, sd, wk, gin);
  HT_CHECK_LAUNCH();
  auto apply = [&](auto kern, size_t lds) -> int {
    int r = ensure_dynamic_lds((const void*)kern, lds);
    if (r) return r;
    hipLaunchKernelGGL(kern, dim3((unsigned)nitems), dim3(256), lds, s, Y, which, sd, wk, items, gin, gout);
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

template int launch_corth<float>(float*, int, const SliceDesc*, const int2*, const int2*, int, int, int, double*,
                                 double*, hipStream_t);
template int launch_corth<double>(double*, int, const SliceDesc*, const int2*, const int2*, int, int, int, double*,
                                  double*, hipStream_t);
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
