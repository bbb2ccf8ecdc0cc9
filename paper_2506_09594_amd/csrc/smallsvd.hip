// Small projected SVD and shrinkage, one workgroup per slice, FP64.
//
// One workgroup per slice of the slice table.  Inputs are Gram partials
// written by earlier kernels: those of the basis Q1 (the last CholeskyQR pass
// of the sketch) and those of Bt = A_j^T Q1.  The
// second CholeskyQR step is applied here in the l x l space: with
// R2 = chol(Q1^T Q1) the orthonormal basis is Q = Q1 R2^{-1}, so
//   B = Q^T A_j = R2^{-T} Bt^T,   W = B B^T = R2^{-T} (Bt^T Bt) R2^{-1}.
// W = U diag(s^2) U^T is diagonalized by the parallel cyclic Jacobi method
// (round-robin pair ordering, l/2 disjoint rotations per step).  With the k =
// min(r, l) largest s shrunk by the proximity operator, the reconstruction
// Q U[:, :k] diag(prox(s)) V_B[:, :k]^T equals Q1 K' Bt^T with
//   K' = R2^{-1} U diag(w) U^T R2^{-T},  w_i = prox(s_i)/s_i (i < k), 0 otherwise,
// because V_B[:, i]^T = U[:, i]^T B / s_i.  The kernel writes K' (l x l).
//
// One Jacobi step applies all l/2 disjoint rotations at once: for pairs s and
// t the 2 x 2 block of W on rows of s and columns of t becomes J_s^T W[s, t] J_t,
// produced from old values only into a second buffer.  The rotations of a step
// are computed during the step before it by a wavefront of their own: the lane
// that owns pair u of the next step forms the three entries of the updated W
// that its rotation needs (with the same 2 x 2 block routine as the update, so
// they equal the stored values bit for bit) and publishes (c, s, p, q) together
// with the pair of every index.  A step is therefore one barrier: the other
// wavefronts apply the published rotations while the next ones are computed.
// For odd l the matrices carry a zero row and column for the padding player of
// the round-robin schedule, whose rotations are the identity, so no item
// branches on it.  W is scaled to unit maximum diagonal first, so the rotation
// formulas cannot overflow.
#include <type_traits>

#include "chol.hpp"

namespace ht {

namespace {

constexpr int LMAX = 80;

size_t svd_lds_bytes(int l) {
  const size_t L2 = (size_t)l + (l & 1);  // with the padding player
  const size_t gp = L2 + 1;
  return (3 * L2 * gp + gp + 3 * LMAX) * 8 + LMAX * 4;
}

// Threads per workgroup: the Jacobi step has (l/2)^2 block items and l^2/2
// rotation items of V.
template <int LB>
constexpr int svd_threads() { return LB <= 32 ? 256 : 512; }

// Symmetric Schur rotation (c, s) that annihilates W[p][q] (Golub-Van Loan,
// written as t = 2 apq sgn(d) / (|d| + sqrt(d^2 + 4 apq^2)), d = aqq - app);
// identity when |apq| is at most tol, or at most tol * sqrt(|app aqq|).  Entries
// are at most 1 in magnitude (W is normalized), so nothing overflows.
__device__ __forceinline__ void schur2(double app, double aqq, double apq, double tol, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (fabs(apq) > tol && apq * apq > tol * tol * fabs(app * aqq)) {
    const double d = aqq - app;
    const double h = sqrt(d * d + 4.0 * apq * apq);
    const double t = 2.0 * apq * (d >= 0.0 ? 1.0 : -1.0) * fast_rcp(fabs(d) + h);
    c = fast_rsqrt(1.0 + t * t);
    s = t * c;
  }
}

// Pair t of step `step` with the padding player kept as an index (L2 - 1 for
// odd l): m = L2 - 1, step, t < m.
__device__ __forceinline__ void rr_pair_pad(int step, int t, int m, int& p, int& q) {
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

// Pair index of player x (<= m) in step `step`; the inverse of rr_pair_pad.
__device__ __forceinline__ int rr_locate(int step, int x, int m, int half) {
  if (x == m || x == step) return 0;
  int d = x - step;
  if (d < 0) d += m;
  return d < half ? d : m - d;
}

// Rotation of one pair of a step, as published for the next one; po, qo are
// the row offsets p gp, q gp.
struct JRot {
  double c, s;
  int p, q, po, qo;
};

// New 2 x 2 block J_s^T W[s, t] J_t from the old block (rows p_s, q_s; columns
// p_t, q_t) and the rotations (c, s) of the two pairs.  Explicit fused
// multiply-adds fix the rounding, so every caller gets identical values.
__device__ __forceinline__ void rotate_block(double w00, double w01, double w10, double w11, double cs, double ss,
                                             double ct, double st, double& n00, double& n01, double& n10,
                                             double& n11) {
  const double r00 = fma(cs, w00, -(ss * w10)), r01 = fma(cs, w01, -(ss * w11));
  const double r10 = fma(ss, w00, cs * w10), r11 = fma(ss, w01, cs * w11);
  n00 = fma(ct, r00, -(st * r01));
  n01 = fma(st, r00, ct * r01);
  n10 = fma(ct, r10, -(st * r11));
  n11 = fma(st, r10, ct * r11);
}

template <typename T, int LB, int NT>
__global__ __launch_bounds__(NT) void k_smallsvd(double* __restrict__ g2_all, const double* __restrict__ gw_all,
                                                 const SliceDesc* __restrict__ sd, const int2* __restrict__ wk,
                                                 const int2* __restrict__ slices, double tau_host, const double* __restrict__ tau_dev,
                                                 const double* __restrict__ mu_dev, Penalty pen,
                                                 T* __restrict__ Kall, double* __restrict__ sigma_out, int sigma_ld,
                                                 int* __restrict__ kept_out, int* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double s_scr;
  __shared__ int s_kept, s_flag[3];             // step flags, three-way rotation
  __shared__ int s_open;                        // some pair of the current W still rotates
  __shared__ JRot s_jr[2][LB / 2];              // rotations per pair, by step parity

  const int j = slices ? slices[blockIdx.x].x : (int)blockIdx.x;  // a class of slices, or all
  const int tid = threadIdx.x;
  const SliceDesc d = sd[j];
  const int l = slice_width(d, wk, j), kkeep = slice_kept(d, wk, j);
  if (l <= 0) return;  // slice not part of this pass
  const int L2 = l + (l & 1);  // players of the round-robin schedule (padding for odd l)
  const int gp = L2 + 1;
  const int nt_q = (d.n1 + kGramRows - 1) / kGramRows, nt_b = (d.n2 + kGramRows - 1) / kGramRows;
  const double delta_rel = 8.0 * (double)d.n1 * 2.220446049250313e-16;
  const double tau = mu_dev ? 1.0 / (*mu_dev) : (tau_dev ? tau_dev[d.tensor] : tau_host);
  const int ll = l * l;
  double* gq = g2_all + d.g2;  // the slice's partials; reused to park R2^{-1}
  double* B0 = reinterpret_cast<double*>(smem_raw);  // G, then a Jacobi buffer
  double* B1 = B0 + (size_t)L2 * gp;                 // W~, then W
  double* V = B1 + (size_t)L2 * gp;                  // R2^{-1}, then eigenvectors
  double* dR = V + (size_t)L2 * gp;
  double* lam = dR + gp;
  double* wv = lam + LMAX;
  double* sig = wv + LMAX;
  int* perm = reinterpret_cast<int*>(sig + LMAX);

  sum_gram_partials(B0, gp, gq, nt_q, l);
  sum_gram_partials(B1, gp, gw_all + d.g1, nt_b, l);
  __syncthreads();
  if (status && tid < 64) {  // a non-finite entry of the slice reaches a diagonal entry of the Gram sums
    bool bad = false;
    for (int a = tid; a < l; a += 64) bad |= !isfinite(B0[a * gp + a]) || !isfinite(B1[a * gp + a]);
    const bool any_bad = __ballot(bad) != 0;
    if (tid == 0) status[j] = any_bad ? 1 : 0;
  }
  if constexpr (LB <= 64) {
    // wave 0: R2 = chol(G2) and R2^{-1} in registers (lane b owns column b)
    if (tid < 64) chol_inverse_regs<LB>(B0, gp, l, delta_rel, V);
    __syncthreads();
  } else {
    if (l <= 64) {  // a narrow slice in a wide launch (uniform branch)
      if (tid < 64) chol_inverse_regs<64>(B0, gp, l, delta_rel, V);
      __syncthreads();
    } else {
      chol_deflate(B0, dR, gp, l, delta_rel, &s_scr);
      tri_inverse<LB>(B0, dR, gp, l, V);  // V = R2^{-1} (upper)
    }
  }
  for (int idx = tid; idx < ll; idx += NT) gq[idx] = V[(idx / l) * gp + (idx % l)];

  // B0 = W~ R2^{-1};  B1 = R2^{-T} B0 (= W, then symmetrized);  V = I
  for (int idx = tid; idx < ll; idx += NT) {
    const int a = idx / l, b = idx % l;
    double s = 0.0;
    for (int c = 0; c <= b; ++c) s += B1[a * gp + c] * V[c * gp + b];
    B0[a * gp + b] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < ll; idx += NT) {
    const int a = idx / l, b = idx % l;
    double s = 0.0;
    for (int c = 0; c <= a; ++c) s += V[c * gp + a] * B0[c * gp + b];
    B1[a * gp + b] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < L2 * L2; idx += NT) {
    const int a = idx / L2, b = idx % L2;
    if (a < l && b < l) {
      if (a < b) {
        const double m = 0.5 * (B1[a * gp + b] + B1[b * gp + a]);
        B1[a * gp + b] = m;
        B1[b * gp + a] = m;
      }
    } else {
      B1[a * gp + b] = 0.0;  // the padding row and column
    }
    V[a * gp + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    double md = 0.0;
    for (int a = tid; a < l; a += 64) md = fmax(md, fabs(B1[a * gp + a]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) md = fmax(md, __shfl_xor(md, off, 64));
    if (tid == 0) s_scr = md;
  }
  __syncthreads();
  // A pair is rotated only when its off-diagonal entry is above both tol
  // relative to sqrt(|app aqq|) and tol * max diag.  FP64 output: tol = 1e-15,
  // the rounding level of W.  FP32 output: tol = 1e-10; a skipped entry moves
  // an eigenvalue by about apq^2 / gap and a vector by about apq / gap, far
  // below the single-precision rounding of B and of the result.
  const double scale = s_scr > 0.0 ? s_scr : 1.0;  // W <- W / max diag
  const double inv_scale = 1.0 / scale;
  for (int idx = tid; idx < ll; idx += NT) B1[(idx / l) * gp + (idx % l)] *= inv_scale;
  __syncthreads();
  const double abs_tol = std::is_same<T, double>::value ? 1e-15 : 1e-10;

  // ---- parallel cyclic Jacobi, ping-pong between B1 and B0 -----------------
  const int half = L2 / 2;
  const int m = L2 - 1;  // steps per sweep
  constexpr int NWV = NT / 64;
  constexpr int NI = NT - 64;  // item threads: every wavefront but the last
  const bool look = tid >= NI;  // the last wavefront computes the next rotations
  const int lu = tid - NI;
  // fixed work of an item thread in every step: block items (s, t) and V items
  // (t, x); an index past the end is clamped to item 0 and only its stores are
  // masked, so every load of a step issues before any arithmetic.
  const int nblk = half * half, nvit = half * l;
  constexpr int NBI = ((LB / 2) * (LB / 2) + NI - 1) / NI;
  constexpr int NVI = ((LB / 2) * LB + NI - 1) / NI;
  int bs[NBI], bt[NBI], vt[NVI], vxo[NVI];
  bool bok[NBI], vok[NVI];
#pragma unroll
  for (int u = 0; u < NBI; ++u) {
    const int item = tid + u * NI;
    bok[u] = !look && item < nblk;
    bs[u] = bok[u] ? item / half : 0;
    bt[u] = bok[u] ? item % half : 0;
  }
#pragma unroll
  for (int u = 0; u < NVI; ++u) {
    const int item = tid + u * NI;
    vok[u] = !look && item < nvit;
    vt[u] = vok[u] ? item / l : 0;
    vxo[u] = vok[u] ? (item % l) * gp : 0;
  }
  if (tid < 3) s_flag[tid] = 0;
  __syncthreads();
  double* Wc = B1;
  double* Wn = B0;
  // rotations of the first step, from W itself
  if (look && lu < half) {
    int p, q;
    rr_pair_pad(0, lu, m, p, q);
    double c = 1.0, sn = 0.0;
    schur2(Wc[p * gp + p], Wc[q * gp + q], Wc[p * gp + q], abs_tol, c, sn);
    s_jr[0][lu] = JRot{c, sn, p, q, p * gp, q * gp};
    if (sn != 0.0) s_flag[0] = 1;
  }
  __syncthreads();
  // Step g applies the rotations in s_jr[g & 1] (published during step g - 1)
  // and publishes those of step g + 1.  s_flag[g % 3] says whether step g
  // rotates at all; it is set during step g - 1, read after the barrier that
  // ends it, and cleared during step g + 1, so set, read and clear are always
  // separated by a barrier.  m consecutive steps without a rotation test every
  // pair once on an unchanged W: the iteration has converged.
  int step = 0, still = 0;
  for (int g = 0; g < 30 * m; ++g) {
    const int fb = g & 1;
    const int ns = (step + 1 == m) ? 0 : step + 1;
    const bool any = s_flag[g % 3] != 0;
    if (tid == 0) s_flag[(g + 2) % 3] = 0;
    if (look) {
      const int u = lu < half ? lu : 0;
      int p2, q2;
      rr_pair_pad(ns, u, m, p2, q2);
      double app, aqq, apq;
      if (!any) {
        app = Wc[p2 * gp + p2];
        aqq = Wc[q2 * gp + q2];
        apq = Wc[p2 * gp + q2];
      } else {
        // entries (p2, p2), (q2, q2), (p2, q2) of W after this step
        const JRot r1 = s_jr[fb][rr_locate(step, p2, m, half)];
        const JRot r2 = s_jr[fb][rr_locate(step, q2, m, half)];
        const double x00 = Wc[r1.po + r1.p], x01 = Wc[r1.po + r1.q], x10 = Wc[r1.qo + r1.p], x11 = Wc[r1.qo + r1.q];
        const double y00 = Wc[r2.po + r2.p], y01 = Wc[r2.po + r2.q], y10 = Wc[r2.qo + r2.p], y11 = Wc[r2.qo + r2.q];
        const double z00 = Wc[r1.po + r2.p], z01 = Wc[r1.po + r2.q], z10 = Wc[r1.qo + r2.p], z11 = Wc[r1.qo + r2.q];
        const bool s1 = p2 == r1.q, s2 = q2 == r2.q;  // second member of its pair
        double n00, n01, n10, n11;
        rotate_block(x00, x01, x10, x11, r1.c, r1.s, r1.c, r1.s, n00, n01, n10, n11);
        app = s1 ? n11 : n00;
        rotate_block(y00, y01, y10, y11, r2.c, r2.s, r2.c, r2.s, n00, n01, n10, n11);
        aqq = s2 ? n11 : n00;
        rotate_block(z00, z01, z10, z11, r1.c, r1.s, r2.c, r2.s, n00, n01, n10, n11);
        apq = s1 ? (s2 ? n11 : n10) : (s2 ? n01 : n00);
      }
      double c = 1.0, sn = 0.0;
      schur2(app, aqq, apq, abs_tol, c, sn);
      if (lu < half) {
        s_jr[fb ^ 1][lu] = JRot{c, sn, p2, q2, p2 * gp, q2 * gp};
        if (sn != 0.0) s_flag[(g + 1) % 3] = 1;
      }
    } else if (any) {
      JRot ra[NBI], rb[NBI], rv[NVI];
#pragma unroll
      for (int u = 0; u < NBI; ++u) {
        ra[u] = s_jr[fb][bs[u]];
        rb[u] = s_jr[fb][bt[u]];
      }
#pragma unroll
      for (int u = 0; u < NVI; ++u) rv[u] = s_jr[fb][vt[u]];
      double w[NBI][4], v[NVI][2];
#pragma unroll
      for (int u = 0; u < NBI; ++u) {
        w[u][0] = Wc[ra[u].po + rb[u].p];
        w[u][1] = Wc[ra[u].po + rb[u].q];
        w[u][2] = Wc[ra[u].qo + rb[u].p];
        w[u][3] = Wc[ra[u].qo + rb[u].q];
      }
#pragma unroll
      for (int u = 0; u < NVI; ++u) {
        v[u][0] = V[vxo[u] + rv[u].p];
        v[u][1] = V[vxo[u] + rv[u].q];
      }
#pragma unroll
      for (int u = 0; u < NBI; ++u) {
        double n00, n01, n10, n11;
        rotate_block(w[u][0], w[u][1], w[u][2], w[u][3], ra[u].c, ra[u].s, rb[u].c, rb[u].s, n00, n01, n10, n11);
        if (bok[u]) {
          Wn[ra[u].po + rb[u].p] = n00;
          Wn[ra[u].po + rb[u].q] = n01;
          Wn[ra[u].qo + rb[u].p] = n10;
          Wn[ra[u].qo + rb[u].q] = n11;
        }
      }
#pragma unroll
      for (int u = 0; u < NVI; ++u) {
        const double np = fma(rv[u].c, v[u][0], -(rv[u].s * v[u][1]));
        const double nq = fma(rv[u].s, v[u][0], rv[u].c * v[u][1]);
        if (vok[u]) {
          V[vxo[u] + rv[u].p] = np;
          V[vxo[u] + rv[u].q] = nq;
        }
      }
    }
    __syncthreads();
    if (any) {
      double* tmp = Wc;
      Wc = Wn;
      Wn = tmp;
      still = 0;
    } else if (++still >= m) {
      break;
    } else if (still == 1) {
      // The first quiet step after rotations: W is unchanged from here on
      // unless some pair passes the rotation test, so testing every pair now
      // decides what the remaining m - 1 steps of the check would find.
      if (tid == 0) s_open = 0;
      __syncthreads();
      for (int idx = tid; idx < ll; idx += NT) {
        const int p = idx / l, q = idx % l;
        if (p < q) {
          const double apq = Wc[p * gp + q];
          if (fabs(apq) > abs_tol && apq * apq > abs_tol * abs_tol * fabs(Wc[p * gp + p] * Wc[q * gp + q])) s_open = 1;
        }
      }
      __syncthreads();
      if (s_open == 0) break;
    }
    step = ns;
  }
  (void)NWV;
  __syncthreads();

  // ---- order, shrink, K = U diag(w) U^T, K' = R2^{-1} K R2^{-T} -------------
  for (int a = tid; a < l; a += NT) lam[a] = Wc[a * gp + a] * scale;
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
    sig[i] = sv;
    if (sigma_out) sigma_out[(int64_t)j * sigma_ld + i] = sv;
  }
  if (sigma_out)
    for (int i = l + tid; i < sigma_ld; i += NT) sigma_out[(int64_t)j * sigma_ld + i] = 0.0;
  __syncthreads();
  double* Kb = Wn;  // free buffer
  double* Ri = Wc;  // R2^{-1} reloaded from global
  for (int idx = tid; idx < ll; idx += NT) {
    const int a = idx / l, b = idx % l;
    double t = 0.0;
    for (int i = 0; i < kkeep; ++i) {
      const int e = perm[i];
      t += V[a * gp + e] * wv[i] * V[b * gp + e];
    }
    Kb[a * gp + b] = t;
  }
  __syncthreads();
  for (int idx = tid; idx < ll; idx += NT) Ri[(idx / l) * gp + (idx % l)] = gq[idx];
  __syncthreads();
  for (int idx = tid; idx < ll; idx += NT) {  // V = K R2^{-T}
    const int a = idx / l, b = idx % l;
    double t = 0.0;
    for (int c = b; c < l; ++c) t += Kb[a * gp + c] * Ri[b * gp + c];
    V[a * gp + b] = t;
  }
  __syncthreads();
  T* K = Kall + d.kq;
  for (int idx = tid; idx < ll; idx += NT) {  // K' = R2^{-1} V, column-major
    const int a = idx % l, b = idx / l;
    double t = 0.0;
    for (int c = a; c < l; ++c) t += Ri[a * gp + c] * V[c * gp + b];
    K[a + (int64_t)b * l] = (T)t;
  }
  if (kept_out && tid == 0) kept_out[j] = s_kept;
}

}  // namespace

template <typename T>
int launch_smallsvd(double* g2, const double* gw, const SliceDesc* sd, const int2* wk, const int2* slices, int nslices,
                    int lmax, int sigma_ld, double tau, const double* tau_dev, const double* mu_dev, Penalty pen,
                    T* K, double* sigma_out, int* kept_out, int* status, hipStream_t s) {
  if (lmax > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  if (nslices == 0) return HT_OK;
  auto launch = [&](auto kern, int nt) -> int {
    int rc = ensure_dynamic_lds((const void*)kern, svd_lds_bytes(HT_MAX_WIDTH));
    if (rc) return rc;
    hipLaunchKernelGGL(kern, dim3((unsigned)nslices), dim3(nt), svd_lds_bytes(lmax), s, g2, gw, sd, wk, slices,
                       tau, tau_dev, mu_dev, pen, K, sigma_out, sigma_ld, kept_out, status);
    HT_CHECK_LAUNCH();
    return HT_OK;
  };
  if (lmax <= 16) return launch(k_smallsvd<T, 16, svd_threads<16>()>, svd_threads<16>());
  if (lmax <= 32) return launch(k_smallsvd<T, 32, svd_threads<32>()>, svd_threads<32>());
  if (lmax <= 48) return launch(k_smallsvd<T, 48, svd_threads<48>()>, svd_threads<48>());
  if (lmax <= 64) return launch(k_smallsvd<T, 64, svd_threads<64>()>, svd_threads<64>());
  return launch(k_smallsvd<T, 80, svd_threads<80>()>, svd_threads<80>());
}

template int launch_smallsvd<float>(double*, const double*, const SliceDesc*, const int2*, const int2*, int, int, int,
                                    double, const double*, const double*, Penalty, float*, double*, int*, int*,
                                    hipStream_t);
template int launch_smallsvd<double>(double*, const double*, const SliceDesc*, const int2*, const int2*, int, int,
                                     int, double, const double*, const double*, Penalty, double*, double*, int*, int*,
                                     hipStream_t);

}  // namespace ht
