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
// One Jacobi step applies all l/2 disjoint rotations at once: one lane per pair
// computes its rotation from the current matrix, then for pairs s and t the
// 2 x 2 block of W on rows of s and columns of t becomes J_s^T W[s, t] J_t,
// produced from old values only into a second buffer.  W is scaled to unit
// maximum diagonal first, so the rotation formulas cannot overflow.
#include "chol.hpp"

namespace ht {

namespace {

constexpr int NT = 256;
constexpr int LMAX = 80;

size_t svd_lds_bytes(int l) {
  const size_t gp = (size_t)l + 1;
  const size_t L2 = (size_t)l + (l & 1);
  (void)L2;
  return (3 * (size_t)l * gp + gp + 3 * LMAX + 2 * 64) * 8 + (LMAX + 2 * 64) * 4;
}

// Pair t of step `step` in the round-robin schedule on L2 (even) players;
// q = -1 when the partner is the padding player (odd l).
__device__ __forceinline__ void rr_pair(int step, int t, int L2, int l, int& p, int& q) {
  const int m = L2 - 1;  // step, t < m, so each reduction is one conditional subtract
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
  if (q >= l) q = -1;
}

// Symmetric Schur rotation (c, s) that annihilates W[p][q] (Golub-Van Loan,
// written as t = 2 apq sgn(d) / (|d| + sqrt(d^2 + 4 apq^2)), d = aqq - app);
// identity when the entry is below the rounding-level thresholds.  Entries are
// at most 1 in magnitude (W is normalized), so nothing overflows.
__device__ __forceinline__ void schur2(double app, double aqq, double apq, double abs_tol, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (fabs(apq) > abs_tol && apq * apq > 1e-30 * fabs(app * aqq)) {
    const double d = aqq - app;
    const double h = sqrt(d * d + 4.0 * apq * apq);
    const double t = 2.0 * apq * (d >= 0.0 ? 1.0 : -1.0) * fast_rcp(fabs(d) + h);
    c = fast_rsqrt(1.0 + t * t);
    s = t * c;
  }
}

template <typename T, int LB>
__global__ __launch_bounds__(NT) void k_smallsvd(double* __restrict__ g2_all, const double* __restrict__ gw_all,
                                                 const SliceDesc* __restrict__ sd, const int2* __restrict__ wk,
                                                 int prod_rows, double tau_host, const double* __restrict__ tau_dev,
                                                 const double* __restrict__ mu_dev, Penalty pen,
                                                 T* __restrict__ Kall, double* __restrict__ sigma_out, int sigma_ld,
                                                 int* __restrict__ kept_out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double s_scr;
  __shared__ int s_rot[2], s_kept, s_step[2];  // flags double-buffered by parity

  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  const SliceDesc d = sd[j];
  const int l = slice_width(d, wk, j), kkeep = slice_kept(d, wk, j);
  if (l <= 0) return;  // slice not part of this pass
  const int gp = l + 1;
  const int nt_q = (d.n1 + 63) / 64, nt_b = (d.n2 + prod_rows - 1) / prod_rows;
  const double delta_rel = 8.0 * (double)d.n1 * 2.220446049250313e-16;
  const double tau = mu_dev ? 1.0 / (*mu_dev) : (tau_dev ? tau_dev[d.tensor] : tau_host);
  const int ll = l * l;
  double* gq = g2_all + d.g2;  // the slice's partials; reused to park R2^{-1}
  double* B0 = reinterpret_cast<double*>(smem_raw);  // G, then a Jacobi buffer
  double* B1 = B0 + (size_t)l * gp;                  // W~, then W
  double* V = B1 + (size_t)l * gp;                   // R2^{-1}, then eigenvectors
  double* dR = V + (size_t)l * gp;
  double* lam = dR + gp;
  double* wv = lam + LMAX;
  double* sig = wv + LMAX;
  double* rc = sig + LMAX;
  double* rs = rc + 64;
  int* perm = reinterpret_cast<int*>(rs + 64);

  sum_gram_partials(B0, gp, gq, nt_q, l);
  sum_gram_partials(B1, gp, gw_all + d.g1, nt_b, l);
  __syncthreads();
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
  for (int idx = tid; idx < ll; idx += NT) {
    const int a = idx / l, b = idx % l;
    if (a < b) {
      const double m = 0.5 * (B1[a * gp + b] + B1[b * gp + a]);
      B1[a * gp + b] = m;
      B1[b * gp + a] = m;
    }
    V[a * gp + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double md = 0.0;
    for (int a = 0; a < l; ++a) md = fmax(md, fabs(B1[a * gp + a]));
    s_scr = md;
  }
  __syncthreads();
  // A pair is rotated only when its off-diagonal entry is above both 1e-15
  // relative to sqrt(|app aqq|) and 1e-15 * max diag: below that it is at the
  // rounding level of W and rotating it would not change the result.
  const double scale = s_scr > 0.0 ? s_scr : 1.0;  // W <- W / max diag
  const double inv_scale = 1.0 / scale;
  for (int idx = tid; idx < ll; idx += NT) B1[(idx / l) * gp + (idx % l)] *= inv_scale;
  __syncthreads();
  const double abs_tol = 1e-15;

  // ---- parallel cyclic Jacobi, ping-pong between B1 and B0 -----------------
  const int L2 = l + (l & 1);
  const int half = L2 / 2;
  // fixed work of this thread in every step: block items (s, t) and V items (t, x)
  const int nblk = half * half, nvit = half * l;
  constexpr int NBI = ((LB / 2) * (LB / 2) + NT - 1) / NT;  // block items per thread (LB >= l)
  constexpr int NVI = ((LB / 2) * LB + NT - 1) / NT;        // V items per thread
  int bs[NBI], bt[NBI], vt[NVI], vx[NVI];
#pragma unroll
  for (int u = 0; u < NBI; ++u) {
    const int item = tid + u * NT;
    bs[u] = item < nblk ? item / half : -1;
    bt[u] = item < nblk ? item % half : 0;
  }
#pragma unroll
  for (int u = 0; u < NVI; ++u) {
    const int item = tid + u * NT;
    vt[u] = item < nvit ? item / l : -1;
    vx[u] = item < nvit ? item % l : 0;
  }
  if (tid == 0) {
    s_step[0] = s_step[1] = 0;
    s_rot[0] = s_rot[1] = 0;
  }
  __syncthreads();
  double* Wc = B1;
  double* Wn = B0;
  // Pair indices come from the schedule arithmetic, so after the barrier every
  // load of the update (rotation parameters, W and V entries) issues at once.
  // A flag of parity b is cleared only after every thread has passed the
  // barriers that follow its last read, so no barrier is needed around it.
  int gstep = 0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    const int sp = sweep & 1;
    for (int step = 0; step < L2 - 1; ++step, ++gstep) {
      const int fp = gstep & 1;
      __syncthreads();  // previous step's update complete; previous flags read
      if (tid == 0) {
        s_step[fp ^ 1] = 0;
        if (step == 0) s_rot[sp ^ 1] = 0;
      }
      if (tid < half) {
        int p, q;
        rr_pair(step, tid, L2, l, p, q);
        double c = 1.0, sn = 0.0;
        if (q >= 0) schur2(Wc[p * gp + p], Wc[q * gp + q], Wc[p * gp + q], abs_tol, c, sn);
        rc[tid] = c;
        rs[tid] = sn;
        if (sn != 0.0) {
          s_step[fp] = 1;
          s_rot[sp] = 1;
        }
      }
      __syncthreads();
      if (!s_step[fp]) continue;  // nothing to rotate in this step: W and V unchanged
#pragma unroll
      for (int u = 0; u < NBI; ++u) {
        if (bs[u] < 0) continue;
        const int st = bs[u], tt = bt[u];
        int ps, qs, pt, qt;
        rr_pair(step, st, L2, l, ps, qs);
        rr_pair(step, tt, L2, l, pt, qt);
        const double cs = rc[st], ss = rs[st], ct = rc[tt], snt = rs[tt];
        const double w00 = Wc[ps * gp + pt];
        const double w01 = qt >= 0 ? Wc[ps * gp + qt] : 0.0;
        const double w10 = qs >= 0 ? Wc[qs * gp + pt] : 0.0;
        const double w11 = (qs >= 0 && qt >= 0) ? Wc[qs * gp + qt] : 0.0;
        const double r00 = cs * w00 - ss * w10, r01 = cs * w01 - ss * w11;
        const double r10 = ss * w00 + cs * w10, r11 = ss * w01 + cs * w11;
        Wn[ps * gp + pt] = ct * r00 - snt * r01;
        if (qt >= 0) Wn[ps * gp + qt] = snt * r00 + ct * r01;
        if (qs >= 0) Wn[qs * gp + pt] = ct * r10 - snt * r11;
        if (qs >= 0 && qt >= 0) Wn[qs * gp + qt] = snt * r10 + ct * r11;
      }
#pragma unroll
      for (int u = 0; u < NVI; ++u) {
        if (vt[u] < 0) continue;
        const int tt = vt[u], x = vx[u];
        int pt, qt;
        rr_pair(step, tt, L2, l, pt, qt);
        if (qt < 0) continue;  // the padding partner: no rotation
        const double snt = rs[tt], ct = rc[tt];
        const double vp = V[x * gp + pt], vq = V[x * gp + qt];
        if (snt != 0.0) {
          V[x * gp + pt] = ct * vp - snt * vq;
          V[x * gp + qt] = snt * vp + ct * vq;
        }
      }
      double* tmp = Wc;
      Wc = Wn;
      Wn = tmp;
    }
    __syncthreads();
    if (!s_rot[sp]) break;
  }
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
int launch_smallsvd(double* g2, const double* gw, const SliceDesc* sd, const int2* wk, int nslices, int lmax,
                    int prod_rows, double tau, const double* tau_dev, const double* mu_dev, Penalty pen, T* K,
                    double* sigma_out, int* kept_out, hipStream_t s) {
  if (lmax > HT_MAX_WIDTH) HT_FAIL(HT_ERR_UNSUPPORTED, "sketch width above HT_MAX_WIDTH");
  if (nslices == 0) return HT_OK;
  auto launch = [&](auto kern) -> int {
    int rc = ensure_dynamic_lds((const void*)kern, svd_lds_bytes(HT_MAX_WIDTH));
    if (rc) return rc;
    hipLaunchKernelGGL(kern, dim3((unsigned)nslices), dim3(NT), svd_lds_bytes(lmax), s, g2, gw, sd, wk, prod_rows,
                       tau, tau_dev, mu_dev, pen, K, sigma_out, lmax, kept_out);
    HT_CHECK_LAUNCH();
    return HT_OK;
  };
  if (lmax <= 16) return launch(k_smallsvd<T, 16>);
  if (lmax <= 32) return launch(k_smallsvd<T, 32>);
  if (lmax <= 48) return launch(k_smallsvd<T, 48>);
  if (lmax <= 64) return launch(k_smallsvd<T, 64>);
  return launch(k_smallsvd<T, 80>);
}

template int launch_smallsvd<float>(double*, const double*, const SliceDesc*, const int2*, int, int, int, double,
                                    const double*, const double*, Penalty, float*, double*, int*, hipStream_t);
template int launch_smallsvd<double>(double*, const double*, const SliceDesc*, const int2*, int, int, int, double,
                                     const double*, const double*, Penalty, double*, double*, int*, hipStream_t);

}  // namespace ht
