// Launch wrappers of the htsvt kernels (host side declarations).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "device.hpp"
#include "layout.hpp"

namespace ht {

// Rows per FP64 Gram partial: every producer of a thin block writes one l x l
// partial per 64 rows of it, so a slice of m rows has ceil(m / 64) partials.
constexpr int kGramRows = 64;

// Largest sketch width of a complex slice (its l x l kernels hold two FP64
// planes per matrix).
constexpr int kMaxComplexWidth = 64;
// Complex rows per work item of the BF16 products of complex slices (items
// (slice, first complex row) with this step).
constexpr int kCplxProdRows = 64;
// Complex reconstruction items: strips of kCmulRows complex rows, groups of up
// to kCmulGroup column tiles of 64 (item.y = strip * groups + group).
constexpr int kCmulRows = 128, kCmulGroup = 8;

// Work items.  Every per-slice launch takes an item list: item i of a product
// or orthonormalization launch is (slice, first row of its tile); of the
// transform, (tensor, first tube position); of the reconstruction nt product,
// (slice, 64 x 64 tile index with row tiles fastest).  Widths: lmax is the
// largest slice width of the launch (selects the kernel's register capacity);
// wk, when not null, holds each slice's (l, k) and overrides the slice table.

// Largest power-of-two tube count TP <= 256 with TP * P * elem_bytes <= budget (0 if none).
int transform_tile_width(int64_t P, size_t elem_bytes, size_t budget);

// Raise a kernel's dynamic-LDS limit once per (device, kernel).
int ensure_dynamic_lds(const void* kernel, size_t bytes);

// Forward (inverse = 0) or inverse transform of every tensor of the table;
// TO = uint16_t rounds the result to BF16.  lds = largest TP * P * sizeof(T).
template <typename T, typename TO>
int launch_transform(const T* in, TO* out, const TensorDesc* tds, const int2* items, int nitems, size_t lds,
                     const T* table, int inverse, hipStream_t s);

// FP32 transform of tensors whose transformed modes are exactly two of length
// 16 (mode tables with n = {16, 16}, slice strides {1, 16} in either order);
// items are (tensor, t0) with t0 a multiple of kT16Tube, each taking tube
// positions t0 .. t0 + kT16Tube - 1 (fewer at the end; NT a multiple of 16,
// tensor offsets even).  in and out must be 8-byte (BF16 out: 4-byte) aligned,
// else HT_ERR_UNSUPPORTED.
constexpr int kT16Tube = 32;
template <typename TO>
int launch_transform16(const float* in, TO* out, const TensorDesc* tds, const int2* items, int nitems,
                       const float* table, int inverse, hipStream_t s);

// Same for tensors under the unitary DFT (complex slices, see TensorDesc):
// forward stores the canonical slots of A, inverse reads the slots of C.
// nf > 0 selects the fused form (every tensor's first fused mode has length
// nf, 16-byte tile accesses; see ModeTable::first), nf = 0 the general one.
template <typename T, typename TO>
int launch_transform_cplx(const T* in, TO* out, const TensorDesc* tds, const int2* items, int nitems, size_t lds,
                          const T* table, const int32_t* cmap, int inverse, int nmax, int nf, hipStream_t s);

// Gaussian sketch matrices of every slice (T storage, FP64 copy and/or the
// BF16 rounding of the T values), at the slices' Omega offsets, or densely at
// s * dense_stride when dense_stride > 0.
template <typename T>
int launch_omega(T* om, double* om64, uint16_t* omh, const SliceDesc* sd, const int2* wk, int nslices,
                 int64_t max_per_slice, uint32_t call, const int32_t* call_dev, uint32_t stream_base, uint64_t seed,
                 int64_t dense_stride, hipStream_t s);

// Thin products on the vector ALUs (64-row tiles; Gram partials per tile).
//   sketch nn: Y = A Omega or A Z;  tn: Z = A^T Q;  recon: QK = Q1 K', C = QK Bt^T.
template <typename T>
int launch_gemm_nn(const T* A, const T* W, T* Y, const SliceDesc* sd, const int2* wk, const int2* items, int nitems,
                   int lmax, double* gpart, hipStream_t s);
template <typename T>
int launch_gemm_tn(const T* A, const T* Q, T* Z, const SliceDesc* sd, const int2* wk, const int2* items, int nitems,
                   int lmax, double* gpart, hipStream_t s);
template <typename T>
int launch_recon_qk(const T* Q, const T* K, T* QK, const SliceDesc* sd, const int2* wk, const int2* items, int nitems,
                    int lmax, hipStream_t s);
template <typename T>
int launch_gemm_nt(const T* X, const T* W, T* C, const SliceDesc* sd, const int2* wk, const int2* items, int nitems,
                   hipStream_t s);

// FP32 and BF16 sketch products on the matrix cores; rows = 64 or 128 output
// rows per workgroup (Gram partials per 64 rows).  The streaming form of the
// FP32 nn product takes 256-row items, real slices with n1 % 4 == 0, widths
// up to 64 and n2 <= kStreamMaxK (its thin operand is staged in LDS whole).
int launch_mfma_nn(const float* A, const float* W, float* Y, const SliceDesc* sd, const int2* wk, const int2* items,
                   int nitems, int lmax, int rows, double* gpart, hipStream_t s);
int launch_mfma_tn(const float* A, const float* Q, float* Z, const SliceDesc* sd, const int2* wk, const int2* items,
                   int nitems, int lmax, int rows, double* gpart, hipStream_t s);
constexpr int kStreamRows = 256, kStreamMaxK = 512;
// Key of the Gaussian sketch draws (as launch_omega): call index (*call_dev
// when set), stream base added to the tensor index, seed.
struct OmegaKey {
  uint32_t call;
  const int32_t* call_dev;
  uint32_t stream_base;
  uint64_t seed;
};
// W == nullptr: the sketch Omega_s is drawn inside the product (the same values
// launch_omega writes, rounded to FP32) from `key` instead of read.
int launch_mfma_nn_stream(const float* A, const float* W, float* Y, const SliceDesc* sd, const int2* wk,
                          const int2* items, int nitems, int lmax, int kmax, double* gpart, const OmegaKey& key,
                          hipStream_t s);
// Q1 K' on the matrix cores (FP32, widths up to 64; items as launch_recon_qk:
// slice and first row of a 64-row tile).
int launch_mfma_qk(const float* Q, const float* K, float* QK, const SliceDesc* sd, const int2* wk, const int2* items,
                   int nitems, int lmax, hipStream_t s);
// Reconstruction C = QK Bt^T on the matrix cores (FP32; items as launch_gemm_nt).
int launch_mfma_nt(const float* X, const float* W, float* C, const SliceDesc* sd, const int2* wk, const int2* items,
                   int nitems, int lmax, hipStream_t s);
int launch_bf16_nn(const uint16_t* A, const float* W, float* Y, const SliceDesc* sd, const int2* wk,
                   const int2* items, int nitems, int lmax, int rows, double* gpart, hipStream_t s);
int launch_bf16_tn(const uint16_t* A, const float* Q, float* Z, const SliceDesc* sd, const int2* wk,
                   const int2* items, int nitems, int lmax, int rows, double* gpart, hipStream_t s);

// Complex slices (stacked layout) on the matrix cores, l <= kMaxComplexWidth,
// items of 64 complex rows (FP32) or kCplxProdRows (BF16): nn Y = A W (wreal:
// W is the real Omega, n2 x l),
// tn Z = A^H Q, with complex Gram partials; reconstruction QK = Q1 K' and
// C = QK Bt^H (items of kCmulRows complex rows and column-tile groups).
int launch_mfma_cnn(const float* A, const float* W, float* Y, int wreal, const SliceDesc* sd, const int2* wk,
                    const int2* items, int nitems, int lmax, double* gpart, hipStream_t s);
int launch_mfma_ctn(const float* A, const float* Q, float* Z, const SliceDesc* sd, const int2* wk, const int2* items,
                    int nitems, int lmax, double* gpart, hipStream_t s);
int launch_bf16_cnn(const uint16_t* A, const uint16_t* W, float* Y, int wreal, const SliceDesc* sd, const int2* wk,
                    const int2* items, int nitems, int lmax, double* gpart, hipStream_t s);
int launch_bf16_ctn(const uint16_t* A, const uint16_t* Q, float* Z, const SliceDesc* sd, const int2* wk,
                    const int2* items, int nitems, int lmax, double* gpart, hipStream_t s);
int launch_mfma_cqk(const float* Q, const float* K, float* QK, const SliceDesc* sd, const int2* wk, const int2* items,
                    int nitems, int lmax, hipStream_t s);
// C = QK Bt^H for BF16-mixed plans: split-BF16 operands (three BF16 products
// per term), items as launch_mfma_cnt.
int launch_bf16x3_cnt(const float* X, const float* W, float* C, const SliceDesc* sd, const int2* wk,
                      const int2* items, int nitems, int lmax, hipStream_t s);
int launch_mfma_cnt(const float* X, const float* W, float* C, const SliceDesc* sd, const int2* wk, const int2* items,
                    int nitems, int lmax, hipStream_t s);

// One CholeskyQR pass with deflation, in place on the basis `which` (0: Y of
// n1 rows, 1: Z of n2 rows) from the Gram partials of the producing product
// (gin at the slice's g1 offset, one per 64 rows).  Optionally
// writes the Gram partials of the result (gout at the slice's g2 offset, one
// per 64 rows).  Items are 64-row tiles.  Widths above 64 overwrite the first
// partial of every slice with R^{-1}.
template <typename T>
int launch_orth_apply(T* Y, int which, const SliceDesc* sd, const int2* wk, const int2* items, int nitems, int lmax,
                      int nslices, double* gin, double* gout, hipStream_t s);

// Small SVD and shrinkage in FP64, one workgroup per slice.  Inputs: Gram
// partials of the basis Q1 (g2 at the slice's g2 offset, one per 64 rows of
// n1) and of Bt = A^T Q1 (gw at its g1 offset, one per 64 rows of n2).
// With R2 = chol(Q1^T Q1), B = R2^{-T} Bt^T, W = B B^T = U diag(s^2) U^T;
// writes K' = R2^{-1} U diag(w) U^T R2^{-T} (l x l, at the slice's kq offset)
// with w_i = prox(s_i)/s_i, i < k.  tau: 1 / *mu_dev if mu_dev, else
// tau_dev[tensor] if tau_dev, else the scalar.  The first l*l doubles of every
// slice's g2 partials are overwritten (scratch).  slices, when not null, lists
// the slices of this launch (x = slice index; nslices entries; a width class),
// else slices 0 .. nslices - 1.  lmax bounds the widths of the launch;
// sigma_out rows have sigma_ld entries.  status (optional): per slice, 1 when
// a Gram matrix held a NaN or an infinity, else 0.
template <typename T>
int launch_smallsvd(double* g2, const double* gw, const SliceDesc* sd, const int2* wk, const int2* slices, int nslices,
                    int lmax, int sigma_ld, double tau, const double* tau_dev, const double* mu_dev, Penalty pen,
                    T* K, double* sigma_out, int* kept_out, int* status, hipStream_t s);

// Complex slices (unitary or plain DFT on every mode 3..d; cplx.hip): the
// stacked [Re; Im] storage described in layout.hpp, widths up to
// kMaxComplexWidth.  Gram partials: one per 64 complex rows, 2 l^2 doubles.
// CholeskyQR with deflation of the complex basis `which` (0: Y, 1: Z): one
// factor launch per slice (R^{-1} parked over the first partial of gin), then
// Q = Y R^{-1} per 64-complex-row item; gout as launch_orth_apply.
// FP32 blocks without gout take `tiles` instead: the same 64-row items in slice
// order, split into contiguous ranges over resident workgroups.  Yh (nullable):
// a BF16 copy of the result at the same element offsets (the operand of the
// BF16 products that follow).
template <typename T>
int launch_corth(T* Y, uint16_t* Yh, int which, const SliceDesc* sd, const int2* wk, const int2* items, int nitems,
                 const int2* tiles, int ntiles, int lmax, int nslices, double* gin, double* gout, hipStream_t s);
// Small SVD and shrinkage of complex slices (arguments as launch_smallsvd;
// K' is written stacked, 2 l x l).
template <typename T>
int launch_csvd(double* g2, const double* gw, const SliceDesc* sd, const int2* wk, const int2* slices, int nslices,
                int lmax, int sigma_ld, double tau, const double* tau_dev, const double* mu_dev, Penalty pen, T* K,
                double* sigma_out, int* kept_out, int* status, hipStream_t s);
// Complex sketch products on the vector units: trans = 0: Y = A W (wreal: W is
// the real Omega, n2 x l), trans = 1: Z = A^H Q; items of 64 complex rows.
template <typename T>
int launch_cgemm(const T* A, const T* W, T* Y, int trans, int wreal, const SliceDesc* sd, const int2* wk,
                 const int2* items, int nitems, int lmax, double* gpart, hipStream_t s);
// Complex reconstruction on the vector units: mode 0: QK = Q1 K' (items of 64
// complex rows), mode 1: C = QK Bt^H (64 x 64 tiles as launch_gemm_nt).
template <typename T>
int launch_crecon(const T* X, const T* W, T* C, int mode, const SliceDesc* sd, const int2* wk, const int2* items,
                  int nitems, hipStream_t s);

// Learned widths (mlp.hip).  Network parameters: one flat FP32 vector of
// mlp_param_count() entries.  Gradient steps use a partial buffer of
// mlp_grad_parts(n) rows of mlp_param_count() floats plus as many loss partials.
int mlp_param_count();
int mlp_grad_parts(int n);
int launch_mlp_forward(const float* th, const float* X, float* z, int n, hipStream_t s);
// Gradient of the mean squared error (grad, loss optional) and, when th is not
// null, one Adam step on th, m, v (th_in and th may alias).
int launch_mlp_grad_step(const float* th_in, const float* X, const float* y, int n, float* part, float* lpart,
                         float* grad, float* loss, float* th, float* m, float* v, int step, float lr, float beta1,
                         float beta2, float eps, hipStream_t s);
// ||A_s||_F^2 into anorm[2 s + 1] (A in T, or BF16 bits when bf16 != 0).
template <typename T>
int launch_anorm(const T* A, int bf16, const SliceDesc* sd, int nslices, double* anorm, hipStream_t s);
// Features of every slice from the previous call (sig rows of lmax, kept,
// widths used wk_prev, anorm[2 s]) and the widths of this call into wk
// (mode 1: fixed widths; mode 2: predicted when lstate[0] says the previous
// call's statistics are valid).
int launch_width(const float* th, int mode, const SliceDesc* sd, int nslices, int lmax, const double* sig,
                 const int* kept, const int2* wk_prev, const double* anorm, const int* lstate, double tau,
                 const double* tau_dev, const double* mu_dev, uint32_t call, const int32_t* call_dev, float* feat,
                 int2* wk, hipStream_t s);
// Redo set wk2 (fixed width, or 0 = skip), final widths wkf, anorm[2 s] <-
// anorm[2 s + 1], counters lstate[1] (predicted slices), lstate[2] (redone).
int launch_fallback(const SliceDesc* sd, int nslices, int lmax, const int2* wk1, const double* sig, const int* kept,
                    double* anorm, double tau, const double* tau_dev, const double* mu_dev, Penalty pen, int force,
                    int2* wk2, int2* wkf, int* lstate, hipStream_t s);
int launch_track_finalize(int nslices, const int2* wk1, int2* wkf, double* anorm, hipStream_t s);
int launch_lstate_set(int* lstate, int valid, int clear_counts, hipStream_t s);

// ADMM update (see htsvt.h) and the per-iteration scalar bookkeeping.
template <typename T>
int launch_admm_input(const T* M, const T* E, const T* Y, const AdmmState* st, T* Xin, int64_t N, hipStream_t s);
// Models HT_RPCA_TUBE / HT_RPCA_SLICE first form the squared group norms into
// gsq (NT or N / NT doubles; NT = n1 n2).
template <typename T>
int launch_admm_update(const T* M, const uint8_t* mask, const T* Lnew, T* L, T* E, T* Y, T* Xin,
                       AdmmState* st, int64_t N, int model, Penalty psi, double lambda, double vartheta,
                       double mu_max, double* gsq, int64_t NT, hipStream_t s);
int launch_admm_finalize(AdmmState* st, double vartheta, double mu_max, hipStream_t s);
int launch_admm_reset(AdmmState* st, double mu0, hipStream_t s);
// st->rse = ||L - truth||_F / ||truth||_F (FP64 block partials in part, 2 per
// block, nblocks blocks, summed in a fixed order), or NaN when truth is null.
template <typename T>
int launch_admm_rse(const T* L, const T* truth, int64_t N, double* part, int nblocks, AdmmState* st, hipStream_t s);

}  // namespace ht
