// Launch wrappers of the htsvt kernels (host side declarations).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "device.hpp"

namespace ht {

// Mode matrices of the transformed modes, as seen by the transform kernel.
struct ModeTable {
  int nmodes;
  int n[HT_MAX_ORDER];
  int stride[HT_MAX_ORDER];  // stride of mode m in the face-slice index
  int off[HT_MAX_ORDER];     // offset of the n x n row-major matrix in the table
};

int transform_tile_width(int64_t P, size_t elem_bytes);

// Raise a kernel's dynamic-LDS limit once per (device, kernel).
int ensure_dynamic_lds(const void* kernel, size_t bytes);

template <typename T>
int launch_transform(const T* in, T* out, int64_t NT, int P, const ModeTable& mt, const T* table, hipStream_t s);

// Forward transform of an FP32 tensor with the result rounded to BF16.
int launch_transform_bf16(const float* in, uint16_t* out, int64_t NT, int P, const ModeTable& mt, const float* table,
                          hipStream_t s);

template <typename T>
int launch_omega(T* om, double* om64, int P, int64_t per_slice, uint32_t call, const int32_t* call_dev,
                 uint32_t stream_id, uint64_t seed, const int32_t* canon, hipStream_t s);

// Batched thin products over P slices (slice strides in elements).
//   nn:  Y_j (m x l)  = A_j (m x kd) W_j (kd x l)
//   tn:  Z_j (n x l)  = A_j^T (n x m) Q_j (m x l)
//   nt:  C_j (m x n)  = X_j (m x l) W_j^T (l x n)
//   gpart (optional): FP64 Gram partial of every 64-row output tile, laid out
//   [slice][tile][l][l] with ceil(rows / 64) tiles per slice.
template <typename T>
int launch_gemm_nn(const T* A, int64_t sA, int lda, const T* W, int64_t sW, int ldw, T* Y, int64_t sY, int ldy,
                   int m, int kd, int l, int P, double* gpart, hipStream_t s);
template <typename T>
int launch_gemm_tn(const T* A, int64_t sA, int lda, const T* Q, int64_t sQ, int ldq, T* Z, int64_t sZ, int ldz,
                   int m, int n, int l, int P, double* gpart, hipStream_t s);
template <typename T>
int launch_gemm_nt(const T* X, int64_t sX, int ldx, const T* W, int64_t sW, int ldw, T* C, int64_t sC, int ldc,
                   int m, int n, int l, int P, hipStream_t s);

// FP32 thin products on the matrix cores (128-row tiles; Gram partials per
// 128-row tile).  Require 16-byte aligned columns (leading dimensions and
// slice strides multiples of 4).
int mfma_tile_rows();
int launch_mfma_nn(const float* A, int64_t sA, int lda, const float* W, int64_t sW, int ldw, float* Y, int64_t sY,
                   int ldy, int m, int kd, int l, int P, double* gpart, hipStream_t s);
int launch_mfma_tn(const float* A, int64_t sA, int lda, const float* Q, int64_t sQ, int ldq, float* Z, int64_t sZ,
                   int ldz, int m, int n, int l, int P, double* gpart, hipStream_t s);

// BF16 thin products on the matrix cores (A in BF16, thin operands FP32 in
// memory, rounded to BF16 when staged; FP32 results; 128-row tiles).
int launch_bf16_nn(const uint16_t* A, int64_t sA, int lda, const float* W, int64_t sW, int ldw, float* Y,
                   int64_t sY, int ldy, int m, int kd, int l, int P, double* gpart, hipStream_t s);
int launch_bf16_tn(const uint16_t* A, int64_t sA, int lda, const float* Q, int64_t sQ, int ldq, float* Z,
                   int64_t sZ, int ldz, int m, int n, int l, int P, double* gpart, hipStream_t s);

// One CholeskyQR pass with deflation, in place on Y_j (m x l), from the Gram
// partials written by the producing product (gin, nparts per slice).
// Optionally writes the Gram partials of the result (gout, ceil(m/64) per
// slice).
template <typename T>
int launch_orth_apply(T* Y, int64_t sY, int ldy, int m, int l, int P, const double* gin, int nparts, double* gout,
                      hipStream_t s);

// Small SVD and shrinkage in FP64.  Inputs: Gram partials of the basis Q1
// (g2, ntiles_q per slice) and of Bt = A^T Q1 (gw, ntiles_b per slice).  With
// R2 = chol(Q1^T Q1), B = R2^{-T} Bt^T, W = B B^T = U diag(s^2) U^T; writes
// K' = R2^{-1} U diag(w) U^T R2^{-T} (l x l) with w_i = prox(s_i)/s_i, i < k.
// The first l*l doubles of every slice's g2 partials are overwritten (scratch).
template <typename T>
int launch_smallsvd(double* g2, int ntiles_q, int m_q, const double* gw, int ntiles_b, int l, int k, int P,
                    double tau, const double* mu_dev, Penalty pen, T* K, double* sigma_out, int* kept_out,
                    hipStream_t s);

// ADMM update (see htsvt.h) and the per-iteration scalar bookkeeping.
template <typename T>
int launch_admm_input(const T* M, const T* E, const T* Y, const AdmmState* st, T* Xin, int64_t N, hipStream_t s);
template <typename T>
int launch_admm_update(const T* M, const uint8_t* mask, const T* Lnew, T* L, T* E, T* Y, T* Xin,
                       AdmmState* st, int64_t N, int model, Penalty psi, double lambda, double vartheta,
                       double mu_max, hipStream_t s);
int launch_admm_finalize(AdmmState* st, double vartheta, double mu_max, hipStream_t s);
int launch_admm_reset(AdmmState* st, double mu0, hipStream_t s);

}  // namespace ht
