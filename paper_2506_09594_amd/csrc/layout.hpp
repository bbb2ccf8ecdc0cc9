// Device-visible description of a plan: one or many tensors, each cut into
// transformed face slices.  Every per-slice kernel finds its operands through
// the slice table and takes its work from an item list, so one launch covers
// all slices of all tensors of a batch whatever their sizes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "htsvt.h"

namespace ht {

// Mode matrices of the transformed modes of one tensor, as seen by the
// transform kernel.
struct ModeTable {
  int nmodes;
  int n[HT_MAX_ORDER];
  int stride[HT_MAX_ORDER];  // stride of mode m in the face-slice index
  int off[HT_MAX_ORDER];     // offset of the n x n row-major matrix in the table
  // DFT tensors, fused transform: first, the shortest mode (length <= 8),
  // applied while the tile loads; last, the longest, which the inverse applies
  // while the tile is stored; every mode a power of two <= 32.  -1 when the
  // tensor takes the general form
  int first, last;
};

// One tensor of a plan.  X and out are packed buffers holding the tensors one
// after another, each in Fortran order; A and C hold the transformed slices
// the method works on.  For a real transform slice j of the tensor is the
// n1 x n2 block at a + j n1 n2.  Under the unitary DFT on every mode 3..d only
// one slice of each conjugate pair is kept (slot s of the tensor), stored as
// the stacked real block [Re; Im] (2 n1 x n2, column-major) at a + 2 s n1 n2;
// cmap[j] is the slot of slice j, with bit 31 set when j is the conjugate
// partner of the slot's slice.
struct TensorDesc {
  int64_t x;      // offset of the tensor in X / out
  int64_t a;      // offset of its slices in A / C
  int64_t NT;     // n1 * n2: elements per face slice
  int64_t cmap;   // offset of its slot map in the plan's map (complex tensors)
  int32_t P;      // face slices
  int32_t TP;     // tube positions per transform tile (power of two)
  int32_t lgTP;
  int32_t slice0; // index of its first slice in the slice table
  int32_t cplx;   // unitary DFT on every transformed mode (complex slices)
  int32_t n1;
  int32_t nslots; // stored slots (complex: one per conjugate pair; the slot map
                  // is followed by (canonical slice, partner or -1) per slot)
  ModeTable fwd, inv;  // complex matrices (interleaved re, im) when cplx
};

// One transformed face slice.  Thin blocks are laid out for the plan's
// maximum width lmax; a slice uses the first l columns.  A complex slice
// (cplx = 1, DFT on every transformed mode) of n1 x n2 complex entries is the
// stacked real block [Re; Im] (2 n1 x n2) at a; its thin blocks are stacked
// too (Y: 2 n1 x l, Z: 2 n2 x l, K: 2 l x l) and l, k count complex columns.
struct SliceDesc {
  int64_t a;   // offset of the n1 x n2 slice in A and C (elements)
  int64_t y;   // offset of its n1 x lmax block in Y and QK
  int64_t z;   // offset of its n2 x lmax block in Omega and Z
  int64_t kq;  // offset of its lmax x lmax block in K
  int64_t g1;  // offset (doubles) of its product Gram partials (ceil(max(n1,n2)/64) tiles)
  int64_t g2;  // offset (doubles) of its basis Gram partials (ceil(n1/64) tiles)
  int32_t n1, n2;   // rows and columns (complex entries for a complex slice)
  int32_t l, k;     // sketch width and number of kept singular values
  int32_t tensor;   // index of the tensor (the Philox stream word is stream_base + tensor)
  int32_t local;    // slice index within the tensor (the Philox counter word)
  int32_t p;        // oversampling of the tensor (learned widths)
  int32_t cplx;     // complex slice (stacked real and imaginary parts)
  int32_t nc;       // columns of C written by the reconstruction (n2)
  int32_t pad;
};

// Element (r, k) of the real embedding [[Ar, -Ai], [Ai, Ar]] (2 n1o x 2 n2o)
// of a complex matrix stored as the stacked block [Ar; Ai] (lda = 2 n1o rows,
// n2o columns), without forming it; cplx = 0: the stored block itself.  The
// embedding times a stacked [Wr; Wi] is the stacked complex product.
__host__ __device__ inline int64_t embed_index(int r, int k, int lda, int cplx, int n1o, int n2o, bool& neg) {
  neg = false;
  if (cplx && k >= n2o) {
    neg = r < n1o;
    return (int64_t)(neg ? r + n1o : r - n1o) + (int64_t)(k - n2o) * lda;
  }
  return (int64_t)r + (int64_t)k * lda;
}

// Width and kept count of slice s: from the slice table, or from an optional
// per-slice (l, k) array written on the device (learned widths; l = 0 skips
// the slice in that launch).
__host__ __device__ inline int slice_width(const SliceDesc& d, const int2* wk, int s) {
  return wk ? wk[s].x : d.l;
}
__host__ __device__ inline int slice_kept(const SliceDesc& d, const int2* wk, int s) {
  return wk ? wk[s].y : d.k;
}

}  // namespace ht
