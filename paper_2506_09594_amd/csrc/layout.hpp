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
};

// One tensor of a plan (element offsets are into the packed X / A / C / out
// buffers, which hold the tensors one after another, each in Fortran order).
struct TensorDesc {
  int64_t x;      // offset of the tensor (and of its slice 0 in A and C)
  int64_t NT;     // n1 * n2: elements per face slice
  int32_t P;      // face slices
  int32_t TP;     // tube positions per transform tile (power of two)
  int32_t lgTP;
  int32_t slice0; // index of its first slice in the slice table
  ModeTable fwd, inv;
};

// One transformed face slice.  Thin blocks are laid out for the plan's
// maximum width lmax; a slice uses the first l columns.
struct SliceDesc {
  int64_t a;   // offset of the n1 x n2 slice in A and C (elements)
  int64_t y;   // offset of its n1 x lmax block in Y and QK
  int64_t z;   // offset of its n2 x lmax block in Omega and Z
  int64_t kq;  // offset of its lmax x lmax block in K
  int64_t g1;  // offset (doubles) of its product Gram partials (ceil(max(n1,n2)/64) tiles)
  int64_t g2;  // offset (doubles) of its basis Gram partials (ceil(n1/64) tiles)
  int32_t n1, n2;
  int32_t l, k;     // sketch width and number of kept singular values
  int32_t tensor;   // index of the tensor (the Philox stream word is stream_base + tensor)
  int32_t local;    // slice index within the tensor (the Philox counter word)
  int32_t p;        // oversampling of the tensor (learned widths)
  int32_t pad;
};

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
