// Shared host/device helpers of the htsvt library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "htsvt.h"

namespace ht {

void set_error(const std::string& msg);

#define HT_CHECK_HIP(expr)                                                         \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::ht::set_error(std::string(#expr) + " failed: " + hipGetErrorString(e_));   \
      return HT_ERR_HIP;                                                           \
    }                                                                              \
  } while (0)

#define HT_CHECK_LAUNCH()                                                          \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess) {                                                        \
      ::ht::set_error(std::string("kernel launch failed: ") + hipGetErrorString(e_)); \
      return HT_ERR_HIP;                                                           \
    }                                                                              \
  } while (0)

#define HT_FAIL(code, msg)        \
  do {                            \
    ::ht::set_error(msg);         \
    return (code);                \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Penalty as seen by the kernels.
struct Penalty {
  int kind;
  double p0, p1;
};

// Scalars the solver keeps on the device so that an iteration reads them
// from memory (mu drives tau = 1/mu and the sketch key is the iteration).
struct AdmmState {
  double mu;
  int32_t iteration;
  int32_t pad0;
  double dL, dE, resid;                       // stopping terms of the last iteration
  unsigned long long red_dL, red_dE, red_res;  // running max (bit patterns of non-negative doubles; NaN is largest)
  double rse;                                  // recovery error against the registered truth (NaN if none)
};

}  // namespace ht
