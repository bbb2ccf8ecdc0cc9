// Device-side building blocks: the counter-based Gaussian generator and the
// scalar proximity operators.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace ht {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplies with the Weyl key schedule.  Counter and key are updated in place.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    const uint32_t hi0 = __umulhi(m0, c[0]), lo0 = m0 * c[0];
    const uint32_t hi1 = __umulhi(m1, c[2]), lo1 = m1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Four N(0,1) draws of group g of key (slice, call, stream, seed): uniforms
// (x + 1/2) 2^-32 from each word, Box-Muller on the pairs (w0, w1), (w2, w3).
__device__ __forceinline__ void gaussian4(uint64_t g, uint32_t slice, uint32_t call, uint32_t stream,
                                          uint64_t seed, double z[4]) {
  uint32_t c[4] = {(uint32_t)g, slice, call, stream};
  philox4x32_10(c, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
  const double s = 1.0 / 4294967296.0;
  const double two_pi = 6.283185307179586;
  double u0 = ((double)c[0] + 0.5) * s, u1 = ((double)c[1] + 0.5) * s;
  double u2 = ((double)c[2] + 0.5) * s, u3 = ((double)c[3] + 0.5) * s;
  double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
  double s1, c1, s3, c3;
  sincos(two_pi * u1, &s1, &c1);
  sincos(two_pi * u3, &s3, &c3);
  z[0] = r01 * c1;
  z[1] = r01 * s1;
  z[2] = r23 * c3;
  z[3] = r23 * s3;
}

// FP32 -> BF16 bits, round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Two FP32 values -> packed BF16 bits (low half: a), round to nearest even, on
// the hardware conversion.
__device__ __forceinline__ uint32_t f32x2_to_bf16x2(float a, float b) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 h2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2{a, b}, h2));
}

// ---------------------------------------------------------------------------
// Penalties and their proximity operators, for v >= 0 (callers pass |v| and
// restore the sign).  Prox_{phi,mu}(v) = argmin_x mu phi(x) + (x - v)^2 / 2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pen_value(const Penalty& p, double x) {
  switch (p.kind) {
    case HT_PEN_L1:
      return x;
    case HT_PEN_MCP:
      return x <= p.p0 ? x - x * x / (2.0 * p.p0) : 0.5 * p.p0;
    case HT_PEN_SCAD: {
      const double a = p.p0, b = p.p1;
      if (x <= b) return x;
      if (x <= a * b) return (2.0 * a * b * x - x * x - b * b) / (2.0 * (a - 1.0) * b);
      return 0.5 * (a + 1.0) * b;
    }
    case HT_PEN_LOG:
      return log1p(x / p.p0);
    default:  // HT_PEN_CAPPED_L1 (FIRM has its closed-form prox and never gets here)
      return fmin(x, p.p0);
  }
}

__device__ __forceinline__ double prox_obj(const Penalty& p, double mu, double v, double x) {
  const double d = x - v;
  return mu * pen_value(p, x) + 0.5 * d * d;
}

// Keep the candidate with the strictly lower objective; on ties the smaller x.
__device__ __forceinline__ void prox_consider(const Penalty& p, double mu, double v, double x,
                                              double& best_x, double& best_f) {
  const double f = prox_obj(p, mu, v, x);
  if (f < best_f || (f == best_f && x < best_x)) {
    best_x = x;
    best_f = f;
  }
}

__device__ inline double prox_pos(const Penalty& p, double v, double mu) {
  if (!(mu > 0.0)) return v;
  switch (p.kind) {
    case HT_PEN_L1:
      return v > mu ? v - mu : 0.0;
    case HT_PEN_MCP: {
      const double g = p.p0;
      if (g > mu) {  // firm shrinkage with thresholds (mu, g)
        if (v <= mu) return 0.0;
        if (v <= g) return g * (v - mu) / (g - mu);
        return v;
      }
      return v > sqrt(g * mu) ? v : 0.0;  // hard threshold
    }
    case HT_PEN_SCAD: {
      const double a = p.p0, b = p.p1;
      double bx = 0.0, bf = prox_obj(p, mu, v, 0.0);
      prox_consider(p, mu, v, fmin(fmax(v - mu, 0.0), b), bx, bf);
      const double den = 1.0 - mu / ((a - 1.0) * b);
      if (den != 0.0) {
        double x = (v - mu * a / (a - 1.0)) / den;
        prox_consider(p, mu, v, fmin(fmax(x, b), a * b), bx, bf);
      }
      prox_consider(p, mu, v, b, bx, bf);
      prox_consider(p, mu, v, a * b, bx, bf);
      prox_consider(p, mu, v, fmax(v, a * b), bx, bf);
      return bx;
    }
    case HT_PEN_FIRM: {  // firm shrinkage with thresholds (mu, a mu), a = p0 > 1
      const double a = p.p0;
      if (v <= mu) return 0.0;
      if (v <= a * mu) return a * (v - mu) / (a - 1.0);
      return v;
    }
    case HT_PEN_LOG: {
      const double e = p.p0;
      double bx = 0.0, bf = prox_obj(p, mu, v, 0.0);
      const double disc = (v + e) * (v + e) - 4.0 * mu;
      if (disc >= 0.0) {
        const double x = 0.5 * ((v - e) + sqrt(disc));  // the local minimizer branch
        if (x > 0.0) prox_consider(p, mu, v, x, bx, bf);
      }
      return bx;
    }
    default: {  // capped-l1
      const double t = p.p0;
      double bx = 0.0, bf = prox_obj(p, mu, v, 0.0);
      prox_consider(p, mu, v, fmin(fmax(v - mu, 0.0), t), bx, bf);
      prox_consider(p, mu, v, fmax(v, t), bx, bf);
      return bx;
    }
  }
}

// Zero threshold of the proximity operator: t0 = sup{v >= 0 : Prox_{phi,mu}(v) = 0}
// (the operator is nondecreasing, so every v <= t0 maps to 0 and every v > t0
// to a positive value).  Closed forms where the prox has one (L1, FIRM: mu;
// MCP: mu for gamma > mu, else sqrt(gamma mu); capped-L1: min(mu, sqrt(2 mu
// theta))), bisection on prox_pos itself otherwise (SCAD, LOG).
__device__ inline double prox_zero_threshold(const Penalty& p, double mu) {
  if (!(mu > 0.0)) return 0.0;
  switch (p.kind) {
    case HT_PEN_L1:
    case HT_PEN_FIRM:
      return mu;
    case HT_PEN_MCP:
      return p.p0 > mu ? mu : sqrt(p.p0 * mu);
    case HT_PEN_CAPPED_L1:
      return fmin(mu, sqrt(2.0 * mu * p.p0));
    default: {
      double lo = 0.0, hi = mu;
      for (int i = 0; i < 64 && prox_pos(p, hi, mu) == 0.0; ++i) {
        lo = hi;
        hi *= 2.0;
      }
      for (int i = 0; i < 80; ++i) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (prox_pos(p, mid, mu) == 0.0)
          lo = mid;
        else
          hi = mid;
      }
      return lo;
    }
  }
}

__device__ __forceinline__ double prox_signed(const Penalty& p, double v, double mu) {
  const double r = prox_pos(p, fabs(v), mu);
  return v < 0.0 ? -r : r;
}

}  // namespace ht
