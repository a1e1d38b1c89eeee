// Device-side helpers shared by the forward, backward and input kernels, so
// that a recomputed spike (or input) is bit-identical to the one the forward
// used.
#pragma once

#include <hip/hip_runtime.h>

namespace evs {

__device__ inline float sigm_fast(float z) { return __frcp_rn(1.0f + __expf(-z)); }

// Lin-log luminance of Eq. (1) (Sec. 3.2) of one linear RGB pixel:
// L = scale (0.2126 R + 0.7152 G + 0.0722 B), then ln L at and above the knee
// and toe * L below it (toe = ln(knee) / knee, so the branches meet).  Every
// operation is spelled out (no contraction), so the stand-alone input kernel
// and the forward's fused input staging compute identical bits.
__device__ inline float linlog_lum(float r, float g, float b, float scale, float knee, float toe) {
  const float L = __fmul_rn(scale, __fmaf_rn(0.0722f, b, __fmaf_rn(0.7152f, g, __fmul_rn(0.2126f, r))));
  return L >= knee ? logf(L) : __fmul_rn(toe, L);
}

// XCD-aware tile order: the hardware deals workgroups round-robin over the
// 8 XCDs; give each XCD a contiguous run of the n tiles so that the halo
// rows and the cache lines that neighbouring tiles share are fetched into the
// same L2 (a 16-pixel tile row is half a 128-byte line).  b is the block
// index in a grid dimension of n blocks, the dimension the hardware walks
// first; any n is a bijection.
__device__ inline int xcd_remap(int b, int n) {
  const int x = b & 7, k = b >> 3;
  const int q = n >> 3, r = n & 7;
  const int start = x * q + (x < r ? x : r);
  return start + k;
}

// Smooth step of the surrogate (Sec. 3.3, Eq. 4) and its slope.
//   kind 0: logistic sigmoid 1 / (1 + exp(-alpha z))
//   kind 1: arctangent 1/2 + arctan(pi/2 alpha z) / pi
__device__ inline float surr_step(float z, float alpha, int kind) {
  if (kind == 1) return 0.5f + atanf(1.57079633f * alpha * z) * 0.318309886f;
  return sigm_fast(alpha * z);
}
__device__ inline float surr_slope(float z, float alpha, int kind) {
  if (kind == 1) {
    const float q = 1.57079633f * alpha * z;
    return 0.5f * alpha / fmaf(q, q, 1.0f);
  }
  const float a = sigm_fast(alpha * z);
  return alpha * a * (1.0f - a);
}

// BiLIF fire + reset (Eq. 2-3): returns the spike and updates v in place (v
// holds the charged potential h on entry).  relaxed: 0 hard spikes; 1 or 2
// the smooth spike step(h - theta) - step(-h - theta) of the sigmoid (1) or
// arctangent (2) step.
__device__ inline float bilif(float& v, float theta, float alpha, int relaxed) {
  const float h = v;
  float s;
  if (relaxed) {
    s = surr_step(h - theta, alpha, relaxed - 1) - surr_step(-h - theta, alpha, relaxed - 1);
  } else {
    // h >= theta -> +1, h <= -theta -> -1, else 0 (theta > 0; a NaN h gives 0):
    // one compare of |h| and the sign of h copied onto 1.0
    const float sgn1 = __builtin_bit_cast(float, (__builtin_bit_cast(unsigned, h) & 0x80000000u) | 0x3f800000u);
    s = __builtin_fabsf(h) >= theta ? sgn1 : 0.0f;
  }
  v = fmaf(-theta, s, h);
  return s;
}

// The spike the forward emitted for the charged potential h.
__device__ inline float spike_of(float h, float theta, float alpha, int relaxed) {
  float v = h;
  return bilif(v, theta, alpha, relaxed);
}

// Surrogate derivative of the spike (Eq. 4):
// psi(h) = step'(h - theta) + step'(-h - theta), kind 0 sigmoid, 1 arctangent.
// Only gradients use it, so its exponential and reciprocals are the
// hardware's (within 1 ulp) rather than correctly rounded, in kernels where
// the vector ALU is shared with the matrix pipe.
//
// Sigmoid: the slope alpha sig(alpha z)(1 - sig(alpha z)) equals
// alpha e / (1 + e)^2 with e = exp(-alpha z), and psi is even in h.  With
// u = |h|, a = exp(alpha (theta - u)) and b = exp(-alpha (u + theta)) =
// a exp(-2 alpha theta), psi = alpha (a / (1+a)^2 + b / (1+b)^2): one
// exponential, and one reciprocal r of (1+a)(1+b), which gives
// 1/(1+a) = (1+b) r and 1/(1+b) = (1+a) r.  Since u >= 0, a <= exp(alpha
// theta) and b <= 1; the exponent is capped at 2^64 (it binds only where
// alpha (theta - u) > 44, where psi < alpha 2^-63), so (1+a)(1+b) stays
// finite for any theta and alpha.
__device__ inline float surrogate(float h, float theta, float alpha, int kind) {
  if (kind == 1) {
    const float qa = 1.57079633f * alpha * (h - theta), qb = 1.57079633f * alpha * (-h - theta);
    return 0.5f * alpha * (__builtin_amdgcn_rcpf(fmaf(qa, qa, 1.0f)) + __builtin_amdgcn_rcpf(fmaf(qb, qb, 1.0f)));
  }
  const float l2e = 1.44269504f;                       // log2(e)
  const float z = fminf(fmaf(__builtin_fabsf(h), -alpha * l2e, alpha * theta * l2e), 64.0f);
  const float a = __builtin_amdgcn_exp2f(z);
  const float b = a * __builtin_amdgcn_exp2f(-2.0f * alpha * theta * l2e);
  const float p = 1.0f + a, q = 1.0f + b;
  const float r = __builtin_amdgcn_rcpf(p * q);
  const float ip = q * r, iq = p * r;
  return alpha * fmaf(a * ip, ip, (b * iq) * iq);
}

}  // namespace evs
