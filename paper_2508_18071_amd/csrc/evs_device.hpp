// Device-side helpers shared by the forward and backward kernels, so that a
// recomputed spike is bit-identical to the one the forward emitted.
#pragma once

#include <hip/hip_runtime.h>

namespace evs {

__device__ inline float sigm_fast(float z) { return __frcp_rn(1.0f + __expf(-z)); }

// BiLIF fire + reset (Eq. 2-3): returns the spike and updates v in place (v
// holds the charged potential h on entry).  relaxed: the smooth spike
// sigma(alpha(h - theta)) - sigma(alpha(-h - theta)).
__device__ inline float bilif(float& v, float theta, float alpha, bool relaxed) {
  const float h = v;
  float s;
  if (relaxed) {
    s = sigm_fast(alpha * (h - theta)) - sigm_fast(alpha * (-h - theta));
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
__device__ inline float spike_of(float h, float theta, float alpha, bool relaxed) {
  float v = h;
  return bilif(v, theta, alpha, relaxed);
}

// Surrogate derivative of the spike (Eq. 4, sigmoid of slope alpha):
// psi(h) = sigma'(h - theta) + sigma'(-h - theta), sigma' = alpha s (1 - s).
__device__ inline float surrogate(float h, float theta, float alpha) {
  const float a = sigm_fast(alpha * (h - theta));
  const float b = sigm_fast(alpha * (-h - theta));
  return alpha * (a * (1.0f - a) + b * (1.0f - b));
}

}  // namespace evs
