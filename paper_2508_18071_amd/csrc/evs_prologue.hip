// Network input of Eq. (1) and contrast-crossing target events (arXiv
// 2508.18071, Sec. 3.2 and Sec. 3.1).
//
// Both are per-pixel scans over time: one thread owns one pixel of one clip
// and walks its frames in order, so every frame is read as coalesced rows
// and the running state (previous log level, event reference level) stays
// in a register.  HBM-bound.
#include <cmath>

#include "evs_device.hpp"
#include "evs_ops.hpp"

namespace evs {
namespace {

constexpr int kThreads = 256;

// lin-log luminance of Eq. (1) of the pixel at f (planes HW apart)
__device__ inline float linlog_at(const float* f, size_t HW, float scale, float knee, float toe) {
  return linlog_lum(f[0], f[HW], f[2 * HW], scale, knee, toe);
}

// x_out[n][k-1][0][p] = L_log[k] - L_log[k-1], k = 1..T, from frames 0..T
__global__ __launch_bounds__(kThreads) void k_logdiff(const float* __restrict__ rgb, int N, int T, long long HW,
                                                      float scale, float knee, float toe,
                                                      float* __restrict__ x_out) {
  const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= (long long)N * HW) return;
  const long long n = idx / HW, p = idx - n * HW;
  const float* f = rgb + (size_t)n * (T + 1) * 3 * HW + p;
  float* o = x_out + (size_t)n * T * HW + p;
  float prev = linlog_at(f, HW, scale, knee, toe);
  for (int k = 1; k <= T; ++k) {
    const float l = linlog_at(f + (size_t)k * 3 * HW, HW, scale, knee, toe);
    o[(size_t)(k - 1) * HW] = __fsub_rn(l, prev);
    prev = l;
  }
}

// ideal contrast camera: the reference starts at frame 0's level; at frame
// t >= 1, d = l - ref emits n = sgn(d) floor(|d| / C) events, ref += n C
__global__ __launch_bounds__(kThreads) void k_contrast(const float* __restrict__ rgb, int N, int T, long long HW,
                                                       float scale, float knee, float toe, float C,
                                                       int8_t* __restrict__ e_out) {
  const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= (long long)N * HW) return;
  const long long n = idx / HW, p = idx - n * HW;
  const float* f = rgb + (size_t)n * T * 3 * HW + p;
  int8_t* e = e_out + (size_t)n * T * 2 * HW + p;
  float ref = linlog_at(f, HW, scale, knee, toe);
  e[0] = 0;
  e[HW] = 0;
  for (int t = 1; t < T; ++t) {
    const float d = linlog_at(f + (size_t)t * 3 * HW, HW, scale, knee, toe) - ref;
    const float q = floorf(fabsf(d) / C);
    const float nev = d > 0.f ? q : (d < 0.f ? -q : 0.f);
    ref = fmaf(nev, C, ref);
    e[(size_t)t * 2 * HW] = (int8_t)fminf(fmaxf(nev, 0.f), 127.f);
    e[(size_t)t * 2 * HW + HW] = (int8_t)fminf(fmaxf(-nev, 0.f), 127.f);
  }
}

int check_prologue_args(const void* in, const void* out, int N, int T, int H, int W, float scale, float knee) {
  if (!in || !out) return fail(EVS_EINVAL, "NULL input or output");
  if (N < 1 || T < 1 || H < 1 || W < 1) return fail(EVS_EINVAL, "N, T, H, W must be >= 1");
  if (!(scale > 0.f) || !(knee > 0.f) || !(scale < 3.0e38f) || !(knee < 3.0e38f))
    return fail(EVS_EINVAL, "lum_scale and knee must be positive and finite");
  if ((double)N * (T + 1) * 3 * H * W > 9.0e18) return fail(EVS_EOVERFLOW, "input too large");
  if ((double)N * H * W > 2.0e9 * kThreads) return fail(EVS_EOVERFLOW, "too many pixels for one launch");
  return EVS_OK;
}

}  // namespace

int logdiff(const float* rgb, int N, int T, int H, int W, float scale, float knee, float* x_out, hipStream_t st) {
  int s = check_prologue_args(rgb, x_out, N, T, H, W, scale, knee);
  if (s) return s;
  const long long HW = (long long)H * W;
  const long long n = (long long)N * HW;
  const float toe = (float)(std::log((double)knee) / (double)knee);
  hipLaunchKernelGGL(k_logdiff, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, rgb, N, T,
                     HW, scale, knee, toe, x_out);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}

int contrast_events(const float* rgb, int N, int T, int H, int W, float scale, float knee, float C, int8_t* e_out,
                    hipStream_t st) {
  int s = check_prologue_args(rgb, e_out, N, T, H, W, scale, knee);
  if (s) return s;
  if (!(C > 0.f) || !(C < 3.0e38f)) return fail(EVS_EINVAL, "contrast threshold C must be positive and finite");
  const long long HW = (long long)H * W;
  const long long n = (long long)N * HW;
  const float toe = (float)(std::log((double)knee) / (double)knee);
  hipLaunchKernelGGL(k_contrast, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, rgb, N, T,
                     HW, scale, knee, toe, C, e_out);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}

}  // namespace evs
