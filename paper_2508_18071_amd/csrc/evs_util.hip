// Small fill / copy kernels.  Fills are kernels rather than hipMemsetAsync so
// that a captured graph replays them correctly.
#include "evs_ops.hpp"

namespace evs {
namespace {

__global__ void k_fill_i32(int32_t* p, size_t n, int32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f32(float* p, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_copy_f32(float* d, const float* s, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) d[i] = s[i];
}

unsigned grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  return (unsigned)(g < 4096 ? (g ? g : 1) : 4096);
}

}  // namespace

int zero_i32(int32_t* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, n, 0);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}
int zero_f32(float* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(256), 0, s, p, n, 0.f);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}
int copy_f32(float* d, const float* src, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(n)), dim3(256), 0, s, d, src, n);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}

}  // namespace evs

namespace evs {
namespace {
__global__ void k_fill_hash(float* p, size_t n, uint32_t seed, float lo, float hi) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ seed;
    h ^= h >> 16; h *= 0x7feb352du; h ^= h >> 15; h *= 0x846ca68bu; h ^= h >> 16;
    p[i] = lo + (hi - lo) * ((float)(h >> 8) * (1.0f / 16777216.0f));
  }
}
}  // namespace

int fill_uniform(float* p, size_t n, uint32_t seed, float lo, float hi, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_hash, dim3(grid_for(n)), dim3(256), 0, s, p, n, seed, lo, hi);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}
}  // namespace evs

namespace evs {
namespace {
// Adds n to a status-word counter, saturating at INT32_MAX.
__device__ inline void sat_add(int32_t* word, unsigned n) {
  int old = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const int nv = (unsigned)old + n > 0x7fffffffu ? 0x7fffffff : old + (int)n;
    const int prev = atomicCAS(word, old, nv);
    if (prev == old) return;
    old = prev;
  }
}

// NaN values among p[0, n): 16-byte loads over the aligned body (vec), one
// count per workgroup added to *word.  With range > 0, any value with
// |v| >= range (infinities included) also sets `flag` in *flags.
__global__ __launch_bounds__(256) void k_count_nan(const float* __restrict__ p, size_t n, int vec,
                                                   int32_t* __restrict__ word, float range,
                                                   int32_t* __restrict__ flags, int flag) {
  unsigned c = 0, big = 0;
  const float lim = range > 0.f ? range : __builtin_inff();
  auto out = [&](float v) __attribute__((always_inline)) { return __builtin_fabsf(v) >= lim ? 1u : 0u; };
  const size_t stride = (size_t)gridDim.x * 256;
  size_t i0 = blockIdx.x * (size_t)256 + threadIdx.x;
  size_t body = 0;
  if (vec) {
    body = n / 4;
    const float4* q = reinterpret_cast<const float4*>(p);
    for (size_t i = i0; i < body; i += stride) {
      const float4 v = q[i];
      c += (v.x != v.x) + (v.y != v.y) + (v.z != v.z) + (v.w != v.w);
      big |= out(v.x) | out(v.y) | out(v.z) | out(v.w);
    }
    body *= 4;
  }
  for (size_t i = body + i0; i < n; i += stride) {
    c += p[i] != p[i];
    big |= out(p[i]);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
  const bool any_big = __builtin_amdgcn_ballot_w64(big != 0u) != 0ull;
  __shared__ unsigned part[4], bigw[4];
  if ((threadIdx.x & 63) == 0) {
    part[threadIdx.x >> 6] = c;
    bigw[threadIdx.x >> 6] = any_big ? 1u : 0u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned tot = part[0] + part[1] + part[2] + part[3];
    if (tot) sat_add(word, tot);
    if (range > 0.f && (bigw[0] | bigw[1] | bigw[2] | bigw[3])) atomicOr(flags, flag);
  }
}
}  // namespace

int count_nan(const float* p, size_t n, int32_t* word, hipStream_t s, float range, int32_t* flags, int flag) {
  if (n == 0) return EVS_OK;
  const int vec = (reinterpret_cast<uintptr_t>(p) & 15) == 0 ? 1 : 0;
  size_t g = (n + 256 * 16 - 1) / (256 * 16);
  g = g < 2048 ? (g ? g : 1) : 2048;
  hipLaunchKernelGGL(k_count_nan, dim3((unsigned)g), dim3(256), 0, s, p, n, vec, word, range, flags, flag);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}
}  // namespace evs
