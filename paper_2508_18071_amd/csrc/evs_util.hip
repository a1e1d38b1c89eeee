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
