// Bidirectional, polarity-split EMD loss with spike-count term and its
// (sub)gradient (arXiv 2508.18071, Sec. 3.3, Eq. 7-11).
//
// One thread owns one (clip, pixel) and both polarity sequences over time.
// With d_t = S_t - E_t, D_i = sum_{t<=i} d_t (prefix) and the suffix sums
// R_m = D_{T-1} - D_{m-1}, the loss of a sequence is (1/2T) sum_i |D_i| + |R_i|
// and its gradient is (1/2T) [ sum_{i>=j} sgn D_i + sum_{m<=j} sgn R_m ].
// Two streaming passes over time (totals and the sum of sgn D, then loss
// and gradient together) keep the per-thread state O(1) for any T; reads
// are coalesced across the pixel dimension.  Per-thread losses are summed
// in a fixed order (block tree, then one block over the partials), so the
// loss is reproducible.
#include <mutex>

#include "evs_ops.hpp"

namespace evs {
namespace {

constexpr int kThreads = 256;

__device__ inline float sgnf(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

// S^k_t for k = 0 (ON) / 1 (OFF)
__device__ inline float s_pol(const float* s, size_t off, int C, int k, size_t cstride) {
  if (C == 2) return s[off + k * cstride];
  const float v = s[off];
  return k == 0 ? (v > 0.f ? v : 0.f) : (v < 0.f ? -v : 0.f);
}

__global__ __launch_bounds__(kThreads) void k_emd(const float* __restrict__ s, const int8_t* __restrict__ e,
                                                 int N, int T, int C, int HW, float lambda,
                                                 float* __restrict__ grad, double* __restrict__ partial) {
  const long long gid = (long long)blockIdx.x * kThreads + threadIdx.x;
  const long long total_px = (long long)N * HW;
  double loss = 0.0;
  if (gid < total_px) {
    const int n = (int)(gid / HW);
    const int px = (int)(gid - (long long)n * HW);
    const size_t sfr = (size_t)C * HW, efr = (size_t)2 * HW;
    const size_t sbase = (size_t)n * T * sfr + px, ebase = (size_t)n * T * efr + px;
    const float inv2t = 0.5f / (float)T;
    // pass 1: totals per polarity, spike/target counts, and the sum of sgn D
    // over all frames (tot runs through the prefix sums D on the way)
    float tot[2] = {0.f, 0.f};
    float sumsgnD[2] = {0.f, 0.f};
    float cnt_s = 0.f, cnt_e = 0.f;
    // unrolled so that several frames' loads are in flight at once (one
    // thread per pixel: few waves per SIMD, so each thread's loads must
    // overlap; the sums keep their order)
#pragma unroll 8
    for (int t = 0; t < T; ++t) {
      for (int k = 0; k < 2; ++k) {
        const float sv = s_pol(s, sbase + t * sfr, C, k, HW);
        const float ev = (float)e[ebase + t * efr + k * HW];
        tot[k] += sv - ev;
        sumsgnD[k] += sgnf(tot[k]);
        cnt_s += fabsf(sv);
        cnt_e += ev;
      }
    }
    const float cdiff = cnt_s - cnt_e;
    // pass 2: loss (suffix sums R = total - prefix before the frame) and the
    // gradient, whose reverse sums of sgn D start at the total
    const float lam_sg = lambda * sgnf(cdiff);
    float Dp[2] = {0.f, 0.f};
    float revD[2] = {sumsgnD[0], sumsgnD[1]};     // sum_{i>=t} sgn D_i
    float fwdR[2] = {0.f, 0.f};                   // sum_{m<=t} sgn R_m
    double l = 0.0;
#pragma unroll 8
    for (int t = 0; t < T; ++t) {
      float g[2];
      for (int k = 0; k < 2; ++k) {
        const float sv = s_pol(s, sbase + t * sfr, C, k, HW);
        const float ev = (float)e[ebase + t * efr + k * HW];
        const float R = tot[k] - Dp[k];           // suffix sum from t
        Dp[k] += sv - ev;
        l += (double)fabsf(Dp[k]) + (double)fabsf(R);
        fwdR[k] += sgnf(R);
        g[k] = (revD[k] + fwdR[k]) * inv2t + lam_sg * sgnf(sv);
        revD[k] -= sgnf(Dp[k]);
      }
      if (grad) {
        if (C == 2) {
          grad[sbase + t * sfr] = g[0];
          grad[sbase + t * sfr + HW] = g[1];
        } else {
          const float v = s[sbase + t * sfr];
          // d/dS of the split parts: S+ = S [S>0], S- = -S [S<0]
          grad[sbase + t * sfr] = v > 0.f ? g[0] : (v < 0.f ? -g[1] : 0.f);
        }
      }
    }
    loss = l * (double)inv2t + (double)lambda * (double)fabsf(cdiff);
  }
  // fixed-order block reduction
  __shared__ double red[kThreads];
  red[threadIdx.x] = loss;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_reduce(const double* __restrict__ partial, int n, float* __restrict__ out) {
  __shared__ double red[1024];
  double acc = 0.0;
  // each thread sums a contiguous run, then a fixed tree
  const int per = (n + 1023) / 1024;
  const int b = threadIdx.x * per;
  for (int i = b; i < b + per && i < n; ++i) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)red[0];
}

}  // namespace

size_t emd_workspace_bytes(int N, int T, int C, int H, int W) {
  (void)T; (void)C;
  const long long px = (long long)N * H * W;
  const long long blocks = (px + kThreads - 1) / kThreads;
  return align256((size_t)blocks * sizeof(double));
}

namespace {

int emd_check(const float* s, const int8_t* e, int N, int T, int C, int H, int W, float lambda, float* loss) {
  if (!s || !e || !loss) return fail(EVS_EINVAL, "emd_loss: s, e and loss must be non-NULL");
  if (N < 1 || T < 1 || H < 1 || W < 1) return fail(EVS_EINVAL, "emd_loss: sizes must be >= 1");
  if (C != 1 && C != 2) return fail(EVS_EUNSUPPORTED, "emd_loss: C must be 1 or 2");
  if ((long long)H * W > (1LL << 30)) return fail(EVS_EOVERFLOW, "emd_loss: frame too large");
  if ((long long)N * H * W > (1LL << 38)) return fail(EVS_EOVERFLOW, "emd_loss: too many pixels");
  if (!(lambda >= 0.f)) return fail(EVS_EINVAL, "emd_loss: lambda must be >= 0");
  return EVS_OK;
}

int emd_launch(const float* s, const int8_t* e, int N, int T, int C, int H, int W, float lambda, float* loss,
               float* grad, double* partial, hipStream_t st) {
  const long long blocks = ((long long)N * H * W + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_emd, dim3((unsigned)blocks), dim3(kThreads), 0, st, s, e, N, T, C, H * W, lambda, grad,
                     partial);
  EVS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partial, (int)blocks, loss);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}

// Static scratch of the allocation-free entry point: the per-block partial
// losses, one double per 256 pixels of N x H x W, fully rewritten by every
// call (nothing has to start at zero).  Every GPU the library runs on holds
// its own copy until the process ends; calls that overlap on one GPU share
// it and race.
constexpr long long kScratchBlocks = 1 << 17;            // 1 MiB: N x H x W up to 2^25 pixels
static __device__ __align__(256) double scratch[kScratchBlocks];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices];

// This GPU's scratch array, looked up once per device with that device
// current (the array's name is a host-side stand-in, not a device address);
// nullptr with the message set on failure.
double* scratch_on_current_device() {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) {
    hip_check(err, "hipGetDevice");
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    fail(EVS_EUNSUPPORTED, "emd_loss_noalloc: device index above 63");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (err != hipSuccess) {
      hip_check(err, "hipGetSymbolAddress(scratch)");
      return nullptr;
    }
    if (!ptr) {
      fail(EVS_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
      return nullptr;
    }
    g_scratch_ptr[dev] = reinterpret_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

int emd_loss(const float* s, const int8_t* e, int N, int T, int C, int H, int W, float lambda,
             float* loss, float* grad, void* ws, size_t ws_bytes, hipStream_t st) {
  int rc = emd_check(s, e, N, T, C, H, W, lambda, loss);
  if (rc) return rc;
  const size_t need = emd_workspace_bytes(N, T, C, H, W);
  if (!ws || ws_bytes < need) return fail(EVS_EWORKSPACE, "emd_loss: workspace too small");
  return emd_launch(s, e, N, T, C, H, W, lambda, loss, grad, reinterpret_cast<double*>(ws), st);
}

int emd_loss_noalloc(const float* s, const int8_t* e, int N, int T, int C, int H, int W, float lambda, float* loss,
                     float* grad, hipStream_t st) {
  int rc = emd_check(s, e, N, T, C, H, W, lambda, loss);
  if (rc) return rc;
  if ((long long)N * H * W > kScratchBlocks * kThreads)
    return fail(EVS_EWORKSPACE, "emd_loss_noalloc: N x H x W above 2^25 pixels, the size of its static scratch "
                                "(evs_emd_loss takes a workspace of any size)");
  double* partial = scratch_on_current_device();
  if (!partial) return EVS_EHIP;
  return emd_launch(s, e, N, T, C, H, W, lambda, loss, grad, partial, st);
}

}  // namespace evs
