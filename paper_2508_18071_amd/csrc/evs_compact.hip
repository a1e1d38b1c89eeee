// Dense spike frames -> event list (t, x, y, channel, polarity), in
// (t, channel, y, x) order (the event tuple of arXiv 2508.18071, Sec. 3.1).
//
// The dense int8 array is cut into chunks of one (t, channel) plane each.
// Pass 1 counts the non-zero spikes of every chunk; pass 2 turns the counts
// into output offsets (exclusive scan in one workgroup); pass 3 re-reads the
// chunk and writes each event at its offset.  Inside a chunk, each lane
// reads 4 consecutive spikes per round; the lane's exclusive offset inside
// the wave comes from three ballots of the bit planes of its count (0..4)
// with mbcnt, and wave totals are scanned in LDS, so the output order is
// the dense order without any sort and the result is deterministic.
#include "evs_ops.hpp"

namespace evs {
namespace {

constexpr int kThreads = 256;            // 4 waves
constexpr int kRounds = 16;              // rounds of 4 x 256 spikes per chunk
constexpr int kChunk = kThreads * 4 * kRounds;   // 16384 spikes per workgroup

__device__ inline unsigned lane_prefix(unsigned long long mask) {
  // number of lanes below this one whose bit is set in mask
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ inline unsigned nz_bytes(unsigned w) {
  // one bit per non-zero byte of w (bits 0, 8, 16, 24 -> 0..3)
  unsigned m = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) m |= (((w >> (8 * b)) & 0xffu) ? 1u : 0u) << b;
  return m;
}

template <bool WRITE>
__global__ __launch_bounds__(kThreads) void k_compact(const int8_t* __restrict__ s, int HW, int W,
                                                      int chunks_per_plane, int C,
                                                      int32_t* __restrict__ counts,
                                                      const long long* __restrict__ offsets,
                                                      uint64_t* __restrict__ events, long long cap) {
  const int chunk = blockIdx.x;                 // chunk within the plane
  const long long plane = blockIdx.y;           // t * C + c
  const int t = (int)(plane / C), c = (int)(plane - (long long)t * C);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int8_t* base = s + plane * HW;
  const long long block_id = plane * chunks_per_plane + chunk;
  __shared__ int wave_tot[4];
  __shared__ int wave_off[4];
  long long run = WRITE ? offsets[block_id] : 0;
  int total = 0;
  const bool vec = (HW & 3) == 0;
  for (int r = 0; r < kRounds; ++r) {
    const int p0 = chunk * kChunk + r * (kThreads * 4) + 4 * threadIdx.x;   // first of 4 spikes
    unsigned w = 0;
    if (vec && p0 + 3 < HW) {
      w = *reinterpret_cast<const unsigned*>(base + p0);
    } else {
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (p0 + b < HW) w |= ((unsigned)(uint8_t)base[p0 + b]) << (8 * b);
    }
    const unsigned nzm = nz_bytes(w);
    const unsigned cnt = __builtin_popcount(nzm);
    const unsigned long long b0 = __ballot(cnt & 1u), b1 = __ballot(cnt & 2u), b2 = __ballot(cnt & 4u);
    const unsigned pre = lane_prefix(b0) + 2u * lane_prefix(b1) + 4u * lane_prefix(b2);
    const int wt = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
    if (lane == 0) wave_tot[wave] = wt;
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = 0;
      for (int k = 0; k < 4; ++k) { wave_off[k] = acc; acc += wave_tot[k]; }
      wave_tot[0] = acc;      // round total (read after the next barrier)
    }
    __syncthreads();
    const int round_total = wave_tot[0];
    if (WRITE) {
      long long o = run + wave_off[wave] + pre;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if ((nzm >> b) & 1u) {
          const int p = p0 + b;
          const int y = p / W, x = p - y * W;
          const int8_t v = (int8_t)((w >> (8 * b)) & 0xffu);
          const uint64_t ev = (uint64_t)(uint32_t)t | ((uint64_t)x << 32) | ((uint64_t)y << 44) |
                              ((uint64_t)c << 56) | ((uint64_t)(v < 0 ? 1u : 0u) << 63);
          if (o < cap) events[o] = ev;
          ++o;
        }
      }
    }
    run += round_total;
    total += round_total;
    __syncthreads();          // wave_tot/wave_off reused next round
  }
  if (!WRITE && threadIdx.x == 0) counts[block_id] = total;
}

// Exclusive scan of the chunk counts in one workgroup (fixed order); the
// grand total goes to *count.
__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ counts, long long n,
                                               long long* __restrict__ offsets, int64_t* __restrict__ count) {
  __shared__ long long part[1024];
  const long long per = (n + 1023) / 1024;
  const long long b = threadIdx.x * per;
  long long acc = 0;
  for (long long i = b; i < b + per && i < n; ++i) acc += counts[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long run = 0;
    for (int k = 0; k < 1024; ++k) { const long long v = part[k]; part[k] = run; run += v; }
    count[0] = run;
  }
  __syncthreads();
  long long run = part[threadIdx.x];
  for (long long i = b; i < b + per && i < n; ++i) { offsets[i] = run; run += counts[i]; }
}

}  // namespace

size_t compact_workspace_bytes(int T, int C, int H, int W) {
  const long long HW = (long long)H * W;
  const long long cpp = (HW + kChunk - 1) / kChunk;
  const long long blocks = cpp * T * C;
  return align256((size_t)blocks * 4) + align256((size_t)blocks * 8);
}

int compact_events(const int8_t* s, int T, int C, int H, int W, uint64_t* events, int64_t cap,
                   int64_t* count, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!s || !count || (cap > 0 && !events)) return fail(EVS_EINVAL, "compact_events: NULL pointer");
  if (T < 1 || C < 1 || H < 1 || W < 1 || cap < 0) return fail(EVS_EINVAL, "compact_events: bad sizes");
  if (W > 4096 || H > 4096 || C > 128) return fail(EVS_EOVERFLOW, "compact_events: x/y/channel field overflow");
  const long long HW = (long long)H * W;
  const long long cpp = (HW + kChunk - 1) / kChunk;
  const long long planes = (long long)T * C;
  if (planes > 65535 * 1024LL) return fail(EVS_EOVERFLOW, "compact_events: too many frames");
  const size_t need = compact_workspace_bytes(T, C, H, W);
  if (!ws || ws_bytes < need) return fail(EVS_EWORKSPACE, "compact_events: workspace too small");
  int32_t* counts = reinterpret_cast<int32_t*>(ws);
  long long* offsets = reinterpret_cast<long long*>(reinterpret_cast<char*>(ws) + align256((size_t)cpp * planes * 4));
  // grid.y holds the (t, c) planes; split across z only if the y limit is exceeded
  if (planes > 65535) return fail(EVS_EUNSUPPORTED, "compact_events: more than 65535 (t, c) planes per call");
  dim3 grid((unsigned)cpp, (unsigned)planes);
  hipLaunchKernelGGL(k_compact<false>, grid, dim3(kThreads), 0, st, s, (int)HW, W, (int)cpp, C, counts,
                     (const long long*)nullptr, (uint64_t*)nullptr, 0LL);
  EVS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, counts, cpp * planes, offsets, count);
  EVS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_compact<true>, grid, dim3(kThreads), 0, st, s, (int)HW, W, (int)cpp, C, counts,
                     offsets, events, (long long)cap);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}

}  // namespace evs
