// Dense spike frames -> event list (t, x, y, channel, polarity), in
// (t, channel, y, x) order (the event tuple of arXiv 2508.18071, Sec. 3.1).
//
// The dense int8 array is cut into chunks of one (t, channel) plane each.
// Pass 1 counts the non-zero spikes of every chunk; pass 2 turns the counts
// into output offsets (exclusive scan in two levels: blocks of 1024 chunk
// counts, then the block totals); pass 3 re-reads the
// chunk and writes its events at that offset.  In pass 3 each lane loads 16
// consecutive spikes per round; its exclusive offset inside the wave comes
// from five ballots of the bit planes of its count (0..16) with mbcnt, the
// wave totals are scanned in LDS, the round's events are gathered in LDS in
// dense order and then written out by all lanes as one contiguous run of
// 8-byte stores.  No sort is needed and the result is deterministic.
#include "evs_ops.hpp"

namespace evs {
namespace {

constexpr int kThreads = 256;                    // 4 waves
constexpr int kSpl = 16;                         // spikes per lane and round (one 16-byte load)
constexpr int kRound = kThreads * kSpl;          // 4096 spikes per round
constexpr int kRounds = 4;
constexpr int kChunk = kRound * kRounds;         // 16384 spikes per workgroup
constexpr int kScanB = 1024;                     // chunk counts per block of the offset scan

__device__ inline unsigned lane_prefix(unsigned long long mask) {
  // number of lanes below this one whose bit is set in mask
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// bit 8k+7 set for every non-zero byte k of w
__device__ inline unsigned nz_hi(unsigned w) { return (((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w) & 0x80808080u; }

// spikes p0 .. p0+15 of a plane (zero past its end)
__device__ inline uint4 load16(const int8_t* base, int p0, int HW, bool vec) {
  if (vec && p0 + 15 < HW) return *reinterpret_cast<const uint4*>(base + p0);
  unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int b = 0; b < 16; ++b)
    if (p0 + b < HW) w[b >> 2] |= ((unsigned)(uint8_t)base[p0 + b]) << (8 * (b & 3));
  return uint4{w[0], w[1], w[2], w[3]};
}

__device__ inline int count16(uint4 v) {
  return __builtin_popcount(nz_hi(v.x)) + __builtin_popcount(nz_hi(v.y)) + __builtin_popcount(nz_hi(v.z)) +
         __builtin_popcount(nz_hi(v.w));
}

// pass 1: non-zero spikes of every chunk
__global__ __launch_bounds__(kThreads) void k_count(const int8_t* __restrict__ s, int HW, int chunks_per_plane,
                                                    int vec, int32_t* __restrict__ counts) {
  const int chunk = blockIdx.x;
  const long long plane = blockIdx.y;
  const int8_t* base = s + plane * HW;
  int n = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r)
    n += count16(load16(base, chunk * kChunk + r * kRound + kSpl * threadIdx.x, HW, vec != 0));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) n += __shfl_xor(n, off);
  __shared__ int wsum[4];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) counts[plane * chunks_per_plane + chunk] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// pass 3: events of every chunk at its offset
__global__ __launch_bounds__(kThreads) void k_write(const int8_t* __restrict__ s, int HW, int W,
                                                    int chunks_per_plane, int C, int vec,
                                                    const long long* __restrict__ offsets,
                                                    const long long* __restrict__ boff,
                                                    uint64_t* __restrict__ events, long long cap) {
  const int chunk = blockIdx.x;
  const long long plane = blockIdx.y;            // t * C + c
  const int t = (int)(plane / C), c = (int)(plane - (long long)t * C);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int8_t* base = s + plane * HW;
  __shared__ uint2 stage[kRound];                // the round's events, dense order
  __shared__ int wave_tot[4];
  __shared__ int wave_off[5];
  const long long idx = plane * chunks_per_plane + chunk;
  long long run = offsets[idx] + boff[idx / kScanB];
  for (int r = 0; r < kRounds; ++r) {
    const int p0 = chunk * kChunk + r * kRound + kSpl * threadIdx.x;
    const uint4 v = load16(base, p0, HW, vec != 0);
    const unsigned cnt = (unsigned)count16(v);
    const unsigned long long b0 = __ballot(cnt & 1u), b1 = __ballot(cnt & 2u), b2 = __ballot(cnt & 4u),
                             b3 = __ballot(cnt & 8u), b4 = __ballot(cnt & 16u);
    const unsigned pre = lane_prefix(b0) + 2u * lane_prefix(b1) + 4u * lane_prefix(b2) + 8u * lane_prefix(b3) +
                         16u * lane_prefix(b4);
    if (lane == 0)
      wave_tot[wave] = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2) + 8 * __popcll(b3) + 16 * __popcll(b4);
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = 0;
      for (int k = 0; k < 4; ++k) { wave_off[k] = acc; acc += wave_tot[k]; }
      wave_off[4] = acc;                           // round total
    }
    __syncthreads();
    const int total = wave_off[4];
    if (cnt) {
      int slot = wave_off[wave] + (int)pre;
      int y = p0 / W, x = p0 - y * W;
      const unsigned ww[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int b = 0; b < kSpl; ++b) {
        const unsigned byte = (ww[b >> 2] >> (8 * (b & 3))) & 0xffu;
        if (byte) {
          const unsigned neg = byte >> 7;          // -1 is 0xff
          stage[slot++] = uint2{(unsigned)t, (unsigned)x | ((unsigned)y << 12) | ((unsigned)c << 24) | (neg << 31)};
        }
        if (++x == W) { x = 0; ++y; }
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < total; i += kThreads) {
      const long long o = run + i;
      if (o < cap) reinterpret_cast<uint2*>(events)[o] = stage[i];
    }
    run += total;
    __syncthreads();                               // stage and wave_off reused next round
  }
}

// Exclusive scan of the chunk counts in two levels (integer sums: the
// result does not depend on the order).  Level 1: blocks of kScanB counts
// scanned in one workgroup each (wave scans by shuffles, then the wave
// totals), offsets relative to the block and the block totals.  Level 2:
// the block totals scanned in place by one workgroup; the grand total goes
// to *count, and a total above the capacity sets the overflow flag of the
// status word (if given).  k_write adds the two levels.
__global__ __launch_bounds__(kScanB) void k_scan_local(const int32_t* __restrict__ counts, long long n,
                                                       long long* __restrict__ offsets, long long* __restrict__ btot) {
  __shared__ int wsum[kScanB / 64];
  const long long i = (long long)blockIdx.x * kScanB + threadIdx.x;
  const int v = i < n ? counts[i] : 0;                 // <= kChunk: block sums fit in 32 bits
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(inc, off);
    if (lane >= off) inc += u;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int r = 0;
    for (int k = 0; k < kScanB / 64; ++k) { const int t = wsum[k]; wsum[k] = r; r += t; }
    btot[blockIdx.x] = r;
  }
  __syncthreads();
  if (i < n) offsets[i] = (long long)(wsum[wave] + inc - v);
}

__global__ __launch_bounds__(1024) void k_scan_top(long long* __restrict__ btot, long long nb,
                                                   int64_t* __restrict__ count, long long cap,
                                                   int32_t* __restrict__ status) {
  __shared__ long long part[1024];
  const long long per = (nb + 1023) / 1024;
  const long long b = threadIdx.x * per;
  long long acc = 0;
  for (long long k = b; k < b + per && k < nb; ++k) acc += btot[k];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long run = 0;
    for (int k = 0; k < 1024; ++k) { const long long v = part[k]; part[k] = run; run += v; }
    count[0] = run;
    if (status && run > cap) atomicOr(status + EVS_STATUS_FLAGS, EVS_FLAG_EVENT_OVERFLOW);
  }
  __syncthreads();
  long long run = part[threadIdx.x];
  for (long long k = b; k < b + per && k < nb; ++k) {
    const long long t = btot[k];
    btot[k] = run;
    run += t;
  }
}

}  // namespace

size_t compact_workspace_bytes(int T, int C, int H, int W) {
  const long long HW = (long long)H * W;
  const long long cpp = (HW + kChunk - 1) / kChunk;
  const long long blocks = cpp * T * C;
  const long long nb = (blocks + kScanB - 1) / kScanB;
  return align256((size_t)blocks * 4) + align256((size_t)blocks * 8) + align256((size_t)nb * 8);
}

int compact_events(const int8_t* s, int T, int C, int H, int W, uint64_t* events, int64_t cap,
                   int64_t* count, void* ws, size_t ws_bytes, int32_t* status, hipStream_t st) {
  if (!s || !count || (cap > 0 && !events)) return fail(EVS_EINVAL, "compact_events: NULL pointer");
  if (T < 1 || C < 1 || H < 1 || W < 1 || cap < 0) return fail(EVS_EINVAL, "compact_events: bad sizes");
  if (W > 4096 || H > 4096 || C > 128) return fail(EVS_EOVERFLOW, "compact_events: x/y/channel field overflow");
  if ((reinterpret_cast<uintptr_t>(status) & 3u) != 0)
    return fail(EVS_EINVAL, "compact_events: dev_status must be 4-byte aligned");
  const long long HW = (long long)H * W;
  const long long cpp = (HW + kChunk - 1) / kChunk;
  const long long planes = (long long)T * C;
  if (planes > 65535 * 1024LL) return fail(EVS_EOVERFLOW, "compact_events: too many frames");
  const size_t need = compact_workspace_bytes(T, C, H, W);
  if (!ws || ws_bytes < need) return fail(EVS_EWORKSPACE, "compact_events: workspace too small");
  int32_t* counts = reinterpret_cast<int32_t*>(ws);
  long long* offsets = reinterpret_cast<long long*>(reinterpret_cast<char*>(ws) + align256((size_t)cpp * planes * 4));
  const long long n = cpp * planes, nb = (n + kScanB - 1) / kScanB;
  long long* boff = reinterpret_cast<long long*>(reinterpret_cast<char*>(offsets) + align256((size_t)n * 8));
  // grid.y holds the (t, c) planes; split across z only if the y limit is exceeded
  if (planes > 65535) return fail(EVS_EUNSUPPORTED, "compact_events: more than 65535 (t, c) planes per call");
  dim3 grid((unsigned)cpp, (unsigned)planes);
  // 16-byte loads when every plane starts 16-byte aligned
  const int vec = ((reinterpret_cast<uintptr_t>(s) & 15) == 0 && (HW & 15) == 0) ? 1 : 0;
  hipLaunchKernelGGL(k_count, grid, dim3(kThreads), 0, st, s, (int)HW, (int)cpp, vec, counts);
  EVS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanB), 0, st, counts, n, offsets, boff);
  EVS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, boff, nb, count, (long long)cap, status);
  EVS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_write, grid, dim3(kThreads), 0, st, s, (int)HW, W, (int)cpp, C, vec, offsets, boff, events,
                     (long long)cap);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}

}  // namespace evs
