// The paper's temporal EvSNet on gfx950 (arXiv 2508.18071, Sec. 3.3,
// Eq. 5-6): per pixel, a kernel-7 Conv1d encoder h0 = ReLU(conv0 X),
// residual blocks h_i = ReLU(h_{i-1} + conv(ReLU(conv h_{i-1}))), i = 1..3,
// a point-wise projection to one value per frame and a BiLIF unit (Eq. 2-3).
//
// Dataflow: every pixel is independent, so one wave owns 16 pixels and
// streams their sequences through time; waves never synchronise.  A conv
// output frame is a 16 (channels) x 16 (pixels) MFMA tile with the pixels as
// the B/D columns, so lane (pixel j, lane group g) receives channels
// 4g .. 4g+3 of pixel j.  The K dimension (tap, channel) is ordered so that
// lane group g also supplies exactly those four channels of every tap to the
// next conv: no activation ever leaves the lane that produced it.  Each conv
// input is a ring of its last 7 frames in registers (7 slots of 4 bf16
// channels, plus an eighth slot mirroring the first, so that every pair of
// consecutive frames is one aligned 4-register B operand): the 7 taps are
// four 16x16x32 bf16 MFMAs over frame pairs, the last pair's second frame
// (the oldest one, about to be replaced) meeting zero weights.  Conv L
// produces frame s - 3(L+1) at step s, so it consumes the frame conv L-1
// produced in the same step; the step loop is unrolled by the ring period so
// every slot is a compile-time register.  Frames outside [0, T) are zero in
// every ring (the convs' zero padding).  Operands are bf16 (input, weights,
// stored activations), sums and biases FP32 (the biases enter as the MFMA
// accumulator), the BiLIF state FP32.
#include <hip/hip_runtime.h>

#include "evs_device.hpp"
#include "evs_ops.hpp"

namespace evs {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef unsigned u16 __attribute__((ext_vector_type(16)));

constexpr int kC = 16;                 // hidden width
constexpr int kTaps = 7;               // kernel size of every encoder conv
constexpr int kConvs = 7;              // conv0 + 2 per residual block
constexpr int kRing = 7;               // frames per ring (= taps)
constexpr int kDelay = 3;              // frames of delay added per conv
constexpr int kLag = kDelay * kConvs;  // frame lag of the projection and BiLIF
constexpr int kNW = 4;                 // waves per workgroup
constexpr int kDbgCh = 7 * kC + 2;     // channels of one debug frame

constexpr int mod7(int a) { return ((a % kRing) + kRing) % kRing; }

typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
// round to bf16 (nearest even) in hardware: two values packed low, high
__device__ inline unsigned pack2(float lo, float hi) {
  const bf2 p = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(unsigned, p);
}
// ReLU of two packed bf16 values (rounding keeps the sign, so this equals
// rounding the ReLU): a signed 16-bit max with 0 clears every negative half.
// The empty asm only pins the packed value: without it the conversion is
// split into one conversion per value plus a permute, and the integer max of
// a bit-cast float followed by a bf16 conversion is miscompiled by this clang
// (only element 0 of the vector is converted).  fmaxf would cost an extra
// canonicalising max per value.
typedef short s2 __attribute__((ext_vector_type(2)));
__device__ inline unsigned relu2(unsigned p) {
  asm("" : "+v"(p));
  return __builtin_bit_cast(unsigned, __builtin_elementwise_max(__builtin_bit_cast(s2, p), s2{0, 0}));
}
__device__ inline float lo_bf16(unsigned u) { return __builtin_bit_cast(float, u << 16); }
__device__ inline float hi_bf16(unsigned u) { return __builtin_bit_cast(float, u & 0xffff0000u); }

__device__ inline f4 mfma32(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// Ring slot K (compile time): frames f with f mod 7 == K; slot 7 mirrors 0.
template <int K>
__device__ __forceinline__ u4 ring_pair(const u16& r) {
  return __builtin_shufflevector(r, r, 2 * K, 2 * K + 1, 2 * K + 2, 2 * K + 3);
}
template <int K>
__device__ __forceinline__ u2 ring_slot(const u16& r) {
  return __builtin_shufflevector(r, r, 2 * K, 2 * K + 1);
}
template <int K>
__device__ __forceinline__ void ring_put(u16& r, u2 v) {
  r[2 * K] = v.x;
  r[2 * K + 1] = v.y;
  if constexpr (K == 0) {
    r[2 * kRing] = v.x;
    r[2 * kRing + 1] = v.y;
  }
}

// Offsets of the layers in the flat weight array (see evs.h).
__host__ __device__ constexpr int w_conv_off(int L) {     // weights of conv L >= 1
  return kC * kTaps + kC + (L - 1) * (kC * kC * kTaps + kC);
}
__host__ __device__ constexpr int w_bias_off(int L) {
  return L == 0 ? kC * kTaps : w_conv_off(L) + kC * kC * kTaps;
}
__host__ __device__ constexpr int w_pw_off() { return w_conv_off(kConvs); }
constexpr int kWeightFloats = w_pw_off() + kC + 1;

// Per-wave streaming state, all in registers.
struct Tnet {
  u4 aw[kConvs - 1][3];   // conv 1..6, taps (2q, 2q+1) x channels 4g..4g+3 of output row j
  u4 a6[kConvs - 1];      // conv 1..6, tap 6 (elements 4..7 zero)
  u4 a0;                  // conv0: taps 0..6 in lane group 0, zero elsewhere
  u4 ap;                  // projection weights of channels 4g..4g+3 (every row; elements 4..7 zero)
  u16 ring[kConvs - 1];   // ring[L]: output frames of conv L (the input of conv L+1)
  u4 xw;                  // X of frames s-6 .. s as bf16 (element 7 zero)
  float xr[kRing];        // prefetched X, slot f mod 7
  float v, bp;            // BiLIF membrane; projection bias
};

struct Io {
  const f4* bias;         // LDS: bias of conv L, rows 4g..4g+3 at [4L + g]
  const float* xc;        // X of the clip, frame 0 (uniform)
  int8_t* oc;             // spikes of the clip, frame 0 (uniform)
  float* dc;              // debug frames of the clip (uniform)
  size_t HW;
  int T, g, pix, pixc;    // pixc: pix clamped into the frame (tail lanes read a real pixel)
  bool valid;
  float theta, leak;
};

// Chunk modes: warm-up (s0 = W0 in {0, 7, 14} at compile time: the convs
// whose frame would lie before the clip are left out), steady (every conv has
// a frame inside the clip and every prefetch lies inside it), drain (frames
// past the clip are zeroed by selects).  No mode branches per conv, so a
// chunk stays one basic block.
enum { kWarm = 0, kSteady = 1, kDrain = 2 };

// Conv L at step s (K7 = s mod 7): output frame t = s - 3(L+1) from the
// ring of conv L-1, whose newest frame t+3 was written earlier in this step.
template <int K7, int L, int MODE, int W0, bool DBG>
__device__ __forceinline__ void conv(Tnet& st, const Io& io, int s, u2& h3) {
  if constexpr (MODE == kWarm && W0 + K7 - kDelay * (L + 1) < 0) return;   // the ring slot stays zero
  const int t = s - kDelay * (L + 1);
  constexpr int so = mod7(K7 - kDelay * (L + 1));   // slot of frame t
  f4 acc = io.bias[4 * L + io.g];
  if constexpr (L == 0) {
    acc = mfma32(st.a0, st.xw, acc);
  } else {
    constexpr int b0 = mod7(so - 3);                  // slot of frame t-3 (tap 0)
    acc = mfma32(st.aw[L - 1][0], ring_pair<b0>(st.ring[L - 1]), acc);
    acc = mfma32(st.aw[L - 1][1], ring_pair<mod7(b0 + 2)>(st.ring[L - 1]), acc);
    acc = mfma32(st.aw[L - 1][2], ring_pair<mod7(b0 + 4)>(st.ring[L - 1]), acc);
    acc = mfma32(st.a6[L - 1], ring_pair<mod7(b0 + 6)>(st.ring[L - 1]), acc);
  }
  if constexpr (L == 2 || L == 4 || L == 6) {        // residual: h_{i-1} at frame t
    const u2 r = ring_slot<so>(st.ring[L - 2]);
    acc[0] += lo_bf16(r.x);
    acc[1] += hi_bf16(r.x);
    acc[2] += lo_bf16(r.y);
    acc[3] += hi_bf16(r.y);
  }
  u2 o = {relu2(pack2(acc[0], acc[1])), relu2(pack2(acc[2], acc[3]))};
  if constexpr (MODE != kSteady) {                    // zero padding past the clip
    const bool real = t < io.T;
    o.x = real ? o.x : 0u;
    o.y = real ? o.y : 0u;
  }
  if constexpr (L < kConvs - 1)
    ring_put<so>(st.ring[L], o);
  else
    h3 = o;
  if constexpr (DBG) {
    if (io.valid && t < io.T) {
      float* d = io.dc + ((size_t)t * kDbgCh + L * kC + 4 * io.g) * io.HW + io.pix;
      d[0] = lo_bf16(o.x);
      d[io.HW] = hi_bf16(o.x);
      d[2 * io.HW] = lo_bf16(o.y);
      d[3 * io.HW] = hi_bf16(o.y);
    }
  }
}

template <int K7, int MODE, int W0, bool DBG>
__device__ __forceinline__ void step(Tnet& st, const Io& io, int s0, u2& spk) {
  const int s = s0 + K7;
  // frame s enters the X window; frame s+7 is fetched into the freed slot
  // (past the clip: a clamped, in-bounds load replaced by zero)
  const float xs = st.xr[K7];
  if constexpr (MODE == kSteady) {
    st.xr[K7] = (io.xc + (size_t)(s + kRing) * io.HW)[io.pixc];
  } else {
    const int f = s + kRing;
    const float xv = (io.xc + (size_t)(f < io.T ? f : io.T - 1) * io.HW)[io.pixc];
    st.xr[K7] = f < io.T ? xv : 0.f;
  }
  st.xw.x = __builtin_amdgcn_alignbit(st.xw.y, st.xw.x, 16);
  st.xw.y = __builtin_amdgcn_alignbit(st.xw.z, st.xw.y, 16);
  st.xw.z = __builtin_amdgcn_alignbit(st.xw.w, st.xw.z, 16);
  st.xw.w = pack2(xs, 0.f);
  u2 h3 = {0u, 0u};
  conv<K7, 0, MODE, W0, DBG>(st, io, s, h3);
  conv<K7, 1, MODE, W0, DBG>(st, io, s, h3);
  conv<K7, 2, MODE, W0, DBG>(st, io, s, h3);
  conv<K7, 3, MODE, W0, DBG>(st, io, s, h3);
  conv<K7, 4, MODE, W0, DBG>(st, io, s, h3);
  conv<K7, 5, MODE, W0, DBG>(st, io, s, h3);
  conv<K7, 6, MODE, W0, DBG>(st, io, s, h3);
  // projection (every row of the A operand holds wp, so every lane receives
  // u of its pixel) and BiLIF of frame s - 21 (none during the warm-up; past
  // the clip the state no longer matters and the spike is not stored)
  if constexpr (MODE == kWarm) return;
  const int t = s - kLag;
  const float u = mfma32(st.ap, u4{h3.x, h3.y, 0u, 0u}, f4{st.bp, st.bp, st.bp, st.bp})[0];
  float hv = fmaf(io.leak, st.v, u);
  const float charged = hv;
  const float sp = bilif(hv, io.theta, 0.f, 0);
  st.v = hv;
  // the spike as byte K7 % 4 of word K7 / 4 (stored once per chunk)
  const unsigned b = (unsigned)(int)sp & 0xffu;
  if constexpr (K7 < 4)
    spk.x |= b << (8 * K7);
  else
    spk.y |= b << (8 * (K7 - 4));
  if constexpr (DBG) {
    if (io.valid && io.g == 0 && t < io.T) {
      io.dc[((size_t)t * kDbgCh + 7 * kC) * io.HW + io.pix] = u;
      io.dc[((size_t)t * kDbgCh + 7 * kC + 1) * io.HW + io.pix] = charged;
    }
  }
}

// Seven steps (one ring period).  The scheduler works step by step:
// interleaving steps raises register pressure past the budget of two waves
// per SIMD.
template <int MODE, int W0, bool DBG>
__device__ __forceinline__ void chunk(Tnet& st, const Io& io, int s0) {
  u2 spk = {0u, 0u};
  step<0, MODE, W0, DBG>(st, io, s0, spk);
  __builtin_amdgcn_sched_barrier(0);
  step<1, MODE, W0, DBG>(st, io, s0, spk);
  __builtin_amdgcn_sched_barrier(0);
  step<2, MODE, W0, DBG>(st, io, s0, spk);
  __builtin_amdgcn_sched_barrier(0);
  step<3, MODE, W0, DBG>(st, io, s0, spk);
  __builtin_amdgcn_sched_barrier(0);
  step<4, MODE, W0, DBG>(st, io, s0, spk);
  __builtin_amdgcn_sched_barrier(0);
  step<5, MODE, W0, DBG>(st, io, s0, spk);
  __builtin_amdgcn_sched_barrier(0);
  step<6, MODE, W0, DBG>(st, io, s0, spk);
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (MODE == kWarm) return;
  // every lane holds the 7 spikes of its pixel: lane group g stores those of
  // steps g and g + 4 (frames s0 + k - 21)
  if (io.valid) {
    const int t1 = s0 + io.g - kLag, t2 = t1 + 4;
    if (MODE == kSteady || t1 < io.T) io.oc[(size_t)t1 * io.HW + io.pix] = (int8_t)(spk.x >> (8 * io.g));
    if (io.g < 3 && (MODE == kSteady || t2 < io.T))
      io.oc[(size_t)t2 * io.HW + io.pix] = (int8_t)(spk.y >> (8 * io.g));
  }
}

template <bool DBG>
__global__ __launch_bounds__(kNW * 64) __attribute__((amdgpu_waves_per_eu(2))) void k_tnet(
    const float* __restrict__ w, const float* __restrict__ x, int N, int T, int HW, float theta, float leak,
    int8_t* __restrict__ out, float* __restrict__ dbg) {
  __shared__ f4 bias[4 * kConvs];
  if (threadIdx.x < kC * kConvs) {
    const int L = threadIdx.x / kC, c = threadIdx.x % kC;
    reinterpret_cast<float*>(bias)[threadIdx.x] = w[w_bias_off(L) + c];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int bpc = (HW + 15) / 16;                   // pixel blocks per clip
  const int blk = blockIdx.x * kNW + wave;
  if (blk >= N * bpc) return;                       // no barriers below: a wave may leave
  const int n = blk / bpc, pix = (blk % bpc) * 16 + j;
  const bool valid = pix < HW;
  const int pixc = valid ? pix : HW - 1;            // tail lanes read a real pixel, store nothing

  // ---- weights as MFMA A fragments: row j = output channel; lane group g
  // holds (tap 2q, channels 4g..4g+3), (tap 2q+1, channels 4g..4g+3)
  Tnet st;
#pragma unroll
  for (int L = 1; L < kConvs; ++L) {
    const float* wl = w + w_conv_off(L) + (j * kC + 4 * g) * kTaps;   // [ci][tap] of row j, ci = 4g + c
#pragma unroll
    for (int q = 0; q < 3; ++q)
      st.aw[L - 1][q] = u4{pack2(wl[0 * kTaps + 2 * q], wl[1 * kTaps + 2 * q]),
                           pack2(wl[2 * kTaps + 2 * q], wl[3 * kTaps + 2 * q]),
                           pack2(wl[0 * kTaps + 2 * q + 1], wl[1 * kTaps + 2 * q + 1]),
                           pack2(wl[2 * kTaps + 2 * q + 1], wl[3 * kTaps + 2 * q + 1])};
    st.a6[L - 1] = u4{pack2(wl[0 * kTaps + 6], wl[1 * kTaps + 6]), pack2(wl[2 * kTaps + 6], wl[3 * kTaps + 6]), 0u, 0u};
  }
  {
    float v0[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v0[e] = (g == 0 && e < kTaps) ? w[j * kTaps + e] : 0.f;
    st.a0 = u4{pack2(v0[0], v0[1]), pack2(v0[2], v0[3]), pack2(v0[4], v0[5]), pack2(v0[6], v0[7])};
  }
  {
    const float* wp = w + w_pw_off() + 4 * g;
    st.ap = u4{pack2(wp[0], wp[1]), pack2(wp[2], wp[3]), 0u, 0u};
  }
  st.bp = w[w_pw_off() + kC];
#pragma unroll
  for (int L = 0; L < kConvs - 1; ++L) st.ring[L] = u16{};
  st.xw = u4{0u, 0u, 0u, 0u};
  st.v = 0.f;

  Io io;
  io.bias = bias;
  io.HW = (size_t)HW;
  io.xc = x + (size_t)n * T * HW;
  io.oc = out + (size_t)n * T * HW;
  io.dc = DBG ? dbg + (size_t)n * T * kDbgCh * HW : nullptr;
  io.T = T;
  io.g = g;
  io.pix = pix;
  io.pixc = pixc;
  io.valid = valid;
  io.theta = theta;
  io.leak = leak;
#pragma unroll
  for (int k = 0; k < kRing; ++k) st.xr[k] = k < T ? (io.xc + (size_t)k * HW)[pixc] : 0.f;

  // steps s = 0 .. T+20 (the projection lags the input by 21 frames)
  chunk<kWarm, 0, DBG>(st, io, 0);
  chunk<kWarm, 7, DBG>(st, io, 7);
  chunk<kWarm, 14, DBG>(st, io, 14);
  int s0 = kLag;
  for (; s0 + 2 * kRing <= T; s0 += kRing) chunk<kSteady, 0, DBG>(st, io, s0);
  for (; s0 < T + kLag; s0 += kRing) chunk<kDrain, 0, DBG>(st, io, s0);
}

}  // namespace

size_t tnet_weight_floats() { return (size_t)kWeightFloats; }

int tnet_forward(const evs_tnet& net, const float* weights, const float* x, int N, int T, int H, int W, int8_t* s_out,
                 float* debug, hipStream_t st) {
  if (net.hidden != kC) return fail(EVS_EUNSUPPORTED, "tnet: hidden width must be 16");
  if (!(net.theta > 0.f) || !(net.theta < 3.0e38f)) return fail(EVS_EINVAL, "tnet: theta must be positive and finite");
  if (!(net.leak >= 0.f && net.leak <= 1.f)) return fail(EVS_EINVAL, "tnet: leak must be in [0, 1]");
  if (!weights || !x || !s_out) return fail(EVS_EINVAL, "tnet: NULL weights, input or output");
  if (N < 1 || T < 1 || H < 1 || W < 1) return fail(EVS_EINVAL, "tnet: N, T, H, W must be >= 1");
  const double HW = (double)H * W;
  if ((double)N * T * HW > 9.0e18 || HW > 2.0e9) return fail(EVS_EOVERFLOW, "tnet: input too large");
  if (debug && (double)N * T * kDbgCh * HW > 2.0e9) return fail(EVS_EOVERFLOW, "tnet: debug output too large");
  if ((double)T + kLag + 2 * kRing > 2.0e9) return fail(EVS_EOVERFLOW, "tnet: too many frames");
  const long long blocks = (long long)N * ((H * (long long)W + 15) / 16);
  const long long grid = (blocks + kNW - 1) / kNW;
  if (grid > 2000000000LL) return fail(EVS_EOVERFLOW, "tnet: too many pixels");
  if (debug)
    hipLaunchKernelGGL(k_tnet<true>, dim3((unsigned)grid), dim3(kNW * 64), 0, st, weights, x, N, T, (int)HW, net.theta,
                       net.leak, s_out, debug);
  else
    hipLaunchKernelGGL(k_tnet<false>, dim3((unsigned)grid), dim3(kNW * 64), 0, st, weights, x, N, T, (int)HW,
                       net.theta, net.leak, s_out, debug);
  EVS_HIP(hipGetLastError());
  return EVS_OK;
}

}  // namespace evs
