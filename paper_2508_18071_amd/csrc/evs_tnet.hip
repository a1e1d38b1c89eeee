// The paper's temporal EvSNet on gfx950 (arXiv 2508.18071, Sec. 3.3,
// Eq. 5-6): per pixel, a kernel-7 Conv1d encoder h0 = ReLU(conv0 X),
// residual blocks h_i = ReLU(h_{i-1} + conv(ReLU(conv h_{i-1}))), i = 1..3,
// a point-wise projection to one value per frame and a BiLIF unit (Eq. 2-3).
//
// Dataflow: every pixel is independent, so one wave owns 16 pixels (the
// MFMA column block) and streams their sequences through time; waves never
// synchronise.  Each conv keeps its input as a ring of the last 8 frames in
// LDS ([slot][pixel][16 channels] bf16), so a conv output frame is one
// 16x16x32 bf16 MFMA chain over K = (tap, channel) = 7 x 16 (4 k-steps).
// Conv L produces frame s - 4(L+1) at step s: its inputs were all written at
// earlier steps, so the seven convs of a step are independent and their MFMA
// chains interleave.  Frames outside [0, T) are zero in every ring (the
// convs' zero padding).  Operands are bf16 (input, weights, stored
// activations), sums and biases FP32, the BiLIF state FP32.
#include <hip/hip_runtime.h>

#include "evs_device.hpp"
#include "evs_ops.hpp"

namespace evs {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kC = 16;            // hidden width
constexpr int kTaps = 7;          // kernel size of every encoder conv
constexpr int kConvs = 7;         // conv0 + 2 per residual block
constexpr int kRing = 8;          // frames per ring
constexpr int kSlotBytes = 16 * kC * 2;           // 16 pixels x 16 channels bf16
constexpr int kRingBytes = kRing * kSlotBytes;    // 4 KB
constexpr int kRings = kConvs - 1;                // conv6 feeds the projection directly
constexpr int kWaveLds = kRings * kRingBytes;     // 24 KB per wave
constexpr int kNW = 6;                            // waves per workgroup
constexpr int kDelay = 4;                         // frames of delay added per conv

typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
// round to bf16 (nearest even) in hardware: two values packed low, high
__device__ inline unsigned pack2(float lo, float hi) {
  const bf2 p = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(unsigned, p);
}
__device__ inline float bf16_round_dev(float f) { return (float)(__bf16)f; }
__device__ inline float lo_bf16(unsigned u) { return __builtin_bit_cast(float, u << 16); }
__device__ inline float hi_bf16(unsigned u) { return __builtin_bit_cast(float, u & 0xffff0000u); }

__device__ inline f4 mfma_bf16(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// Offsets of the layers in the flat weight array (see evs.h).
__host__ __device__ constexpr int w_conv_off(int L) {     // weights of conv L >= 1
  return kC * kTaps + kC + (L - 1) * (kC * kC * kTaps + kC);
}
__host__ __device__ constexpr int w_pw_off() { return w_conv_off(kConvs); }
constexpr int kWeightFloats = w_pw_off() + kC + 1;

// Per-wave streaming state, kept in registers.
struct Tnet {
  u4 a0;                        // conv0 A fragment
  u4 aw[kConvs - 1][4];         // conv 1..6 A fragments, 4 k-steps each
  f4 bias[kConvs];              // biases of this lane's rows 4g .. 4g+3
  f4 wp;                        // projection weights of those rows (bf16 values)
  float bp;
  unsigned xw[4];               // bf16 X of the last 7 frames (entry 7 = 0)
  float xnext, v;
};

// One step s (K8 = s mod 8, so every ring slot is a compile-time offset):
// conv L produces frame s - 4(L+1) from ring frames written at earlier
// steps; the projection and BiLIF handle frame s - 28.
template <bool DBG, int K8>
__device__ __forceinline__ void tnet_step(Tnet& st, int s, int T, int HW, char* ring, int lb, int wb, int wd,
                                          int g, bool valid, float theta, float leak, const float*& xnp,
                                          int8_t* op, float* dbgp, int j) {
  f4 h3 = {0.f, 0.f, 0.f, 0.f};
  // conv 6 .. conv 0: a conv reads its residual source before the conv that
  // produced it overwrites that slot in this step
#pragma unroll
  for (int L = kConvs - 1; L >= 0; --L) {
    const int t = s - kDelay * (L + 1);
    f4 acc = st.bias[L];
    if (L == 0) {
      acc = mfma_bf16(st.a0, u4{st.xw[0], st.xw[1], st.xw[2], st.xw[3]}, acc);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // lane groups g/2 = 0, 1 read taps 2q and 2q+1 (tap 7: zero weights)
        const int c = (K8 - kDelay * (L + 1) - 3 + 2 * q + 8 * kRing) % kRing;   // slot of tap 2q
        const int ro = (L - 1) * kRingBytes;
        u4 b;
        if (q == 3) {
          // taps 6 (and 7 -> read tap 6 again): no lane-group offset
          b = *reinterpret_cast<const u4*>(ring + lb - (g >> 1) * kSlotBytes + ro + c * kSlotBytes);
        } else if (c == kRing - 1) {
          // tap 2q+1 wraps to slot 0
          b = *reinterpret_cast<const u4*>(ring + lb + wd + ro + c * kSlotBytes);
        } else {
          b = *reinterpret_cast<const u4*>(ring + lb + ro + c * kSlotBytes);
        }
        acc = mfma_bf16(st.aw[L - 1][q], b, acc);
      }
    }
    const int so = ((K8 - kDelay * (L + 1)) % kRing + kRing) % kRing;       // output slot (frame t)
    if (L == 2 || L == 4 || L == 6) {              // residual: h_{i-1} at frame t
      const uint2 r2 = *reinterpret_cast<const uint2*>(ring + wb + (L - 2) * kRingBytes + so * kSlotBytes);
      acc[0] += lo_bf16(r2.x);
      acc[1] += hi_bf16(r2.x);
      acc[2] += lo_bf16(r2.y);
      acc[3] += hi_bf16(r2.y);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = fmaxf(acc[r], 0.f);
    const bool real = t >= 0 && t < T;
    if (L < kConvs - 1) {
      const uint2 o = real ? uint2{pack2(acc[0], acc[1]), pack2(acc[2], acc[3])} : uint2{0u, 0u};
      *reinterpret_cast<uint2*>(ring + wb + L * kRingBytes + so * kSlotBytes) = o;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) h3[r] = bf16_round_dev(acc[r]);
    }
    if (DBG && real && valid) {
      float* d = dbgp + ((size_t)t * (7 * kC + 2) + L * kC + 4 * g) * HW;
#pragma unroll
      for (int r = 0; r < 4; ++r) d[(size_t)r * HW] = bf16_round_dev(acc[r]);
    }
  }
  // projection and BiLIF of frame s - 28
  {
    const int t = s - kDelay * kConvs;
    float p = st.wp[0] * h3[0];
    p = fmaf(st.wp[1], h3[1], p);
    p = fmaf(st.wp[2], h3[2], p);
    p = fmaf(st.wp[3], h3[3], p);
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    const float u = p + st.bp;
    if (t >= 0 && t < T) {
      float hv = fmaf(leak, st.v, u);
      const float charged = hv;
      const float sp = bilif(hv, theta, 0.f, 0);
      st.v = hv;
      if (valid && g == 0) {
        op[(size_t)t * HW] = (int8_t)sp;
        if (DBG) {
          dbgp[((size_t)t * (7 * kC + 2) + 7 * kC) * HW] = u;
          dbgp[((size_t)t * (7 * kC + 2) + 7 * kC + 1) * HW] = charged;
        }
      }
    }
  }
  // X window: frames s-6 .. s for the next step
  st.xw[0] = __builtin_amdgcn_alignbit(st.xw[1], st.xw[0], 16);
  st.xw[1] = __builtin_amdgcn_alignbit(st.xw[2], st.xw[1], 16);
  st.xw[2] = __builtin_amdgcn_alignbit(st.xw[3], st.xw[2], 16);
  st.xw[3] = pack2(st.xnext, 0.f);
  st.xnext = (valid && s + 1 < T) ? *xnp : 0.f;
  xnp += HW;
}

template <bool DBG>
__global__ __launch_bounds__(kNW * 64) void k_tnet(const float* __restrict__ w, const float* __restrict__ x, int N,
                                                   int T, int HW, float theta, float leak, int8_t* __restrict__ out,
                                                   float* __restrict__ dbg) {
  __shared__ __attribute__((aligned(16))) char lds[kNW * kWaveLds];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int bpc = (HW + 15) / 16;                   // pixel blocks per clip
  const int blk = blockIdx.x * kNW + wave;
  if (blk >= N * bpc) return;                       // no barriers below: a wave may leave
  const int n = blk / bpc, pix = (blk % bpc) * 16 + j;
  const bool valid = pix < HW;
  char* const ring = lds + wave * kWaveLds;
  for (int e = lane; e < kWaveLds / 16; e += 64) reinterpret_cast<u4*>(ring)[e] = u4{0u, 0u, 0u, 0u};

  // ---- weights as MFMA A fragments (row = output channel j, lane group g
  // holds K = 8g..8g+7 = taps 2q + g/2, channels 8(g&1)..+7), biases and
  // point-wise weights for this lane's rows 4g..4g+3
  Tnet st;
  {
    unsigned d[4];
    for (int e2 = 0; e2 < 4; ++e2) {
      float vv[2];
      for (int h = 0; h < 2; ++h) {
        const int tap = 2 * e2 + h;
        vv[h] = (g == 0 && tap < kTaps) ? w[j * kTaps + tap] : 0.f;
      }
      d[e2] = pack2(vv[0], vv[1]);
    }
    st.a0 = u4{d[0], d[1], d[2], d[3]};
  }
#pragma unroll
  for (int L = 1; L < kConvs; ++L)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int tap = 2 * q + (g >> 1);
      unsigned d[4];
      for (int e2 = 0; e2 < 4; ++e2) {
        float vv[2];
        for (int h = 0; h < 2; ++h) {
          const int ci = 8 * (g & 1) + 2 * e2 + h;
          vv[h] = tap < kTaps ? w[w_conv_off(L) + (j * kC + ci) * kTaps + tap] : 0.f;
        }
        d[e2] = pack2(vv[0], vv[1]);
      }
      st.aw[L - 1][q] = u4{d[0], d[1], d[2], d[3]};
    }
#pragma unroll
  for (int L = 0; L < kConvs; ++L)
#pragma unroll
    for (int r = 0; r < 4; ++r) st.bias[L][r] = w[(L == 0 ? kC * kTaps : w_conv_off(L) + kC * kC * kTaps) + 4 * g + r];
#pragma unroll
  for (int r = 0; r < 4; ++r) st.wp[r] = bf16_round_dev(w[w_pw_off() + 4 * g + r]);
  st.bp = w[w_pw_off() + kC];
  st.xw[0] = st.xw[1] = st.xw[2] = st.xw[3] = 0u;
  st.v = 0.f;

  const float* xp = x + (size_t)n * T * HW + pix;
  st.xnext = valid ? xp[0] : 0.f;
  const float* xnp = xp + HW;                       // frame 1
  int8_t* op = out + (size_t)n * T * HW + pix;
  float* dbgp = DBG ? dbg + (size_t)n * T * (7 * kC + 2) * HW + pix : nullptr;
  // ring addressing: byte offsets inside this wave's rings; lane groups
  // g/2 = 1 read the slot after that of lane groups g/2 = 0 (wd: the same
  // slot wrapped to 0)
  const int lb = j * 32 + (g & 1) * 16 + (g >> 1) * kSlotBytes;
  const int wd = -(g >> 1) * kRing * kSlotBytes;
  const int wb = j * 32 + g * 8;
  const int steps = T + kDelay * kConvs;
  for (int s0 = 0; s0 < steps; s0 += kRing) {
#define EVS_TNET_STEP(K)                                                                                     \
    if (s0 + K < steps)                                                                                      \
      tnet_step<DBG, K>(st, s0 + K, T, HW, ring, lb, wb, wd, g, valid, theta, leak, xnp, op, dbgp, j);
    EVS_TNET_STEP(0) EVS_TNET_STEP(1) EVS_TNET_STEP(2) EVS_TNET_STEP(3)
    EVS_TNET_STEP(4) EVS_TNET_STEP(5) EVS_TNET_STEP(6) EVS_TNET_STEP(7)
#undef EVS_TNET_STEP
  }
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
  if (debug && (double)N * T * (7 * kC + 2) * HW > 2.0e9) return fail(EVS_EOVERFLOW, "tnet: debug output too large");
  if ((double)T + kDelay * kConvs > 2.0e9) return fail(EVS_EOVERFLOW, "tnet: too many frames");
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
