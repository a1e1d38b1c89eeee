// Layer-by-layer EvSNet forward (arXiv 2508.18071, Sec. 3.3, Eq. 2-3) for
// the network shapes the fused kernels of evs_forward.hip do not cover:
// more than three layers, hidden layers of different widths, or widths with
// no fused build.  One launch per (frame, layer): a workgroup takes a 16x16
// pixel tile, stages the haloed input of the layer (x, or the spikes the
// layer below wrote for this frame) in LDS, and each thread updates the
// BiLIF neurons of its pixel: h = leak v + sum_{ci, tap} W[c][ci][tap]
// s[ci][p + tap] (zero padding), then fire and reset.  The membrane state
// of every layer lives in a [N][sum C][H][W] buffer, each pixel read and
// written only by its own thread, so no launch waits on a neighbour's
// state; the spikes between layers go through two [N][C][H][W] float
// buffers.  Arithmetic: FP32 products and sums for FP32 nets; BF16 nets
// multiply the bf16-rounded x and W (exact in FP32) and sum in FP32.  The
// outputs (spikes, checkpoints, the public trace, the backward's
// pixel-major trace, the final state) have the layouts of the fused path.
#include "evs_internal.hpp"
#include "evs_device.hpp"
#include "evs_ops.hpp"

namespace evs {
namespace {

constexpr int LT = 16;               // tile edge (output pixels)
constexpr int LNT = LT * LT;         // threads per workgroup: one pixel each
constexpr int LE = LT + 2;           // haloed tile edge
constexpr int kMaxC = 32;            // widest layer

struct LayerArgs {
  const float* in;                   // the layer's input frame [cin][H][W] of clip 0
  long long in_nstride;              // elements between clips
  const float* w;                    // [cout][cin][3][3] (bf16-rounded for BF16 nets)
  int cin, cout, H, W, tiles_x, bf_in;
  float theta, leak, alpha;
  int relaxed;                       // 0 hard, 1 sigmoid step, 2 arctangent step
  float* v;                          // state planes of this layer [cout][H][W], clip 0
  long long v_nstride;
  float* s_next;                     // spikes for the layer above [cout][H][W], or null
  long long sn_nstride;
  char* s_out;                       // last layer: the frame's [cout][H][W] block of s_out, clip 0
  long long so_nstride;              // elements between clips
  int s_fp32;
  float* ckpt;                       // checkpoint planes of this layer (state before the frame), or null
  long long ck_nstride;
  float* trace;                      // public trace: plane 0 of this layer in the frame's block, or null
  long long tr_nstride;
  int tb_y0, tb_x0, tb_h, tb_w;
  char* rtrace;                      // pixel-major trace: this layer's [H][W][rt_cw] block, or null
  long long rt_nstride;              // elements between clips
  int rt_cw, rt_f16;
  unsigned t16;                      // fp16 traces: bits of the smallest fp16 >= theta
};

// An fp16 trace value: h rounded toward zero, a firing neuron's magnitude
// raised to at least t16 (the smallest fp16 >= theta), so the stored value
// gives the same spike; NaN stays NaN.
__device__ inline unsigned short trace_f16(float h, float s, unsigned t16) {
  const unsigned q = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(h, 0.f)) & 0xffffu;
  unsigned mag = q & 0x7fffu;
  if (s != 0.f && mag < t16) mag = t16;
  return (unsigned short)(mag | (q & 0x8000u));
}

template <int COP>
__global__ __launch_bounds__(LNT) void k_layer(LayerArgs a) {
  __shared__ float tile[kMaxC * LE * LE];
  const int n = blockIdx.y;
  const int ty0 = (blockIdx.x / a.tiles_x) * LT, tx0 = (blockIdx.x % a.tiles_x) * LT;
  const int H = a.H, W = a.W;
  const size_t HW = (size_t)H * W;
  const float* in = a.in + n * a.in_nstride;
  for (int e = threadIdx.x; e < a.cin * LE * LE; e += LNT) {
    const int ci = e / (LE * LE), r = (e / LE) % LE, c = e % LE;
    const int y = ty0 - 1 + r, x = tx0 - 1 + c;
    float v = (y >= 0 && y < H && x >= 0 && x < W) ? in[(size_t)ci * HW + (size_t)y * W + x] : 0.f;
    if (a.bf_in) v = round_bf16(v);
    tile[e] = v;
  }
  __syncthreads();
  const int ty = threadIdx.x / LT, tx = threadIdx.x % LT;
  const int y = ty0 + ty, x = tx0 + tx;
  if (y >= H || x >= W) return;                      // past the only barrier
  const size_t pix = (size_t)y * W + x;
  float* const v = a.v + n * a.v_nstride;
  float acc[COP];
#pragma unroll
  for (int co = 0; co < COP; ++co) {
    const float v0 = co < a.cout ? v[co * HW + pix] : 0.f;
    if (a.ckpt && co < a.cout) a.ckpt[n * a.ck_nstride + co * HW + pix] = v0;
    acc[co] = a.leak * v0;
  }
  for (int ci = 0; ci < a.cin; ++ci) {
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const float xv = tile[(ci * LE + ty + tap / 3) * LE + tx + tap % 3];
#pragma unroll
      for (int co = 0; co < COP; ++co) {
        const float wv = co < a.cout ? a.w[(co * a.cin + ci) * 9 + tap] : 0.f;
        acc[co] = fmaf(wv, xv, acc[co]);
      }
    }
  }
  const bool in_box = a.trace && y >= a.tb_y0 && y < a.tb_y0 + a.tb_h && x >= a.tb_x0 && x < a.tb_x0 + a.tb_w;
#pragma unroll
  for (int co = 0; co < COP; ++co) {
    if (co >= a.cout) break;
    const float h = acc[co];
    if (in_box)
      a.trace[n * a.tr_nstride + (size_t)co * a.tb_h * a.tb_w + (size_t)(y - a.tb_y0) * a.tb_w + (x - a.tb_x0)] = h;
    float vv = h;
    const float s = bilif(vv, a.theta, a.alpha, a.relaxed);
    v[co * HW + pix] = vv;
    if (a.rtrace) {
      const size_t e = n * a.rt_nstride + pix * a.rt_cw + co;
      if (a.rt_f16) reinterpret_cast<unsigned short*>(a.rtrace)[e] = trace_f16(h, s, a.t16);
      else reinterpret_cast<float*>(a.rtrace)[e] = h;
    }
    if (a.s_next) a.s_next[n * a.sn_nstride + co * HW + pix] = s;
    if (a.s_out) {
      const size_t o = n * a.so_nstride + co * HW + pix;
      if (a.s_fp32) reinterpret_cast<float*>(a.s_out)[o] = s;
      else a.s_out[o] = (char)(int)s;
    }
  }
}

// W rounded to bfloat16 (round to nearest even), as float.
__global__ void k_round_w(const float* __restrict__ w, int n, float* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = round_bf16(w[i]);
}

size_t weight_floats(const evs_net& net) {
  size_t n = 0;
  for (int l = 0; l < net.n_layers; ++l) n += (size_t)net.ch[l + 1] * net.ch[l] * 9;
  return n;
}

int max_width(const evs_net& net) {
  int m = 0;
  for (int l = 1; l < net.n_layers; ++l) m = net.ch[l] > m ? net.ch[l] : m;
  return m;
}

}  // namespace

size_t layerwise_workspace_bytes(const evs_net& net, int N, int H, int W) {
  const size_t HW = (size_t)H * W;
  return align256((size_t)N * real_sum_channels(net) * HW * 4)            // state
         + 2 * align256((size_t)N * (max_width(net) > 0 ? max_width(net) : 1) * HW * 4)   // spikes between layers
         + align256(weight_floats(net) * 4);                              // bf16-rounded weights
}

int layerwise_forward(const evs_net& net, const float* w, const LwClip& c, void* ws, hipStream_t st) {
  const int L = net.n_layers, N = c.N, T = c.T, H = c.H, W = c.W;
  const size_t HW = (size_t)H * W;
  const int sumc = real_sum_channels(net);
  const int cin0 = net.ch[0], cout = net.ch[L];
  const bool bf = net.precision == EVS_BF16;
  char* p = reinterpret_cast<char*>(ws);
  float* state = reinterpret_cast<float*>(p);
  p += align256((size_t)N * sumc * HW * 4);
  const int mw = max_width(net) > 0 ? max_width(net) : 1;
  float* sb[2] = {reinterpret_cast<float*>(p), nullptr};
  p += align256((size_t)N * mw * HW * 4);
  sb[1] = reinterpret_cast<float*>(p);
  p += align256((size_t)N * mw * HW * 4);
  const float* wl = w;
  int rc;
  if (bf) {
    float* wr = reinterpret_cast<float*>(p);
    const int nw = (int)weight_floats(net);
    hipLaunchKernelGGL(k_round_w, dim3((nw + 255) / 256), dim3(256), 0, st, w, nw, wr);
    EVS_HIP(hipGetLastError());
    wl = wr;
  }
  // initial state: v_in (per clip, v_in + n * vin_nstride) or zero
  if (c.v_in) {
    for (int n = 0; n < N; ++n)
      if ((rc = copy_f32(state + (size_t)n * sumc * HW, c.v_in + (size_t)n * c.vin_nstride, (size_t)sumc * HW, st)))
        return rc;
  } else if ((rc = zero_f32(state, (size_t)N * sumc * HW, st))) {
    return rc;
  }
  int wofs[9], choff[9], tpo[9];
  for (int l = 0, o = 0, q = 0, r = 0; l < L; ++l) {
    wofs[l] = o;
    o += net.ch[l + 1] * net.ch[l] * 9;
    choff[l] = q;
    q += net.ch[l + 1];
    tpo[l] = r;
    r += l + 1 == L ? 4 : (net.ch[l + 1] + 3) & ~3;
  }
  const int tpf = tpo[L - 1] + 4;
  const int tiles_x = (W + LT - 1) / LT, tiles_y = (H + LT - 1) / LT;
  const dim3 grid((unsigned)(tiles_x * tiles_y), (unsigned)N);
  const int nseg = c.ckpt ? (T + c.ckpt_every - 1) / c.ckpt_every : 0;
  const int tbh = c.tb[2] > 0 ? c.tb[2] : H, tbw = c.tb[2] > 0 ? c.tb[3] : W;
  const int tby = c.tb[2] > 0 ? c.tb[0] : 0, tbx = c.tb[2] > 0 ? c.tb[1] : 0;
  unsigned t16 = 0;
  if (bf) {
    const _Float16 q = (_Float16)net.theta;
    const unsigned b = __builtin_bit_cast(unsigned short, q);
    t16 = (float)q < net.theta ? b + 1 : b;
  }
  for (int t = 0; t < T; ++t) {
    for (int l = 0; l < L; ++l) {
      LayerArgs a{};
      const bool last = l + 1 == L;
      if (l == 0) {
        a.in = c.x + (size_t)t * cin0 * HW;
        a.in_nstride = c.x_nstride;
        a.bf_in = bf ? 1 : 0;
      } else {
        a.in = sb[(l - 1) & 1];
        a.in_nstride = (long long)mw * HW;
      }
      a.w = wl + wofs[l];
      a.cin = net.ch[l];
      a.cout = net.ch[l + 1];
      a.H = H; a.W = W; a.tiles_x = tiles_x;
      a.theta = net.theta; a.leak = net.leak; a.alpha = net.surr_alpha;
      a.relaxed = net.relaxed ? 1 + net.surrogate : 0;
      a.v = state + (size_t)choff[l] * HW;
      a.v_nstride = (long long)sumc * HW;
      if (!last) {
        a.s_next = sb[l & 1];
        a.sn_nstride = (long long)mw * HW;
      } else if (c.s_out) {
        a.s_out = reinterpret_cast<char*>(c.s_out) + (size_t)t * cout * HW * (c.s_fp32 ? 4 : 1);
        a.so_nstride = (long long)T * cout * HW;
        a.s_fp32 = c.s_fp32;
      }
      if (c.ckpt && t % c.ckpt_every == 0) {
        a.ckpt = c.ckpt + ((size_t)(t / c.ckpt_every) * sumc + choff[l]) * HW;
        a.ck_nstride = (long long)nseg * sumc * HW;
      }
      if (c.h_trace) {
        a.trace = c.h_trace + ((size_t)t * sumc + choff[l]) * tbh * tbw;
        a.tr_nstride = (long long)T * sumc * tbh * tbw;
        a.tb_y0 = tby; a.tb_x0 = tbx; a.tb_h = tbh; a.tb_w = tbw;
      }
      if (c.rtrace) {
        const size_t es = c.rt_f16 ? 2 : 4;
        a.rtrace = reinterpret_cast<char*>(c.rtrace) + ((size_t)t * tpf + tpo[l]) * HW * es;
        a.rt_nstride = c.rt_nstride;
        a.rt_cw = last ? 4 : (net.ch[l + 1] + 3) & ~3;
        a.rt_f16 = c.rt_f16;
        a.t16 = t16;
      }
      const int co = a.cout;
      if (co <= 2) hipLaunchKernelGGL(k_layer<2>, grid, dim3(LNT), 0, st, a);
      else if (co <= 8) hipLaunchKernelGGL(k_layer<8>, grid, dim3(LNT), 0, st, a);
      else if (co <= 16) hipLaunchKernelGGL(k_layer<16>, grid, dim3(LNT), 0, st, a);
      else hipLaunchKernelGGL(k_layer<32>, grid, dim3(LNT), 0, st, a);
      EVS_HIP(hipGetLastError());
    }
  }
  if (c.v_out && (rc = copy_f32(c.v_out, state, (size_t)N * sumc * HW, st))) return rc;
  return EVS_OK;
}

}  // namespace evs
