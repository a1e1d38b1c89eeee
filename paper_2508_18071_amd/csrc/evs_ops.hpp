// Internal declarations of the non-forward operations of libevs.
#pragma once

#include "evs_internal.hpp"

namespace evs {

// small utility kernels (evs_util.hip)
int zero_i32(int32_t* p, size_t n, hipStream_t s);
int zero_f32(float* p, size_t n, hipStream_t s);
int copy_f32(float* dst, const float* src, size_t n, hipStream_t s);
int fill_uniform(float* p, size_t n, uint32_t seed, float lo, float hi, hipStream_t s);
// adds the number of NaN values in p[0, n) to the status-word counter *word
// NaN count of p[0, n) added to *word; with range > 0, |v| >= range (or
// infinite) anywhere sets bit `flag` of *flags.
int count_nan(const float* p, size_t n, int32_t* word, hipStream_t s, float range = 0.f, int32_t* flags = nullptr,
              int flag = 0);

// Layer-by-layer forward (evs_layerwise.hip) of the networks the fused
// kernels do not cover (fused_shape false): one clip of N, direct input.
//   x        [N][T][Cin][H][W] frames 0..T-1 of clip n at x + n x_nstride
//   v_in     initial state [sum C][H][W] of clip n at v_in + n vin_nstride, or
//            null (zero); v_out: final state [N][sum C][H][W], or null
//   s_out    [N][T][Cout][H][W] int8 or (s_fp32) float32, or null
//   ckpt     [N][ceil(T / ckpt_every)][sum C][H][W], or null
//   h_trace  public trace [N][T][sum C][tb h][tb w] over tb (tb[2] == 0: the
//            whole frame), or null
//   rtrace   the backward's pixel-major trace, frames [T][planes][H][W]
//            (fp16 if rt_f16), clip n at + n rt_nstride elements, or null
struct LwClip {
  int N, T, H, W;
  const float* x;
  long long x_nstride;
  const float* v_in;
  long long vin_nstride;
  float* v_out;
  void* s_out;
  int s_fp32;
  float* ckpt;
  int ckpt_every;
  float* h_trace;
  int tb[4];
  void* rtrace;
  int rt_f16;
  long long rt_nstride;
};
size_t layerwise_workspace_bytes(const evs_net& net, int N, int H, int W);
int layerwise_forward(const evs_net& net, const float* w, const LwClip& c, void* ws, hipStream_t st);
// true when compiled fused kernels cover the network's shape (at most three
// layers, equal hidden widths)
bool fused_shape(const evs_net& net);

// EMD loss (evs_emd.hip)
size_t emd_workspace_bytes(int N, int T, int C, int H, int W);
int emd_loss(const float* s, const int8_t* e, int N, int T, int C, int H, int W, float lambda,
             float* loss, float* grad, void* ws, size_t ws_bytes, hipStream_t st);
int emd_loss_noalloc(const float* s, const int8_t* e, int N, int T, int C, int H, int W, float lambda,
                     float* loss, float* grad, hipStream_t st);

// event compaction (evs_compact.hip)
size_t compact_workspace_bytes(int T, int C, int H, int W);
int compact_events(const int8_t* s, int T, int C, int H, int W, uint64_t* events, int64_t cap,
                   int64_t* count, void* ws, size_t ws_bytes, int32_t* status, hipStream_t st);

// the paper's temporal EvSNet (evs_tnet.hip)
size_t tnet_weight_floats();
int tnet_forward(const evs_tnet& net, const float* weights, const float* x, int N, int T, int H, int W, int8_t* s_out,
                 float* debug, hipStream_t st);
// network input of Eq. 1 and contrast-crossing targets (evs_prologue.hip)
int logdiff(const float* rgb, int N, int T, int H, int W, float scale, float knee, float* x_out, hipStream_t st);
int contrast_events(const float* rgb, int N, int T, int H, int W, float scale, float knee, float C, int8_t* e_out,
                    hipStream_t st);

// BPTT backward (evs_backward.hip)
size_t backward_workspace_bytes(const evs_net& net, const evs_clip& clip, int ckpt_every);
int backward(const evs_net& net, const void* packed, const evs_clip& clip, const float* ckpt,
             int ckpt_every, const float* grad_s, float* const* grad_w, float* grad_x, float* grad_v,
             void* ws, size_t ws_bytes, int32_t* status, hipStream_t st);

// tile selection (evs_api.cpp); the autotuner (evs_autotune.cpp)
void load_tile_cache_once();
int choose_tile(const evs_net& net, int H, int W, int N = 1);
void remember_tile(const evs_net& net, int H, int W, int tile);
// with_frag: the packed buffer carries the prepacked fragments
// (evs_pack_weights wrote it)
FwdNetArgs make_net_args(const evs_net& net, const void* packed, bool with_frag = true);

}  // namespace evs
