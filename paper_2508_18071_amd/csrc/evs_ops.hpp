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
