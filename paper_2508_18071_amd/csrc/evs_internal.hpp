// Internal helpers shared by the HIP translation units of libevs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>

#include "../../include/evs.h"

namespace evs {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);
int hip_check(hipError_t e, const char* what);

#define EVS_HIP(call)                                  \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) return ::evs::hip_check(_e, #call); \
  } while (0)

// ---------------------------------------------------------------- sizes
inline int real_sum_channels(const evs_net& n) {
  int s = 0;
  for (int l = 1; l <= n.n_layers; ++l) s += n.ch[l];
  return s;
}
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Validation of a network description; returns EVS_OK or an error code
// (with the message set).
int validate_net(const evs_net* net);
int validate_clip(const evs_net& net, const evs_clip& c, bool need_x);

// ---------------------------------------------------------------- bf16
__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u) {           // inf / nan: keep, quiet nan
    return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  }
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}
__host__ __device__ inline float round_bf16(float f) { return bf16_to_f32(f32_to_bf16_rne(f)); }

// ---------------------------------------------------------------- forward
// Per-launch arguments of the forward kernels (one clip batch).
struct FwdClipArgs {
  const float* x;        // [N][T][Cin][H][W], or [N][T+1][3][H][W] RGB (FwdNetArgs::x_rgb)
  void* s_out;           // [N][T][Cout][H][W] int8 or float, may be null
  float* v_out;          // [N][sumC][H][W] final state, may be null
  const float* v_in;     // [N][sumC][H][W] initial state, may be null
  float* h_trace;        // [N][T][sumC][H][W], may be null
  float* ckpt;           // [N][nseg][sumC][H][W], may be null
  int32_t N, T, H, W;
  int32_t s_fp32;
  int32_t ckpt_every;
  int32_t tiles_x, tiles_y;
  // element strides between the clips of a batch (x, initial state, trace)
  int64_t x_nstride, vin_nstride, trace_nstride;
  // image window recorded in h_trace (the whole frame by default)
  int32_t tb_y0, tb_x0, tb_h, tb_w;
  // h_trace holds fp16 values (the backward's segment potentials of BF16
  // nets, rounded so that each stored value gives the forward's spike), else
  // float
  int32_t trace_f16;
  // h_trace is pixel-major (the backward's segment potentials): per frame,
  // layer after layer, each layer [H][W][CP] with CP its width rounded up to
  // a multiple of 4 (the output layer: 4), so that a lane's four channels of
  // a pixel are one store and one load; else [sumC][h][w] over the window
  int32_t trace_pm;
};

constexpr int kMaxLayers = EVS_MAX_LAYERS;
struct FwdNetArgs {
  const float* w;        // packed fp32 weights, layer after layer [Cout][Cin][3][3]
  int32_t n_layers;
  int32_t ch[kMaxLayers + 1];   // real channel counts
  int32_t wofs[kMaxLayers];     // float offsets of each layer in w
  int32_t sum_c;
  float theta, leak, alpha;
  int32_t relaxed;       // 0 hard spikes, 1 relaxed (sigmoid step), 2 relaxed (arctangent step)
  // x holds T+1 RGB frames and the input is their lin-log luminance
  // difference (Eq. 1): scale, knee and toe slope ln(knee) / knee
  int32_t x_rgb;
  float lum_scale, knee, toe;
  // the prepacked MFMA fragments of the packed weight buffer (a header of
  // kFragHeaderWords words, then the LDS image of the weight area), or null
  const uint32_t* frag;
};

// Header of the prepacked fragments: magic, layout signature of the kernel
// configuration they were built for, the real channel counts (8 bits each),
// the layer count, the two weight-scale words of FP32 nets, image bytes.
constexpr int kFragHeaderWords = 8;
constexpr uint32_t kFragMagic = 0x45565346u;

// Batched (persistent) launch: a clip table passed by value.
constexpr int kMaxBatchClips = 24;
struct BatchTable {
  int32_t n_clips;
  int32_t n_items;                   // total (clip, tile) items
  int32_t item_start[kMaxBatchClips + 1];  // prefix sums of tiles per clip (LPT clip order)
  FwdClipArgs clip[kMaxBatchClips];
};

// Forward dispatch (evs_forward.hip).
int launch_forward(const evs_net& net, const FwdNetArgs& na, const FwdClipArgs& ca,
                   int tile_id, hipStream_t stream);
int launch_forward_batched(const evs_net& net, const FwdNetArgs& na, const BatchTable& bt,
                           int tile_id, int32_t* counter, hipStream_t stream);
int forward_tile_count(const evs_net& net);
const char* forward_tile_name(const evs_net& net, int tile_id);
void forward_tile_dims(const evs_net& net, int tile_id, int* th, int* tw);
int forward_default_tile(const evs_net& net, int H, int W, int N);
int forward_batched_tile(const evs_net& net, int preferred);   // -1: none compiled
// Prepacked fragments: bytes of the block (header + image) for `net`, 0
// when no kernel of the net takes them; forward_prepack writes the block.
size_t forward_frag_bytes(const evs_net& net);
int forward_prepack(const evs_net& net, const FwdNetArgs& na, uint32_t* dst, hipStream_t stream);

}  // namespace evs
