// C ABI of libevs: argument validation, workspace sizing, tile selection and
// dispatch to the HIP kernels.  Declared in include/evs.h.
#include <cmath>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "evs_internal.hpp"
#include "evs_ops.hpp"

namespace evs {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int status, const std::string& msg) {
  set_error(msg);
  return status;
}

int hip_check(hipError_t e, const char* what) {
  return fail(EVS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int validate_net(const evs_net* net) {
  if (!net) return fail(EVS_EINVAL, "net is NULL");
  const int L = net->n_layers;
  if (L < 1 || L > kMaxLayers) return fail(EVS_EINVAL, "n_layers must be 1..8");
  if (net->ch[0] != 1 && net->ch[0] != 3) return fail(EVS_EUNSUPPORTED, "input channels must be 1 or 3");
  for (int l = 1; l < L; ++l)
    if (net->ch[l] < 1 || net->ch[l] > 32) return fail(EVS_EUNSUPPORTED, "hidden width must be 1..32");
  if (net->ch[L] < 1 || net->ch[L] > 2) return fail(EVS_EUNSUPPORTED, "output channels must be 1 or 2");
  if (!(net->theta > 0.f) || !(net->theta < 3.0e38f)) return fail(EVS_EINVAL, "theta must be positive and finite");
  if (!(net->leak >= 0.f && net->leak <= 1.f)) return fail(EVS_EINVAL, "leak must be in [0, 1]");
  if (!(net->surr_alpha > 0.f)) return fail(EVS_EINVAL, "surr_alpha must be positive");
  if (net->precision != EVS_FP32 && net->precision != EVS_BF16) return fail(EVS_EINVAL, "bad precision");
  if (net->relaxed && net->precision != EVS_FP32) return fail(EVS_EUNSUPPORTED, "relaxed spikes need FP32");
  if (net->surrogate != EVS_SURR_SIGMOID && net->surrogate != EVS_SURR_ATAN)
    return fail(EVS_EINVAL, "surrogate must be EVS_SURR_SIGMOID or EVS_SURR_ATAN");
  if (net->input != EVS_INPUT_DIRECT && net->input != EVS_INPUT_RGB_LOGDIFF)
    return fail(EVS_EINVAL, "input must be EVS_INPUT_DIRECT or EVS_INPUT_RGB_LOGDIFF");
  if (net->input == EVS_INPUT_RGB_LOGDIFF) {
    if (net->ch[0] != 1) return fail(EVS_EINVAL, "RGB log-difference input feeds a one-channel net (ch[0] = 1)");
    if (net->precision != EVS_FP32) return fail(EVS_EUNSUPPORTED, "RGB log-difference input needs FP32");
    if (!(net->lum_scale > 0.f) || !(net->knee > 0.f) || !(net->lum_scale < 3.0e38f) || !(net->knee < 3.0e38f))
      return fail(EVS_EINVAL, "lum_scale and knee must be positive and finite");
  }
  return EVS_OK;
}

int validate_clip(const evs_net& net, const evs_clip& c, bool need_x) {
  if (c.N < 1 || c.T < 1 || c.H < 1 || c.W < 1) return fail(EVS_EINVAL, "clip N, T, H, W must be >= 1");
  if (c.H > 4096 || c.W > 4096) return fail(EVS_EUNSUPPORTED, "frame size above 4096");
  if ((double)c.N * (c.T + 1) * 3 * c.H * c.W > 9.0e18) return fail(EVS_EOVERFLOW, "clip too large");
  if (need_x && !c.x) return fail(EVS_EINVAL, "clip x is NULL");
  if (net.relaxed && c.s_out && !c.s_fp32) return fail(EVS_EINVAL, "relaxed spikes need s_fp32 = 1");
  if (c.trace_box[2] > 0 || c.trace_box[3] > 0) {
    const int* b = c.trace_box;
    if (b[0] < 0 || b[1] < 0 || b[2] < 1 || b[3] < 1 || b[0] + b[2] > c.H || b[1] + b[3] > c.W)
      return fail(EVS_EINVAL, "trace_box must lie inside the frame");
  }
  return EVS_OK;
}

// ---------------------------------------------------------------- tiles
namespace {
std::mutex g_tile_mu;
// key: (L, ch0, ch1, ch2, ch3, precision, H, W) -> tile id
std::map<std::tuple<int, int, int, int, int, int, int, int>, int> g_tuned;
std::map<std::tuple<int, int, int, int, int, int>, int> g_forced;

std::tuple<int, int, int, int, int, int> net_key(const evs_net& n) {
  return {n.n_layers, n.ch[0], n.ch[1], n.ch[2], n.ch[3], n.precision};
}
std::tuple<int, int, int, int, int, int, int, int> shape_key(const evs_net& n, int H, int W) {
  return {n.n_layers, n.ch[0], n.ch[1], n.ch[2], n.ch[3], n.precision, H, W};
}
}  // namespace

int choose_tile(const evs_net& net, int H, int W, int N) {
  load_tile_cache_once();
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto f = g_forced.find(net_key(net));
  if (f != g_forced.end() && f->second >= 0) return f->second;
  auto t = g_tuned.find(shape_key(net, H, W));
  if (t != g_tuned.end()) return t->second;
  return forward_default_tile(net, H, W, N);
}

void remember_tile(const evs_net& net, int H, int W, int tile) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tuned[shape_key(net, H, W)] = tile;
}

std::map<std::tuple<int, int, int, int, int, int, int, int>, int> tuned_snapshot() {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  return g_tuned;
}

void set_tuned(const std::tuple<int, int, int, int, int, int, int, int>& k, int tile) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tuned[k] = tile;
}

size_t packed_floats(const evs_net& net);

// Byte offset of the prepacked fragment block in a packed weight buffer:
// after the FP32 weights, 256-byte aligned.
size_t frag_offset(const evs_net& net) { return align256(packed_floats(net) * sizeof(float)); }

FwdNetArgs make_net_args(const evs_net& net, const void* packed, bool with_frag) {
  FwdNetArgs na{};
  na.w = reinterpret_cast<const float*>(packed);
  na.frag = with_frag && forward_frag_bytes(net) > 0
                ? reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(packed) + frag_offset(net))
                : nullptr;
  na.n_layers = net.n_layers;
  int ofs = 0;
  for (int l = 0; l <= kMaxLayers; ++l) na.ch[l] = l <= net.n_layers ? net.ch[l] : 0;
  for (int l = 0; l < net.n_layers; ++l) {
    na.wofs[l] = ofs;
    ofs += net.ch[l + 1] * net.ch[l] * 9;
  }
  na.sum_c = real_sum_channels(net);
  na.theta = net.theta;
  na.leak = net.leak;
  na.alpha = net.surr_alpha;
  na.relaxed = net.relaxed ? 1 + net.surrogate : 0;     // 0 hard, 1 sigmoid, 2 arctangent
  na.x_rgb = net.input == EVS_INPUT_RGB_LOGDIFF ? 1 : 0;
  na.lum_scale = net.lum_scale;
  na.knee = net.knee;
  na.toe = na.x_rgb ? (float)(std::log((double)net.knee) / (double)net.knee) : 0.f;
  return na;
}

size_t packed_floats(const evs_net& net) {
  size_t n = 0;
  for (int l = 0; l < net.n_layers; ++l) n += (size_t)net.ch[l + 1] * net.ch[l] * 9;
  return n;
}

}  // namespace evs

using namespace evs;

extern "C" {

const char* evs_status_str(int s) {
  switch (s) {
    case EVS_OK: return "ok";
    case EVS_EINVAL: return "invalid argument";
    case EVS_EUNSUPPORTED: return "unsupported configuration";
    case EVS_EWORKSPACE: return "workspace missing or too small";
    case EVS_EHIP: return "HIP runtime error";
    case EVS_EOVERFLOW: return "size overflow";
    default: return "unknown status";
  }
}

const char* evs_last_error(void) { return g_last_error.c_str(); }

const char* evs_version(void) { return "evs-mi355x 0.1 (gfx950)"; }

size_t evs_packed_weights_bytes(const evs_net* net) {
  if (validate_net(net) != EVS_OK) return (size_t)-1;
  const size_t fb = forward_frag_bytes(*net);
  return fb ? frag_offset(*net) + fb : packed_floats(*net) * sizeof(float);
}

int evs_pack_weights(const evs_net* net, const float* const* w, void* packed, void* stream) {
  int st = validate_net(net);
  if (st) return st;
  if (!w || !packed) return fail(EVS_EINVAL, "weights or packed buffer is NULL");
  for (int l = 0; l < net->n_layers; ++l)
    if (!w[l]) return fail(EVS_EINVAL, "a layer weight pointer is NULL");
  char* dst = reinterpret_cast<char*>(packed);
  for (int l = 0; l < net->n_layers; ++l) {
    const size_t b = (size_t)net->ch[l + 1] * net->ch[l] * 9 * sizeof(float);
    EVS_HIP(hipMemcpyAsync(dst, w[l], b, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    dst += b;
  }
  // the MFMA fragments of the forward kernels, built once from the copy
  if (forward_frag_bytes(*net) > 0) {
    const FwdNetArgs na = make_net_args(*net, packed, false);
    uint32_t* fb = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(packed) + frag_offset(*net));
    if ((st = forward_prepack(*net, na, fb, (hipStream_t)stream))) return st;
  }
  return EVS_OK;
}

size_t evs_workspace_bytes(const evs_net* net, const evs_clip* clips, int32_t n_clips,
                           int32_t ckpt_every, int32_t op) {
  if (!clips || n_clips < 1) return (size_t)-1;
  switch (op) {
    case EVS_OP_FORWARD: {
      if (validate_net(net) != EVS_OK) return (size_t)-1;
      size_t b = 0;
      if (!fused_shape(*net)) {
        // layer by layer: the clips run one after the other in one workspace
        for (int i = 0; i < n_clips; ++i) {
          if (validate_clip(*net, clips[i], false) != EVS_OK) return (size_t)-1;
          const evs_clip& c = clips[i];
          size_t bi = layerwise_workspace_bytes(*net, c.N, c.H, c.W);
          // RGB input: the Eq. (1) frames are formed first
          if (net->input == EVS_INPUT_RGB_LOGDIFF) bi += align256((size_t)c.N * c.T * c.H * c.W * 4);
          b = bi > b ? bi : b;
        }
        return b;
      }
      for (int i = 0; i < n_clips; ++i) {
        if (validate_clip(*net, clips[i], false) != EVS_OK) return (size_t)-1;
        if (clips[i].v_state)
          b += align256((size_t)clips[i].N * real_sum_channels(*net) * clips[i].H * clips[i].W * 4);
      }
      if (n_clips > 1) b += 256;   // work counter
      return b;
    }
    case EVS_OP_BACKWARD:
      if (validate_net(net) != EVS_OK || n_clips != 1) return (size_t)-1;
      return backward_workspace_bytes(*net, clips[0], ckpt_every);
    case EVS_OP_EMD:
      return emd_workspace_bytes(clips[0].N, clips[0].T, net ? net->ch[net->n_layers] : 2, clips[0].H,
                                 clips[0].W);
    case EVS_OP_COMPACT:
      return compact_workspace_bytes(clips[0].T, net ? net->ch[net->n_layers] : 2, clips[0].H, clips[0].W);
    default:
      return (size_t)-1;
  }
}

int evs_forward(const evs_net* net, const void* packed, const evs_clip* clips, int32_t n_clips,
                float* ckpt, int32_t ckpt_every, void* ws, size_t ws_bytes, int32_t* dev_status, void* stream) {
  int st = validate_net(net);
  if (st) return st;
  if (!packed) return fail(EVS_EINVAL, "packed weights are NULL");
  if (!clips || n_clips < 1 || n_clips > kMaxBatchClips)
    return fail(EVS_EINVAL, "n_clips must be 1..24");
  for (int i = 0; i < n_clips; ++i)
    if ((st = validate_clip(*net, clips[i], true))) return st;
  if (ckpt && (ckpt_every < 1 || n_clips != 1)) return fail(EVS_EINVAL, "ckpt needs ckpt_every >= 1 and one clip");
  if ((reinterpret_cast<uintptr_t>(dev_status) & 3u) != 0) return fail(EVS_EINVAL, "dev_status must be 4-byte aligned");
  const size_t need = evs_workspace_bytes(net, clips, n_clips, ckpt_every, EVS_OP_FORWARD);
  if (need > 0 && (!ws || ws_bytes < need)) return fail(EVS_EWORKSPACE, "forward workspace too small");
  hipStream_t s = (hipStream_t)stream;
  // NaN inputs: one streaming pass over each clip's x, only when asked for;
  // for nets whose input layer splits x into fp16 parts (FP32, three input
  // channels, hidden layers, hard spikes) the same pass flags |x| >= 65520
  if (dev_status) {
    const bool fp16_split = net->precision == EVS_FP32 && net->input == EVS_INPUT_DIRECT && net->ch[0] == 3 &&
                            net->n_layers >= 2 && !net->relaxed && fused_shape(*net);
    for (int i = 0; i < n_clips; ++i) {
      const evs_clip& c = clips[i];
      const size_t frames = net->input == EVS_INPUT_RGB_LOGDIFF ? (size_t)c.T + 1 : (size_t)c.T;
      const size_t chans = net->input == EVS_INPUT_RGB_LOGDIFF ? 3 : (size_t)net->ch[0];
      if ((st = count_nan(c.x, (size_t)c.N * frames * chans * c.H * c.W, dev_status + EVS_STATUS_NAN_X, s,
                          fp16_split ? 65520.f : 0.f, dev_status + EVS_STATUS_FLAGS, EVS_FLAG_X_RANGE)))
        return st;
    }
  }
  if (!fused_shape(*net)) {
    // no fused kernel for this shape: layer by layer, clip after clip; RGB
    // input goes through the Eq. (1) kernel into the workspace first (the
    // fused kernels form the same values while staging)
    const int sumc = real_sum_channels(*net);
    for (int i = 0; i < n_clips; ++i) {
      const evs_clip& c = clips[i];
      const long long HW = (long long)c.H * c.W;
      LwClip lc{};
      lc.N = c.N; lc.T = c.T; lc.H = c.H; lc.W = c.W;
      lc.x = c.x;
      lc.x_nstride = (long long)c.T * net->ch[0] * HW;
      if (net->input == EVS_INPUT_RGB_LOGDIFF) {
        float* xd = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) +
                                             align256(layerwise_workspace_bytes(*net, c.N, c.H, c.W)));
        if ((st = logdiff(c.x, c.N, c.T, c.H, c.W, net->lum_scale, net->knee, xd, s))) return st;
        lc.x = xd;
        lc.x_nstride = (long long)c.T * HW;
      }
      lc.v_in = c.v_state;
      lc.vin_nstride = (long long)sumc * HW;
      lc.v_out = c.v_state;
      lc.s_out = c.s_out;
      lc.s_fp32 = c.s_fp32;
      lc.ckpt = ckpt;
      lc.ckpt_every = ckpt ? ckpt_every : 0;
      lc.h_trace = c.h_trace;
      for (int k = 0; k < 4; ++k) lc.tb[k] = c.trace_box[k];
      if ((st = layerwise_forward(*net, reinterpret_cast<const float*>(packed), lc, ws, s))) return st;
    }
    return EVS_OK;
  }
  const FwdNetArgs na = make_net_args(*net, packed);
  const int sumc = na.sum_c;
  char* wsp = reinterpret_cast<char*>(ws);

  auto clip_args = [&](const evs_clip& c, int tile, FwdClipArgs& ca) -> int {
    int th = 0, tw = 0;
    forward_tile_dims(*net, tile, &th, &tw);
    if (th == 0) return fail(EVS_EUNSUPPORTED, "no compiled forward kernel for this network shape");
    ca = FwdClipArgs{};
    ca.x = c.x;
    ca.s_out = c.s_out;
    ca.s_fp32 = c.s_fp32;
    ca.h_trace = c.h_trace;
    ca.N = c.N; ca.T = c.T; ca.H = c.H; ca.W = c.W;
    ca.tiles_x = (c.W + tw - 1) / tw;
    ca.tiles_y = (c.H + th - 1) / th;
    const int64_t HW = (int64_t)c.H * c.W;
    ca.x_nstride = net->input == EVS_INPUT_RGB_LOGDIFF ? (int64_t)(c.T + 1) * 3 * HW : (int64_t)c.T * net->ch[0] * HW;
    ca.vin_nstride = (int64_t)sumc * HW;
    if (c.trace_box[2] > 0) {
      ca.tb_y0 = c.trace_box[0]; ca.tb_x0 = c.trace_box[1]; ca.tb_h = c.trace_box[2]; ca.tb_w = c.trace_box[3];
    } else {
      ca.tb_y0 = 0; ca.tb_x0 = 0; ca.tb_h = c.H; ca.tb_w = c.W;
    }
    ca.trace_nstride = (int64_t)c.T * sumc * ca.tb_h * ca.tb_w;
    if (c.v_state) {
      // the initial state is read from a private copy so that workgroups
      // writing the final state cannot race with halo reads of the initial one
      const size_t b = (size_t)c.N * sumc * c.H * c.W * 4;
      float* copy = reinterpret_cast<float*>(wsp);
      wsp += align256(b);
      int cst = copy_f32(copy, c.v_state, b / 4, s);
      if (cst) return cst;
      ca.v_in = copy;
      ca.v_out = c.v_state;
    }
    return EVS_OK;
  };

  if (n_clips == 1) {
    const int tile = choose_tile(*net, clips[0].H, clips[0].W, clips[0].N);
    FwdClipArgs ca;
    if ((st = clip_args(clips[0], tile, ca))) return st;
    ca.ckpt = ckpt;
    ca.ckpt_every = ckpt ? ckpt_every : 0;
    return launch_forward(*net, na, ca, tile, s);
  }
  // batched: one tile shape for all clips (the one tuned for the largest clip)
  int big = 0;
  for (int i = 1; i < n_clips; ++i)
    if ((double)clips[i].H * clips[i].W > (double)clips[big].H * clips[big].W) big = i;
  const int tile = forward_batched_tile(*net, choose_tile(*net, clips[big].H, clips[big].W));
  if (tile < 0) return fail(EVS_EUNSUPPORTED, "no batched kernel compiled for this network");
  if (net->relaxed) return fail(EVS_EUNSUPPORTED, "batched forward: relaxed spikes not supported");
  if (net->input != EVS_INPUT_DIRECT) return fail(EVS_EUNSUPPORTED, "batched forward: direct input only");
  for (int i = 0; i < n_clips; ++i)
    if (clips[i].s_fp32 || clips[i].h_trace)
      return fail(EVS_EUNSUPPORTED, "batched forward: int8 spikes only, no traces");
  // longest-first order of clips: the work per tile is proportional to T
  int order[kMaxBatchClips];
  for (int i = 0; i < n_clips; ++i) order[i] = i;
  for (int i = 1; i < n_clips; ++i)
    for (int k = i; k > 0 && clips[order[k]].T > clips[order[k - 1]].T; --k) std::swap(order[k], order[k - 1]);
  BatchTable bt{};
  bt.n_clips = n_clips;
  int items = 0;
  for (int i = 0; i < n_clips; ++i) {
    FwdClipArgs& ca = bt.clip[i];
    if ((st = clip_args(clips[order[i]], tile, ca))) return st;
    bt.item_start[i] = items;
    const long long add = (long long)ca.tiles_x * ca.tiles_y * ca.N;
    if (items + add > 2000000000LL) return fail(EVS_EOVERFLOW, "too many work items");
    items += (int)add;
  }
  bt.item_start[n_clips] = items;
  bt.n_items = items;
  int32_t* counter = reinterpret_cast<int32_t*>(wsp);
  if ((st = zero_i32(counter, 8, s))) return st;      // one work queue per XCD
  return launch_forward_batched(*net, na, bt, tile, counter, s);
}

int32_t evs_tile_count(const evs_net* net) {
  if (validate_net(net) != EVS_OK) return -1;
  return forward_tile_count(*net);
}

const char* evs_tile_name(const evs_net* net, int32_t tile_id) {
  if (validate_net(net) != EVS_OK) return nullptr;
  return forward_tile_name(*net, tile_id);
}

int evs_set_tile(const evs_net* net, int32_t tile_id) {
  int st = validate_net(net);
  if (st) return st;
  if (tile_id >= forward_tile_count(*net)) return fail(EVS_EINVAL, "tile id out of range");
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_forced[net_key(*net)] = tile_id;
  return EVS_OK;
}

}  // extern "C"
