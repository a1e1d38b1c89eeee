// Tile autotuner, its persistent cache, and hipGraph capture helpers.
//
// evs_autotune times every compiled tile variant of a network on a
// synthetic clip of the requested frame size with HIP events and remembers
// the fastest for later evs_forward calls.  The cache lives in the process
// and, if EVS_AUTOTUNE_CACHE names a file, is loaded from and saved to it
// as a JSON list of {"key": [L, c0, c1, c2, c3, precision, H, W], "tile": id}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "evs_ops.hpp"

namespace evs {

using ShapeKey = std::tuple<int, int, int, int, int, int, int, int>;
std::map<ShapeKey, int> tuned_snapshot();
void set_tuned(const ShapeKey& k, int tile);

namespace {
std::once_flag g_load_once;
std::mutex g_file_mu;

const char* cache_path() {
  const char* p = std::getenv("EVS_AUTOTUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

void load_file() {
  const char* path = cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  std::fclose(f);
  size_t pos = 0;
  while ((pos = txt.find("\"key\"", pos)) != std::string::npos) {
    int k[8], tile;
    const size_t lb = txt.find('[', pos);
    if (lb == std::string::npos) break;
    if (std::sscanf(txt.c_str() + lb, "[%d,%d,%d,%d,%d,%d,%d,%d], \"tile\": %d", &k[0], &k[1], &k[2], &k[3], &k[4],
                    &k[5], &k[6], &k[7], &tile) == 9)
      set_tuned(ShapeKey{k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7]}, tile);
    pos = lb + 1;
  }
}

void save_file() {
  const char* path = cache_path();
  if (!path) return;
  std::lock_guard<std::mutex> lk(g_file_mu);
  const auto snap = tuned_snapshot();
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "[\n");
  size_t i = 0;
  for (const auto& kv : snap) {
    const auto& k = kv.first;
    std::fprintf(f, "  {\"key\": [%d,%d,%d,%d,%d,%d,%d,%d], \"tile\": %d}%s\n", std::get<0>(k), std::get<1>(k),
                 std::get<2>(k), std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k),
                 kv.second, ++i < snap.size() ? "," : "");
  }
  std::fprintf(f, "]\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}
}  // namespace

void load_tile_cache_once() { std::call_once(g_load_once, load_file); }

}  // namespace evs

using namespace evs;

extern "C" {

int evs_autotune(const evs_net* net, int32_t H, int32_t W, int32_t T, int32_t* chosen, void* stream) {
  int st = validate_net(net);
  if (st) return st;
  if (H < 1 || W < 1 || T < 1 || H > 4096 || W > 4096) return fail(EVS_EINVAL, "autotune: bad frame size");
  load_tile_cache_once();
  const int n = forward_tile_count(*net);
  if (n < 1) {
    // a shape without fused kernels runs layer by layer: nothing to choose
    if (chosen) *chosen = -1;
    return EVS_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t HW = (size_t)H * W;
  const int cin = net->ch[0], cout = net->ch[net->n_layers];
  size_t wfl = 0;
  for (int l = 0; l < net->n_layers; ++l) wfl += (size_t)net->ch[l + 1] * net->ch[l] * 9;
  float *x = nullptr, *w = nullptr;
  int8_t* out = nullptr;
  hipEvent_t e0, e1;
  // RGB log-difference nets read T+1 RGB frames
  const size_t xfl = net->input == EVS_INPUT_RGB_LOGDIFF ? (size_t)(T + 1) * 3 * HW : (size_t)T * cin * HW;
  EVS_HIP(hipMalloc(&x, xfl * 4));
  EVS_HIP(hipMalloc(&w, wfl * 4));
  EVS_HIP(hipMalloc(&out, (size_t)T * cout * HW));
  EVS_HIP(hipEventCreate(&e0));
  EVS_HIP(hipEventCreate(&e1));
  int best = 0;
  float best_ms = 1e30f;
  if ((st = fill_uniform(x, xfl, 1u, 0.f, 2.f, s)) ||
      (st = fill_uniform(w, wfl, 2u, -0.5f, 0.5f, s))) goto done;
  {
    const FwdNetArgs na = make_net_args(*net, w, false);   // plain weights: no prepacked block
    FwdClipArgs ca{};
    ca.x = x;
    ca.s_out = out;
    ca.N = 1; ca.T = T; ca.H = H; ca.W = W;
    ca.x_nstride = (int64_t)xfl;
    for (int tile = 0; tile < n; ++tile) {
      int th, tw;
      forward_tile_dims(*net, tile, &th, &tw);
      ca.tiles_x = (W + tw - 1) / tw;
      ca.tiles_y = (H + th - 1) / th;
      if ((st = launch_forward(*net, na, ca, tile, s))) goto done;     // warm-up
      std::vector<float> ms;
      for (int r = 0; r < 3; ++r) {
        (void)hipEventRecord(e0, s);
        if ((st = launch_forward(*net, na, ca, tile, s))) goto done;
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) { st = fail(EVS_EHIP, "autotune: event sync"); goto done; }
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        ms.push_back(t);
      }
      std::sort(ms.begin(), ms.end());
      if (ms[1] < best_ms) { best_ms = ms[1]; best = tile; }
    }
  }
  remember_tile(*net, H, W, best);
  save_file();
  if (chosen) *chosen = best;
done:
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(x);
  (void)hipFree(w);
  (void)hipFree(out);
  return st;
}

// ---------------------------------------------------------------- graphs
int evs_graph_begin(void* stream) {
  if (!stream) return fail(EVS_EINVAL, "graph capture needs a non-default stream");
  EVS_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
  return EVS_OK;
}

int evs_graph_end(void* stream, void** graph_exec) {
  if (!stream || !graph_exec) return fail(EVS_EINVAL, "graph_end: NULL argument");
  hipGraph_t g = nullptr;
  EVS_HIP(hipStreamEndCapture((hipStream_t)stream, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_check(e, "hipGraphInstantiate");
  *graph_exec = ex;
  return EVS_OK;
}

int evs_graph_launch(void* graph_exec, void* stream) {
  if (!graph_exec) return fail(EVS_EINVAL, "graph_launch: NULL graph");
  EVS_HIP(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream));
  return EVS_OK;
}

int evs_graph_destroy(void* graph_exec) {
  if (graph_exec) EVS_HIP(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
  return EVS_OK;
}

}  // extern "C"
