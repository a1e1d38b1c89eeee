// extern "C" entry points of the non-forward operations (declared in
// include/evs.h); each forwards to its implementation file.
#include "evs_ops.hpp"

extern "C" {
int evs_backward(const evs_net* net, const void* packed, const evs_clip* clip, const float* ckpt, int32_t k,
                 const float* grad_s, float* const* grad_w, float* grad_x, float* grad_v, void* ws, size_t wsb,
                 int32_t* dev_status, void* stream) {
  if (!net || !clip) return evs::fail(EVS_EINVAL, "backward: net or clip is NULL");
  return evs::backward(*net, packed, *clip, ckpt, k, grad_s, grad_w, grad_x, grad_v, ws, wsb, dev_status,
                       (hipStream_t)stream);
}
int evs_emd_loss(const float* s, const int8_t* e, int32_t N, int32_t T, int32_t C, int32_t H, int32_t W,
                 float lambda_count, float* loss, float* grad_s, void* ws, size_t wsb, void* stream) {
  return evs::emd_loss(s, e, N, T, C, H, W, lambda_count, loss, grad_s, ws, wsb, (hipStream_t)stream);
}
int evs_emd_loss_noalloc(const float* s, const int8_t* e, int32_t N, int32_t T, int32_t C, int32_t H, int32_t W,
                         float lambda_count, float* loss, float* grad_s, void* stream) {
  return evs::emd_loss_noalloc(s, e, N, T, C, H, W, lambda_count, loss, grad_s, (hipStream_t)stream);
}
int evs_compact_events(const int8_t* s, int32_t T, int32_t C, int32_t H, int32_t W, uint64_t* events,
                       int64_t capacity, int64_t* count, void* ws, size_t wsb, int32_t* dev_status, void* stream) {
  return evs::compact_events(s, T, C, H, W, events, capacity, count, ws, wsb, dev_status, (hipStream_t)stream);
}
size_t evs_tnet_weight_floats(const evs_tnet* net) {
  if (!net || net->hidden != 16) return (size_t)-1;
  return evs::tnet_weight_floats();
}
int evs_tnet_forward(const evs_tnet* net, const float* weights, const float* x, int32_t N, int32_t T, int32_t H,
                     int32_t W, int8_t* s_out, float* debug, void* stream) {
  if (!net) return evs::fail(EVS_EINVAL, "tnet: net is NULL");
  return evs::tnet_forward(*net, weights, x, N, T, H, W, s_out, debug, (hipStream_t)stream);
}
int evs_logdiff(const float* rgb, int32_t N, int32_t T, int32_t H, int32_t W, float lum_scale, float knee,
                float* x_out, void* stream) {
  return evs::logdiff(rgb, N, T, H, W, lum_scale, knee, x_out, (hipStream_t)stream);
}
int evs_contrast_events(const float* rgb, int32_t N, int32_t T, int32_t H, int32_t W, float lum_scale, float knee,
                        float C, int8_t* e_out, void* stream) {
  return evs::contrast_events(rgb, N, T, H, W, lum_scale, knee, C, e_out, (hipStream_t)stream);
}
}
