/*
 * evs.h -- C ABI of the MI355X EvSNet library (libevs.so).
 *
 * EvSNet (arXiv 2508.18071, Sec. 3.3) turns noisy rendered video into
 * bipolar event streams: every frame passes through 3x3 convolution layers,
 * and every layer feeds bipolar leaky integrate-and-fire (BiLIF) units whose
 * membrane potential is carried through time at every pixel.  This library
 * computes, on one AMD Instinct MI355X (gfx950):
 *
 *   evs_forward         the network over a clip (or a batch of clips)
 *   evs_backward        the surrogate-gradient BPTT backward (Eq. 4)
 *   evs_emd_loss        the bidirectional polarity-split EMD loss (Eq. 7-11)
 *   evs_compact_events  dense spike frames -> (t, x, y, c, polarity) events
 *   evs_logdiff         the network input of Eq. 1 from RGB frames
 *   evs_contrast_events contrast-crossing target events of clean frames
 *
 * Network definition, per frame t and layer l = 1..L (s_0[t] = x[t]):
 *   u_l[t] = conv3x3(s_{l-1}[t], W_l)       zero "same" padding, stride 1,
 *                                           cross-correlation, no bias
 *   h_l[t] = leak * v_l[t-1] + u_l[t]       charge (Eq. 2, leak = 1 - 1/tau)
 *   s_l[t] = +1 if h >= theta, -1 if h <= -theta, else 0     (Eq. 3)
 *   v_l[t] = h_l[t] - theta * s_l[t]        reset
 * with v_l[-1] = 0 unless an initial state is supplied.
 *
 * Conventions shared by every entry point
 *   - Every tensor argument is a DEVICE pointer owned by the caller, dense,
 *     row-major in the index order written next to it; the library never
 *     keeps a pointer after the call returns (its kernels read and write it
 *     asynchronously on `stream`).  Host-memory arguments are marked "host".
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *     only enqueue work: no host synchronisation and no device allocation
 *     happen inside evs_forward, evs_backward, evs_emd_loss or
 *     evs_compact_events, so they may be captured in a hipGraph.  Scratch
 *     memory comes from the caller's workspace `ws` of `ws_bytes` bytes
 *     (size from evs_workspace_bytes; alignment 256 bytes).
 *   - Every call returns an evs_status.  Argument errors are detected on the
 *     host before anything is enqueued; the message is then available from
 *     evs_last_error() on the calling thread.  EVS_EHIP reports a failed HIP
 *     launch.  Outputs are overwritten, never accumulated.
 */
#ifndef EVS_H
#define EVS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EVS_OK = 0,
  EVS_EINVAL = 1,        /* bad argument (null pointer, size, range) */
  EVS_EUNSUPPORTED = 2,  /* valid but not implemented (e.g. channel count) */
  EVS_EWORKSPACE = 3,    /* workspace missing or too small */
  EVS_EHIP = 4,          /* HIP runtime error */
  EVS_EOVERFLOW = 5      /* an index or size does not fit its field */
} evs_status;

typedef enum { EVS_FP32 = 0, EVS_BF16 = 1 } evs_precision;

/* Network description (host struct, read during the call only).
 *   n_layers   L in 1..EVS_MAX_LAYERS (8)
 *   ch[0]      input channels Cin: 3 (RGB) or 1
 *   ch[1..L-1] hidden widths, each in 1..32.  Nets of at most three layers
 *              whose hidden layers have equal widths run the fused kernels
 *              (all layers and frames of a tile in one launch; widths
 *              padded internally to 16 or 32 with zero weights; the tile
 *              calls below list them); other shapes run layer by layer
 *              (one launch per frame and layer, FP32 VALU arithmetic on the
 *              same operands, the same outputs and layouts; RGB input is
 *              formed by evs_logdiff's kernel first).  Entries past ch[L]
 *              are ignored.
 *   ch[L]      output channels in 1..2.  With two outputs, channel 0 is the
 *              ON stream and channel 1 the OFF stream; each is a BiLIF unit
 *              that may itself fire with either sign.
 *   theta      firing threshold V_th > 0 (Eq. 2-3)
 *   leak       beta = 1 - 1/tau in [0, 1]
 *   surr_alpha slope alpha of the surrogate step sigma (see `surrogate`)
 *              used by evs_backward and by relaxed forwards (Eq. 4)
 *   precision  EVS_FP32: FP32 convolutions: sums accumulate in FP32 and
 *              every product is carried to within 2^-22 of its value
 *              (operands split into fp16 parts on the matrix cores, or f32
 *              MFMA, or FP32 multiply-adds on the layer-by-layer path),
 *              except in the input layer of fused nets with three input
 *              channels and hidden layers (hard spikes), where x and W are
 *              split into two fp16 parts each: there every product is within
 *              2^-21 |w x| (plus absolute terms below 2^-35 |w|max at the
 *              fp16 subnormal spacing), and x must satisfy
 *              |x| < 65520 (larger or infinite values give NaN potentials;
 *              the status word flags them, EVS_FLAG_X_RANGE);
 *              EVS_BF16: x and W rounded to bfloat16 (round-to-nearest-even)
 *              and multiplied on BF16 MFMA with FP32 accumulation (exact
 *              products; the layer-by-layer path forms the same products
 *              with FP32 multiply-adds).
 *              Membrane state, threshold compare and reset are FP32 in both.
 *   relaxed    0: hard spikes (Eq. 3).  1: smooth spikes
 *              sigma(h-theta) - sigma(-h-theta) in the output and the reset,
 *              whose exact derivative is the surrogate (FP32 only; used to
 *              check gradients against finite differences).
 *   detach_reset  evs_backward only: 1 stops the gradient through the
 *              reset term theta * s.
 *   surrogate  smooth step sigma of the surrogate and of relaxed spikes:
 *              EVS_SURR_SIGMOID (0) sigma(z) = 1/(1+exp(-alpha z)), or
 *              EVS_SURR_ATAN (1) sigma(z) = 1/2 + arctan(pi/2 alpha z)/pi,
 *              the arctangent surrogate the paper trains with (Sec. 3.3).
 *   input      what evs_forward reads from clip x:
 *              EVS_INPUT_DIRECT (0): the network input itself,
 *              [N][T][ch[0]][H][W].
 *              EVS_INPUT_RGB_LOGDIFF (1): T+1 linear RGB frames
 *              [N][T+1][3][H][W]; the forward forms the one-channel input of
 *              Eq. 1 (Sec. 3.2) as it stages each frame, bit-identical to
 *              evs_logdiff with the same lum_scale and knee.  Needs ch[0] = 1
 *              and FP32; forward only (one clip per call): evs_backward
 *              rejects it, training passes the output of evs_logdiff.
 *   lum_scale, knee  used with EVS_INPUT_RGB_LOGDIFF only, as in
 *              evs_logdiff (255 and 20 in the paper's reading).           */
#define EVS_SURR_SIGMOID 0
#define EVS_SURR_ATAN 1
#define EVS_INPUT_DIRECT 0
#define EVS_INPUT_RGB_LOGDIFF 1
#define EVS_MAX_LAYERS 8
typedef struct evs_net {
  int32_t n_layers;
  int32_t ch[EVS_MAX_LAYERS + 1];
  float theta;
  float leak;
  float surr_alpha;
  int32_t precision;
  int32_t relaxed;
  int32_t detach_reset;
  int32_t surrogate;
  int32_t input;
  float lum_scale;
  float knee;
} evs_net;

/* One clip, or a batch of N clips of equal shape (host struct).
 *   x        [N][T][Cin][H][W] float32, the network input (noisy linear
 *            RGB frames for Cin = 3); [N][T+1][3][H][W] RGB frames for
 *            nets with input = EVS_INPUT_RGB_LOGDIFF
 *   s_out    [N][T][Cout][H][W] spikes: int8 in {-1,0,1} (s_fp32 = 0) or
 *            float32 (s_fp32 = 1; required for relaxed nets); may be NULL
 *   v_state  NULL, or [N][sum_l C_l][H][W] float32 membrane potentials of
 *            all layers (layer-major): read as the initial state and
 *            overwritten with the state after frame T-1.  Splitting a clip
 *            at any frame and carrying v_state gives bit-identical spikes.
 *   h_trace  NULL, or [N][T][sum_l C_l][h][w] float32: the charged
 *            potential h of every layer at every frame (debug/training),
 *            over the window trace_box = {y0, x0, h, w} of the frame, or over
 *            the whole frame (h = H, w = W) when trace_box[2] == 0.        */
typedef struct evs_clip {
  int32_t N, T, H, W;
  const float* x;
  void* s_out;
  int32_t s_fp32;
  float* v_state;
  float* h_trace;
  int32_t trace_box[4];
} evs_clip;

/* Event record produced by evs_compact_events, packed in a uint64:
 *   bits  0..31  t (frame index; physical time t / F_evt, F_evt = 1000)
 *   bits 32..43  x       bits 44..55  y
 *   bits 56..62  channel bit 63 polarity (1 = negative spike)            */
#define EVS_EVENT_T(e)   ((uint32_t)((e) & 0xffffffffu))
#define EVS_EVENT_X(e)   ((uint32_t)(((e) >> 32) & 0xfffu))
#define EVS_EVENT_Y(e)   ((uint32_t)(((e) >> 44) & 0xfffu))
#define EVS_EVENT_C(e)   ((uint32_t)(((e) >> 56) & 0x7fu))
#define EVS_EVENT_NEG(e) ((uint32_t)((e) >> 63))

/* Device status word: a caller-owned DEVICE array of EVS_STATUS_WORDS
 * int32 values that evs_forward, evs_backward and evs_compact_events update
 * from their kernels when it is passed (it may be NULL: nothing is
 * recorded).  Updates accumulate (counts add, flag bits are OR-ed): the
 * library never clears the word, so the caller zeroes it (e.g. a zero-filled
 * tensor) before the calls it wants to watch.  Updating it needs no host
 * synchronisation and no memset, so the calls stay graph-capturable.
 *   [EVS_STATUS_NAN_X]    NaN values in the network input x of evs_forward
 *                         (every value of every clip: [N][T][Cin][H][W],
 *                         or the T+1 RGB frames of RGB-input nets), counted
 *                         by one extra streaming read of x (4 bytes per
 *                         value) that runs only when the word is given.  A
 *                         NaN input propagates (a NaN potential never
 *                         reaches a threshold, so its neurons stay silent);
 *                         the NaN potentials that mask the neurons outside
 *                         the image are not inputs and are not counted.
 *   [EVS_STATUS_NAN_GRAD] NaN values read from grad_s by evs_backward.
 *   [EVS_STATUS_FLAGS]    EVS_FLAG_EVENT_OVERFLOW: evs_compact_events found
 *                         more events than `capacity` (the list was cut; the
 *                         dense spikes and `count` stay exact).
 *                         EVS_FLAG_X_RANGE: evs_forward of an FP32 net whose
 *                         input layer splits x into fp16 parts (see
 *                         `precision`) read a value with |x| >= 65520 or an
 *                         infinity (same pass as the NaN count).
 *   [3]                   reserved (left unchanged).                       */
#define EVS_STATUS_WORDS 4
#define EVS_STATUS_NAN_X 0
#define EVS_STATUS_NAN_GRAD 1
#define EVS_STATUS_FLAGS 2
#define EVS_FLAG_EVENT_OVERFLOW 1
#define EVS_FLAG_X_RANGE 2

/* Operation selector for evs_workspace_bytes. */
typedef enum {
  EVS_OP_FORWARD = 0,
  EVS_OP_BACKWARD = 1,
  EVS_OP_EMD = 2,
  EVS_OP_COMPACT = 3
} evs_op;

/* Workspace bytes needed by `op` for these arguments (0 = none needed).
 * For EVS_OP_EMD / EVS_OP_COMPACT only clip[0].N/T/H/W and net->ch[L] are
 * read.  Returns (size_t)-1 on invalid arguments.                        */
size_t evs_workspace_bytes(const evs_net* net, const evs_clip* clips, int32_t n_clips,
                           int32_t ckpt_every, int32_t op);

/* Size in bytes of the packed weight buffer for `net`.                   */
size_t evs_packed_weights_bytes(const evs_net* net);

/* Pack the per-layer weights into one device buffer read by the kernels
 * (the weights of the 3x3 convolutions of Sec. 3.3).  The buffer holds the
 * FP32 weights layer after layer and, 256-byte aligned after them, the
 * forward kernels' matrix-core operand fragments (BF16-rounded weights, or
 * the two-part splits of FP32 nets with their power-of-two scales) built
 * once here, which every forward workgroup copies instead of building; a
 * kernel whose layout the block was not built for builds its own.  The
 * buffer is tied to the channel counts and precision of `net`.  Enqueued
 * on `stream` (a copy and one kernel); the sources must stay valid until it
 * has run.
 *   w       host array of L device pointers; w[l] is float32
 *           [C_{l+1}][C_l][3][3] (torch Conv2d layout)
 *   packed  device buffer of evs_packed_weights_bytes(net) bytes        */
int evs_pack_weights(const evs_net* net, const float* const* w, void* packed, void* stream);

/* Forward pass (Sec. 3.3, Eq. 2-3 with 3x3 convolution layers).
 *   clips, n_clips  host array of clip descriptors.  n_clips = 1 runs the
 *           single-clip kernel over N x tiles.  n_clips > 1 (at most 24)
 *           runs the persistent batched kernel: (clip, tile) work items in
 *           longest-first order are taken from a device counter in `ws`.
 *   ckpt    NULL, or (n_clips = 1 only) [N][ceil(T/ckpt_every)][sum C][H][W]
 *           float32: the membrane of every layer before frames 0, k, 2k, ...
 *           (k = ckpt_every), as needed by evs_backward.
 *   tile    tiles are chosen by the autotuner cache (evs_autotune) or a
 *           built-in default; results do not depend on the tile choice.
 *   dev_status  NULL or the device status word (counts NaN inputs, flags
 *               inputs outside the fp16 range where `precision` says so). */
int evs_forward(const evs_net* net, const void* packed, const evs_clip* clips, int32_t n_clips,
                float* ckpt, int32_t ckpt_every, void* ws, size_t ws_bytes, int32_t* dev_status,
                void* stream);

/* Surrogate-gradient BPTT backward through the whole clip (Eq. 4).
 * The surrogate is psi(h) = sigma'(h - theta) + sigma'(-h - theta), the
 * derivative of sigma(h - theta) - sigma(-h - theta); one BiLIF step's
 * adjoint with g_v = dL/dv[t] arriving from frame t+1 is
 *     g_h = (G - theta g_v) psi(h) + g_v   (G * psi(h) + g_v if detached)
 *     dL/dv[t-1] = leak * g_h,   dL/du[t] = g_h.
 *   clip    the same x as the forward; clip->v_state is not read (the
 *           initial state is ckpt segment 0); s_out/h_trace are ignored.
 *   ckpt    the checkpoints written by evs_forward with the same ckpt_every
 *   grad_s  [N][T][Cout][H][W] float32 dLoss/ds_L
 *   grad_w  host array of L device pointers, float32 [C_l][C_{l-1}][3][3],
 *           overwritten with dLoss/dW_l (summed over the batch)
 *   grad_x  NULL or [N][T][Cin][H][W] float32 dLoss/dx
 *   grad_v  NULL or [N][sum C][H][W] float32 dLoss/d(initial membrane)
 *   dev_status  NULL or the device status word (counts NaN values of grad_s)
 * Segments are recomputed from their checkpoints in reverse order (with
 * the forward's arithmetic, input range included); the weight gradient is
 * reduced deterministically (no float atomics).  FP32 nets: every product
 * of the gradient convolutions is carried to within 2^-23 of its value
 * (exact three-part bf16 splits on the matrix cores, FP32 MFMA or VALU),
 * sums and recurrences in FP32.                                         */
int evs_backward(const evs_net* net, const void* packed, const evs_clip* clip,
                 const float* ckpt, int32_t ckpt_every, const float* grad_s,
                 float* const* grad_w, float* grad_x, float* grad_v,
                 void* ws, size_t ws_bytes, int32_t* dev_status, void* stream);

/* Bidirectional polarity-split EMD loss plus spike-count term (Eq. 7-11).
 *   s       [N][T][C][H][W] float32 spikes, C = 2 (channel 0 = ON stream,
 *           channel 1 = OFF stream, each scored with its signed values) or
 *           C = 1 (bipolar; split into S*[S>0] and -S*[S<0] as in Eq. 9)
 *   e       [N][T][2][H][W] int8 target counts (>= 0): [..][0] ON, [..][1] OFF
 *   loss    device float32 scalar: sum over clips, channels and pixels of
 *           (1/2T) sum_i (|D_i| + |R_i|), D = prefix and R = suffix sums of
 *           S - E over time, plus lambda_count * sum over pixels of
 *           | sum_t |S| - sum_t E |.
 *   grad_s  NULL or [N][T][C][H][W] float32 dloss/ds (subgradient 0 at 0)
 * The reduction order is fixed, so results are bitwise reproducible.    */
int evs_emd_loss(const float* s, const int8_t* e, int32_t N, int32_t T, int32_t C,
                 int32_t H, int32_t W, float lambda_count, float* loss, float* grad_s,
                 void* ws, size_t ws_bytes, void* stream);

/* evs_emd_loss without a workspace, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight training loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * evs_emd_loss; its scratch (the per-block partial losses) is a static
 * device array of 1 MiB that every GPU the library runs on holds until the
 * process ends, so N x H x W is limited to 2^25 pixels (EVS_EWORKSPACE
 * above that).  Allocates nothing on any call.  Every call on one GPU uses
 * that GPU's one array: calls that overlap on one GPU (other streams,
 * threads) race and must be serialised by the caller.                    */
int evs_emd_loss_noalloc(const float* s, const int8_t* e, int32_t N, int32_t T, int32_t C,
                         int32_t H, int32_t W, float lambda_count, float* loss, float* grad_s,
                         void* stream);

/* Dense spikes -> event list in (t, c, y, x) order (Sec. 3.1 event tuples).
 *   s         [T][C][H][W] int8 spikes
 *   events    device uint64 array of `capacity` records (format above)
 *   count     device int64: the number of events in s.  If it exceeds
 *             capacity, only the first `capacity` events are written and
 *             EVS_FLAG_EVENT_OVERFLOW is set in dev_status (NULL or the
 *             device status word).
 * Requires W, H <= 4096, C <= 128, T < 2^32.                            */
int evs_compact_events(const int8_t* s, int32_t T, int32_t C, int32_t H, int32_t W,
                       uint64_t* events, int64_t capacity, int64_t* count,
                       void* ws, size_t ws_bytes, int32_t* dev_status, void* stream);

/* Network input of Eq. (1) (Sec. 3.2): per pixel the Rec. 709 luminance
 * L = lum_scale * (0.2126 R + 0.7152 G + 0.0722 B) of linear RGB frames,
 * mapped to ln L at and above the knee and to (ln knee / knee) * L below it,
 * and differenced in time: X_k = L_log[k] - L_log[k-1] for k = 1..T.  The
 * result is the input of a one-channel net (ch[0] = 1).
 *   rgb    [N][T+1][3][H][W] float32 frames 0..T
 *   x_out  [N][T][1][H][W] float32
 *   lum_scale, knee  > 0 (the paper's rho; e.g. 255 and 20)
 * No workspace; graph-capturable.                                        */
int evs_logdiff(const float* rgb, int32_t N, int32_t T, int32_t H, int32_t W,
                float lum_scale, float knee, float* x_out, void* stream);

/* Contrast-crossing events of clean frames (training targets standing in
 * for the event simulator the paper trains against): per pixel, with L_log
 * as in evs_logdiff, the reference level starts at frame 0; at frame t >= 1
 * d = L_log[t] - ref emits n = sgn(d) floor(|d| / C) events, ref += n C.
 *   rgb    [N][T][3][H][W] float32 clean frames
 *   e_out  [N][T][2][H][W] int8: channel 0 ON = max(n, 0), channel 1
 *          OFF = max(-n, 0), clamped to 127; frame 0 is all zero
 *   C      contrast threshold > 0
 * FP32 arithmetic; no workspace; graph-capturable.                       */
int evs_contrast_events(const float* rgb, int32_t N, int32_t T, int32_t H, int32_t W,
                        float lum_scale, float knee, float C, int8_t* e_out, void* stream);

/* The paper's own temporal EvSNet (Sec. 3.3, Eq. 5-6; kernel size 7 and
 * depth M = 3 from Sec. 4): per pixel of a one-channel input sequence X,
 *     h0 = ReLU(conv0 X),
 *     h_i = ReLU(h_{i-1} + conv_{2i}(ReLU(conv_{2i-1} h_{i-1}))), i = 1..3,
 *     u = wp . h3 + bp,  S = BiLIF(u) over time (Eq. 2-3, v starts at 0).
 * Every conv is a kernel-7 cross-correlation over frames with zero padding
 * of 3 frames on both sides (centred: frame t sees t-21 .. t+21 overall)
 * and a bias per output channel; pixels are independent.  Operands are
 * rounded to bfloat16 (input, weights, stored activations h_i, a_i),
 * sums, biases and the BiLIF state are FP32.
 *   net      hidden = 16 (the only width compiled), theta > 0, leak in [0, 1]
 *   weights  device float32, evs_tnet_weight_floats() values in this order:
 *            w0 [16][7], b0 [16]; then for k = 1..6: w_k [16][16][7]
 *            ([out][in][tap]), b_k [16]; then wp [16], bp [1]
 *   x        [N][T][H][W] float32 (e.g. the output of evs_logdiff)
 *   s_out    [N][T][H][W] int8 spikes in {-1, 0, 1}
 *   debug    NULL, or [N][T][7*16 + 2][H][W] float32: the activations h0,
 *            a1, h1, a2, h2, a3, h3 (16 channels each, bf16 values), u and
 *            the charged BiLIF potential leak * v + u, per frame
 * Returns EVS_EUNSUPPORTED for other widths, EVS_EINVAL / EVS_EOVERFLOW
 * for bad arguments (checked before anything is enqueued).              */
typedef struct evs_tnet {
  int32_t hidden;
  float theta;
  float leak;
} evs_tnet;
size_t evs_tnet_weight_floats(const evs_tnet* net);
int evs_tnet_forward(const evs_tnet* net, const float* weights, const float* x, int32_t N, int32_t T,
                     int32_t H, int32_t W, int8_t* s_out, float* debug, void* stream);

/* Time the compiled tile shapes for this network and frame size on
 * `stream` (allocates its own scratch; not capture-safe) and remember the
 * fastest for later evs_forward calls with this (net, H, W).  If the
 * environment variable EVS_AUTOTUNE_CACHE names a file, the cache is
 * loaded from and saved to it.  `chosen` (host, may be NULL) receives the
 * chosen tile id, or -1 for a shape that runs layer by layer (no tiles to
 * choose from; nothing is timed).                                        */
int evs_autotune(const evs_net* net, int32_t H, int32_t W, int32_t T, int32_t* chosen, void* stream);

/* Number of compiled tile variants for `net` (0 for a shape that runs
 * layer by layer), and a description of one (host string, valid until the
 * library is unloaded).                                                  */
int32_t evs_tile_count(const evs_net* net);
const char* evs_tile_name(const evs_net* net, int32_t tile_id);

/* Force a tile variant for later calls with `net` (-1 = automatic).      */
int evs_set_tile(const evs_net* net, int32_t tile_id);

/* hipGraph capture helpers.  evs_graph_begin starts capturing `stream`
 * (must not be the NULL stream); every capture-safe call enqueued on it
 * (evs_forward, evs_backward, evs_emd_loss, evs_compact_events) is recorded
 * instead of run.  evs_graph_end stops the capture and instantiates the
 * graph into *graph_exec (an opaque hipGraphExec_t owned by the caller);
 * evs_graph_launch replays it on a stream; evs_graph_destroy frees it.
 * A replay reuses the device pointers that were captured.                */
int evs_graph_begin(void* stream);
int evs_graph_end(void* stream, void** graph_exec);
int evs_graph_launch(void* graph_exec, void* stream);
int evs_graph_destroy(void* graph_exec);

/* Static strings. */
const char* evs_status_str(int status);
const char* evs_last_error(void);
const char* evs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EVS_H */
