// EvSNet forward on gfx950: conv3x3 layers feeding BiLIF units, fused over
// all layers and all frames of a clip (arXiv 2508.18071, Sec. 3.3, Eq. 2-3).
//
// Dataflow (one workgroup = one spatial tile of TH x TW output pixels):
//   * The tile is processed on a canvas of (TH+2L) x (TW+2L) pixels.  Layer
//     l is evaluated on the canvas shrunk by l pixels on each side, so the
//     halo rings needed by the next layer are recomputed redundantly inside
//     the workgroup (no inter-workgroup exchange per frame).  Each
//     workgroup keeps the membrane state of its canvas neurons in registers
//     for all T frames; halo neurons replicate bit-for-bit the neurons of
//     the neighbouring tile because every pixel is computed by the same
//     instruction sequence.  The pixels of each layer's region are packed
//     densely into 16-pixel MFMA column blocks.
//   * Per frame, the x tile (+halo) is staged in LDS (the next frame's
//     loads overlap the current frame), and every conv runs as a transposed
//     GEMM D[cout][pixel] = W[cout][K] * S[K][pixel] on MFMA with
//     K = (tap, cin) and the pixel operand gathered from LDS; the
//     accumulator fragment IS the membrane state (C input = leak * v), so
//     BiLIF runs in place.
//   * Hidden spikes are exactly -1, 0 or +1, so every conv that reads them
//     runs on a 16-bit matrix core.  BF16 nets: bf16 spikes and bf16-rounded
//     weights.  FP32 nets keep FP32 accuracy: fp16 spikes and each weight,
//     scaled by a power of two per layer, split into two fp16 parts (every
//     product within 2^-22, sums in FP32; the state behind the conv is kept
//     in the scaled units, which is exact).  The spike fragment of a k-step
//     is loaded once and multiplied by the parts.
//   * The first layer of FP32 nets with three input channels splits x and
//     the (power-of-two scaled) W into two fp16 parts each and keeps all
//     four part products (each product within 2^-21 |w x| up to absolute
//     terms at the fp16 subnormal spacing, sums in FP32);
//     other FP32 nets use the f32 MFMA for it, BF16 nets the bf16 one with
//     bf16-rounded input.
//   * The output layer (1-2 channels) puts its (channel, part) pairs on the
//     MFMA rows: row 4c + p holds part p of channel c, and the potentials
//     are the sums of the part rows.
//   * Neurons outside the image (the conv's zero padding) and the tail
//     lanes of the last block start from a NaN potential: a NaN never
//     reaches the threshold, so they emit zero spikes with no per-frame
//     masking.  (Relaxed spikes are smooth functions of h and keep an
//     explicit mask; they are not exact in bf16, so that mode keeps FP32
//     spike buffers and the f32 MFMA / VALU paths.)
//   * Only the HBM traffic of the algorithm remains: x in (12 B/px/frame)
//     and the output spikes (int8).
#include <cmath>

#include "evs_internal.hpp"
#include "evs_device.hpp"

namespace evs {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }
constexpr int align16(int b) { return (b + 15) & ~15; }

// MODE_: 0 = inference; 1 = training/debug features (h traces, membrane
// checkpoints, FP32 spike output); 2 = relaxed (smooth) spikes with the
// features of mode 1; 3 = the backward's segment recompute (the charged
// potentials of every layer into its pixel-major trace, nothing else);
// 8 = the forward of a training step (checkpoints and FP32 spike output,
// no trace).  Only mode 0 leaves the feature code out of the loop.
// MODE_ + 4 (one-channel FP32 nets): x holds RGB frames and the input of
// Eq. (1) is formed while staging.
template <int NL_, int CIN_, int CH_, bool BF16_, int TH_, int TW_, int NW_, int MODE_>
struct Cfg {
  static constexpr int NL = NL_, CIN = CIN_, CH = CH_, TH = TH_, TW = TW_, NW = NW_, MODE = MODE_;
  static constexpr int BMODE = MODE_ == 8 ? 8 : (MODE_ & 3);
  static constexpr bool LOGX = MODE_ >= 4 && MODE_ < 8;
  static constexpr bool BF16 = BF16_, RELAX = BMODE == 2, REC = BMODE == 3;
  // the public trace (planar; relaxed builds also the backward's)
  static constexpr bool TRC = BMODE == 1 || BMODE == 2;
  // checkpoints and FP32 spike output
  static constexpr bool CKS = BMODE == 1 || BMODE == 2 || BMODE == 8;
  // any of the training / debug features (register budget)
  static constexpr bool FULL = BMODE != 0;
  static_assert(!(REC && MODE_ >= 4), "recompute builds take direct input");
  static_assert(!LOGX || (CIN_ == 1 && !BF16_), "RGB input: one-channel FP32 nets");
  static_assert(!(BF16_ && MODE_ == 2), "relaxed spikes are FP32 only");
  static constexpr int CO = 2;                       // output channels (max)
  static constexpr int NH = NL - 1;                  // hidden layers
  // BF16 nets compute layer 1 over whole canvas rows (the two edge columns
  // are junk nobody reads), so a lane's canvas pixel advances by the same
  // amount from block to block and every layer-1 x gather is a per-lane base
  // plus an immediate offset
  static constexpr bool L1LIN = BF16_ && NL >= 2;
  static constexpr int CHT = TH + 2 * NL, CWT = TW + 2 * NL;
  static constexpr int NPIX = CHT * CWT;
  static constexpr int PADF = 32;                    // front pad of every LDS plane (pixels)
  static constexpr int NT = 64 * NW;
  static constexpr int MB = CH / 16;                 // 16-row output blocks
  // layer l (1 = first hidden layer, NL = output layer) covers canvas rows
  // [l, CHT-l) and columns [l, CWT-l)
  static constexpr int rgh(int l) { return CHT - 2 * l; }
  static constexpr int rgw(int l) { return (L1LIN && l == 1) ? CWT : CWT - 2 * l; }
  static constexpr int nblk(int l) { return cdiv(rgh(l) * rgw(l), 16); }
  static constexpr int NB1 = NH >= 1 ? cdiv(nblk(1), NW) : 1;
  static constexpr int NB2 = NH >= 2 ? cdiv(nblk(2), NW) : 1;
  // waves per SIMD the register budget is cut for: four (<= 128 VGPRs) for
  // the inference build of BF16 nets with one hidden layer whose layer-1
  // state is at most 4 blocks per wave (the 8-wave 12x32 tile: two
  // workgroups, 16 waves, per CU; its frame loop has no spill code at that
  // budget, the traced build's has), else two (<= 256 VGPRs)
  static constexpr int WPE = (BF16_ && NH == 1 && NB1 <= 4 && !FULL) ? 4 : 2;
  static constexpr bool S16 = !RELAX;                // hidden spikes stored as bf16
  // FP32 nets: spikes and the weights of the convs that read them in fp16,
  // each weight (scaled by a power of two per layer) as two fp16 parts
  static constexpr bool SF16 = !BF16 && !RELAX;
  static constexpr int NSP = BF16 ? 1 : 2;           // parts of a spike-conv weight
  // Output layer (1-2 channels) of nets with one hidden layer, or two of
  // width 16, in tap-major form: per block of the last hidden layer,
  // Y[(tap, co)][pixel] = sum_ci W[co][ci][tap] s[ci][pixel] on MFMA (rows
  // tap * 2 + co, 18 of 32 live; the spike operand comes from the registers
  // of that layer's epilogue), stored to LDS; the output potential of a
  // pixel is then the sum of the 9 Y values of its neighbourhood.
  static constexpr bool OTAP = S16 && (NH == 1 || (NH == 2 && CH == 16));
  static constexpr bool OMF = S16 && NH >= 1 && !OTAP;   // output layer on MFMA, rows (channel, part)
  static constexpr int KB = CH == 32 ? 9 : 5;        // spike-operand k-steps (32 of K = 9*CH each)
  // FP32 16-wide layer 2: the last k-step holds tap 8 only (lane groups
  // 0-1), so its two weight parts share one MFMA: groups 2-3, which read
  // tap 8's spikes too, carry its low part (9 MFMAs per block, not 10)
  static constexpr bool M2 = SF16 && CH == 16 && NH >= 2;
  static constexpr int NBO = OMF ? cdiv(nblk(NL), NW) : 1;
  // tail lanes of a layer's last block read around and write to this
  // canvas pixel, which lies past the canvas and is read by no real pixel
  static constexpr int JP = NPIX + CWT + 1;
  // pixels of one LDS spike / record plane, a multiple of 16 so that an
  // 8-channel bf16/fp16 plane is a multiple of 256 bytes: the lane groups of
  // a 16-byte spike read that take the two channel halves of one tap then
  // start on the same bank, which is what the LDS needs to serve them in one
  // pass (gfx950 pairs lanes 0-7 with 24-31 and 8-15 with 16-23)
  static constexpr int NPIXL = (PADF + NPIX + 2 * CWT + 4 + 15) / 16 * 16;
  static constexpr int NOUT = OMF ? 1 : cdiv(TH * TW, NT);
  static constexpr int XN = CIN * NPIX;
  static constexpr int XPF = cdiv(XN, NT);
  static constexpr int K1 = 9 * CIN;
  static constexpr int KS1 = BF16 ? cdiv(K1, 32) : cdiv(K1, 4);
  static constexpr int XELEM = BF16 ? 2 : 4;
  // x planes plus one all-zero plane read by the padded K slots of layer 1;
  // FP32 nets with hidden layers fill them by direct global -> LDS loads of
  // 64-pixel chunks into two buffers (frame t+1 lands while t is read)
  // FP32 nets with three input channels (16 or 32 hidden channels) run layer 1
  // on the fp16 pipe as well: each staged x value is split into two fp16
  // parts, stored as 24 bytes per canvas pixel that hold the parts of the
  // pixel and its right neighbour (register staging, no raw x in LDS)
  static constexpr bool XSPLIT = !BF16 && CIN == 3 && NH >= 1 && !RELAX && !LOGX;
  static constexpr bool XDMA = !BF16 && NH >= 1 && !RELAX && !LOGX && !XSPLIT;
  static constexpr int XPP = cdiv(NPIX, NT);         // canvas pixels staged per thread (XSPLIT)
  // 16-channel spike convs run block by block with all weight fragments in
  // registers, so that block i-1's epilogue overlaps block i's MFMAs
  static constexpr bool BO = CH == 16 && S16;
  static constexpr int NFR1 = 4;                     // XSPLIT A fragments: weight parts h, l x 2 k-steps
  static constexpr int XCK = CIN * CHT;              // x chunks: one canvas row of one plane
  static constexpr int XPW = cdiv(XCK, NW);          // chunk loads per wave and frame
  // x buffer: front pad, CIN planes and the zero plane back to back (plane
  // stride NPIX), then room for the neighbourhood of the junk pixel
  static constexpr int XPL = NPIX;
  // room after the zero plane: tap offsets of real pixels, and the linear
  // layer-1 gathers of the tail lanes of the last block
  static constexpr int XTAIL = L1LIN && 16 * NW * NB1 + 2 * CWT + 2 - XPL > 2 * CWT + 4
                                   ? 16 * NW * NB1 + 2 * CWT + 2 - XPL : 2 * CWT + 4;
  static constexpr int XS1 = align16((PADF + (CIN + 1) * XPL + XTAIL) * XELEM);
  static constexpr int XS_BYTES = XSPLIT ? 3 * NPIXL * 8 : XS1 * (XDMA ? 2 : 1);
  static constexpr int SELEM = S16 ? 2 : 4;
  // bf16 spikes are stored as CH/8 planes of [pixel][8 channels] (16 B per
  // pixel): the 16 lanes of a lane group then read 256 contiguous bytes
  static constexpr int SPL = NPIXL * 16;             // bytes of one 8-channel plane
  // (the spikes of the last hidden layer of tap-major nets never reach LDS)
  static constexpr int SP1_BYTES =
      NH >= 1 && !(OTAP && NH == 1) ? (S16 ? SPL * (CH / 8) : align16(NPIXL * CH * SELEM)) : 0;
  // separate layer-2 spike buffer: saves two barriers per frame
  static constexpr bool SEP = NH == 2 && CH == 16 && S16 && !OTAP;
  // tap-major output layer: Y planes over the last hidden layer's region,
  // one float2 (co 0, 1) per tap and pixel, plane length NYPL = NYP + a
  // junk slot for the tail lanes of the last block, rounded to 8 mod 16
  // pixels (the two taps a lane group stores together then fill different
  // banks)
  static constexpr int NYP = OTAP ? rgh(NH) * rgw(NH) : 0;
  static constexpr int NYPL = OTAP ? (NYP + 8) / 16 * 16 + 8 : 0;
  static constexpr int YS_BYTES = OTAP ? 9 * NYPL * 8 : 0;
  static constexpr int KY = (OTAP && SF16 && CH == 32) ? 2 : 1;     // k-steps of the Y product
  // region row length and the column of output column 0 in it
  static constexpr int YRW = OTAP ? rgw(NH) : 1;
  static constexpr int YC0 = OTAP ? NL - ((L1LIN && NH == 1) ? 0 : NH) : 0;
  static constexpr int S2OFF = SEP ? SP1_BYTES : 0;
  static constexpr int SP_BYTES = SP1_BYTES * (SEP ? 2 : 1);
  static constexpr int WL_FLOATS = (OMF || OTAP) ? 0 : 9 * (NH >= 1 ? CH : CIN) * CO;
  static_assert(CH == 16 || CH == 32, "hidden width must be padded to 16 or 32");
  static_assert(NB1 <= 32 && NB2 <= 32 && NBO <= 32 && NOUT <= 32, "mask words overflow");
  static_assert(!OTAP || (NYPL % 16 == 8 && NYPL >= NYP + 1), "Y plane length");
  static_assert(PADF + JP + CWT + 1 < NPIXL, "junk pixel neighbourhood outside the planes");
  static_assert(!L1LIN || PADF + CIN * XPL + 2 * CWT + 16 * NW * NB1 < XS1 / XELEM,
                "linear layer-1 gathers outside the x buffer");
  static_assert(CWT <= 64, "a canvas row must fit one wave");
};

__device__ inline f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
__device__ inline f4 mfma_f16(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
}
__device__ inline f4 mfma_bf16(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                 __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// MFMA of a conv that reads spikes: fp16 operands for FP32 nets, bf16 for
// BF16 nets
template <class C>
__device__ inline f4 mfma_sp(u4 a, u4 b, f4 c) {
  if constexpr (C::SF16) return mfma_f16(a, b, c);
  else return mfma_bf16(a, b, c);
}

// Two fp16 values (exact in fp16) packed low, high.
__device__ inline unsigned pack_f16x2(float lo, float hi) {
  return __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(lo, hi));
}

// s_waitcnt operand that waits until at most N vector memory operations of
// this wave are outstanding (expcnt and lgkmcnt left at their maxima)
template <int N>
constexpr int kVmcntEncoded = (N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14);
static_assert(kVmcntEncoded<0> == 0x0f70, "s_waitcnt encoding");

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ inline unsigned pack_bf16x2(float lo, float hi) {
  // both values are exact in bf16: one hardware conversion of the pair
  const bf16x2 p = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(unsigned, p);
}

// Split three FP32 values into two fp16 parts each, round to nearest:
// h = fp16(x), and l = fp16(2^11 (x - h)) (x - h is exact), the low part
// carried at 2^11 times its value so that it stays in the fp16 normal range
// for |x| >= 2^-14 (the weights it meets are scaled by 2^-11, exactly).  The
// fp16 matrix cores of gfx950 keep subnormal operands, so below that the
// parts stay accurate to the subnormal spacing: |x - h - 2^-11 l| <=
// 2^-22 |x| + 2^-36.  |x| must stay below 65520 (h overflows there).
// Packed as V = [h0 h1 | h2 l0 | l1 l2].
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
__device__ inline void split2_parts(float x0, float x1, float x2, unsigned (&v)[3]) {
  const float x[3] = {x0, x1, x2};
  _Float16 hp[3], lp[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    hp[c] = (_Float16)x[c];
    lp[c] = (_Float16)((x[c] - (float)hp[c]) * 2048.f);
  }
  v[0] = __builtin_bit_cast(unsigned, f16x2{hp[0], hp[1]});
  v[1] = __builtin_bit_cast(unsigned, f16x2{hp[2], lp[0]});
  v[2] = __builtin_bit_cast(unsigned, f16x2{lp[1], lp[2]});
}

// ------------------------------------------------------------------ weights
__device__ inline float wget(const FwdNetArgs& na, int layer, int co, int ci, int tap) {
  // layer 0-based; real channel bounds checked by the caller
  const int cin = na.ch[layer];
  return na.w[na.wofs[layer] + (co * cin + ci) * 9 + tap];
}

// Part p of the exact split w = hi + mid + lo into bf16 values: hi keeps the
// top 8 significant bits of w, mid the next 8 of the (exact) remainder, and
// lo the rest, which has at most 8 significant bits left.
__device__ inline float wpart(float w, int p) {
  const float hi = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, w) & 0xffff0000u);
  const float r1 = w - hi;
  const float mid = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, r1) & 0xffff0000u);
  return p == 0 ? hi : (p == 1 ? mid : r1 - mid);
}

// Layer-1 operand order of the split FP32 nets.  The six parts V(P) of
// canvas pixel P are stored twice, at bytes 24P - 12 and 24P of the x area,
// so the five 8-byte records at 24P + {-24, -16, -8, 8, 16} (index rho 0..4)
// hold
//   V(P-1)[0..3] | V(P-1)[4..5] V(P)[0..1] | V(P)[2..5] | V(P)[4..5] V(P+1)[0..1] | V(P+1)[2..5]
// : the 18 parts of one kernel row (taps dx = -1, 0, +1), the repeated
// V(P)[4..5] aside.  The 15 records of the three kernel rows (and one
// repeated record, zero weights) are dealt so that each lane group reads
// two records a fixed distance apart, one 16-byte pair load per k-step:
// k-step 0 the horizontal neighbours rho 0 | 1 of rows -1, 0, +1 and rho
// 3 | 4 of row -1 (8 bytes apart), k-step 1 the vertical neighbours rho 2
// of rows -1 | 0 and 0 | +1, rho 3 and rho 4 of rows 0 | +1 (one canvas
// row apart).  kXRec[q][g] is (row + 1) * 5 + rho of the first record of
// lane group g in k-step q.
constexpr int kXRec[2][4] = {{0, 5, 10, 3}, {2, 7, 8, 9}};
__device__ __forceinline__ int xrec_first(int q, int g) { return kXRec[q][g]; }
// Record (row, rho) of slot r (0, 1) of lane group g in k-step q, and
// whether it repeats another slot's record (zero weights).
__device__ __forceinline__ int xrec_of(int q, int g, int r, bool& dup) {
  const int f = kXRec[q][g];
  dup = q == 1 && g == 1 && r == 0;                  // row 0, rho 2 again
  return q == 0 ? f + r : f + 5 * r;
}
// Slot v of record (row, rho) holds (tap, channel c, part lo) when xslot
// returns true.
__device__ __forceinline__ bool xslot(int rec, int v, int& tap, int& c, int& lo) {
  const int r = rec % 5;
  int dx, i;
  if (r == 0) { dx = -1; i = v; }
  else if (r == 1) { dx = v < 2 ? -1 : 0; i = v < 2 ? 4 + v : v - 2; }
  else if (r == 2) { dx = 0; i = 2 + v; }
  else if (r == 3) { if (v < 2) return false; dx = 1; i = v - 2; }
  else { dx = 1; i = 2 + v; }
  tap = 3 * (rec / 5) + dx + 1;
  c = i % 3;
  lo = i / 3;
  return true;
}
// Byte offset of record (row, rho) from the 24P of its block pixel (row
// stride cwt), and the distance of the second record of a k-step's pair.
__device__ __forceinline__ int xrec_off(int rec, int cwt) {
  constexpr int kOff[5] = {-24, -16, -8, 8, 16};
  return 24 * cwt * (rec / 5 - 1) + kOff[rec % 5];
}
constexpr int xpair_dist(int q, int cwt) { return q == 0 ? 8 : 24 * cwt; }

// Power-of-two exponent s that brings the largest weight magnitude of a
// layer (bits of |w|max) into [2^14, 2^15): the scaled weights use the fp16
// range without overflow and their low parts stay normal.
__device__ inline int scale_exp(unsigned maxbits) {
  if (maxbits == 0u) return 0;
  const int s = 141 - (int)((maxbits >> 23) & 0xffu);
  return s < -100 ? -100 : (s > 100 ? 100 : s);
}

// Part p of the split w sc = h + l into fp16 values (h = fp16(w sc),
// l = fp16(w sc - h), round to nearest; |w sc - h - l| <= 2^-22 |w sc|).
__device__ inline float wpart16(float w, float sc, int p) {
  const float ws = w * sc;
  const float h = (float)(_Float16)ws;
  return p == 0 ? h : (float)(_Float16)(ws - h);
}

// The bf16 value a spike-operand MFMA multiplies: part p of the FP32 weight,
// or the bf16-rounded weight of a BF16 net (p = 0).
__device__ inline float wbf(const FwdNetArgs& na, int layer, int co, int ci, int tap, bool bf, int p) {
  const float w = wget(na, layer, co, ci, tap);
  return bf ? round_bf16(w) : wpart(w, p);
}

// (tap, first input channel) of the eight K slots that lane group g holds in
// spike-operand k-step kb: 32-channel layers take one tap per k-step (8
// channels per lane group), 16-channel layers two taps (lane groups 0-1 and
// 2-3).  tap 9 marks the empty half of the last 16-channel k-step.
template <int CH>
__device__ __forceinline__ void kslot(int kb, int g, int& tau, int& cib) {
  if constexpr (CH == 32) { tau = kb; cib = 8 * g; }
  else { tau = 2 * kb + (g >> 1); cib = 8 * (g & 1); }
}

// LDS layout of one workgroup (byte offsets).
template <class C>
struct Layout {
  static constexpr int XS = 0;                                  // x tile(s) [pad | CIN+1 planes | tail]
  static constexpr int SP = XS + C::XS_BYTES;                   // spikes: bf16 [CH/8][NPIXL][8], f32 [NPIXL][CH] (x2 if SEP)
  static constexpr int WL = SP + C::SP_BYTES;                   // VALU output weights [9][CI][2] f32
  static constexpr int FR1 = WL + align16(C::WL_FLOATS * 4);    // layer-1 A fragments
  static constexpr int FR1_BYTES =
      C::NH >= 1 ? (C::XSPLIT ? C::NFR1 * C::MB * 64 * 16 : C::KS1 * C::MB * 64 * (C::BF16 ? 16 : 4)) : 0;
  static constexpr int FR2 = FR1 + FR1_BYTES;                   // layer-2 A fragments
  static constexpr int FR2_BYTES =
      C::NH >= 2 ? (C::S16 ? C::KB * C::NSP * C::MB * 64 * 16 : 9 * (C::CH / 16) * C::MB * 64 * 16) : 0;
  static constexpr int FR3 = FR2 + FR2_BYTES;                   // output-layer A fragments
  static constexpr int FR3_BYTES = C::OMF ? C::KB * 64 * 16 : 0;
  static constexpr int FRY = FR3 + FR3_BYTES;                   // tap-major output: Y A fragments
  static constexpr int FRY_BYTES = C::OTAP ? 2 * C::KY * 64 * 16 : 0;
  static constexpr int YS = FRY + FRY_BYTES;                    // Y planes [9][NYPL][2] f32
  static constexpr int XDUMMY = YS + C::YS_BYTES;               // target of the padding x loads
  static constexpr int SCL = XDUMMY + (C::XDMA ? 256 : 0);      // |w|max bits of the fp16 convs (u32 x 3)
  static constexpr int TOTAL = SCL + 16;
  static_assert(TOTAL <= 160 * 1024, "tile does not fit in LDS");
};

// Fill the weight areas of LDS with the MFMA A-operand fragments in the
// per-lane order the k-step loops read them (and the VALU output weights).
// Scale 2^s of the fp16 weights of FP32 nets: slot 0 the hidden -> hidden
// conv, slot 1 the output conv, slot 2 layer 1 of split nets (1 for other
// nets).
template <class C>
__device__ __forceinline__ float spike_scale(const char* lds, int slot) {
  if constexpr (C::SF16) return __builtin_ldexpf(1.f, scale_exp(reinterpret_cast<const unsigned*>(lds + Layout<C>::SCL)[slot]));
  else return 1.f;
}

template <class C>
__device__ __forceinline__ void load_weights(const FwdNetArgs& na, char* lds) {
  using Lo = Layout<C>;
  const int L = na.n_layers - 1;
  if constexpr (C::SF16) {
    // largest |w| of each conv that reads spikes (|w| bits order like |w|)
    unsigned* scl = reinterpret_cast<unsigned*>(lds + Lo::SCL);
    if (threadIdx.x < 4) scl[threadIdx.x] = 0u;
    __syncthreads();
    // (and of layer 1 of split nets, slot 2)
    for (int l = C::XSPLIT ? 0 : 1; l <= L; ++l) {
      if (l >= 1 && l < L && C::NH < 2) continue;
      const int n = na.ch[l + 1] * na.ch[l] * 9;
      unsigned m = 0u;
      for (int e = threadIdx.x; e < n; e += C::NT) {
        const unsigned b = __builtin_bit_cast(unsigned, na.w[na.wofs[l] + e]) & 0x7fffffffu;
        m = b > m ? b : m;
      }
      atomicMax(scl + (l == 0 ? 2 : (l == L ? 1 : 0)), m);
    }
    __syncthreads();
  }
  if constexpr (!C::OMF && !C::OTAP) {
    float* wl = reinterpret_cast<float*>(lds + Lo::WL);
    const int cin = na.ch[L], cout = na.ch[L + 1];
    constexpr int CI = C::NH >= 1 ? C::CH : C::CIN;
    for (int e = threadIdx.x; e < C::WL_FLOATS; e += C::NT) {
      const int co = e % 2, ci = (e / 2) % CI, tap = e / (2 * CI);
      wl[e] = (co < cout && ci < cin) ? wget(na, L, co, ci, tap) : 0.f;
    }
  }
  if constexpr (C::XSPLIT) {
    const int c1 = na.ch[1];
    const float sc = spike_scale<C>(lds, 2);
    // entry (m, f, lane): weight part p = f / 2 over k-step q = f % 2, row
    // co = 16m + lane%16, lane group g = lane/16; the slots of low x parts
    // take the weight part times 2^-11 (rounded to nearest where that leaves
    // the fp16 normal range)
    for (int e = threadIdx.x; e < C::MB * C::NFR1 * 64; e += C::NT) {
      const int lane = e % 64, f = (e / 64) % C::NFR1, m = e / (64 * C::NFR1);
      const int co = 16 * m + (lane & 15), g = lane >> 4;
      const int p = f >> 1, q = f & 1;
      unsigned wd[4];
      for (int e2 = 0; e2 < 4; ++e2) {
        float ww[2];
        for (int h = 0; h < 2; ++h) {
          const int slot = 2 * e2 + h;
          int tap = 0, c = 0, lo = 0;
          bool dup = false;
          const int rec = xrec_of(q, g, slot >> 2, dup);
          const bool real = !dup && xslot(rec, slot & 3, tap, c, lo) && co < c1;
          const float wp = real ? wpart16(wget(na, 0, co, c, tap), sc, p) : 0.f;
          ww[h] = lo ? (float)(_Float16)(wp * 0x1p-11f) : wp;
        }
        wd[e2] = pack_f16x2(ww[0], ww[1]);
      }
      reinterpret_cast<u4*>(lds + Lo::FR1)[e] = u4{wd[0], wd[1], wd[2], wd[3]};
    }
  } else if constexpr (C::NH >= 1) {
    const int c1 = na.ch[1];
    // entry (q, m, lane): row co = 16m + lane%16, lane group g = lane/16
    for (int e = threadIdx.x; e < C::KS1 * C::MB * 64; e += C::NT) {
      const int lane = e % 64, m = (e / 64) % C::MB, q = e / (64 * C::MB);
      const int co = 16 * m + (lane & 15), g = lane >> 4;
      if constexpr (!C::BF16) {
        const int K = 4 * q + g;
        reinterpret_cast<float*>(lds + Lo::FR1)[e] =
            (K < C::K1 && co < c1) ? wget(na, 0, co, K % C::CIN, K / C::CIN) : 0.f;
      } else {
        unsigned wd[4];
        for (int e2 = 0; e2 < 4; ++e2) {
          float ww[2];
          for (int h = 0; h < 2; ++h) {
            const int K = 32 * q + 8 * g + 2 * e2 + h;
            ww[h] = (K < C::K1 && co < c1) ? round_bf16(wget(na, 0, co, K % C::CIN, K / C::CIN)) : 0.f;
          }
          wd[e2] = pack_bf16x2(ww[0], ww[1]);
        }
        reinterpret_cast<u4*>(lds + Lo::FR1)[e] = u4{wd[0], wd[1], wd[2], wd[3]};
      }
    }
  }
  if constexpr (C::NH >= 2) {
    const int c1 = na.ch[1], c2 = na.ch[2];
    const float sc = spike_scale<C>(lds, 0);
    if constexpr (C::S16) {
      // entry ((kb, p, m), lane): part p of the k-step kb fragment, rows co = 16m + lane%16
      for (int e = threadIdx.x; e < C::KB * C::NSP * C::MB * 64; e += C::NT) {
        const int lane = e % 64, m = (e / 64) % C::MB, p = (e / (64 * C::MB)) % C::NSP;
        const int kb = e / (64 * C::MB * C::NSP);
        const int co = 16 * m + (lane & 15), g = lane >> 4;
        int tau, cib;
        kslot<C::CH>(kb, g, tau, cib);
        // merged last k-step (M2): part 0 of it holds tap 8's low part in
        // the slots of tap 9; its part 1 is never multiplied
        const bool merged = C::M2 && kb == C::KB - 1 && tau == 9;
        const int tw = merged ? 8 : tau, pw = merged ? p + 1 : p;
        unsigned wd[4];
        for (int e2 = 0; e2 < 4; ++e2) {
          float ww[2];
          for (int h = 0; h < 2; ++h) {
            const int ci = cib + 2 * e2 + h;
            const bool real = tw < 9 && pw < C::NSP && co < c2 && ci < c1;
            if constexpr (C::SF16) ww[h] = real ? wpart16(wget(na, 1, co, ci, tw), sc, pw) : 0.f;
            else ww[h] = real ? wbf(na, 1, co, ci, tau, C::BF16, p) : 0.f;
          }
          wd[e2] = C::SF16 ? pack_f16x2(ww[0], ww[1]) : pack_bf16x2(ww[0], ww[1]);
        }
        reinterpret_cast<u4*>(lds + Lo::FR2)[e] = u4{wd[0], wd[1], wd[2], wd[3]};
      }
    } else {
      // f32 (relaxed spikes): entry ((tau, hh, m, lane), q4), input channel 4g + q4 + 16hh
      for (int e = threadIdx.x; e < 9 * (C::CH / 16) * C::MB * 64 * 4; e += C::NT) {
        const int q4 = e % 4, lane = (e / 4) % 64, m = (e / 256) % C::MB;
        const int hh = (e / (256 * C::MB)) % (C::CH / 16), tau = e / (256 * C::MB * (C::CH / 16));
        const int co = 16 * m + (lane & 15), g = lane >> 4;
        const int ci = 4 * g + q4 + 16 * hh;
        reinterpret_cast<float*>(lds + Lo::FR2)[e] = (co < c2 && ci < c1) ? wget(na, 1, co, ci, tau) : 0.f;
      }
    }
  }
  if constexpr (C::OTAP) {
    // tap-major output layer: entry ((rb, ks), lane) is the A fragment of
    // row-block rb, k-step ks; row r = 16 rb + lane%16 is (tap r/2, channel
    // r%2).  K slot 8g + e of lane group g (e = 0..7) holds input channel
    //   16 wide: 4g + e%4, weight part e/4 (FP32) or zero for e >= 4 (BF16)
    //   32 wide: 4g + e for e < 4, 16 + 4g + e - 4 for e >= 4, part ks (FP32)
    // which are the channels the epilogue's registers hold for that lane
    // group (rows 4g..4g+3 of each 16-channel accumulator block).
    const int cin = na.ch[L], cout = na.ch[L + 1];
    const float sc = spike_scale<C>(lds, 1);
    for (int e = threadIdx.x; e < 2 * C::KY * 64; e += C::NT) {
      const int lane = e % 64, ks = (e / 64) % C::KY, rb = e / (64 * C::KY);
      const int r = 16 * rb + (lane & 15), g = lane >> 4;
      const int tau = r >> 1, co = r & 1;
      unsigned wd[4];
      for (int e2 = 0; e2 < 4; ++e2) {
        float ww[2];
        for (int h = 0; h < 2; ++h) {
          const int el = 2 * e2 + h;
          int ci, part;
          if constexpr (C::CH == 32) {
            ci = el < 4 ? 4 * g + el : 16 + 4 * g + el - 4;
            part = ks;
          } else {
            ci = 4 * g + (el & 3);
            part = C::SF16 ? (el >> 2) : (el < 4 ? 0 : C::NSP);
          }
          const bool real = tau < 9 && co < cout && ci < cin && part < C::NSP;
          if constexpr (C::SF16) ww[h] = real ? wpart16(wget(na, L, co, ci, tau), sc, part) : 0.f;
          else ww[h] = real ? round_bf16(wget(na, L, co, ci, tau)) : 0.f;
        }
        wd[e2] = C::SF16 ? pack_f16x2(ww[0], ww[1]) : pack_bf16x2(ww[0], ww[1]);
      }
      reinterpret_cast<u4*>(lds + Lo::FRY)[e] = u4{wd[0], wd[1], wd[2], wd[3]};
    }
  }
  if constexpr (C::OMF) {
    // output layer: row i = 4 co + p holds part p of output channel co
    const int cin = na.ch[L], cout = na.ch[L + 1];
    const float sc = spike_scale<C>(lds, 1);
    for (int e = threadIdx.x; e < C::KB * 64; e += C::NT) {
      const int lane = e % 64, kb = e / 64;
      const int i = lane & 15, g = lane >> 4;
      const int co = i >> 2, p = i & 3;
      int tau, cib;
      kslot<C::CH>(kb, g, tau, cib);
      unsigned wd[4];
      for (int e2 = 0; e2 < 4; ++e2) {
        float ww[2];
        for (int h = 0; h < 2; ++h) {
          const int ci = cib + 2 * e2 + h;
          const bool real = tau < 9 && co < cout && p < C::NSP && ci < cin;
          if constexpr (C::SF16) ww[h] = real ? wpart16(wget(na, L, co, ci, tau), sc, p) : 0.f;
          else ww[h] = real ? wbf(na, L, co, ci, tau, C::BF16, p) : 0.f;
        }
        wd[e2] = C::SF16 ? pack_f16x2(ww[0], ww[1]) : pack_bf16x2(ww[0], ww[1]);
      }
      reinterpret_cast<u4*>(lds + Lo::FR3)[e] = u4{wd[0], wd[1], wd[2], wd[3]};
    }
  }
}

// ------------------------------------------------------------------ tile
// Workgroup barrier for LDS data: completes this wave's LDS operations and
// meets the other waves.  Unlike __syncthreads() it leaves outstanding
// global -> LDS loads alone (the x prefetch is waited for by count).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

struct Tile {
  int n, ty0, tx0;
};

__device__ __forceinline__ int tap_off(int tau, int cwt) {
  const int ty = tau / 3;
  return (ty - 1) * cwt + (tau - 3 * ty - 1);
}

// Window of the image whose potentials go to the trace.
struct TraceBox {
  int y0, x0, h, w;
  __device__ bool has(int gy, int gx) const { return gy >= y0 && gy < y0 + h && gx >= x0 && gx < x0 + w; }
  __device__ size_t idx(int gy, int gx) const { return (size_t)(gy - y0) * w + (gx - x0); }
  __device__ size_t plane() const { return (size_t)h * w; }
};

// One frame of the potential trace.  Training / debug builds: float,
// planar [sumC][h][w] over the window; relaxed builds: that, or (pm, the
// backward's traces) pixel-major: layer li at off[li] planes of the frame,
// cw[li] values per pixel.  p == nullptr: no trace.  Layer index li: 0, 1
// the hidden layers, 2 the output layer.  Recompute builds use rs / t16
// (rec_store*).
struct TraceFrame {
  char* p;
  int pm;
  float theta;        // unscaled threshold
  int off[3], cw[3];
  // recompute builds: the frame's layer blocks as buffer resources (hidden
  // 1, hidden 2, output), stores at 32-bit byte offsets; t16 the bits of the
  // smallest fp16 value >= theta (fp16 traces)
  __amdgpu_buffer_rsrc_t rs[3];
  unsigned t16;
  // element index; PM: pixel-major layouts are possible (relaxed builds)
  template <bool PM>
  __device__ size_t idx(int li, int choff, int co, size_t pix, size_t plane) const {
    return (PM && pm) ? (size_t)off[li] * plane + pix * cw[li] + co : (size_t)(choff + co) * plane + pix;
  }
  __device__ void put(size_t e, float h) const { reinterpret_cast<float*>(p)[e] = h; }
  // four consecutive values at e (a multiple of 4): one 16-byte store
  __device__ void put4(size_t e, f4 v) const { *reinterpret_cast<f4*>(reinterpret_cast<float*>(p) + e) = v; }
};

// LDS plane index (front pad included) of pixel 16b + j of layer l's region,
// and whether that neuron is a real one (inside the region and the image).
template <class C>
__device__ __forceinline__ int block_pixel(int l, int b, int j, int gy0, int gx0, int H, int W, bool& ok) {
  const int q = 16 * b + j;
  const int w = C::rgw(l);
  if (q >= C::rgh(l) * w) {
    ok = false;
    return C::PADF + C::JP;
  }
  const int row = l + q / w, col = ((C::L1LIN && l == 1) ? 0 : l) + q % w;
  const int gy = gy0 + row, gx = gx0 + col;
  ok = gy >= 0 && gy < H && gx >= 0 && gx < W;
  return C::PADF + row * C::CWT + col;
}

// Trace stores of the recompute builds.  fp16 (BF16 nets): round toward
// zero, then a firing neuron whose magnitude fell below the threshold is
// raised to t16, the smallest fp16 value >= theta (it is the fp16 neighbour
// above), so the stored value gives the forward's spike; sp holds the
// pair's spikes as 16-bit +-1 / 0 (bf16 or fp16 bits), any nonzero half
// firing.  NaN stays NaN.
__device__ inline unsigned rec_f16_pair(float h0, float h1, unsigned sp, unsigned t16) {
  typedef unsigned short us2 __attribute__((ext_vector_type(2)));
  const unsigned q = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(h0, h1));
  const us2 fire = __builtin_bit_cast(us2, sp & 0x7fff7fffu) >> (unsigned short)13;   // 1 per firing half
  const us2 lo = fire * (unsigned short)t16;
  const us2 mag = __builtin_bit_cast(us2, q & 0x7fff7fffu);
  const us2 m2 = mag > lo ? mag : lo;
  return (__builtin_bit_cast(unsigned, m2)) | (q & 0x80008000u);
}
// A recompute build's store of a lane's four (hidden) or two (output)
// channel values of one pixel at element offset e of a layer block.
template <class C>
__device__ inline void rec_store4(const TraceFrame& tr, int li, unsigned e, f4 h, uint2 sp) {
  if constexpr (C::BF16) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 v = {rec_f16_pair(h[0], h[1], sp.x, tr.t16), rec_f16_pair(h[2], h[3], sp.y, tr.t16)};
    __builtin_amdgcn_raw_buffer_store_b64(v, tr.rs[li], e * 2u, 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, h), tr.rs[li], e * 4u, 0, 0);
  }
}
template <class C>
__device__ inline void rec_store2(const TraceFrame& tr, unsigned e, float h0, float h1, float s0, float s1) {
  if constexpr (C::BF16) {
    __builtin_amdgcn_raw_buffer_store_b32(rec_f16_pair(h0, h1, pack_f16x2(s0, s1), tr.t16), tr.rs[2], e * 2u, 0, 0);
  } else {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 v = {__builtin_bit_cast(unsigned, h0), __builtin_bit_cast(unsigned, h1)};
    __builtin_amdgcn_raw_buffer_store_b64(v, tr.rs[2], e * 4u, 0, 0);
  }
}
template <class C>
__device__ inline void rec_store1(const TraceFrame& tr, unsigned e, float h, float s) {
  if constexpr (C::BF16) {
    const unsigned v = rec_f16_pair(h, 0.f, pack_f16x2(s, 0.f), tr.t16);
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, tr.rs[2], e * 2u, 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, h), tr.rs[2], e * 4u, 0, 0);
  }
}
// Element offset of an output or hidden pixel of the tile interior in the
// recompute trace (pixel-major), or the dead offset past the block when the
// canvas pixel p is not an interior pixel inside the image.
template <class C>
__device__ inline unsigned rec_pix(int p, bool valid, int gy0, int gx0, int H, int W, int cw) {
  const int q = p - C::PADF, row = q / C::CWT, col = q - row * C::CWT;
  const int gy = gy0 + row, gx = gx0 + col;
  const bool in = valid && (unsigned)(row - C::NL) < (unsigned)C::TH && (unsigned)(col - C::NL) < (unsigned)C::TW &&
                  gy < H && gx < W;
  return in ? (unsigned)(gy * W + gx) * (unsigned)cw : 0x20000000u;   // (x 2 or 4 bytes: past the block)
}

// Hidden-layer epilogue for one 16-pixel block: st holds the charged
// potentials h of MB x 4 (channel, pixel) pairs of this lane; fire, reset,
// write spikes to LDS and, optionally, h to the trace.  TOY (the last hidden
// layer of a tap-major net): the spikes are not stored; they are the B
// operand of the Y product of this block (fragments ay), whose rows are
// stored to the Y planes at region pixel yq.
template <class C, bool TOY = false>
__device__ __forceinline__ void hidden_epilogue(f4 (&st)[C::MB], char* lds, int sp_off, int p, bool valid, int g,
                                                float theta, float alpha, int relaxed, const TraceFrame& tr, float tscale,
                                                int cl, int choff, int gy0, int gx0, const TraceBox& tb,
                                                const u4 (*ay)[C::KY] = nullptr, int yq = 0, int li = 0,
                                                unsigned rec_base = 0u) {
  f4 hsave[C::REC ? C::MB : 1];
  if constexpr (C::REC) {
#pragma unroll
    for (int m = 0; m < C::MB; ++m) hsave[m] = st[m] * tscale;
  }
  if (C::TRC && tr.p && valid) {
    const int row = (p - C::PADF) / C::CWT, col = (p - C::PADF) % C::CWT;
    const int gy = gy0 + row, gx = gx0 + col;
    if (row >= C::NL && row < C::NL + C::TH && col >= C::NL && col < C::NL + C::TW && tb.has(gy, gx)) {
      const size_t pix = tb.idx(gy, gx);
#pragma unroll
      for (int m = 0; m < C::MB; ++m) {
        if (C::RELAX && tr.pm) {
          // the lane's four channels 16m + 4g .. +3 of the pixel (padding
          // channels of the layer hold 0 and are stored too)
          if (16 * m + 4 * g < tr.cw[li])
            tr.put4(tr.template idx<true>(li, choff, 16 * m + 4 * g, pix, tb.plane()), st[m] * tscale);
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int co = 16 * m + 4 * g + r;
            if (co < cl) tr.put(tr.template idx<false>(li, choff, co, pix, tb.plane()), st[m][r] * tscale);
          }
        }
      }
    }
  }
  uint2 sw[C::MB];
#pragma unroll
  for (int m = 0; m < C::MB; ++m) {
    f4 s;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v = st[m][r];
      s[r] = bilif(v, theta, alpha, C::RELAX ? relaxed : 0);
      st[m][r] = v;
    }
    // materialise the reset potential here: left to the scheduler, the
    // reset sinks to the next frame and keeps every spike value live
    asm volatile("" : "+v"(st[m]));
    if constexpr (C::RELAX) {
      if (!valid) s = f4{0.f, 0.f, 0.f, 0.f};
    }
    if constexpr (C::S16) {
      sw[m] = C::SF16 ? uint2{pack_f16x2(s[0], s[1]), pack_f16x2(s[2], s[3])}
                      : uint2{pack_bf16x2(s[0], s[1]), pack_bf16x2(s[2], s[3])};
      if constexpr (C::REC) {
        // the lane's channels 16m + 4g .. +3 of the pixel (the layer's
        // padding channels hold 0 and are stored too)
        // rec_base: rec_pix of the block pixel, formed once per tile
        const unsigned e = 16 * m + 4 * g < tr.cw[li] ? rec_base : 0x20000000u;
        rec_store4<C>(tr, li, e + 16 * m + 4 * g, hsave[m], sw[m]);
      }
      // channels 16m + 4g .. +3: plane 2m + g/2, half (g & 1) of the pixel's 16 bytes
      if constexpr (!TOY)
        *reinterpret_cast<uint2*>(lds + Layout<C>::SP + sp_off + (2 * m + (g >> 1)) * C::SPL + p * 16 + 8 * (g & 1)) =
            sw[m];
    } else {
      *reinterpret_cast<f4*>(lds + Layout<C>::SP + sp_off + ((size_t)p * C::CH + 16 * m + 4 * g) * 4) = s;
    }
  }
  if constexpr (TOY) {
    // B operand: K slots 8g..8g+7 of column j are this lane's spikes (the
    // 16-wide form repeats them for the second weight part, or for zero
    // weights)
    const u4 b = C::MB == 2 ? u4{sw[0].x, sw[0].y, sw[C::MB - 1].x, sw[C::MB - 1].y}
                            : u4{sw[0].x, sw[0].y, sw[0].x, sw[0].y};
    f4 y0 = {0.f, 0.f, 0.f, 0.f}, y1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < C::KY; ++ks) {
      y0 = mfma_sp<C>(ay[0][ks], b, y0);
      y1 = mfma_sp<C>(ay[1][ks], b, y1);
    }
    // rows 4g..4g+3 of row-block 0 are taps 2g and 2g+1 (channels 0, 1);
    // rows 16, 17 (lane group 0 of row-block 1) tap 8
    float* const ys = reinterpret_cast<float*>(lds + Layout<C>::YS);
    *reinterpret_cast<float2*>(ys + ((2 * g) * C::NYPL + yq) * 2) = float2{y0[0], y0[1]};
    *reinterpret_cast<float2*>(ys + ((2 * g + 1) * C::NYPL + yq) * 2) = float2{y0[2], y0[3]};
    if (g == 0) *reinterpret_cast<float2*>(ys + (8 * C::NYPL + yq) * 2) = float2{y1[0], y1[1]};
  }
}

// A fragments of the tap-major Y product (row-block, k-step) for this lane.
template <class C>
__device__ __forceinline__ void load_yfrag(const char* lds, int lane, u4 (&ay)[2][C::KY]) {
  const u4* f = reinterpret_cast<const u4*>(lds + Layout<C>::FRY) + lane;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int ks = 0; ks < C::KY; ++ks) ay[rb][ks] = f[(rb * C::KY + ks) * 64];
}

// True for a canvas pixel of the tile interior (an output pixel of the tile).
template <class C>
__device__ __forceinline__ bool interior(int p, int& row, int& col) {
  row = (p - C::PADF) / C::CWT;
  col = (p - C::PADF) % C::CWT;
  return row >= C::NL && row < C::NL + C::TH && col >= C::NL && col < C::NL + C::TW;
}

// Write the membrane state of the interior pixels of a hidden layer.
template <class C, int NB>
__device__ __forceinline__ void write_hidden_state(const f4 (&st)[NB][C::MB], unsigned vm, const int (&ad)[NB],
                                                   int g, float* dst, int cl, int choff, int gy0, int gx0, int W,
                                                   size_t HW, float scale) {
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    int row, col;
    if (((vm >> i) & 1u) && interior<C>(ad[i], row, col)) {
      const size_t pix = (size_t)(gy0 + row) * W + (gx0 + col);
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int co = 16 * m + 4 * g + r;
          if (co < cl) dst[(size_t)(choff + co) * HW + pix] = st[i][m][r] * scale;
        }
    }
  }
}

// Initial membrane state of a hidden layer: v_in (or 0) times `scale` for
// real neurons, `fill` for the others.
template <class C, int NB>
__device__ __forceinline__ void read_hidden_state(f4 (&st)[NB][C::MB], unsigned vm, const int (&ad)[NB], int g,
                                                  const float* src, int cl, int choff, int gy0, int gx0, int W,
                                                  size_t HW, float fill, float scale) {
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int m = 0; m < C::MB; ++m) {
      f4 v = {fill, fill, fill, fill};
      if ((vm >> i) & 1u) {
        v = f4{0.f, 0.f, 0.f, 0.f};
        if (src) {
          const int row = (ad[i] - C::PADF) / C::CWT, col = (ad[i] - C::PADF) % C::CWT;
          const size_t pix = (size_t)(gy0 + row) * W + (gx0 + col);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int co = 16 * m + 4 * g + r;
            if (co < cl) v[r] = src[(size_t)(choff + co) * HW + pix] * scale;
          }
        }
      }
      st[i][m] = v;
    }
}

// Process one tile over frames [0, T) of one clip.
template <class C>
__device__ __forceinline__ void run_tile(const FwdNetArgs& na, const FwdClipArgs& ca, const Tile tl, char* lds) {
  using Lo = Layout<C>;
  uint16_t* const xsb = reinterpret_cast<uint16_t*>(lds + Lo::XS);
  float* const xsf = reinterpret_cast<float*>(lds + Lo::XS);
  const char* const sp1 = lds + Lo::SP;              // layer-1 spikes (and layer-2 ones unless SEP)
  const char* const sp2 = lds + Lo::SP + C::S2OFF;   // layer-2 spikes
  const float* const wl = reinterpret_cast<const float*>(lds + Lo::WL);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int j = lane & 15, g = lane >> 4;
  const int H = ca.H, W = ca.W, T = ca.T;
  const size_t HW = (size_t)H * W;
  const int sumc = na.sum_c;
  const float theta = na.theta, leak = na.leak, alpha = na.alpha;
  // FP32 nets keep the state of the layers behind an fp16 conv (those that
  // read spikes, and layer 1 of split nets) in units of that conv's weight
  // scale 2^s (exact): their threshold is theta 2^s, and traces, checkpoints
  // and the final state are written unscaled
  const float sc1 = C::XSPLIT ? spike_scale<C>(lds, 2) : 1.f;
  const float sc2 = spike_scale<C>(lds, 0), sc3 = spike_scale<C>(lds, 1);
  const float isc1 = 1.f / sc1, isc2 = 1.f / sc2, isc3 = 1.f / sc3;
  const float theta1 = theta * sc1, theta2 = theta * sc2, theta3 = theta * sc3;
  const int relaxed = na.relaxed;                   // 0 hard, 1 sigmoid, 2 arctangent step
  const int c1 = na.ch[1], c2 = na.ch[2];
  const int cout = na.ch[na.n_layers];
  const int choff2 = c1, choffo = (C::NH == 0) ? 0 : (C::NH == 1 ? c1 : c1 + c2);
  // pixel-major trace: widths rounded up to 4, layer offsets (in planes)
  const int cp1 = (c1 + 3) & ~3, cp2 = (c2 + 3) & ~3;
  const int tp1 = cp1, tpo = (C::NH == 0) ? 0 : (C::NH == 1 ? cp1 : cp1 + cp2), tpsum = tpo + 4;
  // recompute builds of BF16 nets: bits of the smallest fp16 value >= theta
  unsigned t16 = 0;
  if constexpr (C::REC && C::BF16) {
    const _Float16 q = (_Float16)theta;
    const unsigned b = __builtin_bit_cast(unsigned short, q);
    t16 = (float)q < theta ? b + 1 : b;
  }
  const int gy0 = tl.ty0 - C::NL, gx0 = tl.tx0 - C::NL;   // image coords of canvas (0,0)

  // ---- LDS pixel of every block lane of every layer, and which neurons are real
  int a1[C::NB1], a2[C::NB2], ao[C::NBO];
  unsigned vm1 = 0, vm2 = 0, vmo = 0;
#pragma unroll
  for (int i = 0; i < C::NB1; ++i) {
    bool ok = false;
    a1[i] = C::NH >= 1 ? block_pixel<C>(1, wave + C::NW * i, j, gy0, gx0, H, W, ok) : 0;
    vm1 |= (ok ? 1u : 0u) << i;
  }
#pragma unroll
  for (int i = 0; i < C::NB2; ++i) {
    bool ok = false;
    a2[i] = C::NH >= 2 ? block_pixel<C>(2, wave + C::NW * i, j, gy0, gx0, H, W, ok) : 0;
    vm2 |= (ok ? 1u : 0u) << i;
  }
  // output neurons (MFMA form): lane group g < 2 holds channel g of pixel j;
  // oo = its offset inside one frame of s_out (-1: not stored)
  int oo[C::NBO];
#pragma unroll
  for (int i = 0; i < C::NBO; ++i) {
    bool ok = false;
    ao[i] = C::OMF ? block_pixel<C>(C::NL, wave + C::NW * i, j, gy0, gx0, H, W, ok) : 0;
    vmo |= (ok ? 1u : 0u) << i;
    const int row = (ao[i] - C::PADF) / C::CWT, col = (ao[i] - C::PADF) % C::CWT;
    oo[i] = (ok && g < cout) ? g * (int)HW + (gy0 + row) * W + (gx0 + col) : -1;
  }
  // recompute builds: trace element offsets of the block pixels (rec_pix),
  // frame-invariant, formed once here (the frame loop hides the block
  // pixels from the optimiser, so they would be formed again every frame)
  unsigned re1[C::NB1] = {}, re2[C::NB2] = {}, reo[C::NBO] = {};
  if constexpr (C::REC) {
    const int cpw1 = (c1 + 3) & ~3, cpw2 = (c2 + 3) & ~3;
#pragma unroll
    for (int i = 0; i < C::NB1; ++i) re1[i] = rec_pix<C>(a1[i], (vm1 >> i) & 1u, gy0, gx0, ca.tb_h, ca.tb_w, cpw1);
#pragma unroll
    for (int i = 0; i < C::NB2; ++i) re2[i] = rec_pix<C>(a2[i], (vm2 >> i) & 1u, gy0, gx0, ca.tb_h, ca.tb_w, cpw2);
#pragma unroll
    for (int i = 0; i < C::NBO; ++i) reo[i] = rec_pix<C>(ao[i], oo[i] >= 0, gy0, gx0, H, W, 4) + g;
  }
  // ---- output pixels of this lane (VALU output layer)
  int op[C::NOUT];
  unsigned ovm = 0;
#pragma unroll
  for (int k = 0; k < C::NOUT; ++k) {
    const int q = tid + C::NT * k;
    const int ty = q / C::TW, tx = q % C::TW;
    const bool inq = q < C::TH * C::TW;
    // LDS canvas pixel (VALU output layer), or the pixel's index in the Y
    // planes (tap-major output layer; idle lanes take output pixel 0)
    if constexpr (C::OTAP) op[k] = (C::NL - C::NH + (inq ? ty : 0)) * C::YRW + C::YC0 + (inq ? tx : 0);
    else op[k] = C::PADF + (inq ? (C::NL + ty) * C::CWT + (C::NL + tx) : C::NL * C::CWT + C::NL);
    const int gy = tl.ty0 + ty, gx = tl.tx0 + tx;
    ovm |= ((inq && gy < H && gx < W) ? 1u : 0u) << k;
  }

  // ---- state registers
  f4 st1[C::NB1][C::MB];
  f4 st2[C::NB2][C::MB];
  float so[C::NOUT][2];
  float vo[C::NBO];         // output potential (MFMA form)
  const float* vin = ca.v_in ? ca.v_in + (size_t)tl.n * ca.vin_nstride : nullptr;
  const float fill = C::RELAX ? 0.f : __builtin_nanf("");
  if constexpr (C::NH >= 1) read_hidden_state<C, C::NB1>(st1, vm1, a1, g, vin, c1, 0, gy0, gx0, W, HW, fill, sc1);
  if constexpr (C::NH >= 2)
    read_hidden_state<C, C::NB2>(st2, vm2, a2, g, vin, c2, choff2, gy0, gx0, W, HW, fill, sc2);
#pragma unroll
  for (int i = 0; i < C::NBO; ++i) {
    vo[i] = 0.f;
    if (C::OMF && vin && oo[i] >= 0) vo[i] = vin[(size_t)choffo * HW + oo[i]] * sc3;
  }
#pragma unroll
  for (int k = 0; k < C::NOUT; ++k) {
    so[k][0] = so[k][1] = 0.f;
    if (!C::OMF && vin && ((ovm >> k) & 1u)) {
      const int q = tid + C::NT * k;
      const size_t pix = (size_t)(tl.ty0 + q / C::TW) * W + (tl.tx0 + q % C::TW);
#pragma unroll
      for (int co = 0; co < 2; ++co)
        if (co < cout) so[k][co] = vin[(size_t)(choffo + co) * HW + pix] * (C::OTAP ? sc3 : 1.f);
    }
  }

  // ---- x staging
  const float* xclip = ca.x + (size_t)tl.n * ca.x_nstride;
  // (a) FP32 nets: direct global -> LDS buffer loads into two x buffers.
  // Chunk wave + NW*k is one canvas row of one x plane, lane = canvas
  // column.  Every wave issues exactly XPW loads per frame (chunks past the
  // last and rows outside the image read through an empty buffer, columns
  // outside the image use an offset past the end: both return zero), so a
  // frame's loads can be waited for by count while the next frame's are in
  // flight.  The per-lane offset is the same for every chunk.
  const unsigned xv = (gx0 + lane >= 0 && gx0 + lane < W) ? (unsigned)(gx0 + lane) * 4u : 0x80000000u;
  auto issue_x = [&](int tt, int buf) __attribute__((always_inline)) {
    if constexpr (C::XDMA) {
      float* const xf = const_cast<float*>(xclip + (size_t)tt * C::CIN * HW);
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(xf, (short)0, (int)(C::CIN * HW * 4), 0x00020000);
      const __amdgpu_buffer_rsrc_t rz = __builtin_amdgcn_make_buffer_rsrc(xf, (short)0, 0, 0x00020000);
      if (lane < C::CWT) {
#pragma unroll
        for (int k = 0; k < C::XPW; ++k) {
          const int id = wave + C::NW * k;
          const int c = id / C::CHT, r = id % C::CHT;
          const bool real = id < C::XCK;
          const bool row_in = real && gy0 + r >= 0 && gy0 + r < H;
          const int dst = real ? Lo::XS + buf * C::XS1 + (C::PADF + id * C::CWT) * 4 : Lo::XDUMMY;
          const unsigned so = row_in ? (unsigned)(c * (int)HW + (gy0 + r) * W) * 4u : 0u;
          __builtin_amdgcn_raw_ptr_buffer_load_lds(row_in ? rs : rz, (__attribute__((address_space(3))) void*)(lds + dst),
                                                   4, xv, so, 0, 0);
        }
      }
    }
  };
  // (b) other nets: register prefetch of the next frame.  With RGB input
  // (LOGX) a lane prefetches the three colours of its canvas pixels of RGB
  // frame tt + 1 and keeps the lin-log luminance of frame tt of the same
  // pixels (xl_prev), so input frame tt is X = L_log[tt + 1] - L_log[tt];
  // pixels outside the image load zeros and give X = 0 (the zero padding).
  // Split FP32 nets (XSPLIT) prefetch the three channels of canvas pixels
  // tid + NT k and store their six fp16 parts V twice (see xslot).
  int xo[C::XSPLIT ? C::XPP : 1];
  if constexpr (C::XSPLIT) {
#pragma unroll
    for (int k = 0; k < C::XPP; ++k) {
      const int q = tid + C::NT * k;
      const int gy = gy0 + q / C::CWT, gx = gx0 + q % C::CWT;
      const bool in = q < C::NPIX && gy >= 0 && gy < H && gx >= 0 && gx < W;
      xo[k] = in ? (gy * W + gx) * 4 : (int)0x80000000u;
    }
  }
  // Other register-staged nets: a 32-bit byte offset per staged element
  // (channel plane and pixel of the frame, or of its red plane with RGB
  // input), or one past the end for elements outside the canvas or the
  // image, which reads zero
  constexpr bool XGEN = !C::XSPLIT && !C::XDMA;
  unsigned xog[XGEN ? C::XPF : 1];
  if constexpr (XGEN) {
#pragma unroll
    for (int k = 0; k < C::XPF; ++k) {
      const int e = tid + C::NT * k;
      const int c = e / C::NPIX, rem = e % C::NPIX;
      const int gy = gy0 + rem / C::CWT, gx = gx0 + rem % C::CWT;
      const bool in = e < C::XN && gy >= 0 && gy < H && gx >= 0 && gx < W;
      xog[k] = in ? (unsigned)((c * H + gy) * W + gx) * 4u : 0x80000000u;
    }
  }
  constexpr int XPR = C::LOGX ? 3 : 1;
  constexpr int NXPF = C::XDMA ? 1 : (C::XSPLIT ? 3 * C::XPP : C::XPF * XPR);
  float xpf[NXPF];
  float xl_prev[C::LOGX ? C::XPF : 1];
  auto fetch_x = [&](int frame) __attribute__((always_inline)) {
    if constexpr (C::XSPLIT) {
      // buffer loads: 32-bit pixel offsets, the channel offset in soffset;
      // pixels outside the canvas or the image use an offset past the end,
      // which reads zero
      float* const xf = const_cast<float*>(xclip + (size_t)frame * 3 * HW);
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(xf, (short)0, (int)(3 * HW * 4), 0x00020000);
#pragma unroll
      for (int k = 0; k < C::XPP; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          xpf[3 * k + c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, xo[k], c * (int)HW * 4, 0));
    } else if constexpr (XGEN) {
      // buffer loads (the colour plane of RGB input in soffset)
      float* const xf = const_cast<float*>(xclip + (size_t)frame * (C::LOGX ? 3 : C::CIN) * HW);
      const __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc(xf, (short)0, (int)((C::LOGX ? 3 : C::CIN) * HW * 4), 0x00020000);
#pragma unroll
      for (int k = 0; k < C::XPF; ++k)
#pragma unroll
        for (int r = 0; r < XPR; ++r)
          xpf[k * XPR + r] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, xog[k], r * (int)HW * 4, 0));
    }
  };
  auto load_x = [&](int tt) __attribute__((always_inline)) { fetch_x(C::LOGX ? tt + 1 : tt); };
  // split nets: records of staged pixel group k (pixels tid + NT k)
  auto store_group = [&](int k) __attribute__((always_inline)) {
    if constexpr (C::XSPLIT) {
      const int q = tid + C::NT * k;
      if (q < C::NPIX) {
        unsigned v[3];
        split2_parts(xpf[3 * k], xpf[3 * k + 1], xpf[3 * k + 2], v);
        char* const px = lds + Lo::XS + (C::PADF + q) * 24;
        *reinterpret_cast<unsigned*>(px - 12) = v[0];
        *reinterpret_cast<uint2*>(px - 8) = uint2{v[1], v[2]};
        *reinterpret_cast<uint2*>(px) = uint2{v[0], v[1]};
        *reinterpret_cast<unsigned*>(px + 8) = v[2];
      }
    }
  };
  // three-layer split nets store the next frame's records inside the
  // layer-2 block loop (group k after block k's MFMAs are issued), the
  // others right after the layer-1 barrier
  constexpr bool STAGE_IN_L2 = C::XSPLIT && C::NH == 2 && C::BO;
  auto store_x = [&]() __attribute__((always_inline)) {
    if constexpr (C::XSPLIT) {
#pragma unroll
      for (int k = 0; k < C::XPP; ++k) store_group(k);
    } else if constexpr (!C::XDMA) {
#pragma unroll
      for (int k = 0; k < C::XPF; ++k) {
        const int e = tid + C::NT * k;
        if (e < C::XN) {
          const int c = e / C::NPIX, rem = e % C::NPIX;
          float v = xpf[k * XPR];
          if constexpr (C::LOGX) {
            const float l = linlog_lum(xpf[3 * k], xpf[3 * k + 1], xpf[3 * k + 2], na.lum_scale, na.knee, na.toe);
            v = __fsub_rn(l, xl_prev[k]);
            xl_prev[k] = l;
          }
          if constexpr (C::BF16) xsb[c * C::XPL + C::PADF + rem] = __builtin_bit_cast(uint16_t, (__bf16)v);
          else xsf[c * C::XPL + C::PADF + rem] = v;
        }
      }
    }
  };

  // split nets: byte offset (from 24 P of a block pixel P) of the first
  // record of k-step q's pair for this lane's group
  int ro[C::XSPLIT ? 2 : 1];
  if constexpr (C::XSPLIT) {
#pragma unroll
    for (int q = 0; q < 2; ++q) ro[q] = xrec_off(xrec_first(q, g), C::CWT);
  }
  // per-lane x-plane offsets of the layer-1 k-steps (FP32: K = 4q + g)
  int o1[C::BF16 || C::XSPLIT ? 1 : C::KS1];
  if constexpr (!C::BF16 && !C::XSPLIT) {
#pragma unroll
    for (int q = 0; q < C::KS1; ++q) {
      const int K = 4 * q + g;
      const int tap = K / C::CIN, c = K - tap * C::CIN;
      o1[q] = K < C::K1 ? c * C::XPL + tap_off(tap, C::CWT) : C::CIN * C::XPL;
    }
  }

  // tap-major output layer: the last hidden layer's epilogue forms Y (layer
  // 1 of two-layer nets, layer 2 of three-layer ones); a block lane stores
  // at its region pixel, tail lanes at the junk slot NYP
  constexpr bool Y1 = C::OTAP && C::NH == 1, Y2 = C::OTAP && C::NH == 2;
  static_assert(!Y2 || C::BO, "tap-major three-layer nets run layer 2 block by block");
  auto yidx = [&](int b) __attribute__((always_inline)) {
    const int q = 16 * b + j;
    return q < C::NYP ? q : C::NYP;
  };
  const int nseg = ca.ckpt_every > 0 ? cdiv(T, ca.ckpt_every) : 0;
  const TraceBox tb{ca.tb_y0, ca.tb_x0, ca.tb_h, ca.tb_w};
  auto write_state = [&](float* dst) __attribute__((always_inline)) {
    if constexpr (C::NH >= 1) write_hidden_state<C, C::NB1>(st1, vm1, a1, g, dst, c1, 0, gy0, gx0, W, HW, isc1);
    if constexpr (C::NH >= 2) write_hidden_state<C, C::NB2>(st2, vm2, a2, g, dst, c2, choff2, gy0, gx0, W, HW, isc2);
#pragma unroll
    for (int k = 0; k < C::NOUT; ++k) {
      if (!C::OMF && ((ovm >> k) & 1u)) {
        const int q = tid + C::NT * k;
        const size_t pix = (size_t)(tl.ty0 + q / C::TW) * W + (tl.tx0 + q % C::TW);
#pragma unroll
        for (int co = 0; co < 2; ++co)
          if (co < cout) dst[(size_t)(choffo + co) * HW + pix] = so[k][co] * (C::OTAP ? isc3 : 1.f);
      }
    }
#pragma unroll
    for (int i = 0; i < C::NBO; ++i)
      if (C::OMF && oo[i] >= 0) dst[(size_t)choffo * HW + oo[i]] = vo[i] * isc3;
  };

  // ---- prologue: frame 0 into LDS, frame 1 in flight (DMA) or in registers
  if constexpr (C::XDMA) {
    issue_x(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (T > 1) issue_x(1, 1);
  } else {
    if constexpr (C::LOGX) {
      fetch_x(0);
#pragma unroll
      for (int k = 0; k < C::XPF; ++k)
        xl_prev[k] = linlog_lum(xpf[3 * k], xpf[3 * k + 1], xpf[3 * k + 2], na.lum_scale, na.knee, na.toe);
    }
    load_x(0);
    store_x();
    if (T > 1) load_x(1);
    __syncthreads();
  }

  for (int t = 0; t < T; ++t) {
    // block pixel indices, opaque to the optimiser inside the frame loop:
    // each (block, k-step) LDS address is then formed when used instead of
    // being hoisted out of the loop into registers of its own
#pragma unroll
    for (int i = 0; i < C::NB1; ++i) asm volatile("" : "+v"(a1[i]));
#pragma unroll
    for (int i = 0; i < C::NB2; ++i) asm volatile("" : "+v"(a2[i]));
#pragma unroll
    for (int i = 0; i < C::NBO; ++i) asm volatile("" : "+v"(ao[i]));
    if constexpr (C::REC) {
      // (the trace offsets too: only they stay in registers, not values
      // derived from them)
#pragma unroll
      for (int i = 0; i < C::NB1; ++i) asm volatile("" : "+v"(re1[i]));
#pragma unroll
      for (int i = 0; i < C::NB2; ++i) asm volatile("" : "+v"(re2[i]));
#pragma unroll
      for (int i = 0; i < C::NBO; ++i) asm volatile("" : "+v"(reo[i]));
    }
    const int (&e1)[C::NB1] = a1;
    const int (&e2)[C::NB2] = a2;
    const int (&eo)[C::NBO] = ao;
    TraceFrame trace_t{nullptr, ca.trace_pm, theta, {0, tp1, tpo}, {cp1, cp2, 4}, {}, t16};
    if constexpr (C::CKS) {
      if (ca.ckpt && (t % ca.ckpt_every) == 0)
        write_state(ca.ckpt + ((size_t)tl.n * nseg + t / ca.ckpt_every) * sumc * HW);
    }
    if constexpr (C::REC) {
      // the frame's three layer blocks of the pixel-major trace
      constexpr unsigned es = C::BF16 ? 2 : 4;
      // (no trace: empty resources, every store dropped)
      char* const fb = reinterpret_cast<char*>(ca.h_trace) + ((size_t)tl.n * ca.trace_nstride + (size_t)t * tpsum * HW) * es;
      const unsigned on = ca.h_trace ? 1u : 0u;
#pragma unroll
      for (int li = 0; li < 3; ++li)
        trace_t.rs[li] = __builtin_amdgcn_make_buffer_rsrc(fb + (size_t)trace_t.off[li] * HW * es, (short)0,
                                                           (int)(on * (unsigned)trace_t.cw[li] * (unsigned)HW * es),
                                                           0x00020000);
    } else if constexpr (C::TRC) {
      if (ca.h_trace)
        trace_t.p = reinterpret_cast<char*>(ca.h_trace) +
                    ((size_t)tl.n * ca.trace_nstride + (size_t)t * ((C::RELAX && ca.trace_pm) ? tpsum : sumc) * tb.plane()) * 4;
    }

    if constexpr (C::NH >= 1) {
      // ================= layer 1: x -> hidden (MFMA), K = tap * CIN + c
#pragma unroll
      for (int i = 0; i < C::NB1; ++i)
#pragma unroll
        for (int m = 0; m < C::MB; ++m) st1[i][m] *= leak;
      u4 ay[2][C::KY];
      if constexpr (Y1) load_yfrag<C>(lds, lane, ay);
      if constexpr (C::XSPLIT) {
        // fp16 MFMA over the split records: per block, the 4 fragment
        // products (weight parts h, l per k-step) accumulate onto leak * v
        // in one chain (dependent MFMAs issue back to back); the records of
        // block i+1 load and the epilogue of block i-1 runs while block i
        // multiplies
        const char* const xr = lds + Lo::XS;
        const u4* const fr = reinterpret_cast<const u4*>(lds + Lo::FR1) + lane;
        u4 af[C::MB][C::NFR1];
#pragma unroll
        for (int m = 0; m < C::MB; ++m)
#pragma unroll
          for (int f = 0; f < C::NFR1; ++f) af[m][f] = fr[(m * C::NFR1 + f) * 64];
        u4 bq[2][2];
        auto ldb = [&](int i, int sl) __attribute__((always_inline)) {
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            // 24-bit multiply (canvas pixel indices are small): one
            // full-rate multiply-add instead of a quarter-rate 32-bit multiply
            const char* const b = xr + (__umul24((unsigned)e1[i], 24u) + ro[q]);
            const uint2 lo = *reinterpret_cast<const uint2*>(b);
            const uint2 hi = *reinterpret_cast<const uint2*>(b + xpair_dist(q, C::CWT));
            bq[sl][q] = u4{lo.x, lo.y, hi.x, hi.y};
          }
        };
        ldb(0, 0);
#pragma unroll
        for (int i = 0; i <= C::NB1; ++i) {
          if (i < C::NB1) {
            if (i + 1 < C::NB1) ldb(i + 1, (i + 1) & 1);
            const u4 (&b)[2] = bq[i & 1];
#pragma unroll
            for (int m = 0; m < C::MB; ++m) {
              f4& h = st1[i][m];
              h = mfma_f16(af[m][2], b[0], h);       // low weight parts first
              h = mfma_f16(af[m][3], b[1], h);
              h = mfma_f16(af[m][0], b[0], h);
              h = mfma_f16(af[m][1], b[1], h);
            }
          }
          if (i > 0)
            hidden_epilogue<C, Y1>(st1[i - 1], lds, 0, e1[i - 1], (vm1 >> (i - 1)) & 1u, g, theta1, alpha, relaxed,
                                   trace_t, isc1, c1, 0, gy0, gx0, tb, ay, yidx(wave + C::NW * (i - 1)), 0,
                                   re1[i - 1]);
        }
      } else if constexpr (!C::BF16) {
        // f32 MFMA; the operands of k-step q+1 load while those of q multiply
        const float* xb = reinterpret_cast<const float*>(lds + Lo::XS + (C::XDMA ? (t & 1) * C::XS1 : 0));
        const float* fr1 = reinterpret_cast<const float*>(lds + Lo::FR1) + lane;
        float bq[2][C::NB1], aq[2][C::MB];
        auto ld1 = [&](int q, int s) __attribute__((always_inline)) {
#pragma unroll
          for (int m = 0; m < C::MB; ++m) aq[s][m] = fr1[(q * C::MB + m) * 64];
#pragma unroll
          for (int i = 0; i < C::NB1; ++i) bq[s][i] = xb[e1[i] + o1[q]];
        };
        ld1(0, 0);
#pragma unroll
        for (int q = 0; q < C::KS1; ++q) {
          if (q + 1 < C::KS1) ld1(q + 1, (q + 1) & 1);
#pragma unroll
          for (int m = 0; m < C::MB; ++m)
#pragma unroll
            for (int i = 0; i < C::NB1; ++i) st1[i][m] = mfma_f32(aq[q & 1][m], bq[q & 1][i], st1[i][m]);
        }
      } else {
#pragma unroll 1
        for (int q = 0; q < C::KS1; ++q) {
          const u4* fr = reinterpret_cast<const u4*>(lds + Lo::FR1) + q * C::MB * 64 + lane;
          u4 a[C::MB];
#pragma unroll
          for (int m = 0; m < C::MB; ++m) a[m] = fr[m * 64];
          int o[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int K = 32 * q + 8 * g + e;
            const int tap = K / C::CIN, c = K - tap * C::CIN;
            o[e] = K < C::K1 ? c * C::XPL + tap_off(tap, C::CWT) : C::CIN * C::XPL;
          }
          // lane (j, wave) of block i sits at canvas pixel l1b + 16 NW i
          // (whole-row layer-1 region); tail lanes of the last block read
          // inside the buffer's tail room and are not stored
          const uint16_t* xl = xsb + C::PADF + C::CWT + 16 * wave + j;
          u4 bv[C::NB1];
#pragma unroll
          for (int i = 0; i < C::NB1; ++i) {
            unsigned wd[4];
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) {
              const unsigned r0 = xl[o[2 * e2] + 16 * C::NW * i], r1 = xl[o[2 * e2 + 1] + 16 * C::NW * i];
              wd[e2] = r0 | (r1 << 16);
            }
            bv[i] = u4{wd[0], wd[1], wd[2], wd[3]};
          }
#pragma unroll
          for (int m = 0; m < C::MB; ++m)
#pragma unroll
            for (int i = 0; i < C::NB1; ++i) st1[i][m] = mfma_bf16(a[m], bv[i], st1[i][m]);
        }
      }
      if constexpr (!C::XSPLIT) {
#pragma unroll
        for (int i = 0; i < C::NB1; ++i)
          hidden_epilogue<C, Y1>(st1[i], lds, 0, e1[i], (vm1 >> i) & 1u, g, theta1, alpha, relaxed, trace_t, isc1, c1,
                                 0, gy0, gx0, tb, ay, yidx(wave + C::NW * i), 0, re1[i]);
      }
      lds_barrier();                                   // B1: s1 visible, x buffer (t & 1) free
      if constexpr (C::XDMA) {
        // three-layer nets issue after the layer-2 epilogue: the compiler
        // orders every LDS store after LDS DMA still in flight, and the
        // output layer + next layer-1 MFMAs are the longest store-free stretch
        if (C::NH == 1 && t + 2 < T) issue_x(t + 2, t & 1);
      } else if constexpr (!STAGE_IN_L2) {
        if (t + 1 < T) store_x();
        if (t + 2 < T) load_x(t + 2);
      }
    }

    if constexpr (C::NH >= 2) {
      // ================= layer 2: hidden -> hidden (MFMA), K = tap * CH + ci
#pragma unroll
      for (int i = 0; i < C::NB2; ++i)
#pragma unroll
        for (int m = 0; m < C::MB; ++m) st2[i][m] *= leak;
      if constexpr (C::BO) {
        // block by block: the fragments of all k-steps and parts stay in
        // registers; block i+1's spikes load and block i-1's epilogue runs
        // while block i multiplies (per block the MFMA order is the same as
        // k-step by k-step: kb outer, part inner)
        const u4* fr2 = reinterpret_cast<const u4*>(lds + Lo::FR2) + lane;
        u4 aw[C::KB][C::NSP];
#pragma unroll
        for (int kb = 0; kb < C::KB; ++kb)
#pragma unroll
          for (int p = 0; p < C::NSP; ++p) aw[kb][p] = fr2[(kb * C::NSP + p) * 64];
        u4 ay[2][C::KY];
        if constexpr (Y2) load_yfrag<C>(lds, lane, ay);
        u4 bq[2][C::KB];
        auto ldb2 = [&](int i, int sl) __attribute__((always_inline)) {
#pragma unroll
          for (int kb = 0; kb < C::KB; ++kb) {
            int tau, cib;
            kslot<C::CH>(kb, g, tau, cib);
            const int o = (cib >> 3) * C::SPL + tap_off(tau > 8 ? 8 : tau, C::CWT) * 16;   // tap 9: zero weights
            bq[sl][kb] = *reinterpret_cast<const u4*>(sp1 + e2[i] * 16 + o);
          }
        };
        ldb2(0, 0);
#pragma unroll
        for (int i = 0; i <= C::NB2; ++i) {
          if (i < C::NB2) {
            if (i + 1 < C::NB2) ldb2(i + 1, (i + 1) & 1);
#pragma unroll
            for (int kb = 0; kb < C::KB; ++kb)
#pragma unroll
              for (int p = 0; p < C::NSP; ++p)
                if (!(C::M2 && kb == C::KB - 1 && p > 0)) st2[i][0] = mfma_sp<C>(aw[kb][p], bq[i & 1][kb], st2[i][0]);
          }
          if (STAGE_IN_L2 && i < C::XPP && t + 1 < T) store_group(i);
          if (i > 0)
            hidden_epilogue<C, Y2>(st2[i - 1], lds, C::S2OFF, e2[i - 1], (vm2 >> (i - 1)) & 1u, g, theta2, alpha,
                                   relaxed, trace_t, isc2, c2, choff2, gy0, gx0, tb, ay, yidx(wave + C::NW * (i - 1)),
                                   1, re2[i - 1]);
        }
        if constexpr (STAGE_IN_L2) {
#pragma unroll
          for (int k = C::NB2 + 1; k < C::XPP; ++k)
            if (t + 1 < T) store_group(k);
          if (t + 2 < T) load_x(t + 2);
        }
      } else if constexpr (C::S16) {
        // the spike fragment of k-step kb is loaded once and multiplied by
        // the NSP weight parts; k-step kb+1 loads while kb multiplies
        const u4* fr2 = reinterpret_cast<const u4*>(lds + Lo::FR2) + lane;
        u4 bq[2][C::NB2], aq[2][C::NSP][C::MB];
        auto ld2 = [&](int kb, int s) __attribute__((always_inline)) {
          int tau, cib;
          kslot<C::CH>(kb, g, tau, cib);
          const int o = (cib >> 3) * C::SPL + tap_off(tau > 8 ? 8 : tau, C::CWT) * 16;   // tap 9: zero weights
#pragma unroll
          for (int i = 0; i < C::NB2; ++i) bq[s][i] = *reinterpret_cast<const u4*>(sp1 + e2[i] * 16 + o);
#pragma unroll
          for (int p = 0; p < C::NSP; ++p)
#pragma unroll
            for (int m = 0; m < C::MB; ++m) aq[s][p][m] = fr2[((kb * C::NSP + p) * C::MB + m) * 64];
        };
        ld2(0, 0);
#pragma unroll
        for (int kb = 0; kb < C::KB; ++kb) {
          if (kb + 1 < C::KB) ld2(kb + 1, (kb + 1) & 1);
#pragma unroll
          for (int p = 0; p < C::NSP; ++p)
#pragma unroll
            for (int m = 0; m < C::MB; ++m)
#pragma unroll
              for (int i = 0; i < C::NB2; ++i)
                if (!(C::M2 && kb == C::KB - 1 && p > 0)) st2[i][m] = mfma_sp<C>(aq[kb & 1][p][m], bq[kb & 1][i], st2[i][m]);
        }
      } else {
        const float* spf = reinterpret_cast<const float*>(sp1);
#pragma unroll 1
        for (int tau = 0; tau < 9; ++tau) {
          const int to = tap_off(tau, C::CWT);
#pragma unroll
          for (int hh = 0; hh < C::CH / 16; ++hh) {
            const f4* fr = reinterpret_cast<const f4*>(lds + Lo::FR2) +
                           ((tau * (C::CH / 16) + hh) * C::MB) * 64 + lane;
            f4 a[C::MB];
#pragma unroll
            for (int m = 0; m < C::MB; ++m) a[m] = fr[m * 64];
            f4 bv[C::NB2];
#pragma unroll
            for (int i = 0; i < C::NB2; ++i)
              bv[i] = *reinterpret_cast<const f4*>(spf + (size_t)(e2[i] + to) * C::CH + 16 * hh + 4 * g);
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
              for (int m = 0; m < C::MB; ++m)
#pragma unroll
                for (int i = 0; i < C::NB2; ++i) st2[i][m] = mfma_f32(a[m][q4], bv[i][q4], st2[i][m]);
          }
        }
      }
      if constexpr (!C::SEP && !C::OTAP) lds_barrier();   // B2: all reads of s1 done
      if constexpr (!C::BO) {
#pragma unroll
        for (int i = 0; i < C::NB2; ++i)
          hidden_epilogue<C>(st2[i], lds, C::S2OFF, e2[i], (vm2 >> i) & 1u, g, theta2, alpha, relaxed, trace_t, isc2,
                             c2, choff2, gy0, gx0, tb, nullptr, 0, 1, re2[i]);
      }
      if constexpr (C::XDMA) {
        if (t + 2 < T) issue_x(t + 2, t & 1);
        // x(t+1) was issued one frame ago: wait for it, not for x(t+2)
        if (t + 2 < T) __builtin_amdgcn_s_waitcnt(kVmcntEncoded<C::XPW>);
        else __builtin_amdgcn_s_waitcnt(0);
      }
      lds_barrier();                                   // B3: s2 visible
    } else if constexpr (C::XDMA) {
      if (t + 2 < T) __builtin_amdgcn_s_waitcnt(kVmcntEncoded<C::XPW>);
      else __builtin_amdgcn_s_waitcnt(0);
    }

    if constexpr (C::OMF) {
      // ================= output layer on MFMA: rows 4co + p, K = tap * CH + ci
      const char* const sob = C::NH == 2 ? sp2 : sp1;
      const u4* fr3 = reinterpret_cast<const u4*>(lds + Lo::FR3) + lane;
      int8_t* const s8 = reinterpret_cast<int8_t*>(ca.s_out) + ((size_t)tl.n * T + t) * cout * HW;
      float* const s32 = reinterpret_cast<float*>(ca.s_out) + ((size_t)tl.n * T + t) * cout * HW;
      // fire/reset of output block i; lanes of group g < 2 hold output
      // channel g of pixel j (rows 4g + p of the accumulator)
      auto out_epilogue = [&](int i, const f4& acc) __attribute__((always_inline)) {
        if (g < 2) {
          const float h = C::NSP == 2 ? acc[0] + acc[1] : acc[0];
          if (C::TRC && oo[i] >= 0 && trace_t.p) {
            const int row = (ao[i] - C::PADF) / C::CWT, col = (ao[i] - C::PADF) % C::CWT;
            const int gy = gy0 + row, gx = gx0 + col;
            if (tb.has(gy, gx)) trace_t.put(trace_t.template idx<C::RELAX>(2, choffo, g, tb.idx(gy, gx), tb.plane()), h * isc3);
          }
          float v = h;
          const float sp = bilif(v, theta3, alpha, false);
          if constexpr (C::REC)
            rec_store1<C>(trace_t, reo[i], h * isc3, sp);
          asm volatile("" : "+v"(v));
          vo[i] = v;
          if (oo[i] >= 0 && ca.s_out) {
            if (C::CKS && ca.s_fp32) s32[oo[i]] = sp;
            else s8[oo[i]] = (int8_t)sp;
          }
        }
      };
      if constexpr (C::BO) {
        // block by block, as layer 2: all k-step fragments in registers,
        // block i-1's epilogue overlaps block i's MFMAs
        u4 a3[C::KB];
#pragma unroll
        for (int kb = 0; kb < C::KB; ++kb) a3[kb] = fr3[kb * 64];
        u4 bq[2][C::KB];
        f4 acc[2];
        auto ldb3 = [&](int i, int sl) __attribute__((always_inline)) {
#pragma unroll
          for (int kb = 0; kb < C::KB; ++kb) {
            int tau, cib;
            kslot<C::CH>(kb, g, tau, cib);
            const int o = (cib >> 3) * C::SPL + tap_off(tau > 8 ? 8 : tau, C::CWT) * 16;
            bq[sl][kb] = *reinterpret_cast<const u4*>(sob + eo[i] * 16 + o);
          }
        };
        ldb3(0, 0);
#pragma unroll
        for (int i = 0; i <= C::NBO; ++i) {
          if (i < C::NBO) {
            if (i + 1 < C::NBO) ldb3(i + 1, (i + 1) & 1);
            acc[i & 1] = f4{leak * vo[i], 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < C::KB; ++kb) acc[i & 1] = mfma_sp<C>(a3[kb], bq[i & 1][kb], acc[i & 1]);
          }
          if (i > 0) out_epilogue(i - 1, acc[(i - 1) & 1]);
        }
      } else {
        f4 acc[C::NBO];
#pragma unroll
        for (int i = 0; i < C::NBO; ++i) acc[i] = f4{leak * vo[i], 0.f, 0.f, 0.f};
        u4 bq[2][C::NBO], aq[2];
        auto ld3 = [&](int kb, int s) __attribute__((always_inline)) {
          int tau, cib;
          kslot<C::CH>(kb, g, tau, cib);
          const int o = (cib >> 3) * C::SPL + tap_off(tau > 8 ? 8 : tau, C::CWT) * 16;
#pragma unroll
          for (int i = 0; i < C::NBO; ++i) bq[s][i] = *reinterpret_cast<const u4*>(sob + eo[i] * 16 + o);
          aq[s] = fr3[kb * 64];
        };
        ld3(0, 0);
#pragma unroll
        for (int kb = 0; kb < C::KB; ++kb) {
          if (kb + 1 < C::KB) ld3(kb + 1, (kb + 1) & 1);
#pragma unroll
          for (int i = 0; i < C::NBO; ++i) acc[i] = mfma_sp<C>(aq[kb & 1], bq[kb & 1][i], acc[i]);
        }
#pragma unroll
        for (int i = 0; i < C::NBO; ++i) out_epilogue(i, acc[i]);
      }
    } else if constexpr (C::OTAP) {
      // ================= tap-major output layer: u = sum over the 9 taps of
      // the neighbour's Y (fixed order), h = leak v + u, BiLIF; lane = one
      // output pixel, both channels; potentials in the output conv's weight
      // scale (threshold theta3), traces and state unscaled
      const float* const ys = reinterpret_cast<const float*>(lds + Lo::YS);
      int8_t* const s8 = reinterpret_cast<int8_t*>(ca.s_out) + ((size_t)tl.n * T + t) * cout * HW;
      float* const s32 = reinterpret_cast<float*>(ca.s_out) + ((size_t)tl.n * T + t) * cout * HW;
#pragma unroll
      for (int k = 0; k < C::NOUT; ++k) {
        float u0 = 0.f, u1 = 0.f;
#pragma unroll
        for (int tau = 0; tau < 9; ++tau) {
          const int o = op[k] + (tau / 3 - 1) * C::YRW + (tau % 3 - 1);
          const float2 y = *reinterpret_cast<const float2*>(ys + (tau * C::NYPL + o) * 2);
          u0 += y.x;
          u1 += y.y;
        }
        const bool ok = (ovm >> k) & 1u;
        const int q = tid + C::NT * k;
        const int gy = tl.ty0 + q / C::TW, gx = tl.tx0 + q % C::TW;
        const size_t pix = (size_t)gy * W + gx;
        float hs[2], ss[2];
#pragma unroll
        for (int co = 0; co < 2; ++co) {
          const float h = leak * so[k][co] + (co == 0 ? u0 : u1);
          if (C::TRC && ok && co < cout && trace_t.p && tb.has(gy, gx))
            trace_t.put(trace_t.template idx<C::RELAX>(2, choffo, co, tb.idx(gy, gx), tb.plane()), h * isc3);
          float v = h;
          const float sp = bilif(v, theta3, alpha, false);
          so[k][co] = v;
          hs[co] = h * isc3;
          ss[co] = sp;
          if (ok && co < cout && ca.s_out) {
            if (C::CKS && ca.s_fp32) s32[(size_t)co * HW + pix] = sp;
            else s8[(size_t)co * HW + pix] = (int8_t)sp;
          }
        }
        // both channels of the pixel (a second channel of a one-channel net
        // has no weights and stays 0)
        if constexpr (C::REC) rec_store2<C>(trace_t, ok ? (unsigned)pix * 4u : 0x20000000u, hs[0], hs[1], ss[0], ss[1]);
      }
    } else {
      // ================= output layer (VALU), weights broadcast from LDS
      float u[C::NOUT][2];
#pragma unroll
      for (int k = 0; k < C::NOUT; ++k) { u[k][0] = leak * so[k][0]; u[k][1] = leak * so[k][1]; }
#pragma unroll 1
      for (int tau = 0; tau < 9; ++tau) {
        const int to = tap_off(tau, C::CWT);
        if constexpr (C::NH == 0) {
#pragma unroll
          for (int c = 0; c < C::CIN; ++c) {
            const float w0 = wl[(tau * C::CIN + c) * 2], w1 = wl[(tau * C::CIN + c) * 2 + 1];
#pragma unroll
            for (int k = 0; k < C::NOUT; ++k) {
              const float xv = xsf[c * C::XPL + op[k] + to];
              u[k][0] = fmaf(w0, xv, u[k][0]);
              u[k][1] = fmaf(w1, xv, u[k][1]);
            }
          }
        } else {
          const float* sfin = reinterpret_cast<const float*>(sp2);
#pragma unroll
          for (int c4 = 0; c4 < C::CH / 4; ++c4) {
            const f4 wa = *reinterpret_cast<const f4*>(wl + (tau * C::CH + 4 * c4) * 2);
            const f4 wb = *reinterpret_cast<const f4*>(wl + (tau * C::CH + 4 * c4) * 2 + 4);
#pragma unroll
            for (int k = 0; k < C::NOUT; ++k) {
              const f4 sv = *reinterpret_cast<const f4*>(sfin + (size_t)(op[k] + to) * C::CH + 4 * c4);
              u[k][0] = fmaf(wa[0], sv[0], u[k][0]); u[k][1] = fmaf(wa[1], sv[0], u[k][1]);
              u[k][0] = fmaf(wa[2], sv[1], u[k][0]); u[k][1] = fmaf(wa[3], sv[1], u[k][1]);
              u[k][0] = fmaf(wb[0], sv[2], u[k][0]); u[k][1] = fmaf(wb[1], sv[2], u[k][1]);
              u[k][0] = fmaf(wb[2], sv[3], u[k][0]); u[k][1] = fmaf(wb[3], sv[3], u[k][1]);
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < C::NOUT; ++k) {
        const bool ok = (ovm >> k) & 1u;
        const int q = tid + C::NT * k;
        const size_t pix = (size_t)(tl.ty0 + q / C::TW) * W + (tl.tx0 + q % C::TW);
#pragma unroll
        for (int co = 0; co < 2; ++co) {
          if (C::TRC && ok && co < cout && trace_t.p) {
            const int gy = tl.ty0 + q / C::TW, gx = tl.tx0 + q % C::TW;
            if (tb.has(gy, gx)) trace_t.put(trace_t.template idx<C::RELAX>(2, choffo, co, tb.idx(gy, gx), tb.plane()), u[k][co]);
          }
          float v = u[k][co];
          const float s = bilif(v, theta, alpha, C::RELAX ? relaxed : 0);
          if constexpr (C::REC) rec_store1<C>(trace_t, ok ? (unsigned)pix * 4u + co : 0x20000000u, u[k][co], s);
          so[k][co] = v;
          if (ok && co < cout && ca.s_out) {
            const size_t o = (((size_t)tl.n * T + t) * cout + co) * HW + pix;
            if (C::CKS && ca.s_fp32) reinterpret_cast<float*>(ca.s_out)[o] = s;
            else reinterpret_cast<int8_t*>(ca.s_out)[o] = (int8_t)s;
          }
        }
      }
    }
    if constexpr (C::NH == 0) {
      lds_barrier();
      if (t + 1 < T) store_x();
      if (t + 2 < T) load_x(t + 2);
    }
    // B4: spikes / xs / Y consumed before the next frame overwrites them (the
    // separate layer-2 buffer, or in three-layer tap-major nets the Y planes
    // written only by layer 2, make B1 or B3 of the next frame the guard)
    if constexpr (!C::SEP && !(C::OTAP && C::NH == 2)) lds_barrier();
  }
  if constexpr (C::XDMA) __builtin_amdgcn_s_waitcnt(0);
  if (ca.v_out) write_state(ca.v_out + (size_t)tl.n * sumc * HW);
}

// Signature of the weight area's layout (offsets relative to its start, the
// shape parameters that decide its contents): kernels of one network shape
// that share it can take the same prepacked image whatever their tile.
template <class C>
constexpr uint32_t frag_sig() {
  using Lo = Layout<C>;
  uint32_t h = 2166136261u;
  const uint32_t v[] = {(uint32_t)(Lo::YS - Lo::WL), (uint32_t)(Lo::FR1 - Lo::WL), (uint32_t)(Lo::FR2 - Lo::WL),
                        (uint32_t)(Lo::FR3 - Lo::WL), (uint32_t)(Lo::FRY - Lo::WL), (uint32_t)C::BF16,
                        (uint32_t)C::CH, (uint32_t)C::NL, (uint32_t)C::CIN, (uint32_t)C::XSPLIT, (uint32_t)C::OTAP,
                        (uint32_t)C::OMF, (uint32_t)C::SF16};
  for (uint32_t x : v) h = (h ^ x) * 16777619u;
  return h;
}
template <class C>
constexpr bool takes_frag() { return !C::RELAX && !C::LOGX; }

template <class C>
__device__ __forceinline__ void init_lds(const FwdNetArgs& na, char* lds) {
  using Lo = Layout<C>;
  // zero canvas and pads once: pads are read only by junk (masked) pixels
  unsigned* z = reinterpret_cast<unsigned*>(lds);
  for (int e = threadIdx.x; e < (C::XS_BYTES + C::SP_BYTES) / 4; e += C::NT) z[e] = 0u;
  // the prepacked weight area when it was built for this layout and these
  // channel counts (uniform branch), else built here from the weights
  bool pre = false;
  if constexpr (takes_frag<C>()) {
    if (na.frag) {
      const uint32_t* hd = na.frag;
      const uint32_t chw = (uint32_t)na.ch[0] | ((uint32_t)na.ch[1] << 8) | ((uint32_t)na.ch[2] << 16) |
                           ((uint32_t)na.ch[3] << 24);
      pre = hd[0] == kFragMagic && hd[1] == frag_sig<C>() && hd[2] == chw && hd[3] == (uint32_t)na.n_layers &&
            hd[6] == (uint32_t)(Lo::YS - Lo::WL);
    }
  }
  if (pre) {
    const u4* src = reinterpret_cast<const u4*>(na.frag + kFragHeaderWords);
    u4* dst = reinterpret_cast<u4*>(lds + Lo::WL);
    for (int e = threadIdx.x; e < (Lo::YS - Lo::WL) / 16; e += C::NT) dst[e] = src[e];
    // |w|max bits: slots 0, 1 in header words 4, 5, slot 2 in word 7
    if (threadIdx.x < 3)
      reinterpret_cast<unsigned*>(lds + Lo::SCL)[threadIdx.x] = na.frag[threadIdx.x == 2 ? 7 : 4 + threadIdx.x];
  } else {
    load_weights<C>(na, lds);
  }
}

// Prepack: build the weight area once (one workgroup) and store it with its
// header for the kernels to copy.
template <class C>
__global__ __launch_bounds__(C::NT) void k_prepack(FwdNetArgs na, uint32_t* dst) {
  using Lo = Layout<C>;
  __shared__ __attribute__((aligned(16))) char lds[Lo::TOTAL];
  na.frag = nullptr;
  load_weights<C>(na, lds);
  __syncthreads();
  const u4* src = reinterpret_cast<const u4*>(lds + Lo::WL);
  u4* out = reinterpret_cast<u4*>(dst + kFragHeaderWords);
  for (int e = threadIdx.x; e < (Lo::YS - Lo::WL) / 16; e += C::NT) out[e] = src[e];
  if (threadIdx.x == 0) {
    dst[0] = kFragMagic;
    dst[1] = frag_sig<C>();
    dst[2] = (uint32_t)na.ch[0] | ((uint32_t)na.ch[1] << 8) | ((uint32_t)na.ch[2] << 16) | ((uint32_t)na.ch[3] << 24);
    dst[3] = (uint32_t)na.n_layers;
    dst[4] = reinterpret_cast<const unsigned*>(lds + Lo::SCL)[0];
    dst[5] = reinterpret_cast<const unsigned*>(lds + Lo::SCL)[1];
    dst[6] = (uint32_t)(Lo::YS - Lo::WL);
    dst[7] = reinterpret_cast<const unsigned*>(lds + Lo::SCL)[2];
  }
}
template <class C>
void launch_prepack(const FwdNetArgs& na, uint32_t* dst, hipStream_t st, hipError_t* err) {
  hipLaunchKernelGGL(k_prepack<C>, dim3(1), dim3(C::NT), 0, st, na, dst);
  *err = hipGetLastError();
}
template <class C>
constexpr size_t frag_block_bytes() {
  return (size_t)kFragHeaderWords * 4 + (size_t)(Layout<C>::YS - Layout<C>::WL);
}

template <class C>
__global__ __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(C::WPE))) void fwd_kernel(FwdNetArgs na, FwdClipArgs ca) {
  __shared__ __attribute__((aligned(16))) char lds[Layout<C>::TOTAL];
  init_lds<C>(na, lds);
  __syncthreads();
  const int ntiles = ca.tiles_x * ca.tiles_y;
  const int tile = xcd_remap(blockIdx.x, ntiles);
  Tile tl;
  tl.n = blockIdx.y;
  tl.ty0 = (tile / ca.tiles_x) * C::TH;
  tl.tx0 = (tile % ca.tiles_x) * C::TW;
  run_tile<C>(na, ca, tl, lds);
}

// Work queues of the persistent kernel: the items are cut into one
// contiguous range per XCD (the hardware deals workgroups round-robin over
// the 8 XCDs), so neighbouring tiles, which share halo rows of x, run on
// the same L2; a workgroup whose range is empty takes items from the others.
constexpr int kQueues = 8;

// Next item for a workgroup on XCD `x` (thread 0 only), -1 when all are taken.
__device__ inline int pop_item(int32_t* counter, int n_items, int x) {
  const int per = (n_items + kQueues - 1) / kQueues;
  for (int k = 0; k < kQueues; ++k) {
    const int y = (x + k) % kQueues;
    const int lo = y * per, hi = lo + per < n_items ? lo + per : n_items;
    if (lo >= hi) continue;
    const int i = atomicAdd(counter + y, 1);
    if (lo + i < hi) return lo + i;
  }
  return -1;
}

// Persistent batched kernel: workgroups pop (clip, tile) items from the
// per-XCD queues; items are ordered clip by clip, clips longest-first.
template <class C>
__global__ __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(C::WPE))) void fwd_batched_kernel(FwdNetArgs na, BatchTable bt, int32_t* counter) {
  __shared__ __attribute__((aligned(16))) char lds[Layout<C>::TOTAL];
  __shared__ int item_sh;
  init_lds<C>(na, lds);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item_sh = pop_item(counter, bt.n_items, blockIdx.x % kQueues);
    __syncthreads();
    const int item = item_sh;
    if (item < 0) break;
    int c = 0;
    while (c + 1 < bt.n_clips && bt.item_start[c + 1] <= item) ++c;
    const FwdClipArgs ca = bt.clip[c];            // by value: scalar registers, loaded once per item
    const int local = item - bt.item_start[c];
    const int per_n = ca.tiles_x * ca.tiles_y;
    Tile tl;
    tl.n = local / per_n;
    const int tile = local % per_n;
    tl.ty0 = (tile / ca.tiles_x) * C::TH;
    tl.tx0 = (tile % ca.tiles_x) * C::TW;
    // LDS canvas must start from zeros for every item (pads and junk)
    unsigned* z = reinterpret_cast<unsigned*>(lds);
    for (int e = threadIdx.x; e < (C::XS_BYTES + C::SP_BYTES) / 4; e += C::NT) z[e] = 0u;
    __syncthreads();
    run_tile<C>(na, ca, tl, lds);
  }
}

// ------------------------------------------------------------------ registry
struct Variant {
  int nl, cin, ch, bf16, th, tw;
  const char* name;
  void (*single_fast)(const FwdNetArgs&, const FwdClipArgs&, hipStream_t, hipError_t*);
  void (*single_full)(const FwdNetArgs&, const FwdClipArgs&, hipStream_t, hipError_t*);
  // the backward's segment recompute (pixel-major trace only)
  void (*single_rec)(const FwdNetArgs&, const FwdClipArgs&, hipStream_t, hipError_t*);
  // the forward of a training step (checkpoints, FP32 spikes, no trace)
  void (*single_train)(const FwdNetArgs&, const FwdClipArgs&, hipStream_t, hipError_t*);
  void (*single_relaxed)(const FwdNetArgs&, const FwdClipArgs&, hipStream_t, hipError_t*);
  void (*batched)(const FwdNetArgs&, const BatchTable&, int32_t*, int ncu, hipStream_t, hipError_t*);
  // RGB-input kernels of one-channel nets: inference, training/debug, relaxed
  void (*logx[3])(const FwdNetArgs&, const FwdClipArgs&, hipStream_t, hipError_t*);
  // 1: one of the shape's default candidates, which differ only in how
  // their tile count fills the CUs (see forward_default_tile)
  int dflt;
};
// The prepack of a shape (its first variant's inference configuration).
struct Prepack {
  void (*launch)(const FwdNetArgs&, uint32_t*, hipStream_t, hipError_t*);
  size_t bytes;
};

template <class C>
void launch_single(const FwdNetArgs& na, const FwdClipArgs& ca, hipStream_t st, hipError_t* err) {
  dim3 grid(ca.tiles_x * ca.tiles_y, ca.N);
  hipLaunchKernelGGL(fwd_kernel<C>, grid, dim3(C::NT), 0, st, na, ca);
  *err = hipGetLastError();
}
// Persistent launch: as many workgroups as the CUs hold at once (two per CU
// for the 4-wave tiles), capped by the number of work items.
template <class C>
void launch_batched(const FwdNetArgs& na, const BatchTable& bt, int32_t* counter, int ncu,
                    hipStream_t st, hipError_t* err) {
  static int per_cu = 0;                       // queried once per kernel (host-side only)
  if (per_cu == 0) {
    int n = 1;
    *err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fwd_batched_kernel<C>, C::NT, 0);
    if (*err != hipSuccess) return;
    per_cu = n < 1 ? 1 : n;
  }
  const int cap = per_cu * ncu;
  const int n_wg = bt.n_items < cap ? bt.n_items : cap;
  hipLaunchKernelGGL(fwd_batched_kernel<C>, dim3(n_wg), dim3(C::NT), 0, st, na, bt, counter);
  *err = hipGetLastError();
}

#define EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, MODE) Cfg<NL, CIN, CH, (bool)BF, TH, TW, NW, MODE>
#define EVS_FAST_FULL(NL, CIN, CH, BF, TH, TW, NW)                                                   \
  &launch_single<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, 0)>, &launch_single<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, 1)>, \
      &launch_single<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, 3)>, &launch_single<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, 8)>
// a tile variant: inference kernel + training/debug kernel + the backward's
// recompute kernel + the training-step forward kernel; _R adds the relaxed-spike kernel (one tile per FP32
// shape), _B the batched one
#define EVS_VARIANT(NL, CIN, CH, BF, TH, TW, NW, NAME) \
  Variant{NL, CIN, CH, BF, TH, TW, NAME, EVS_FAST_FULL(NL, CIN, CH, BF, TH, TW, NW), nullptr, nullptr}
#define EVS_VARIANT_R(NL, CIN, CH, TH, TW, NW, NAME)                                 \
  Variant{NL, CIN, CH, 0, TH, TW, NAME, EVS_FAST_FULL(NL, CIN, CH, 0, TH, TW, NW),   \
          &launch_single<EVS_CFG(NL, CIN, CH, 0, TH, TW, NW, 2)>, nullptr}
#define EVS_VARIANT_B(NL, CIN, CH, BF, TH, TW, NW, NAME)                             \
  Variant{NL, CIN, CH, BF, TH, TW, NAME, EVS_FAST_FULL(NL, CIN, CH, BF, TH, TW, NW), \
          nullptr, &launch_batched<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, 0)>}
// one-channel FP32 nets: _R plus the RGB-input (Eq. 1) kernels
#define EVS_VARIANT_RX(NL, CH, TH, TW, NW, NAME)                                              \
  Variant{NL, 1, CH, 0, TH, TW, NAME, EVS_FAST_FULL(NL, 1, CH, 0, TH, TW, NW),                  \
          &launch_single<EVS_CFG(NL, 1, CH, 0, TH, TW, NW, 2)>, nullptr,                        \
          {&launch_single<EVS_CFG(NL, 1, CH, 0, TH, TW, NW, 4)>,                                \
           &launch_single<EVS_CFG(NL, 1, CH, 0, TH, TW, NW, 5)>,                                \
           &launch_single<EVS_CFG(NL, 1, CH, 0, TH, TW, NW, 6)>}}
#define EVS_VARIANT_RB(NL, CIN, CH, TH, TW, NW, NAME)                                \
  Variant{NL, CIN, CH, 0, TH, TW, NAME, EVS_FAST_FULL(NL, CIN, CH, 0, TH, TW, NW),   \
          &launch_single<EVS_CFG(NL, CIN, CH, 0, TH, TW, NW, 2)>,                    \
          &launch_batched<EVS_CFG(NL, CIN, CH, 0, TH, TW, NW, 0)>}
// default candidates (one workgroup per CU each)
#define EVS_VARIANT_RB_D(NL, CIN, CH, TH, TW, NW, NAME)                              \
  Variant{NL, CIN, CH, 0, TH, TW, NAME, EVS_FAST_FULL(NL, CIN, CH, 0, TH, TW, NW),   \
          &launch_single<EVS_CFG(NL, CIN, CH, 0, TH, TW, NW, 2)>,                    \
          &launch_batched<EVS_CFG(NL, CIN, CH, 0, TH, TW, NW, 0)>, {}, 1}
#define EVS_VARIANT_D(NL, CIN, CH, BF, TH, TW, NW, NAME) \
  Variant{NL, CIN, CH, BF, TH, TW, NAME, EVS_FAST_FULL(NL, CIN, CH, BF, TH, TW, NW), nullptr, nullptr, {}, 1}

// Tile variants per network shape; the first one of a shape is its default.
// (Three-layer 16-wide nets have no 30x32 / 30x40 tiles: with the Y planes
// of the tap-major output layer they need more than 160 KB of LDS.)
const Variant kVariants[] = {
    // single-layer nets (input -> output), f32
    EVS_VARIANT_RX(1, 16, 32, 32, 8, "L1 cin1 f32 32x32 w8"),
    EVS_VARIANT_R(1, 3, 16, 32, 32, 8, "L1 cin3 f32 32x32 w8"),
    // two-layer nets cin -> hidden(<=16) -> out
    EVS_VARIANT_RB(2, 3, 16, 16, 32, 8, "L2 h16 f32 16x32 w8"),
    EVS_VARIANT(2, 3, 16, 0, 30, 40, 8, "L2 h16 f32 30x40 w8"),
    EVS_VARIANT(2, 3, 16, 0, 20, 32, 4, "L2 h16 f32 20x32 w4"),
    EVS_VARIANT_RX(2, 16, 30, 40, 8, "L2 cin1 h16 f32 30x40 w8"),
    EVS_VARIANT(2, 3, 16, 1, 30, 40, 8, "L2 h16 bf16 30x40 w8"),
    // two-layer nets with hidden width <= 32
    EVS_VARIANT_D(2, 3, 32, 0, 24, 32, 8, "L2 h32 f32 24x32 w8"),
    EVS_VARIANT_D(2, 3, 32, 0, 23, 32, 8, "L2 h32 f32 23x32 w8"),
    EVS_VARIANT_R(2, 3, 32, 22, 32, 8, "L2 h32 f32 22x32 w8"),
    EVS_VARIANT(2, 3, 32, 0, 16, 44, 8, "L2 h32 f32 16x44 w8"),
    EVS_VARIANT_B(2, 3, 32, 1, 12, 32, 8, "L2 h32 bf16 12x32 w8"),
    EVS_VARIANT_B(2, 3, 32, 1, 12, 32, 4, "L2 h32 bf16 12x32 w4"),
    EVS_VARIANT_B(2, 3, 32, 1, 24, 32, 8, "L2 h32 bf16 24x32 w8"),
    EVS_VARIANT(2, 3, 32, 1, 30, 40, 8, "L2 h32 bf16 30x40 w8"),
    EVS_VARIANT(2, 3, 32, 1, 16, 32, 4, "L2 h32 bf16 16x32 w4"),
    // three-layer nets
    EVS_VARIANT_RB_D(3, 3, 16, 24, 32, 8, "L3 h16 f32 24x32 w8"),
    EVS_VARIANT_D(3, 3, 16, 0, 23, 32, 8, "L3 h16 f32 23x32 w8"),
    EVS_VARIANT_B(3, 3, 16, 0, 12, 32, 4, "L3 h16 f32 12x32 w4"),
    EVS_VARIANT(3, 3, 16, 0, 16, 24, 4, "L3 h16 f32 16x24 w4"),
    // (16x32: the default of 256x256 crops in fours, 512 tiles in 2 full rounds)
    EVS_VARIANT_D(3, 3, 16, 0, 16, 32, 8, "L3 h16 f32 16x32 w8"),
    EVS_VARIANT_D(3, 3, 16, 1, 24, 32, 8, "L3 h16 bf16 24x32 w8"),
    EVS_VARIANT_D(3, 3, 16, 1, 23, 32, 8, "L3 h16 bf16 23x32 w8"),
    EVS_VARIANT_D(3, 3, 16, 1, 16, 32, 8, "L3 h16 bf16 16x32 w8"),
    EVS_VARIANT(3, 3, 16, 1, 16, 32, 4, "L3 h16 bf16 16x32 w4"),
    EVS_VARIANT(3, 3, 32, 1, 24, 32, 8, "L3 h32 bf16 24x32 w8"),
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Prepack per network shape, built with the shape's first tile (the weight
// area does not depend on the tile; a kernel whose layout signature differs
// builds its own).
struct ShapePrepack {
  int nl, cin, ch, bf16;
  Prepack pp;
};
#define EVS_PREPACK(NL, CIN, CH, BF, TH, TW, NW)                                       \
  ShapePrepack{NL, CIN, CH, BF, Prepack{&launch_prepack<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, 0)>, \
                                        frag_block_bytes<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, 0)>()}}
const ShapePrepack kPrepacks[] = {
    EVS_PREPACK(1, 1, 16, 0, 32, 32, 8), EVS_PREPACK(1, 3, 16, 0, 32, 32, 8),
    EVS_PREPACK(2, 3, 16, 0, 16, 32, 8), EVS_PREPACK(2, 1, 16, 0, 30, 40, 8),
    EVS_PREPACK(2, 3, 16, 1, 30, 40, 8), EVS_PREPACK(2, 3, 32, 0, 24, 32, 8),
    EVS_PREPACK(2, 3, 32, 1, 12, 32, 8), EVS_PREPACK(3, 3, 16, 0, 24, 32, 8),
    EVS_PREPACK(3, 3, 16, 1, 24, 32, 8), EVS_PREPACK(3, 3, 32, 1, 24, 32, 8),
};

int padded_hidden(const evs_net& net) {
  int mx = 0;
  for (int l = 1; l < net.n_layers; ++l) mx = net.ch[l] > mx ? net.ch[l] : mx;
  return mx <= 16 ? 16 : 32;
}

bool matches(const Variant& v, const evs_net& net) {
  return v.nl == net.n_layers && v.cin == net.ch[0] && v.bf16 == (net.precision == EVS_BF16) &&
         (net.n_layers == 1 || v.ch == padded_hidden(net)) && (net.n_layers < 3 || net.ch[1] == net.ch[2]);
}

const ShapePrepack* find_prepack(const evs_net& net) {
  for (const ShapePrepack& p : kPrepacks)
    if (p.nl == net.n_layers && p.cin == net.ch[0] && p.bf16 == (net.precision == EVS_BF16) &&
        (net.n_layers == 1 || p.ch == padded_hidden(net)) && (net.n_layers < 3 || net.ch[1] == net.ch[2]))
      return &p;
  return nullptr;
}

const Variant* find_variant(const evs_net& net, int tile_id) {
  int k = 0;
  for (int i = 0; i < kNumVariants; ++i) {
    if (!matches(kVariants[i], net)) continue;
    if (k == tile_id) return &kVariants[i];
    ++k;
  }
  return nullptr;
}

}  // namespace

size_t forward_frag_bytes(const evs_net& net) {
  const ShapePrepack* p = find_prepack(net);
  return p ? (p->pp.bytes + 255) / 256 * 256 : 0;
}

int forward_prepack(const evs_net& net, const FwdNetArgs& na, uint32_t* dst, hipStream_t stream) {
  const ShapePrepack* p = find_prepack(net);
  if (!p) return EVS_OK;
  hipError_t e = hipSuccess;
  p->pp.launch(na, dst, stream, &e);
  if (e != hipSuccess) return hip_check(e, "weight prepack launch");
  return EVS_OK;
}

int forward_tile_count(const evs_net& net) {
  int k = 0;
  for (int i = 0; i < kNumVariants; ++i) k += matches(kVariants[i], net) ? 1 : 0;
  return k;
}

bool fused_shape(const evs_net& net) { return forward_tile_count(net) > 0; }

const char* forward_tile_name(const evs_net& net, int tile_id) {
  const Variant* v = find_variant(net, tile_id);
  return v ? v->name : nullptr;
}

void forward_tile_dims(const evs_net& net, int tile_id, int* th, int* tw) {
  const Variant* v = find_variant(net, tile_id);
  *th = v ? v->th : 0;
  *tw = v ? v->tw : 0;
}

int forward_batched_tile(const evs_net& net, int preferred) {
  const Variant* v = find_variant(net, preferred);
  if (v && v->batched) return preferred;
  const int n = forward_tile_count(net);
  for (int t = 0; t < n; ++t)
    if (find_variant(net, t)->batched) return t;
  return -1;
}

// Default tile: the first compiled variant of the shape, or, among its
// default candidates (whole-CU workgroups that differ only in tile height),
// the one with the least estimated time: whole rounds of workgroups over the
// CUs, ceil(tiles / CUs), times the canvas pixels of one tile.  A 720p frame
// has 1200 tiles of 24x32 (4.69 rounds on 256 CUs, run as 5) but 1280 of
// 23x32 (5 full rounds of a 3% smaller canvas).
int forward_default_tile(const evs_net& net, int H, int W, int N) {
  if (forward_tile_count(net) <= 0) return -1;
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0, n = 0;
    ncu = (hipGetDevice(&dev) == hipSuccess &&
           hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) ? n : 256;
  }
  int best = 0, k = 0;
  double best_cost = -1.0;
  for (int i = 0; i < kNumVariants; ++i) {
    const Variant& v = kVariants[i];
    if (!matches(v, net)) continue;
    if (v.dflt) {
      const int L = net.n_layers;
      const double tiles = (double)((H + v.th - 1) / v.th) * ((W + v.tw - 1) / v.tw) * (N > 0 ? N : 1);
      const double cost = std::ceil(tiles / ncu) * (v.th + 2 * L) * (v.tw + 2 * L);
      if (best_cost < 0.0 || cost < best_cost) {
        best_cost = cost;
        best = k;
      }
    }
    ++k;
  }
  return best;
}

int launch_forward(const evs_net& net, const FwdNetArgs& na, const FwdClipArgs& ca, int tile_id,
                   hipStream_t stream) {
  const Variant* v = find_variant(net, tile_id);
  if (!v) return fail(EVS_EUNSUPPORTED, "no compiled forward kernel for this network shape");
  hipError_t e = hipSuccess;
  const bool full = ca.h_trace || ca.ckpt || ca.s_fp32;
  if (na.x_rgb) {
    // results do not depend on the tile: take the first variant of the shape that has the kernels
    const int n = forward_tile_count(net);
    for (int t = 0; t < n && !v->logx[0]; ++t) v = find_variant(net, t);
    if (!v->logx[0]) return fail(EVS_EUNSUPPORTED, "no RGB-input kernel compiled for this network shape");
    v->logx[na.relaxed ? 2 : (full ? 1 : 0)](na, ca, stream, &e);
  } else if (na.relaxed) {
    // results do not depend on the tile: take the first variant of the shape that has the kernel
    const int n = forward_tile_count(net);
    for (int t = 0; t < n && !v->single_relaxed; ++t) v = find_variant(net, t);
    if (!v->single_relaxed) return fail(EVS_EUNSUPPORTED, "no relaxed-spike kernel compiled for this network shape");
    v->single_relaxed(na, ca, stream, &e);
  } else if (ca.trace_pm) {
    // the backward's segment recompute: its pixel-major trace (fp16 exactly
    // for BF16 nets), nothing else
    if (ca.ckpt || ca.s_out || ca.v_out || (ca.trace_f16 != 0) != (net.precision == EVS_BF16))
      return fail(EVS_EINVAL, "recompute launch: trace only, fp16 exactly for BF16 nets");
    v->single_rec(na, ca, stream, &e);
  } else if (full && !ca.h_trace) {
    // checkpoints / FP32 spikes without a trace: the forward of a training step
    v->single_train(na, ca, stream, &e);
  } else {
    (full ? v->single_full : v->single_fast)(na, ca, stream, &e);
  }
  if (e != hipSuccess) return hip_check(e, "forward kernel launch");
  return EVS_OK;
}

int launch_forward_batched(const evs_net& net, const FwdNetArgs& na, const BatchTable& bt, int tile_id,
                           int32_t* counter, hipStream_t stream) {
  const Variant* v = find_variant(net, tile_id);
  if (!v) return fail(EVS_EUNSUPPORTED, "no compiled forward kernel for this network shape");
  if (!v->batched) return fail(EVS_EUNSUPPORTED, "no batched kernel compiled for this tile variant");
  if (na.x_rgb) return fail(EVS_EUNSUPPORTED, "batched forward: direct input only");
  int dev = 0, ncu = 0;
  EVS_HIP(hipGetDevice(&dev));
  EVS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  hipError_t e = hipSuccess;
  v->batched(na, bt, counter, ncu, stream, &e);
  if (e != hipSuccess) return hip_check(e, "batched forward kernel launch");
  return EVS_OK;
}

}  // namespace evs
