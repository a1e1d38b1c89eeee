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
//     instruction sequence.
//   * Per frame, the x tile (+halo) is staged in LDS (register prefetch of
//     frame t+1 overlaps frame t), hidden layers run as transposed GEMMs
//     D[cout][pixel] = W[cout][K] * S[K][pixel] on MFMA (f32 16x16x4 or
//     bf16 16x16x32 with f32 accumulation), with K = (tap, cin) and the
//     spike operand gathered from LDS; the accumulator fragment IS the
//     membrane state (C input = leak * v), so BiLIF runs in place.  The
//     spikes of a hidden layer go back to LDS (f32 or bf16, exact) for the
//     next layer.  The output layer (1-2 channels) runs on the VALU with
//     its weights broadcast from LDS.
//   * Only the HBM traffic of the algorithm remains: x in (12 B/px/frame)
//     and the output spikes (int8).
#include "evs_internal.hpp"
#include "evs_device.hpp"

namespace evs {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }
constexpr int align16(int b) { return (b + 15) & ~15; }

// FULL_ = true compiles the training/debug features (h traces, membrane
// checkpoints, relaxed spikes); the inference build leaves them out so that
// the hot loop carries no dead address arithmetic.
template <int NL_, int CIN_, int CH_, bool BF16_, int TH_, int TW_, int NW_, bool FULL_>
struct Cfg {
  static constexpr int NL = NL_, CIN = CIN_, CH = CH_, TH = TH_, TW = TW_, NW = NW_;
  static constexpr bool BF16 = BF16_, FULL = FULL_;
  static constexpr int CO = 2;                       // output channels (max)
  static constexpr int NH = NL - 1;                  // hidden layers
  static constexpr int CHT = TH + 2 * NL, CWT = TW + 2 * NL;
  static constexpr int NPIX = CHT * CWT;
  static constexpr int PADF = 32;                    // zeroed front pad (pixels)
  static constexpr int NT = 64 * NW;
  static constexpr int MB = CH / 16;                 // 16-row output blocks
  static constexpr int npb(int l) { return cdiv((CHT - 2 * l) * CWT, 16); }
  static constexpr int NPB1 = NH >= 1 ? npb(1) : 1;
  static constexpr int NPB2 = NH >= 2 ? npb(2) : 1;
  static constexpr int NB1 = cdiv(NPB1, NW);
  static constexpr int NB2 = cdiv(NPB2, NW);
  // BF16 nets run the output layer on MFMA too (16-row blocks, Cout rows
  // used); FP32 nets run it on the VALU, one lane per output pixel.
  static constexpr bool OMF = BF16 && NH >= 1;
  static constexpr int NPBO = cdiv(TH * CWT, 16);    // output blocks (rows NL..NL+TH-1)
  static constexpr int NBO = OMF ? cdiv(NPBO, NW) : 1;
  static constexpr int KSO = CH == 32 ? 9 : 5;
  // Every wave runs all of its NB blocks (the tail blocks past the layer's
  // region compute masked junk), so the canvas is padded to hold them and
  // their 3x3 neighbourhood.
  static constexpr int imax(int a, int b) { return a > b ? a : b; }
  // wave-specialised schedule: layer-1 blocks over 4 waves, layer-2 blocks over 4
  static constexpr int NB1V = cdiv(NPB1, 4), NB2M = cdiv(NPB2, 4);
  static constexpr int NPIXL =
      PADF + imax(imax(imax(NPIX, (NL + 1) * CWT + 16 * NW * NBO + 2),
                       imax(2 * CWT + 16 * NW * NB1 + 2, 3 * CWT + 16 * NW * NB2 + 2)),
                  imax(2 * CWT + 64 * NB1V + 2, 3 * CWT + 64 * NB2M + 2)) + 16;
  static constexpr int NOUT = OMF ? 1 : cdiv(TH * TW, NT);
  static constexpr int XN = CIN * NPIX;
  static constexpr int XPF = cdiv(XN, NT);
  static constexpr int K1 = 9 * CIN;
  static constexpr int KS1 = BF16 ? cdiv(K1, 32) : cdiv(K1, 4);
  static constexpr int KS2 = BF16 ? (CH == 32 ? 9 : 5) : 9 * CH / 4;
  static constexpr int XELEM = BF16 ? 2 : 4;
  // x planes plus one all-zero plane read by the padded K slots of layer 1
  static constexpr int XS_BYTES = align16((CIN + 1) * NPIXL * XELEM);
  // The FP32 three-layer inference kernel runs a software pipeline (output
  // layer of frame t-1 fused into the layer-2 MFMA loop of frame t) and keeps
  // separate layer-1 / layer-2 spike buffers.  Spikes are exact in bf16, so
  // the pipelined and BF16 kernels store them in 16 bits.
  static constexpr bool PIPE = !BF16 && NH == 2 && !FULL && NW == 8 && CH == 16;
  static constexpr bool SPB16 = BF16;                            // layer-1 (shared) buffer in bf16
  static constexpr int SELEM = SPB16 ? 2 : 4;
  static constexpr int SP1_BYTES = NH >= 1 ? align16(NPIXL * CH * SELEM) : 0;
  static constexpr int SP2_OFF = PIPE ? SP1_BYTES : 0;          // layer-2 buffer (bf16) inside SP
  static constexpr int SP_BYTES = SP1_BYTES + (PIPE ? align16(NPIXL * CH * 2) : 0);
  static constexpr int WL_FLOATS = 9 * (NH >= 1 ? CH : CIN) * CO;
  static_assert(CH == 16 || CH == 32, "hidden width must be padded to 16 or 32");
  static_assert(NB1 <= 32 && NB2 <= 32 && NBO <= 32 && NOUT <= 32 && (BF16 ? 8 * KS1 : KS1) <= 32,
                "mask words overflow");
  static constexpr int toff(int tau) { return (tau / 3 - 1) * CWT + (tau % 3 - 1); }
};

__device__ inline f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma_bf16(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                 __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}


__device__ inline unsigned pack_bf16x2(float lo, float hi) {
  // spikes are exactly representable: take the upper halves of the floats
  return (__builtin_bit_cast(unsigned, lo) >> 16) | (__builtin_bit_cast(unsigned, hi) & 0xffff0000u);
}

// ------------------------------------------------------------------ weights
__device__ inline float wget(const FwdNetArgs& na, int layer, int co, int ci, int tap, bool bf) {
  // layer 0-based; real channel bounds checked by the caller
  const int cin = na.ch[layer];
  float w = na.w[na.wofs[layer] + (co * cin + ci) * 9 + tap];
  return bf ? round_bf16(w) : w;
}

// LDS layout of one workgroup (byte offsets).
template <class C>
struct Layout {
  static constexpr int XS = 0;                                  // x tile [CIN][NPIXL]
  static constexpr int SP = XS + C::XS_BYTES;                   // spikes [NPIXL][CH]
  static constexpr int WL = SP + C::SP_BYTES;                   // out weights [9][CI][2] f32
  static constexpr int FR1 = WL + align16(C::WL_FLOATS * 4);    // layer-1 A fragments
  static constexpr int FR1_BYTES = C::NH >= 1 ? C::KS1 * C::MB * 64 * (C::BF16 ? 16 : 4) : 0;
  static constexpr int FR2 = FR1 + FR1_BYTES;                   // layer-2 A fragments
  static constexpr int FR2_BYTES = C::NH >= 2 ? C::KS2 * C::MB * 64 * (C::BF16 ? 16 : 4) : 0;
  static constexpr int FR3 = FR2 + FR2_BYTES;                   // output-layer A fragments (MFMA form)
  static constexpr int FR3_BYTES = C::OMF ? C::KSO * 64 * 16 : 0;
  static constexpr int TOTAL = FR3 + FR3_BYTES;
  static_assert(TOTAL <= 160 * 1024, "tile does not fit in LDS");
};

// Fill the weight areas of LDS: output-layer weights wl[tap][ci][co] (co
// padded to 2) and the MFMA A-operand fragments of the hidden layers in the
// per-lane order the k-step loops read them.
template <class C>
__device__ __forceinline__ void load_weights(const FwdNetArgs& na, char* lds) {
  using Lo = Layout<C>;
  {
    float* wl = reinterpret_cast<float*>(lds + Lo::WL);
    const int L = na.n_layers - 1;
    const int cin = na.ch[L], cout = na.ch[L + 1];
    constexpr int CI = C::NH >= 1 ? C::CH : C::CIN;
    for (int e = threadIdx.x; e < C::WL_FLOATS; e += C::NT) {
      const int co = e % 2, ci = (e / 2) % CI, tap = e / (2 * CI);
      wl[e] = (co < cout && ci < cin) ? wget(na, L, co, ci, tap, C::BF16) : 0.f;
    }
  }
  if constexpr (C::NH >= 1) {
    const int c1 = na.ch[1];
    // entry (q, m, lane): row co = 16m + lane%16, lane group g = lane/16
    for (int e = threadIdx.x; e < C::KS1 * C::MB * 64; e += C::NT) {
      const int lane = e % 64, m = (e / 64) % C::MB, q = e / (64 * C::MB);
      const int co = 16 * m + (lane & 15), g = lane >> 4;
      if constexpr (!C::BF16) {
        const int K = 4 * q + g;
        reinterpret_cast<float*>(lds + Lo::FR1)[e] =
            (K < C::K1 && co < c1) ? wget(na, 0, co, K % C::CIN, K / C::CIN, false) : 0.f;
      } else {
        unsigned wd[4];
        for (int e2 = 0; e2 < 4; ++e2) {
          float ww[2];
          for (int h = 0; h < 2; ++h) {
            const int K = 32 * q + 8 * g + 2 * e2 + h;
            ww[h] = (K < C::K1 && co < c1) ? wget(na, 0, co, K % C::CIN, K / C::CIN, true) : 0.f;
          }
          wd[e2] = pack_bf16x2(ww[0], ww[1]);
        }
        reinterpret_cast<u4*>(lds + Lo::FR1)[e] = u4{wd[0], wd[1], wd[2], wd[3]};
      }
    }
  }
  if constexpr (C::NH >= 2) {
    const int c1 = na.ch[1], c2 = na.ch[2];
    if constexpr (!C::BF16) {
      // entry ((tau, hh, m, lane), q4): k-step (tau, 4hh+q4), input channel 4g + q4 + 16hh
      for (int e = threadIdx.x; e < 9 * (C::CH / 16) * C::MB * 64 * 4; e += C::NT) {
        const int q4 = e % 4, lane = (e / 4) % 64, m = (e / 256) % C::MB;
        const int hh = (e / (256 * C::MB)) % (C::CH / 16), tau = e / (256 * C::MB * (C::CH / 16));
        const int co = 16 * m + (lane & 15), g = lane >> 4;
        const int ci = 4 * g + q4 + 16 * hh;
        reinterpret_cast<float*>(lds + Lo::FR2)[e] = (co < c2 && ci < c1) ? wget(na, 1, co, ci, tau, false) : 0.f;
      }
    } else {
      for (int e = threadIdx.x; e < C::KS2 * C::MB * 64; e += C::NT) {
        const int lane = e % 64, m = (e / 64) % C::MB, q = e / (64 * C::MB);
        const int co = 16 * m + (lane & 15), g = lane >> 4;
        int tau, cib;
        if constexpr (C::CH == 32) { tau = q; cib = 8 * g; }
        else { tau = 2 * q + (g >> 1); cib = 8 * (g & 1); }
        unsigned wd[4];
        for (int e2 = 0; e2 < 4; ++e2) {
          float ww[2];
          for (int h = 0; h < 2; ++h) {
            const int ci = cib + 2 * e2 + h;
            ww[h] = (tau < 9 && co < c2 && ci < c1) ? wget(na, 1, co, ci, tau, true) : 0.f;
          }
          wd[e2] = pack_bf16x2(ww[0], ww[1]);
        }
        reinterpret_cast<u4*>(lds + Lo::FR2)[e] = u4{wd[0], wd[1], wd[2], wd[3]};
      }
    }
  }
}

// A fragments of the output layer in its MFMA form (BF16 nets): rows are the
// output channels (16 rows, Cout used), K = (tap, ci) laid out like the
// hidden->hidden layer.
template <class C>
__device__ __forceinline__ void load_out_frags(const FwdNetArgs& na, char* lds) {
  if constexpr (C::OMF) {
    const int L = na.n_layers - 1;
    const int cin = na.ch[L], cout = na.ch[L + 1];
    for (int e = threadIdx.x; e < C::KSO * 64; e += C::NT) {
      const int lane = e % 64, q = e / 64;
      const int co = lane & 15, g = lane >> 4;
      int tau, cib;
      if constexpr (C::CH == 32) { tau = q; cib = 8 * g; }
      else { tau = 2 * q + (g >> 1); cib = 8 * (g & 1); }
      unsigned wd[4];
      for (int e2 = 0; e2 < 4; ++e2) {
        float ww[2];
        for (int h = 0; h < 2; ++h) {
          const int ci = cib + 2 * e2 + h;
          ww[h] = (tau < 9 && co < cout && ci < cin) ? wget(na, L, co, ci, tau, true) : 0.f;
        }
        wd[e2] = pack_bf16x2(ww[0], ww[1]);
      }
      reinterpret_cast<u4*>(lds + Layout<C>::FR3)[e] = u4{wd[0], wd[1], wd[2], wd[3]};
    }
  }
}

// ------------------------------------------------------------------ tile
struct Tile {
  int n, ty0, tx0;
};

__device__ __forceinline__ int tap_off(int tau, int cwt) {
  const int ty = tau / 3;
  return (ty - 1) * cwt + (tau - 3 * ty - 1);
}

// Hidden-layer epilogue for one 16-pixel block: st holds the charged
// potentials h of MB x 4 (channel, pixel) pairs of this lane; fire, reset,
// write spikes to LDS and, optionally, h to the trace.
// Window of the image whose potentials go to the trace.
struct TraceBox {
  int y0, x0, h, w;
  __device__ bool has(int gy, int gx) const { return gy >= y0 && gy < y0 + h && gx >= x0 && gx < x0 + w; }
  __device__ size_t idx(int gy, int gx) const { return (size_t)(gy - y0) * w + (gx - x0); }
  __device__ size_t plane() const { return (size_t)h * w; }
};

template <class C, bool B16 = C::SPB16>
__device__ __forceinline__ void hidden_epilogue(f4 (&st)[C::MB], char* lds, int sp_off, int pr, bool valid, int g,
                                                float theta, float alpha, bool relaxed, float* trace_t,
                                                int cl, int choff, int gy0, int gx0, const TraceBox& tb) {
  if (C::FULL && trace_t && valid) {
    const int row = pr / C::CWT, col = pr % C::CWT;
    const int gy = gy0 + row, gx = gx0 + col;
    if (row >= C::NL && row < C::NL + C::TH && col >= C::NL && col < C::NL + C::TW && tb.has(gy, gx)) {
      const size_t pix = tb.idx(gy, gx);
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int co = 16 * m + 4 * g + r;
          if (co < cl) trace_t[(size_t)(choff + co) * tb.plane() + pix] = st[m][r];
        }
    }
  }
  const int p = C::PADF + pr;
#pragma unroll
  for (int m = 0; m < C::MB; ++m) {
    f4 s;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v = st[m][r];
      s[r] = bilif(v, theta, alpha, C::FULL && relaxed);
      st[m][r] = v;
    }
    if (!valid) s = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (B16) {
      uint2 w2 = {pack_bf16x2(s[0], s[1]), pack_bf16x2(s[2], s[3])};
      *reinterpret_cast<uint2*>(lds + Layout<C>::SP + sp_off + ((size_t)p * C::CH + 16 * m + 4 * g) * 2) = w2;
    } else {
      *reinterpret_cast<f4*>(lds + Layout<C>::SP + sp_off + ((size_t)p * C::CH + 16 * m + 4 * g) * 4) = s;
    }
  }
}

// Write the membrane state of the interior pixels of a hidden layer.
template <class C, int NB>
__device__ __forceinline__ void write_hidden_state(const f4 (&st)[NB][C::MB], unsigned vm, int layer, int wave,
                                                   int j, int g, float* dst, int cl, int choff, int gy0,
                                                   int gx0, int W, size_t HW, int nw = C::NW) {
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int pr = layer * C::CWT + 16 * (wave + nw * i) + j;
    const int row = pr / C::CWT, col = pr % C::CWT;
    if (((vm >> i) & 1u) && row >= C::NL && row < C::NL + C::TH && col >= C::NL && col < C::NL + C::TW) {
      const size_t pix = (size_t)(gy0 + row) * W + (gx0 + col);
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int co = 16 * m + 4 * g + r;
          if (co < cl) dst[(size_t)(choff + co) * HW + pix] = st[i][m][r];
        }
    }
  }
}

template <class C, int NB>
__device__ __forceinline__ void read_hidden_state(f4 (&st)[NB][C::MB], unsigned vm, int layer, int wave, int j,
                                                  int g, const float* src, int cl, int choff, int gy0, int gx0,
                                                  int W, size_t HW, int nw = C::NW) {
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int m = 0; m < C::MB; ++m) {
      f4 v = {0.f, 0.f, 0.f, 0.f};
      if (src && ((vm >> i) & 1u)) {
        const int pr = layer * C::CWT + 16 * (wave + nw * i) + j;
        const size_t pix = (size_t)(gy0 + pr / C::CWT) * W + (gx0 + pr % C::CWT);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int co = 16 * m + 4 * g + r;
          if (co < cl) v[r] = src[(size_t)(choff + co) * HW + pix];
        }
      }
      st[i][m] = v;
    }
}

// ---------------------------------------------------------------------------
// Wave-specialised schedule of the FP32 three-layer inference kernel.
//
// Waves 0-3 (one per SIMD) own layer 2: its membrane state and all of its
// MFMAs.  Waves 4-7 own layer 1 and the output layer.  Per frame t:
//   phase A   waves 0-3: fire/reset of layer 2 for frame t-1 (-> S2, bf16)
//             waves 4-7: layer-1 MFMA + fire/reset for frame t (-> S1, f32)
//   barrier;  all: stage x(t+1), prefetch x(t+2)
//   phase B   waves 0-3: layer-2 MFMA of frame t (reads S1)
//             waves 4-7: output layer of frame t-1 on the VALU (reads S2)
//   barrier
// In phase B every SIMD holds one MFMA-issuing wave and one VALU-issuing
// wave, so the output layer runs under the MFMA work.  Each neuron sees the
// same arithmetic in the same order as in the plain schedule: the results
// are bit-identical.
// ---------------------------------------------------------------------------
template <class C>
__device__ __forceinline__ void run_tile_pipe(const FwdNetArgs& na, const FwdClipArgs& ca, const Tile tl,
                                              char* lds) {
  static_assert(C::NW == 8 && C::NH == 2 && !C::BF16 && !C::FULL, "specialised schedule: FP32, 3 layers, 8 waves");
  using Lo = Layout<C>;
  constexpr int NB1V = C::NB1V, NB2M = C::NB2M;
  constexpr int NOV = cdiv(C::TH * C::TW, 256);
  float* const xsf = reinterpret_cast<float*>(lds + Lo::XS);
  const float* const s1f = reinterpret_cast<const float*>(lds + Lo::SP);
  const uint16_t* const s2b = reinterpret_cast<const uint16_t*>(lds + Lo::SP + C::SP2_OFF);
  const float* const wl = reinterpret_cast<const float*>(lds + Lo::WL);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool mrole = wave < 4;                       // layer-2 (MFMA) waves
  const int rw = wave & 3;                           // index inside the role
  const int j = lane & 15, g = lane >> 4;
  const int H = ca.H, W = ca.W, T = ca.T;
  const size_t HW = (size_t)H * W;
  const int sumc = na.sum_c;
  const float theta = na.theta, leak = na.leak, alpha = na.alpha;
  const int c1 = na.ch[1], c2 = na.ch[2];
  const int cout = na.ch[3];
  const int choff2 = c1, choffo = c1 + c2;
  const int gy0 = tl.ty0 - C::NL, gx0 = tl.tx0 - C::NL;
  const TraceBox tb{0, 0, 0, 0};

  // ---- block masks (layer 1: VALU waves, layer 2: MFMA waves)
  unsigned vm1 = 0, vm2 = 0, ovm = 0;
#pragma unroll
  for (int i = 0; i < NB1V; ++i) {
    const int b = rw + 4 * i;
    const int pr = C::CWT + 16 * b + j;
    const int row = pr / C::CWT, col = pr % C::CWT;
    const int gy = gy0 + row, gx = gx0 + col;
    vm1 |= ((b < C::NPB1 && row < C::CHT - 1 && gy >= 0 && gy < H && gx >= 0 && gx < W) ? 1u : 0u) << i;
  }
#pragma unroll
  for (int i = 0; i < NB2M; ++i) {
    const int b = rw + 4 * i;
    const int pr = 2 * C::CWT + 16 * b + j;
    const int row = pr / C::CWT, col = pr % C::CWT;
    const int gy = gy0 + row, gx = gx0 + col;
    vm2 |= ((b < C::NPB2 && row < C::CHT - 2 && gy >= 0 && gy < H && gx >= 0 && gx < W) ? 1u : 0u) << i;
  }
  const int vt = tid & 255;                          // lane index inside the VALU group
  int op[NOV];
#pragma unroll
  for (int k = 0; k < NOV; ++k) {
    const int q = vt + 256 * k;
    const int ty = q / C::TW, tx = q % C::TW;
    const bool inq = q < C::TH * C::TW;
    op[k] = C::PADF + (inq ? (C::NL + ty) * C::CWT + (C::NL + tx) : C::NL * C::CWT + C::NL);
    ovm |= ((inq && tl.ty0 + ty < H && tl.tx0 + tx < W) ? 1u : 0u) << k;
  }

  // ---- state: one register array, layer 1 in the VALU waves and layer 2
  // in the MFMA waves (the roles never meet in one wave)
  constexpr int NBS = NB1V > NB2M ? NB1V : NB2M;
  f4 st[NBS][C::MB];
  float so[NOV][2];
  const float* vin = ca.v_in ? ca.v_in + (size_t)tl.n * ca.vin_nstride : nullptr;
  if (!mrole) read_hidden_state<C, NBS>(st, vm1, 1, rw, j, g, vin, c1, 0, gy0, gx0, W, HW, 4);
  else read_hidden_state<C, NBS>(st, vm2, 2, rw, j, g, vin, c2, choff2, gy0, gx0, W, HW, 4);
#pragma unroll
  for (int k = 0; k < NOV; ++k) {
    so[k][0] = so[k][1] = 0.f;
    if (!mrole && vin && ((ovm >> k) & 1u)) {
      const int q = vt + 256 * k;
      const size_t pix = (size_t)(tl.ty0 + q / C::TW) * W + (tl.tx0 + q % C::TW);
#pragma unroll
      for (int co = 0; co < 2; ++co)
        if (co < cout) so[k][co] = vin[(size_t)(choffo + co) * HW + pix];
    }
  }

  // ---- x staging over all 512 threads
  const float* xclip = ca.x + (size_t)tl.n * ca.x_nstride;
  float xpf[C::XPF];
  auto load_x = [&](int tt) __attribute__((always_inline)) {
    const float* xf = xclip + (size_t)tt * C::CIN * HW;
#pragma unroll
    for (int k = 0; k < C::XPF; ++k) {
      const int e = tid + C::NT * k;
      const int c = e / C::NPIX, rem = e % C::NPIX;
      const int gy = gy0 + rem / C::CWT, gx = gx0 + rem % C::CWT;
      float v = 0.f;
      if (e < C::XN && gy >= 0 && gy < H && gx >= 0 && gx < W) v = xf[(size_t)c * HW + (size_t)gy * W + gx];
      xpf[k] = v;
    }
  };
  auto store_x = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < C::XPF; ++k) {
      const int e = tid + C::NT * k;
      if (e < C::XN) xsf[(e / C::NPIX) * C::NPIXL + C::PADF + e % C::NPIX] = xpf[k];
    }
  };

  const int p1base = C::PADF + C::CWT + 16 * rw + j;
  const int p2base = C::PADF + 2 * C::CWT + 16 * rw + j;

  // layer 1 on the VALU waves: MFMA + fire/reset -> S1 (f32)
  auto layer1 = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NB1V; ++i)
#pragma unroll
      for (int m = 0; m < C::MB; ++m) st[i][m] *= leak;
#pragma unroll 1
    for (int q = 0; q < C::KS1; ++q) {
      const float* fr = reinterpret_cast<const float*>(lds + Lo::FR1) + q * C::MB * 64 + lane;
      float a[C::MB];
#pragma unroll
      for (int m = 0; m < C::MB; ++m) a[m] = fr[m * 64];
      const int K = 4 * q + g;
      const int tap = K / C::CIN, c = K - tap * C::CIN;
      const int o = K < C::K1 ? c * C::NPIXL + tap_off(tap, C::CWT) : C::CIN * C::NPIXL;
      float bv[NB1V];
#pragma unroll
      for (int i = 0; i < NB1V; ++i) bv[i] = xsf[p1base + 64 * i + o];
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
#pragma unroll
        for (int i = 0; i < NB1V; ++i) st[i][m] = mfma_f32(a[m], bv[i], st[i][m]);
    }
#pragma unroll
    for (int i = 0; i < NB1V; ++i)
      hidden_epilogue<C, false>(st[i], lds, 0, C::CWT + 16 * (rw + 4 * i) + j, (vm1 >> i) & 1u, g, theta, alpha,
                                false, nullptr, c1, 0, gy0, gx0, tb);
  };
  // layer-2 fire/reset on the MFMA waves -> S2 (bf16)
  auto fire2 = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NB2M; ++i)
      hidden_epilogue<C, true>(st[i], lds, C::SP2_OFF, 2 * C::CWT + 16 * (rw + 4 * i) + j, (vm2 >> i) & 1u, g,
                               theta, alpha, false, nullptr, c2, choff2, gy0, gx0, tb);
  };
  // layer-2 MFMA on the MFMA waves: per tap, the operand loads of the two
  // halves of the blocks are issued before their MFMAs
  auto layer2 = [&]() __attribute__((always_inline)) {
    static_assert(C::CH == 16, "specialised schedule assumes 16 hidden channels");
#pragma unroll
    for (int i = 0; i < NB2M; ++i) st[i][0] *= leak;
    const f4* fr = reinterpret_cast<const f4*>(lds + Lo::FR2) + lane;
#pragma unroll 1
    for (int tau = 0; tau < 9; ++tau) {
      const int to = tap_off(tau, C::CWT);
      const f4 a = fr[tau * 64];
      f4 bv[NB2M];
#pragma unroll
      for (int i = 0; i < NB2M; ++i)
        bv[i] = *reinterpret_cast<const f4*>(s1f + (size_t)(p2base + 64 * i + to) * C::CH + 4 * g);
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
        for (int i = 0; i < NB2M; ++i) st[i][0] = mfma_f32(a[q4], bv[i][q4], st[i][0]);
    }
  };
  // output layer on the VALU waves (frame tt), spikes of layer 2 from S2
  auto output = [&](int tt) __attribute__((always_inline)) {
    float u[NOV][2];
#pragma unroll
    for (int k = 0; k < NOV; ++k) { u[k][0] = leak * so[k][0]; u[k][1] = leak * so[k][1]; }
#pragma unroll 1
    for (int tau = 0; tau < 9; ++tau) {
      const int to = tap_off(tau, C::CWT);
#pragma unroll
      for (int c8 = 0; c8 < C::CH / 8; ++c8) {
        f4 wv[4];
#pragma unroll
        for (int z = 0; z < 4; ++z) wv[z] = *reinterpret_cast<const f4*>(wl + (tau * C::CH + 8 * c8) * 2 + 4 * z);
#pragma unroll
        for (int k = 0; k < NOV; ++k) {
          const u4 rw4 = *reinterpret_cast<const u4*>(s2b + (size_t)(op[k] + to) * C::CH + 8 * c8);
#pragma unroll
          for (int z = 0; z < 4; ++z) {
            const float s0 = __builtin_bit_cast(float, rw4[z] << 16);
            const float sh = __builtin_bit_cast(float, rw4[z] & 0xffff0000u);
            u[k][0] = fmaf(wv[z][0], s0, u[k][0]); u[k][1] = fmaf(wv[z][1], s0, u[k][1]);
            u[k][0] = fmaf(wv[z][2], sh, u[k][0]); u[k][1] = fmaf(wv[z][3], sh, u[k][1]);
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NOV; ++k) {
      const bool ok = (ovm >> k) & 1u;
      const int q = vt + 256 * k;
      const size_t pix = (size_t)(tl.ty0 + q / C::TW) * W + (tl.tx0 + q % C::TW);
#pragma unroll
      for (int co = 0; co < 2; ++co) {
        float v = u[k][co];
        const float sp = bilif(v, theta, alpha, false);
        so[k][co] = v;
        if (ok && co < cout && ca.s_out)
          reinterpret_cast<int8_t*>(ca.s_out)[(((size_t)tl.n * T + tt) * cout + co) * HW + pix] = (int8_t)sp;
      }
    }
  };

  load_x(0);
  store_x();
  if (T > 1) load_x(1);
  __syncthreads();
  for (int t = 0; t < T; ++t) {
    // phase A
    if (mrole) {
      if (t > 0) fire2();
    } else {
      layer1();
    }
    __syncthreads();
    if (t + 1 < T) store_x();
    if (t + 2 < T) load_x(t + 2);
    // phase B
    if (mrole) {
      layer2();
    } else {
      if (t > 0) output(t - 1);
    }
    __syncthreads();
  }
  if (mrole) fire2();
  __syncthreads();
  if (!mrole) output(T - 1);
  if (ca.v_out) {
    float* dst = ca.v_out + (size_t)tl.n * sumc * HW;
    if (!mrole) {
      write_hidden_state<C, NBS>(st, vm1, 1, rw, j, g, dst, c1, 0, gy0, gx0, W, HW, 4);
#pragma unroll
      for (int k = 0; k < NOV; ++k) {
        if ((ovm >> k) & 1u) {
          const int q = vt + 256 * k;
          const size_t pix = (size_t)(tl.ty0 + q / C::TW) * W + (tl.tx0 + q % C::TW);
#pragma unroll
          for (int co = 0; co < 2; ++co)
            if (co < cout) dst[(size_t)(choffo + co) * HW + pix] = so[k][co];
        }
      }
    } else {
      write_hidden_state<C, NBS>(st, vm2, 2, rw, j, g, dst, c2, choff2, gy0, gx0, W, HW, 4);
    }
  }
}

// Process one tile over frames [0, T) of one clip.
template <class C>
__device__ __forceinline__ void run_tile(const FwdNetArgs& na, const FwdClipArgs& ca, const Tile tl, char* lds) {
  if constexpr (C::PIPE) {
    run_tile_pipe<C>(na, ca, tl, lds);
    return;
  }
  using Lo = Layout<C>;
  float* const xsf = reinterpret_cast<float*>(lds + Lo::XS);
  uint16_t* const xsb = reinterpret_cast<uint16_t*>(lds + Lo::XS);
  const float* const spf = reinterpret_cast<const float*>(lds + Lo::SP);
  const uint16_t* const spb = reinterpret_cast<const uint16_t*>(lds + Lo::SP);
  const float* const wl = reinterpret_cast<const float*>(lds + Lo::WL);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int j = lane & 15, g = lane >> 4;
  const int H = ca.H, W = ca.W, T = ca.T;
  const size_t HW = (size_t)H * W;
  const int sumc = na.sum_c;
  const float theta = na.theta, leak = na.leak, alpha = na.alpha;
  const bool relaxed = na.relaxed != 0;
  const int c1 = na.ch[1], c2 = na.ch[2];
  const int cout = na.ch[na.n_layers];
  const int choff2 = c1, choffo = (C::NH == 0) ? 0 : (C::NH == 1 ? c1 : c1 + c2);
  const int gy0 = tl.ty0 - C::NL, gx0 = tl.tx0 - C::NL;   // image coords of canvas (0,0)

  // ---- validity masks of this lane's hidden-layer block pixels
  unsigned vm1 = 0, vm2 = 0;
  if constexpr (C::NH >= 1) {
#pragma unroll
    for (int i = 0; i < C::NB1; ++i) {
      const int b = wave + C::NW * i;
      const int pr = C::CWT * 1 + 16 * b + j;
      const int row = pr / C::CWT, col = pr % C::CWT;
      const int gy = gy0 + row, gx = gx0 + col;
      const bool ok = b < C::NPB1 && row < C::CHT - 1 && gy >= 0 && gy < H && gx >= 0 && gx < W;
      vm1 |= (ok ? 1u : 0u) << i;
    }
  }
  if constexpr (C::NH >= 2) {
#pragma unroll
    for (int i = 0; i < C::NB2; ++i) {
      const int b = wave + C::NW * i;
      const int pr = C::CWT * 2 + 16 * b + j;
      const int row = pr / C::CWT, col = pr % C::CWT;
      const int gy = gy0 + row, gx = gx0 + col;
      const bool ok = b < C::NPB2 && row < C::CHT - 2 && gy >= 0 && gy < H && gx >= 0 && gx < W;
      vm2 |= (ok ? 1u : 0u) << i;
    }
  }
  // ---- output pixels of this lane
  int op[C::NOUT];
  unsigned ovm = 0;
#pragma unroll
  for (int k = 0; k < C::NOUT; ++k) {
    const int q = tid + C::NT * k;
    const int ty = q / C::TW, tx = q % C::TW;
    const bool inq = q < C::TH * C::TW;
    op[k] = C::PADF + (inq ? (C::NL + ty) * C::CWT + (C::NL + tx) : C::NL * C::CWT + C::NL);
    const int gy = tl.ty0 + ty, gx = tl.tx0 + tx;
    ovm |= ((inq && gy < H && gx < W) ? 1u : 0u) << k;
  }

  // output blocks of the MFMA form: canvas rows NL..NL+TH-1, interior columns
  unsigned vmo = 0;
  if constexpr (C::OMF) {
#pragma unroll
    for (int i = 0; i < C::NBO; ++i) {
      const int b = wave + C::NW * i;
      const int pr = C::NL * C::CWT + 16 * b + j;
      const int row = pr / C::CWT, col = pr % C::CWT;
      const int gy = gy0 + row, gx = gx0 + col;
      const bool ok = b < C::NPBO && row < C::NL + C::TH && col >= C::NL && col < C::NL + C::TW && gy < H && gx < W;
      vmo |= (ok ? 1u : 0u) << i;
    }
  }

  // ---- state registers
  f4 st1[C::NB1][C::MB];
  f4 st2[C::NB2][C::MB];
  float so[C::NOUT][2];
  f4 sob[C::NBO];           // output state, MFMA form: rows = channels (lanes g == 0)
  const float* vin = ca.v_in ? ca.v_in + (size_t)tl.n * ca.vin_nstride : nullptr;
  if constexpr (C::NH >= 1) read_hidden_state<C, C::NB1>(st1, vm1, 1, wave, j, g, vin, c1, 0, gy0, gx0, W, HW);
  if constexpr (C::NH >= 2) read_hidden_state<C, C::NB2>(st2, vm2, 2, wave, j, g, vin, c2, choff2, gy0, gx0, W, HW);
#pragma unroll
  for (int i = 0; i < C::NBO; ++i) {
    sob[i] = f4{0.f, 0.f, 0.f, 0.f};
    if (C::OMF && vin && g == 0 && ((vmo >> i) & 1u)) {
      const int pr = C::NL * C::CWT + 16 * (wave + C::NW * i) + j;
      const size_t pix = (size_t)(gy0 + pr / C::CWT) * W + (gx0 + pr % C::CWT);
#pragma unroll
      for (int co = 0; co < 2; ++co)
        if (co < cout) sob[i][co] = vin[(size_t)(choffo + co) * HW + pix];
    }
  }
#pragma unroll
  for (int k = 0; k < C::NOUT; ++k) {
    so[k][0] = so[k][1] = 0.f;
    if (!C::OMF && vin && ((ovm >> k) & 1u)) {
      const int q = tid + C::NT * k;
      const size_t pix = (size_t)(tl.ty0 + q / C::TW) * W + (tl.tx0 + q % C::TW);
#pragma unroll
      for (int co = 0; co < 2; ++co)
        if (co < cout) so[k][co] = vin[(size_t)(choffo + co) * HW + pix];
    }
  }

  // ---- x staging (register prefetch of the next frame)
  const float* xclip = ca.x + (size_t)tl.n * ca.x_nstride;
  float xpf[C::XPF];
#define EVS_LOAD_X(tt)                                                                          \
  do {                                                                                          \
    const float* xf = xclip + (size_t)(tt) * C::CIN * HW;                                       \
    _Pragma("unroll") for (int k = 0; k < C::XPF; ++k) {                                        \
      const int e = tid + C::NT * k;                                                            \
      const int c = e / C::NPIX, rem = e % C::NPIX;                                             \
      const int gy = gy0 + rem / C::CWT, gx = gx0 + rem % C::CWT;                               \
      float v = 0.f;                                                                            \
      if (e < C::XN && gy >= 0 && gy < H && gx >= 0 && gx < W) v = xf[(size_t)c * HW + (size_t)gy * W + gx]; \
      xpf[k] = v;                                                                               \
    }                                                                                           \
  } while (0)
#define EVS_STORE_X()                                                                           \
  do {                                                                                          \
    _Pragma("unroll") for (int k = 0; k < C::XPF; ++k) {                                        \
      const int e = tid + C::NT * k;                                                            \
      if (e < C::XN) {                                                                          \
        const int c = e / C::NPIX, rem = e % C::NPIX;                                           \
        if constexpr (C::BF16) xsb[c * C::NPIXL + C::PADF + rem] = f32_to_bf16_rne(xpf[k]);    \
        else xsf[c * C::NPIXL + C::PADF + rem] = xpf[k];                                        \
      }                                                                                         \
    }                                                                                           \
  } while (0)

  const int nseg = ca.ckpt_every > 0 ? cdiv(T, ca.ckpt_every) : 0;
  const TraceBox tb{ca.tb_y0, ca.tb_x0, ca.tb_h, ca.tb_w};
  auto write_state = [&](float* dst) __attribute__((always_inline)) {
    if constexpr (C::NH >= 1) write_hidden_state<C, C::NB1>(st1, vm1, 1, wave, j, g, dst, c1, 0, gy0, gx0, W, HW);
    if constexpr (C::NH >= 2) write_hidden_state<C, C::NB2>(st2, vm2, 2, wave, j, g, dst, c2, choff2, gy0, gx0, W, HW);
#pragma unroll
    for (int k = 0; k < C::NOUT; ++k) {
      if (!C::OMF && ((ovm >> k) & 1u)) {
        const int q = tid + C::NT * k;
        const size_t pix = (size_t)(tl.ty0 + q / C::TW) * W + (tl.tx0 + q % C::TW);
#pragma unroll
        for (int co = 0; co < 2; ++co)
          if (co < cout) dst[(size_t)(choffo + co) * HW + pix] = so[k][co];
      }
    }
#pragma unroll
    for (int i = 0; i < C::NBO; ++i) {
      if (C::OMF && g == 0 && ((vmo >> i) & 1u)) {
        const int pr = C::NL * C::CWT + 16 * (wave + C::NW * i) + j;
        const size_t pix = (size_t)(gy0 + pr / C::CWT) * W + (gx0 + pr % C::CWT);
#pragma unroll
        for (int co = 0; co < 2; ++co)
          if (co < cout) dst[(size_t)(choffo + co) * HW + pix] = sob[i][co];
      }
    }
  };

  // block pixel bases (canvas index incl. front pad) of block i: pbase + 16*NW*i
  const int p1base = C::PADF + C::CWT + 16 * wave + j;
  const int p2base = C::PADF + 2 * C::CWT + 16 * wave + j;

  // ---- prologue: frame 0 into LDS, frame 1 into registers
  EVS_LOAD_X(0);
  EVS_STORE_X();
  if (T > 1) EVS_LOAD_X(1);
  __syncthreads();

  for (int t = 0; t < T; ++t) {
    float* trace_t = nullptr;
    if constexpr (C::FULL) {
      if (ca.ckpt && (t % ca.ckpt_every) == 0)
        write_state(ca.ckpt + ((size_t)tl.n * nseg + t / ca.ckpt_every) * sumc * HW);
      trace_t = ca.h_trace ? ca.h_trace + (size_t)tl.n * ca.trace_nstride + (size_t)t * sumc * tb.plane()
                           : nullptr;
    }

    if constexpr (C::NH >= 1) {
      // ================= layer 1: x -> hidden (MFMA), K = tap * CIN + c
#pragma unroll
      for (int i = 0; i < C::NB1; ++i)
#pragma unroll
        for (int m = 0; m < C::MB; ++m) st1[i][m] *= leak;
#pragma unroll 1
      for (int q = 0; q < C::KS1; ++q) {
        if constexpr (!C::BF16) {
          const float* fr = reinterpret_cast<const float*>(lds + Lo::FR1) + q * C::MB * 64 + lane;
          float a[C::MB];
#pragma unroll
          for (int m = 0; m < C::MB; ++m) a[m] = fr[m * 64];
          const int K = 4 * q + g;
          const bool kv = K < C::K1;
          const int tap = K / C::CIN, c = K - tap * C::CIN;
          const int o = kv ? c * C::NPIXL + tap_off(tap, C::CWT) : C::CIN * C::NPIXL;
          float bv[C::NB1];
#pragma unroll
          for (int i = 0; i < C::NB1; ++i) bv[i] = xsf[p1base + 16 * C::NW * i + o];
#pragma unroll
          for (int m = 0; m < C::MB; ++m)
#pragma unroll
            for (int i = 0; i < C::NB1; ++i) st1[i][m] = mfma_f32(a[m], bv[i], st1[i][m]);
        } else {
          const u4* fr = reinterpret_cast<const u4*>(lds + Lo::FR1) + q * C::MB * 64 + lane;
          u4 a[C::MB];
#pragma unroll
          for (int m = 0; m < C::MB; ++m) a[m] = fr[m * 64];
          int o[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int K = 32 * q + 8 * g + e;
            const int tap = K / C::CIN, c = K - tap * C::CIN;
            o[e] = K < C::K1 ? c * C::NPIXL + tap_off(tap, C::CWT) : C::CIN * C::NPIXL;
          }
          u4 bv[C::NB1];
#pragma unroll
          for (int i = 0; i < C::NB1; ++i) {
            const int p = p1base + 16 * C::NW * i;
            unsigned wd[4];
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) {
              const unsigned r0 = xsb[p + o[2 * e2]], r1 = xsb[p + o[2 * e2 + 1]];
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
#pragma unroll
      for (int i = 0; i < C::NB1; ++i) {
        const int b = wave + C::NW * i;
        hidden_epilogue<C>(st1[i], lds, 0, C::CWT + 16 * b + j, (vm1 >> i) & 1u, g, theta, alpha, relaxed,
                           trace_t, c1, 0, gy0, gx0, tb);
      }
      __syncthreads();                                   // B1: s1 visible, xs free
      if (t + 1 < T) EVS_STORE_X();
      if (t + 2 < T) EVS_LOAD_X(t + 2);
    }

    if constexpr (C::NH >= 2) {
      // ================= layer 2: hidden -> hidden (MFMA), K = tap * CH + ci
#pragma unroll
      for (int i = 0; i < C::NB2; ++i)
#pragma unroll
        for (int m = 0; m < C::MB; ++m) st2[i][m] *= leak;
      if constexpr (!C::BF16) {
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
              bv[i] = *reinterpret_cast<const f4*>(spf + (size_t)(p2base + 16 * C::NW * i + to) * C::CH + 16 * hh +
                                                   4 * g);
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
              for (int m = 0; m < C::MB; ++m)
#pragma unroll
                for (int i = 0; i < C::NB2; ++i) st2[i][m] = mfma_f32(a[m][q4], bv[i][q4], st2[i][m]);
          }
        }
      } else {
#pragma unroll 1
        for (int q = 0; q < C::KS2; ++q) {
          const u4* fr = reinterpret_cast<const u4*>(lds + Lo::FR2) + q * C::MB * 64 + lane;
          u4 a[C::MB];
#pragma unroll
          for (int m = 0; m < C::MB; ++m) a[m] = fr[m * 64];
          int o;
          if constexpr (C::CH == 32) {
            o = tap_off(q, C::CWT) * C::CH + 8 * g;
          } else {
            int tau = 2 * q + (g >> 1);
            tau = tau > 8 ? 8 : tau;                     // zero weights in that slot
            o = tap_off(tau, C::CWT) * C::CH + 8 * (g & 1);
          }
          u4 bv[C::NB2];
#pragma unroll
          for (int i = 0; i < C::NB2; ++i)
            bv[i] = *reinterpret_cast<const u4*>(spb + (size_t)(p2base + 16 * C::NW * i) * C::CH + o);
#pragma unroll
          for (int m = 0; m < C::MB; ++m)
#pragma unroll
            for (int i = 0; i < C::NB2; ++i) st2[i][m] = mfma_bf16(a[m], bv[i], st2[i][m]);
        }
      }
      __syncthreads();                                   // B2: all reads of s1 done
#pragma unroll
      for (int i = 0; i < C::NB2; ++i) {
        const int b = wave + C::NW * i;
        hidden_epilogue<C>(st2[i], lds, 0, 2 * C::CWT + 16 * b + j, (vm2 >> i) & 1u, g, theta, alpha, relaxed,
                           trace_t, c2, choff2, gy0, gx0, tb);
      }
      __syncthreads();                                   // B3: s2 visible
    }

    if constexpr (C::OMF) {
      // ================= output layer on MFMA (BF16), K = tap * CH + ci
      const int pobase = C::PADF + C::NL * C::CWT + 16 * wave + j;
#pragma unroll
      for (int i = 0; i < C::NBO; ++i) sob[i] *= leak;
#pragma unroll 1
      for (int q = 0; q < C::KSO; ++q) {
        const u4 a = reinterpret_cast<const u4*>(lds + Lo::FR3)[q * 64 + lane];
        int o;
        if constexpr (C::CH == 32) {
          o = tap_off(q, C::CWT) * C::CH + 8 * g;
        } else {
          int tau = 2 * q + (g >> 1);
          tau = tau > 8 ? 8 : tau;
          o = tap_off(tau, C::CWT) * C::CH + 8 * (g & 1);
        }
        u4 bv[C::NBO];
#pragma unroll
        for (int i = 0; i < C::NBO; ++i)
          bv[i] = *reinterpret_cast<const u4*>(spb + (size_t)(pobase + 16 * C::NW * i) * C::CH + o);
#pragma unroll
        for (int i = 0; i < C::NBO; ++i) sob[i] = mfma_bf16(a, bv[i], sob[i]);
      }
      if (g == 0) {
#pragma unroll
        for (int i = 0; i < C::NBO; ++i) {
          const bool ok = (vmo >> i) & 1u;
          const int pr = C::NL * C::CWT + 16 * (wave + C::NW * i) + j;
          const int gy = gy0 + pr / C::CWT, gx = gx0 + pr % C::CWT;
          const size_t pix = (size_t)gy * W + gx;
#pragma unroll
          for (int co = 0; co < 2; ++co) {
            if (C::FULL && ok && co < cout && trace_t && tb.has(gy, gx))
              trace_t[(size_t)(choffo + co) * tb.plane() + tb.idx(gy, gx)] = sob[i][co];
            float v = sob[i][co];
            const float sp = bilif(v, theta, alpha, false);
            sob[i][co] = v;
            if (ok && co < cout && ca.s_out) {
              const size_t o = (((size_t)tl.n * T + t) * cout + co) * HW + pix;
              if (C::FULL && ca.s_fp32) reinterpret_cast<float*>(ca.s_out)[o] = sp;
              else reinterpret_cast<int8_t*>(ca.s_out)[o] = (int8_t)sp;
            }
          }
        }
      }
    } else
    {
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
              const float xv = xsf[c * C::NPIXL + op[k] + to];
              u[k][0] = fmaf(w0, xv, u[k][0]);
              u[k][1] = fmaf(w1, xv, u[k][1]);
            }
          }
        } else if constexpr (!C::BF16) {
#pragma unroll
          for (int c4 = 0; c4 < C::CH / 4; ++c4) {
            const f4 wa = *reinterpret_cast<const f4*>(wl + (tau * C::CH + 4 * c4) * 2);
            const f4 wb = *reinterpret_cast<const f4*>(wl + (tau * C::CH + 4 * c4) * 2 + 4);
#pragma unroll
            for (int k = 0; k < C::NOUT; ++k) {
              const f4 sv = *reinterpret_cast<const f4*>(spf + (size_t)(op[k] + to) * C::CH + 4 * c4);
              u[k][0] = fmaf(wa[0], sv[0], u[k][0]); u[k][1] = fmaf(wa[1], sv[0], u[k][1]);
              u[k][0] = fmaf(wa[2], sv[1], u[k][0]); u[k][1] = fmaf(wa[3], sv[1], u[k][1]);
              u[k][0] = fmaf(wb[0], sv[2], u[k][0]); u[k][1] = fmaf(wb[1], sv[2], u[k][1]);
              u[k][0] = fmaf(wb[2], sv[3], u[k][0]); u[k][1] = fmaf(wb[3], sv[3], u[k][1]);
            }
          }
        } else {
#pragma unroll
          for (int c8 = 0; c8 < C::CH / 8; ++c8) {
            f4 wv[4];
#pragma unroll
            for (int z = 0; z < 4; ++z) wv[z] = *reinterpret_cast<const f4*>(wl + (tau * C::CH + 8 * c8) * 2 + 4 * z);
#pragma unroll
            for (int k = 0; k < C::NOUT; ++k) {
              const u4 raw = *reinterpret_cast<const u4*>(spb + (size_t)(op[k] + to) * C::CH + 8 * c8);
#pragma unroll
              for (int z = 0; z < 4; ++z) {
                const float s0 = __builtin_bit_cast(float, raw[z] << 16);
                const float s1 = __builtin_bit_cast(float, raw[z] & 0xffff0000u);
                u[k][0] = fmaf(wv[z][0], s0, u[k][0]); u[k][1] = fmaf(wv[z][1], s0, u[k][1]);
                u[k][0] = fmaf(wv[z][2], s1, u[k][0]); u[k][1] = fmaf(wv[z][3], s1, u[k][1]);
              }
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
          if (C::FULL && ok && co < cout && trace_t) {
            const int gy = tl.ty0 + q / C::TW, gx = tl.tx0 + q % C::TW;
            if (tb.has(gy, gx)) trace_t[(size_t)(choffo + co) * tb.plane() + tb.idx(gy, gx)] = u[k][co];
          }
          float v = u[k][co];
          const float s = bilif(v, theta, alpha, C::FULL && relaxed);
          so[k][co] = v;
          if (ok && co < cout && ca.s_out) {
            const size_t o = (((size_t)tl.n * T + t) * cout + co) * HW + pix;
            if (C::FULL && ca.s_fp32) reinterpret_cast<float*>(ca.s_out)[o] = s;
            else reinterpret_cast<int8_t*>(ca.s_out)[o] = (int8_t)s;
          }
        }
      }
    }
    if constexpr (C::NH == 0) {
      __syncthreads();
      if (t + 1 < T) EVS_STORE_X();
      if (t + 2 < T) EVS_LOAD_X(t + 2);
    }
    __syncthreads();                                     // B4: spikes / xs consumed
  }
  if (ca.v_out) write_state(ca.v_out + (size_t)tl.n * sumc * HW);
#undef EVS_LOAD_X
#undef EVS_STORE_X
}

template <class C>
__device__ __forceinline__ void init_lds(const FwdNetArgs& na, char* lds) {
  // zero canvas and pads once: pads are read only by junk (masked) pixels
  unsigned* z = reinterpret_cast<unsigned*>(lds);
  for (int e = threadIdx.x; e < (C::XS_BYTES + C::SP_BYTES) / 4; e += C::NT) z[e] = 0u;
  load_weights<C>(na, lds);
  load_out_frags<C>(na, lds);
}

// XCD-aware tile order: the hardware deals workgroups round-robin over the
// 8 XCDs; give each XCD a contiguous run of tiles so that the halos that
// neighbouring tiles share are fetched into the same L2.
__device__ inline int xcd_remap(int b, int n) {
  const int x = b & 7, k = b >> 3;
  const int q = n >> 3, r = n & 7;
  const int start = x * q + (x < r ? x : r);
  return start + k;
}

template <class C>
__global__ __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2))) void fwd_kernel(FwdNetArgs na, FwdClipArgs ca) {
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

// Persistent batched kernel: workgroups pop (clip, tile) items from a device
// counter; items are ordered clip by clip, clips longest-first.
template <class C>
__global__ __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2))) void fwd_batched_kernel(FwdNetArgs na, BatchTable bt, int32_t* counter) {
  __shared__ __attribute__((aligned(16))) char lds[Layout<C>::TOTAL];
  __shared__ int item_sh;
  init_lds<C>(na, lds);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item_sh = atomicAdd(counter, 1);
    __syncthreads();
    const int item = item_sh;
    if (item >= bt.n_items) break;
    int c = 0;
    while (c + 1 < bt.n_clips && bt.item_start[c + 1] <= item) ++c;
    const FwdClipArgs& ca = bt.clip[c];
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
  void (*batched)(const FwdNetArgs&, const BatchTable&, int32_t*, int, hipStream_t, hipError_t*);
};

template <class C>
void launch_single(const FwdNetArgs& na, const FwdClipArgs& ca, hipStream_t st, hipError_t* err) {
  dim3 grid(ca.tiles_x * ca.tiles_y, ca.N);
  hipLaunchKernelGGL(fwd_kernel<C>, grid, dim3(C::NT), 0, st, na, ca);
  *err = hipGetLastError();
}
template <class C>
void launch_batched(const FwdNetArgs& na, const BatchTable& bt, int32_t* counter, int n_wg,
                    hipStream_t st, hipError_t* err) {
  hipLaunchKernelGGL(fwd_batched_kernel<C>, dim3(n_wg), dim3(C::NT), 0, st, na, bt, counter);
  *err = hipGetLastError();
}

#define EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, FULL) Cfg<NL, CIN, CH, (bool)BF, TH, TW, NW, FULL>
// a tile variant: inference kernel + training/debug kernel (+ batched kernel)
#define EVS_VARIANT(NL, CIN, CH, BF, TH, TW, NW, NAME)                                              \
  Variant{NL, CIN, CH, BF, TH, TW, NAME, &launch_single<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, false)>, \
          &launch_single<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, true)>, nullptr}
#define EVS_VARIANT_B(NL, CIN, CH, BF, TH, TW, NW, NAME)                                            \
  Variant{NL, CIN, CH, BF, TH, TW, NAME, &launch_single<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, false)>, \
          &launch_single<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, true)>,                               \
          &launch_batched<EVS_CFG(NL, CIN, CH, BF, TH, TW, NW, false)>}

// Tile variants per network shape; the first one of a shape is its default.
// 4-wave variants are small enough (LDS <= 80 KB) for two workgroups per CU,
// whose MFMA and VALU phases then overlap.
const Variant kVariants[] = {
    // single-layer nets (input -> output), f32
    EVS_VARIANT(1, 1, 16, 0, 32, 32, 8, "L1 cin1 f32 32x32 w8"),
    EVS_VARIANT(1, 3, 16, 0, 32, 32, 8, "L1 cin3 f32 32x32 w8"),
    // two-layer nets cin -> hidden(<=16) -> out
    EVS_VARIANT_B(2, 3, 16, 0, 16, 32, 8, "L2 h16 f32 16x32 w8"),
    EVS_VARIANT(2, 3, 16, 0, 30, 40, 8, "L2 h16 f32 30x40 w8"),
    EVS_VARIANT(2, 3, 16, 0, 20, 32, 4, "L2 h16 f32 20x32 w4"),
    EVS_VARIANT(2, 1, 16, 0, 30, 40, 8, "L2 cin1 h16 f32 30x40 w8"),
    EVS_VARIANT(2, 3, 16, 1, 30, 40, 8, "L2 h16 bf16 30x40 w8"),
    // two-layer nets with hidden width <= 32
    EVS_VARIANT(2, 3, 32, 0, 22, 32, 8, "L2 h32 f32 22x32 w8"),
    EVS_VARIANT(2, 3, 32, 0, 16, 44, 8, "L2 h32 f32 16x44 w8"),
    EVS_VARIANT_B(2, 3, 32, 1, 24, 32, 8, "L2 h32 bf16 24x32 w8"),
    EVS_VARIANT_B(2, 3, 32, 1, 30, 40, 8, "L2 h32 bf16 30x40 w8"),
    EVS_VARIANT_B(2, 3, 32, 1, 16, 32, 4, "L2 h32 bf16 16x32 w4"),
    EVS_VARIANT_B(2, 3, 32, 1, 20, 32, 4, "L2 h32 bf16 20x32 w4"),
    EVS_VARIANT(2, 3, 32, 1, 12, 32, 4, "L2 h32 bf16 12x32 w4"),
    // three-layer nets
    EVS_VARIANT_B(3, 3, 16, 0, 24, 32, 8, "L3 h16 f32 24x32 w8"),
    EVS_VARIANT_B(3, 3, 16, 0, 12, 32, 4, "L3 h16 f32 12x32 w4"),
    EVS_VARIANT(3, 3, 16, 0, 16, 24, 4, "L3 h16 f32 16x24 w4"),
    EVS_VARIANT(3, 3, 16, 1, 30, 40, 8, "L3 h16 bf16 30x40 w8"),
    EVS_VARIANT(3, 3, 16, 1, 16, 32, 4, "L3 h16 bf16 16x32 w4"),
    EVS_VARIANT(3, 3, 32, 1, 24, 32, 8, "L3 h32 bf16 24x32 w8"),
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int padded_hidden(const evs_net& net) {
  int mx = 0;
  for (int l = 1; l < net.n_layers; ++l) mx = net.ch[l] > mx ? net.ch[l] : mx;
  return mx <= 16 ? 16 : 32;
}

bool matches(const Variant& v, const evs_net& net) {
  return v.nl == net.n_layers && v.cin == net.ch[0] && v.bf16 == (net.precision == EVS_BF16) &&
         (net.n_layers == 1 || v.ch == padded_hidden(net));
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

int forward_tile_count(const evs_net& net) {
  int k = 0;
  for (int i = 0; i < kNumVariants; ++i) k += matches(kVariants[i], net) ? 1 : 0;
  return k;
}

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

int forward_default_tile(const evs_net& net, int H, int W) {
  (void)H; (void)W;
  return forward_tile_count(net) > 0 ? 0 : -1;
}

int launch_forward(const evs_net& net, const FwdNetArgs& na, const FwdClipArgs& ca, int tile_id,
                   hipStream_t stream) {
  const Variant* v = find_variant(net, tile_id);
  if (!v) return fail(EVS_EUNSUPPORTED, "no compiled forward kernel for this network shape");
  hipError_t e = hipSuccess;
  const bool full = ca.h_trace || ca.ckpt || na.relaxed || ca.s_fp32;
  (full ? v->single_full : v->single_fast)(na, ca, stream, &e);
  if (e != hipSuccess) return hip_check(e, "forward kernel launch");
  return EVS_OK;
}

int launch_forward_batched(const evs_net& net, const FwdNetArgs& na, const BatchTable& bt, int tile_id,
                           int32_t* counter, hipStream_t stream) {
  const Variant* v = find_variant(net, tile_id);
  if (!v) return fail(EVS_EUNSUPPORTED, "no compiled forward kernel for this network shape");
  if (!v->batched) return fail(EVS_EUNSUPPORTED, "no batched kernel compiled for this tile variant");
  int dev = 0, ncu = 0;
  EVS_HIP(hipGetDevice(&dev));
  EVS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int n_wg = bt.n_items < ncu ? bt.n_items : ncu;
  hipError_t e = hipSuccess;
  v->batched(na, bt, counter, n_wg, stream, &e);
  if (e != hipSuccess) return hip_check(e, "batched forward kernel launch");
  return EVS_OK;
}

}  // namespace evs
