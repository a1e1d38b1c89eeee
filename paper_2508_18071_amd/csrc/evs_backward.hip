// Surrogate-gradient BPTT backward of EvSNet (arXiv 2508.18071, Sec. 3.3,
// Eq. 4), with membrane checkpoints every k frames.
//
// Segments of k frames are visited from the last to the first.  For each:
//   1. the forward kernel recomputes the segment's charged potentials h of
//      every layer from the segment's checkpoint (bit-identical to the
//      original forward: same kernel, same state);
//   2. the top layer's reverse-time adjoint scan per neuron
//          g_h = (G - theta g_v) psi(h) + g_v     (G psi(h) + g_v detached)
//          g_v <- leak * g_h
//      on G = grad_s, with g_v carried across segment boundaries;
//   3. for layers L..1: the weight gradient
//          dW[co][ci][tap] = sum_t,p g_h[co][p] s_in[ci][p+tap]
//      as per-tile partial sums in registers, added to the tile's slot for
//      the whole backward and reduced over the tiles once at the end, in a
//      fixed order (no float atomics: results are bitwise reproducible);
//      then the incoming
//      gradient of the layer below, G = conv_transpose(g_h, W), which for
//      l >= 2 feeds that layer's adjoint scan in the same kernel (G stays in
//      registers), and for l = 1 is grad_x.
// Spikes fed to dW are recomputed from h with the forward's own device
// function, so they equal the forward's spikes bit for bit.
#include "evs_device.hpp"
#include "evs_ops.hpp"

namespace evs {
namespace {

constexpr int TT = 16;            // pixel tile edge of the conv kernels
constexpr int NTH = TT * TT;      // threads per workgroup

inline int pad_in(int c) { return c <= 4 ? 4 : (c <= 16 ? 16 : 32); }
inline int pad_out(int c) { return c <= 2 ? 2 : (c <= 16 ? 16 : 32); }

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

__device__ inline float wq(const float* w, int idx, bool bf) {
  const float v = w[idx];
  return bf ? round_bf16(v) : v;
}

// Storage of a segment's charged potentials h (written by the forward's
// training build) and of the adjoints g_h between the gradient kernels.
// FP32 nets: float both.  BF16 nets: h as fp16 rounded so that the stored
// value gives the forward's spike (the forward's recompute build) and g_h as bf16
// (round to nearest), the operand precision of their bf16 matrix products;
// the adjoint recurrences, the surrogate and every sum stay FP32.
template <bool B16> struct Store;
template <> struct Store<false> { using H = float; using G = float; };
template <> struct Store<true> { using H = _Float16; using G = __bf16; };

__device__ inline float to_f32(float v) { return v; }
__device__ inline float to_f32(_Float16 v) { return (float)v; }
__device__ inline float to_f32(__bf16 v) { return __builtin_bit_cast(float, (unsigned)__builtin_bit_cast(unsigned short, v) << 16); }
template <class T> __device__ inline T from_f32(float v) { return (T)v; }

// Buffer load / store of one element of type T at a byte offset (offsets
// past the resource read 0 and drop the store).
template <class T>
__device__ inline float ld_el(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    return to_f32(__builtin_bit_cast(T, b));
  }
}
template <class T>
__device__ inline void st_el(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, from_f32<T>(v)), r, voff, soff, 0);
  }
}
// byte offset of element e of type T, or the dead offset (reads 0)
constexpr unsigned kDeadOff = 0x80000000u;
template <class T> __device__ inline unsigned el_off(bool live, unsigned e) { return live ? e * (unsigned)sizeof(T) : kDeadOff; }
// four consecutive elements (8- or 16-byte aligned) in one buffer load
template <class T>
__device__ inline f4 ld4_el(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  } else {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    const h4 q = __builtin_bit_cast(h4, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    return f4{(float)q[0], (float)q[1], (float)q[2], (float)q[3]};
  }
}

// Where the potentials of one layer sit in the segment trace the forward
// wrote (pixel-major): frame (n, t) of the segment starts at plane
// (n len + t) tpf, the layer at plane cpo of it, and pixel p's channel c is
// element p cw + c of the layer's block (cw: the layer's width rounded up
// to 4; the output layer's 4).
struct HTrace {
  int tpf, cpo, cw;
  __device__ size_t base(int n, int len, int t, size_t HW) const { return ((size_t)(n * len + t) * tpf + cpo) * HW; }
};

// ---------------------------------------------------------------- adjoint scan
template <class HS, class GS>
__global__ __launch_bounds__(256) void k_adjoint(const HS* __restrict__ hseg, HTrace ht, int sumc, int choff, int C,
                                                 int len, int N, int HW, const float* __restrict__ G,
                                                 long long G_nstride, long long G_tstride,
                                                 GS* __restrict__ gh, float* __restrict__ gv, float theta,
                                                 float leak, float alpha, int surr, int detach,
                                                 int32_t* __restrict__ status) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long total = (long long)N * C * HW;
  if (idx >= total) return;
  int nan = 0;
  const int p = (int)(idx % HW);
  const int c = (int)((idx / HW) % C);
  const int n = (int)(idx / ((long long)HW * C));
  float* gvp = gv + ((size_t)n * sumc + choff + c) * HW + p;
  float g_v = *gvp;
  for (int t = len - 1; t >= 0; --t) {
    const float h = to_f32(hseg[ht.base(n, len, t, HW) + (size_t)p * ht.cw + c]);
    const float Gv = G[(size_t)n * G_nstride + (size_t)t * G_tstride + (size_t)c * HW + p];
    nan += Gv != Gv ? 1 : 0;
    const float psi = surrogate(h, theta, alpha, surr);
    const float g_h = detach ? fmaf(Gv, psi, g_v) : fmaf(fmaf(-theta, g_v, Gv), psi, g_v);
    gh[(((size_t)n * len + t) * C + c) * HW + p] = from_f32<GS>(g_h);
    g_v = leak * g_h;
  }
  *gvp = g_v;
  // every element of grad_s is read by exactly one thread of one call: the
  // NaN count of the status word (saturating)
  if (status && nan) {
    int old = __hip_atomic_load(status + EVS_STATUS_NAN_GRAD, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
      const int nv = old > 0x7fffffff - nan ? 0x7fffffff : old + nan;
      const int prev = atomicCAS(status + EVS_STATUS_NAN_GRAD, old, nv);
      if (prev == old) break;
      old = prev;
    }
  }
}

// ---------------------------------------------------------------- conv transpose
// A layer's weights in [tap][co][ci] order, zero-padded to COUTP x CINP and
// rounded as the forward used them: one (tap, co) row of CINP weights is a
// single uniform (scalar-register) load in the conv-transpose kernel.
__global__ void k_pack_wT(const float* __restrict__ w, int Cout, int Cin, int CINP, int COUTP, int bf,
                          float* __restrict__ wT) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= 9 * COUTP * CINP) return;
  const int ci = e % CINP, co = (e / CINP) % COUTP, tap = e / (CINP * COUTP);
  wT[e] = (co < Cout && ci < Cin) ? wq(w, (co * Cin + ci) * 9 + tap, bf) : 0.f;
}

// G[n][t][ci][y][x] = sum_{co,tap} W[co][ci][tap] * gh[n][t][co][y-dy][x-dx]
// One workgroup per (tile, clip) walks the segment's frames from the last to
// the first, the next frame's haloed g_h tile loading into registers while
// the current one is used from LDS.  The weights are uniform operands (no
// LDS traffic for them).  With ADJ, G never leaves registers: it drives the
// adjoint scan (Eq. 4) of the layer below at the same pixel,
//     g_h = (G - theta g_v) psi(h) + g_v,   g_v <- leak g_h,
// with g_v held in registers for the whole segment, and that layer's g_h is
// written to out [n][t][Cin][H][W]; without ADJ G itself is written (grad_x).
// The arithmetic and its order are those of a separate conv-transpose pass
// followed by a separate scan.
template <int CINP, int COUTP, bool ADJ, class HS, class GS>
__global__ __launch_bounds__(NTH) void k_convT(const GS* __restrict__ gh, int Cout, int Cin, int len, int H,
                                               int W, int tiles_x, const float* __restrict__ wT,
                                               void* __restrict__ outv, long long out_nstride,
                                               long long out_tstride, const HS* __restrict__ hseg, HTrace ht, int sumc,
                                               int choff, float* __restrict__ gv, float theta, float leak,
                                               float alpha, int surr, int detach) {
  constexpr int kTile = COUTP * (TT + 2) * (TT + 2);
  constexpr int kStage = (kTile + NTH - 1) / NTH;
  __shared__ float ghs[COUTP][TT + 2][TT + 2];
  const int tile = xcd_remap(blockIdx.x, gridDim.x), n = blockIdx.y;
  const int ty0 = (tile / tiles_x) * TT, tx0 = (tile % tiles_x) * TT;
  const int HW = H * W;
  const int ty = threadIdx.x / TT, tx = threadIdx.x % TT;
  const int y = ty0 + ty, x = tx0 + tx;
  const bool own = y < H && x < W;
  float pre[kStage];
  auto fetch = [&](int t) __attribute__((always_inline)) {
    const GS* g = gh + ((size_t)n * len + t) * Cout * HW;
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int e = threadIdx.x + NTH * k;
      const int co = e / ((TT + 2) * (TT + 2)), r = (e / (TT + 2)) % (TT + 2), cc = e % (TT + 2);
      const int yy = ty0 - 1 + r, xx = tx0 - 1 + cc;
      pre[k] = (e < kTile && co < Cout && yy >= 0 && yy < H && xx >= 0 && xx < W)
                   ? to_f32(g[(size_t)co * HW + (size_t)yy * W + xx]) : 0.f;
    }
  };
  float g_v[CINP];
  if constexpr (ADJ) {
#pragma unroll
    for (int ci = 0; ci < CINP; ++ci)
      g_v[ci] = (own && ci < Cin) ? gv[((size_t)n * sumc + choff + ci) * HW + (size_t)y * W + x] : 0.f;
  }
  fetch(len - 1);
  for (int t = len - 1; t >= 0; --t) {
    __syncthreads();                                   // the previous frame's tile is consumed
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int e = threadIdx.x + NTH * k;
      if (e < kTile) (&ghs[0][0][0])[e] = pre[k];
    }
    float hv[CINP];
    if constexpr (ADJ) {
      const HS* hp = hseg + ht.base(n, len, t, HW) + ((size_t)y * W + x) * ht.cw;
#pragma unroll
      for (int ci = 0; ci < CINP; ++ci) hv[ci] = (own && ci < Cin) ? to_f32(hp[ci]) : 0.f;
    }
    if (t > 0) fetch(t - 1);                           // in flight while this frame is used
    __syncthreads();
    float acc[CINP];
#pragma unroll
    for (int ci = 0; ci < CINP; ++ci) acc[ci] = 0.f;
#pragma unroll 2
    for (int co = 0; co < Cout; ++co) {
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const float g = ghs[co][ty + 1 - dy][tx + 1 - dx];
        const float* wr = wT + (tap * COUTP + co) * CINP;
#pragma unroll
        for (int ci = 0; ci < CINP; ++ci) acc[ci] = fmaf(wr[ci], g, acc[ci]);
      }
    }
    if (own) {
      if constexpr (ADJ) {
        GS* o = reinterpret_cast<GS*>(outv) + (((size_t)n * len + t) * Cin) * HW + (size_t)y * W + x;
#pragma unroll
        for (int ci = 0; ci < CINP; ++ci) {
          if (ci < Cin) {
            const float psi = surrogate(hv[ci], theta, alpha, surr);
            const float g = detach ? fmaf(acc[ci], psi, g_v[ci]) : fmaf(fmaf(-theta, g_v[ci], acc[ci]), psi, g_v[ci]);
            o[(size_t)ci * HW] = from_f32<GS>(g);
            g_v[ci] = leak * g;
          }
        }
      } else {
        float* o = reinterpret_cast<float*>(outv) + (size_t)n * out_nstride + (size_t)t * out_tstride + (size_t)y * W + x;
#pragma unroll
        for (int ci = 0; ci < CINP; ++ci)
          if (ci < Cin) o[(size_t)ci * HW] = acc[ci];
      }
    }
  }
  if constexpr (ADJ) {
    if (own) {
#pragma unroll
      for (int ci = 0; ci < CINP; ++ci)
        if (ci < Cin) gv[((size_t)n * sumc + choff + ci) * HW + (size_t)y * W + x] = g_v[ci];
    }
  }
}

// The same conv-transpose + adjoint for a layer below with 5..16 channels,
// on the matrix pipe.  Per 16-pixel tile row, G[ci][pixel] is a 16 x 16
// product over K = (tap, co), the weights as the A operand and the haloed
// g_h tile as B, read from LDS at an immediate offset from a per-lane base.
// Lane (pixel j, group g) receives G for channels 4g..4g+3 of pixel j and
// runs the adjoint scan on them; wave w takes tile rows 4w..4w+3.
//   FP32 nets, narrow layer above: v_mfma_f32_16x16x4_f32, lane (ci, k) of
//     the A operand holds W[co][ci][tap] (staged in LDS once per
//     workgroup), K tap-major with co in lane groups of 4 (output widths
//     below 4 padded with zero weights); the g_h planes are 336 floats apart
//     (16 banks mod 64), so the four lane groups of a read hit distinct
//     banks.  FP32 products and sums, in the matrix pipe's own order.
//   FP32 nets, 16-wide layer above (kF3): the bf16 product below with g_h
//     and W each split exactly into three bf16 parts (h = bf16(v),
//     m = bf16(v - h), l = v - h - m) and six part products kept per
//     k-step, (h,h) (h,m) (m,h) (h,l) (m,m) (l,h): the dropped ones are
//     below 2^-23 |w g| together.  g_h is split while it is staged (three
//     pairs of [pixel][8 channels] planes), the weight parts sit in LDS;
//     30 MFMAs per row instead of 36 f32 ones at twice the issue time.
//   BF16 nets, 16-wide layer above (B16): v_mfma_f32_16x16x32_bf16 with
//     the bf16 g_h the layer above stored and the bf16 weights the forward
//     used (exact products, FP32 sums): K slots 8g..8g+7 of k-step s are tap
//     2s + g/2 (tap 9: zero weights), channels 8 (g & 1) .. +7, so the B
//     operand of a lane is one 16-byte read from a tile held as two planes
//     of [pixel][8 channels] bf16 whose stride is a multiple of 256 bytes
//     (the two channel halves of a tap then fill disjoint banks); 5 MFMAs
//     per row instead of 36.
//   BF16 nets, output layer above (2 channels): the same bf16 product with
//     K = 18 (tap, co) pairs in one k-step: lane group g holds taps 4g ..
//     4g + 3 of both channels (tap 8 in group 2, zero weights past it), read
//     from a table of [pixel][2 channels] bf16 pairs; 1 MFMA per row
//     instead of 9.  (The fused weight gradient stays on the FP32 pipe.)
// Part p of the exact split v = h + m + l into bf16 values (round to
// nearest: h = bf16(v), m = bf16(v - h), l = v - h - m, each exact).
__device__ inline float bf16_part(float v, int p) {
  const float h = (float)(__bf16)v;
  if (p == 0) return h;
  const float r = v - h, m = (float)(__bf16)r;
  return p == 1 ? m : r - m;
}

// DW1 (16-wide layer above, the layer below fed by the clip input x): the
// kernel also forms the input layer's weight gradient dW1[co][ci][tap] =
// sum_p g_h1[co][p] x[ci][p + tap] from the g_h1 it has just computed, so
// g_h1 is not written out unless the input gradient needs it (out
// non-null).  Per frame each wave puts its 64 pixels' g_h1 ([pixel][co],
// the A layout of v_mfma_f32_16x16x4_f32: rows co, K = 4 pixels) and its
// own 6 x 18 window of x (B: columns (ci, tap)) into LDS regions only it
// reads, over the g_h tile (after a barrier: the tile is consumed), and
// issues 16 k-steps x 2 column tiles of FP32 MFMAs (products of the g_h1
// values as stored and of x, bf16-rounded for BF16 nets).  Per-wave sums
// stay in registers for the segment and are added in wave order at the end.
// The backward uses it for FP32 nets; BF16 nets keep their separate bf16
// input-layer kernel (faster than FP32 MFMAs at three waves per SIMD).
template <int COUTP, bool B16, bool DW1 = false>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(B16 && !DW1 ? 4 : 3)))
void k_convT_mfma(const typename Store<B16>::G* __restrict__ gh, int Cout, int Cin, int len, int H,
                                                    int W, int tiles_x, const float* __restrict__ wT,
                                                    typename Store<B16>::G* __restrict__ out,
                                                    const typename Store<B16>::H* __restrict__ hseg, HTrace ht,
                                                    int sumc, int choff, float* __restrict__ gv, float theta,
                                                    float leak, float alpha, int surr, int detach, int relaxed,
                                                    float* __restrict__ dw_partial, const float* __restrict__ x1,
                                                    long long x1_ns, int cin0, float* __restrict__ dw1_partial) {
  using HS = typename Store<B16>::H;
  using GS = typename Store<B16>::G;
  constexpr unsigned ESH = sizeof(HS), ESG = sizeof(GS);
  constexpr bool kBF = B16 && COUTP == 16;             // the bf16 product
  constexpr bool kBF2 = B16 && COUTP == 2;             // its two-channel form
  constexpr bool kF3 = !B16 && COUTP == 16;            // the bf16 product on three-part splits
  constexpr int E = TT + 2;                            // haloed tile edge
  constexpr int PS = (E * E + 47) / 64 * 64 + 16;      // plane stride (floats), 16 mod 64
  constexpr int PSB = (E * E * 16 + 255) / 256 * 256;  // bf16 plane stride (bytes), multiple of 256
  constexpr int COG = COUTP < 4 ? 4 : COUTP;           // co slots per tap
  constexpr int KS = 9 * COG / 4;                      // k-steps (f32 product)
  constexpr int KSB = 5;                               // k-steps (bf16 product)
  static_assert(COG % 4 == 0, "co slots come in lane groups of 4");
  static_assert(E * E > NTH && E * E <= 2 * NTH, "a tile plane is staged in two passes");
  static_assert(!DW1 || COUTP == 16, "the fused input-layer gradient sits below a 16-wide layer");
  constexpr int kGhsF = kBF ? 2 * PSB / 4 : (kF3 ? 6 * PSB / 4 : COUTP * PS);
  // DW1 regions over the tile: per wave g_h1 [64 pixels][16 co], then per
  // wave x [3 ci][6 rows][18 columns]; the end-of-segment wave sums reuse it
  constexpr int XWP = 6 * (TT + 2);                    // x window plane (floats)
  constexpr int kG1F = 4 * 64 * 16, kDw1F = kG1F + 4 * 3 * XWP;
  __shared__ __attribute__((aligned(16))) float ghs[DW1 && kDw1F > kGhsF ? kDw1F : kGhsF];
  __shared__ unsigned gp2[kBF2 ? E * E : 1];           // [pixel] (co 0, co 1) bf16 pairs
  const int tile = xcd_remap(blockIdx.x, gridDim.x), n = blockIdx.y;
  const int ty0 = (tile / tiles_x) * TT, tx0 = (tile % tiles_x) * TT;
  const int HW = H * W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  // weights (f32 product): k-step s, lane group g -> tap s / (COG/4), co
  // 4 (s % (COG/4)) + g; held in LDS as [s / 4][lane][s % 4], one 16-byte
  // read per lane for four k-steps (the A operand would otherwise take 36-72
  // registers)
  constexpr int KS4 = (KS + 3) / 4;
  __shared__ f4 wl[kBF || kF3 ? 1 : KS4 * 64];
  u4 wb[kBF ? KSB : 1];
  // kF3: the A operand of part p, k-step s at [p][s][lane], laid out as wb
  __shared__ u4 wl3[kF3 ? 3 * KSB * 64 : 1];
  u4 wb2 = u4{0u, 0u, 0u, 0u};
  if constexpr (kBF2) {
    // row ci = j; K slot 8g + e: tap 4g + e / 2, channel e % 2
    unsigned wd[4];
#pragma unroll
    for (int e2 = 0; e2 < 4; ++e2) {
      const int tap = 4 * g + e2;
      float ww[2];
#pragma unroll
      for (int co = 0; co < 2; ++co) ww[co] = tap < 9 ? wT[(tap * COUTP + co) * 16 + j] : 0.f;
      typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
      const bf2 pr = {(__bf16)ww[0], (__bf16)ww[1]};
      wd[e2] = __builtin_bit_cast(unsigned, pr);
    }
    wb2 = u4{wd[0], wd[1], wd[2], wd[3]};
  }
  if constexpr (kBF) {
    // bf16 A operand in registers: row ci = j, K slot 8g + e of k-step s
#pragma unroll
    for (int s = 0; s < KSB; ++s) {
      const int tap = 2 * s + (g >> 1);
      unsigned wd[4];
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2) {
        float ww[2];
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
          const int co = 8 * (g & 1) + 2 * e2 + h2;
          ww[h2] = tap < 9 ? wT[(tap * COUTP + co) * 16 + j] : 0.f;
        }
        typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
        const bf2 pr = {(__bf16)ww[0], (__bf16)ww[1]};
        wd[e2] = __builtin_bit_cast(unsigned, pr);
      }
      wb[s] = u4{wd[0], wd[1], wd[2], wd[3]};
    }
  } else if constexpr (kF3) {
    for (int idx = threadIdx.x; idx < 3 * KSB * 64; idx += NTH) {
      const int p = idx / (KSB * 64), sk = (idx / 64) % KSB, l = idx % 64;
      const int tap = 2 * sk + (l >> 5);
      unsigned wd[4];
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2) {
        float ww[2];
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
          const int co = 8 * ((l >> 4) & 1) + 2 * e2 + h2;
          ww[h2] = tap < 9 ? bf16_part(wT[(tap * COUTP + co) * 16 + (l & 15)], p) : 0.f;
        }
        typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
        const bf2 pr = {(__bf16)ww[0], (__bf16)ww[1]};   // exact: bf16 values
        wd[e2] = __builtin_bit_cast(unsigned, pr);
      }
      wl3[idx] = u4{wd[0], wd[1], wd[2], wd[3]};
    }
  } else {
    for (int idx = threadIdx.x; idx < KS4 * 4 * 64; idx += NTH) {
      const int s = idx / 64, l = idx % 64;
      const int tap = s / (COG / 4), co = 4 * (s % (COG / 4)) + l / 16;
      wl[(s / 4) * 64 + l][s % 4] = (s < KS && co < COUTP) ? wT[(tap * COUTP + co) * 16 + l % 16] : 0.f;
    }
  }
  // B read of (row r, k-step s): base + r E + imm(s); planes past COUTP
  // (zero weights) read plane g % COUTP, whose values are finite
  const int plane = COUTP < 4 ? g % COUTP : g;
  const float* const bbase = ghs + plane * PS + 4 * wave * E + j;
  const char* const bbase16 = reinterpret_cast<const char*>(ghs) + (g & 1) * PSB + (4 * wave * E + j) * 16;
  // Narrow layers (output widths <= 4) also form their own weight gradient
  // dW[co][ci][tap] = sum_q s[ci][q] g_h[co][q - tap] (s: the spikes of the
  // layer below, from the h this kernel reads anyway) as a 16 (ci) x 18
  // ((co, tap), in two 16-column tiles) product over the wave's 64 pixels per
  // frame: the spikes go through LDS into the A layout, g_h is read from the
  // haloed tile already in LDS.  Per-wave sums stay in registers for the
  // segment and are added in wave order at the end.
  constexpr bool kDW = COUTP <= 4;
  constexpr int kDWCols = COUTP * 9;
  static_assert(!kDW || kDWCols <= 32, "two column tiles");
  constexpr int SBS = NTH + 4;                         // ci stride: lanes j hit banks 4j + g
  __shared__ float sb[kDW ? 16 * SBS : 1];
  f4 dacc[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
  int dwoff[2];
  bool dwcol[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int idx = 16 * nt + j, co = idx / 9, tap = idx % 9;
    dwcol[nt] = kDW && idx < kDWCols && co < Cout;
    // B of pixel (row, col) of the wave's rows: g_h[co][row - dy][col - dx]
    dwoff[nt] = dwcol[nt] ? co * PS + (1 - (tap / 3 - 1)) * E + (1 - (tap % 3 - 1)) + 4 * wave * E + g : 0;
  }
  // this lane's 16 neurons: rows 4 wave + r (uniform in the wave), column j,
  // channels 4g + i.  Their [ch][H][W] planes are read and written through
  // buffer resources bounded to the layer's Cin planes: voff[i] + r W es is
  // the byte offset of neuron (r, i) in a plane of es-byte elements; a lane
  // past the image's right edge has offsets of 2^31 and up, and one past
  // Cin offsets beyond the last plane, so their loads return 0 and their
  // stores are dropped.  Rows past the bottom edge are skipped by a branch
  // that is uniform in the wave.
  const int x = tx0 + j, y0 = ty0 + 4 * wave;
  const unsigned nel = (unsigned)Cin * (unsigned)HW;
  unsigned voff[4], voffG[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned e = (unsigned)(4 * g + i) * (unsigned)HW + (unsigned)(y0 * W + x);
    voff[i] = el_off<float>(x < W, e);
    voffG[i] = el_off<GS>(x < W, e);
  }
  // h of the lane's four channels of a pixel: one load from the
  // pixel-major trace (lanes past the layer's rounded width read 0)
  const unsigned voffH = el_off<HS>(x < W && 4 * g < ht.cw, (unsigned)((y0 * W + x) * ht.cw + 4 * g));
  // staging: this thread loads haloed-tile entries q = tid and tid + 256 of
  // every g_h plane; entries outside the image read 0 the same way
  unsigned qoff[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int q = threadIdx.x + NTH * k;
    const int yy = ty0 - 1 + q / E, xx = tx0 - 1 + q % E;
    qoff[k] = el_off<GS>(q < E * E && yy >= 0 && yy < H && xx >= 0 && xx < W, (unsigned)(yy * W + xx));
  }
  const __amdgpu_buffer_rsrc_t rv =
      __builtin_amdgcn_make_buffer_rsrc(gv + ((size_t)n * sumc + choff) * HW, (short)0, (int)(nel * 4u), 0x00020000);
  float g_v[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) g_v[r][i] = y0 + r < H ? ld_el<float>(rv, voff[i], r * W * 4) : 0.f;
  // DW1: entries e = lane, lane + 64 of the wave's x window (rows y0 - 1 ..
  // y0 + 4, columns tx0 - 1 .. tx0 + 16); outside the image: the dead offset
  // (reads 0, the conv's zero padding).  Column tile nt of the B operand:
  // column idx = 16 nt + j is (ci, tap) = (idx / 9, idx % 9).
  unsigned xoff1[2] = {kDeadOff, kDeadOff};
  float xv1[3][2];
  int xb1[2] = {0, 0};
  bool xc1[2] = {false, false};
  f4 dacc1[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
  if constexpr (DW1) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = lane + 64 * k;
      const int yy = y0 - 1 + e / (TT + 2), xx = tx0 - 1 + e % (TT + 2);
      xoff1[k] = el_off<float>(e < XWP && yy >= 0 && yy < H && xx >= 0 && xx < W, (unsigned)(yy * W + xx));
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int idx = 16 * nt + j, ci = idx / 9, tap = idx % 9;
      xc1[nt] = ci < cin0;
      // pixel (row R, column C) of the wave's block reads window row R + 1 + dy,
      // column C + 1 + dx; this lane's pixel of k-step kk is (kk / 4, 4 (kk % 4) + g)
      xb1[nt] = kG1F + wave * 3 * XWP + (xc1[nt] ? ci : 0) * XWP + (tap / 3) * (TT + 2) + (tap % 3) + g;
    }
  }
  auto load_x1 = [&](int t) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(x1 + (size_t)n * x1_ns + (size_t)t * cin0 * HW), (short)0,
        (int)((unsigned)cin0 * (unsigned)HW * 4u), 0x00020000);
#pragma unroll
    for (int ci = 0; ci < 3; ++ci)
#pragma unroll
      for (int k = 0; k < 2; ++k) xv1[ci][k] = ci < cin0 ? ld_el<float>(rx, xoff1[k] + 4u * ci * HW, 0) : 0.f;
  };
  // a frame's loads: its haloed g_h tile (every load issued before the first
  // LDS store; planes past Cout fall outside the resource and read 0) and the
  // h of this lane's neurons.  Narrow layers above (memory-bound: the scan
  // dominates) load the next frame while the current one is processed.
  constexpr bool kAhead = COUTP <= 4;
  float st0[COUTP], st1[COUTP], hn[4][4];
  auto load_tile = [&](int t) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<GS*>(gh + ((size_t)n * len + t) * Cout * HW), (short)0, (int)((unsigned)Cout * (unsigned)HW * ESG),
        0x00020000);
#pragma unroll
    for (int co = 0; co < COUTP; ++co) st0[co] = ld_el<GS>(rg, qoff[0] + ESG * co * HW, 0);
    if (threadIdx.x < E * E - NTH) {
#pragma unroll
      for (int co = 0; co < COUTP; ++co) st1[co] = ld_el<GS>(rg, qoff[1] + ESG * co * HW, 0);
    }
  };
  auto load_h = [&](int t) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t rh = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<HS*>(hseg + ht.base(n, len, t, HW)), (short)0, (int)((unsigned)ht.cw * (unsigned)HW * ESH),
        0x00020000);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const f4 v = ld4_el<HS>(rh, voffH, r * W * ht.cw * ESH);
#pragma unroll
      for (int i = 0; i < 4; ++i) hn[r][i] = v[i];
    }
  };
  // one staged tile entry (all channels) into LDS: float planes, or the two
  // bf16 planes of [pixel][8 channels] (three pairs of them, one per part,
  // for kF3)
  auto stage_entry = [&](const float (&v)[COUTP], int q) __attribute__((always_inline)) {
    if constexpr (kF3) {
      typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
      float pt[3][COUTP];
#pragma unroll
      for (int c = 0; c < COUTP; ++c) {
        pt[0][c] = bf16_part(v[c], 0);
        const float r = v[c] - pt[0][c];
        pt[1][c] = (float)(__bf16)r;
        pt[2][c] = r - pt[1][c];
      }
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
          unsigned wd[4];
#pragma unroll
          for (int e2 = 0; e2 < 4; ++e2) {
            const bf2 pr = {(__bf16)pt[p][8 * hf + 2 * e2], (__bf16)pt[p][8 * hf + 2 * e2 + 1]};
            wd[e2] = __builtin_bit_cast(unsigned, pr);
          }
          *reinterpret_cast<u4*>(reinterpret_cast<char*>(ghs) + (2 * p + hf) * PSB + q * 16) = u4{wd[0], wd[1], wd[2], wd[3]};
        }
    } else if constexpr (kBF) {
      typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        unsigned wd[4];
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) {
          const bf2 pr = {(__bf16)v[8 * hf + 2 * e2], (__bf16)v[8 * hf + 2 * e2 + 1]};
          wd[e2] = __builtin_bit_cast(unsigned, pr);
        }
        *reinterpret_cast<u4*>(reinterpret_cast<char*>(ghs) + hf * PSB + q * 16) = u4{wd[0], wd[1], wd[2], wd[3]};
      }
    } else {
#pragma unroll
      for (int co = 0; co < COUTP; ++co) ghs[co * PS + q] = v[co];
      if constexpr (kBF2) {
        typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
        const bf2 pr = {(__bf16)v[0], (__bf16)v[1]};     // exact: bf16 values
        gp2[q] = __builtin_bit_cast(unsigned, pr);
      }
    }
  };
  if constexpr (kAhead) {
    load_tile(len - 1);
    load_h(len - 1);
  }
  for (int t = len - 1; t >= 0; --t) {
    __syncthreads();                                   // the previous frame's tile is consumed
    if constexpr (!kAhead) load_tile(t);
    if constexpr (DW1) load_x1(t);
    stage_entry(st0, threadIdx.x);
    if (threadIdx.x < E * E - NTH) stage_entry(st1, threadIdx.x + NTH);
    __syncthreads();
    if constexpr (!kAhead) load_h(t);
    float hv[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) hv[r][i] = hn[r][i];
    if constexpr (kAhead) {
      if (t > 0) {
        load_tile(t - 1);
        load_h(t - 1);
      }
    }
    f4 acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (kF3) {
      const u4* const a3 = wl3 + lane;
#pragma unroll
      for (int s = 0; s < KSB; ++s) {
        const bf8 ah = __builtin_bit_cast(bf8, a3[s * 64]), am = __builtin_bit_cast(bf8, a3[(KSB + s) * 64]),
                  al = __builtin_bit_cast(bf8, a3[(2 * KSB + s) * 64]);
        const int tap = 2 * s + (g >> 1) > 8 ? 8 : 2 * s + (g >> 1);     // tap 9: zero weights
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const int imm = ((1 - dy) * E + (1 - dx)) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const char* const b = bbase16 + r * E * 16 + imm;
          const bf8 bh = __builtin_bit_cast(bf8, *reinterpret_cast<const u4*>(b)),
                    bm = __builtin_bit_cast(bf8, *reinterpret_cast<const u4*>(b + 2 * PSB)),
                    bl = __builtin_bit_cast(bf8, *reinterpret_cast<const u4*>(b + 4 * PSB));
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[r], 0, 0, 0);   // small parts first
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc[r], 0, 0, 0);
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[r], 0, 0, 0);
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, acc[r], 0, 0, 0);
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, acc[r], 0, 0, 0);
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[r], 0, 0, 0);
        }
      }
    } else if constexpr (kBF) {
#pragma unroll
      for (int s = 0; s < KSB; ++s) {
        const int tap = 2 * s + (g >> 1) > 8 ? 8 : 2 * s + (g >> 1);     // tap 9: zero weights
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const int imm = ((1 - dy) * E + (1 - dx)) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const u4 b = *reinterpret_cast<const u4*>(bbase16 + r * E * 16 + imm);
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, wb[s]), __builtin_bit_cast(bf8, b),
                                                           acc[r], 0, 0, 0);
        }
      }
    } else if constexpr (kBF2) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        unsigned bw[4];
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) {
          const int tap = 4 * g + e2 > 8 ? 8 : 4 * g + e2;  // taps past 8: zero weights
          const int dy = tap / 3 - 1, dx = tap % 3 - 1;
          bw[e2] = gp2[(4 * wave + r + 1 - dy) * E + j + 1 - dx];
        }
        acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, wb2),
                                                         __builtin_bit_cast(bf8, u4{bw[0], bw[1], bw[2], bw[3]}), acc[r],
                                                         0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s4 = 0; s4 < KS4; ++s4) {
        const f4 w = wl[s4 * 64 + lane];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int s = 4 * s4 + u;
          if (s < KS) {
            const int tap = s / (COG / 4), cq = s % (COG / 4);
            const int dy = tap / 3 - 1, dx = tap % 3 - 1;
            const int imm = (COUTP < 4 ? 0 : 4 * cq * PS) + (1 - dy) * E + (1 - dx);
#pragma unroll
            for (int r = 0; r < 4; ++r)
              acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[u], bbase[r * E + imm], acc[r], 0, 0, 0);
          }
        }
      }
    }
    // (DW1 without the input gradient: no g_h1 output, a resource of size 0)
    const bool wout = !DW1 || out != nullptr;
    const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
        wout ? out + ((size_t)n * len + t) * Cin * HW : out, (short)0, wout ? (int)(nel * ESG) : 0, 0x00020000);
    float g1[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int i = 0; i < 4; ++i) g1[r][i] = 0.f;
      if (y0 + r < H) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float Gv = acc[r][i];
          const float psi = surrogate(hv[r][i], theta, alpha, surr);
          const float gn = detach ? fmaf(Gv, psi, g_v[r][i]) : fmaf(fmaf(-theta, g_v[r][i], Gv), psi, g_v[r][i]);
          if (wout) st_el<GS>(gn, ro, voffG[i], r * W * ESG);
          g_v[r][i] = leak * gn;
          // the value stored (bf16 for BF16 nets); 0 off the image and past Cin
          if constexpr (DW1) g1[r][i] = x < W && 4 * g + i < Cin ? to_f32(from_f32<GS>(gn)) : 0.f;
        }
      }
    }
    if constexpr (DW1) {
      __syncthreads();                                 // every wave is done with the g_h tile
      float* const g1w = ghs + wave * 64 * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        *reinterpret_cast<f4*>(g1w + (16 * r + j) * 16 + 4 * g) = f4{g1[r][0], g1[r][1], g1[r][2], g1[r][3]};
      float* const xw = ghs + kG1F + wave * 3 * XWP;
#pragma unroll
      for (int ci = 0; ci < 3; ++ci)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int e = lane + 64 * k;
          if (ci < cin0 && e < XWP) xw[ci * XWP + e] = B16 ? round_bf16(xv1[ci][k]) : xv1[ci][k];
        }
      // the regions are this wave's own: its LDS operations run in order
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const float av = g1w[(4 * kk + g) * 16 + j];
        const int imm = (kk / 4) * (TT + 2) + 4 * (kk % 4);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          if (nt == 0 || cin0 > 1) {
            const float bv = xc1[nt] ? ghs[xb1[nt] + imm] : 0.f;
            dacc1[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, dacc1[nt], 0, 0, 0);
          }
        }
      }
    }
    if constexpr (kDW) {
      // the wave's own pixels only: rows 4 wave .. 4 wave + 3 of the tile
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          sb[(4 * g + i) * SBS + (4 * wave + r) * TT + j] =
              y0 + r < H ? spike_of(hv[r][i], theta, alpha, relaxed) : 0.f;
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        // k-step: pixels 4 kk .. 4 kk + 3 of the wave; lane group g takes
        // pixel 4 kk + g = (row kk / 4, column 4 (kk % 4) + g)
        const float av = sb[j * SBS + (4 * wave + kk / 4) * TT + 4 * (kk % 4) + g];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          const float bv = dwcol[nt] ? ghs[dwoff[nt] + (kk / 4) * E + 4 * (kk % 4)] : 0.f;
          dacc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, dacc[nt], 0, 0, 0);
        }
      }
    }
  }
  if constexpr (kDW) {
    // lane (column j, group g) holds dW for ci 4g..4g+3 of column 16 nt + j;
    // the four waves' sums are added in wave order
    __syncthreads();
    float* red = sb;                                   // [wave - 1][lane][8]
    if (wave > 0) {
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[((wave - 1) * 64 + lane) * 8 + 4 * nt + i] = dacc[nt][i];
    }
    __syncthreads();
    if (wave == 0) {
      float* o = dw_partial + ((size_t)blockIdx.y * gridDim.x + tile) * (16 * COUTP * 9);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int idx = 16 * nt + j, co = idx / 9, tap = idx % 9;
        if (idx < kDWCols) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float v = dacc[nt][i];
#pragma unroll
            for (int w2 = 0; w2 < 3; ++w2) v += red[(w2 * 64 + lane) * 8 + 4 * nt + i];
            o[(co * 16 + 4 * g + i) * 9 + tap] += v;     // [co][ci][tap], as the VALU kernel
          }
        }
      }
    }
  }
  if constexpr (DW1) {
    // lane (column j, group g) holds dW1 for co 4g..4g+3 of column 16 nt + j;
    // the four waves' sums are added in wave order
    __syncthreads();
    float* red = ghs;                                  // [wave - 1][lane][8]
    if (wave > 0) {
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[((wave - 1) * 64 + lane) * 8 + 4 * nt + i] = dacc1[nt][i];
    }
    __syncthreads();
    if (wave == 0) {
      // [co][ci (4 slots)][tap], the layout of the separate input-layer kernels
      float* o = dw1_partial + ((size_t)blockIdx.y * gridDim.x + tile) * (16 * 4 * 9);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int idx = 16 * nt + j, ci = idx / 9, tap = idx % 9;
        if (xc1[nt]) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float v = dacc1[nt][i];
#pragma unroll
            for (int w2 = 0; w2 < 3; ++w2) v += red[(w2 * 64 + lane) * 8 + 4 * nt + i];
            o[((4 * g + i) * 4 + ci) * 9 + tap] += v;
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (y0 + r < H) {
#pragma unroll
      for (int i = 0; i < 4; ++i) st_el<float>(g_v[r][i], rv, voff[i], r * W * 4);
    }
}

// ---------------------------------------------------------------- weight gradient
// Per (tile, clip) workgroup over all frames of the segment: partial
// dW[co][ci][tap] in registers; s_in is x (layer 1) or the spikes of the
// layer below recomputed from its h.
// IS: element type of the input (x: float; h of the layer below: its
// storage type); GS: that of g_h.
template <int CINP, int COUTP, class IS, class GS>
__global__ __launch_bounds__(NTH) void k_dw(const GS* __restrict__ gh, int Cout, int Cin, int len, int H,
                                            int W, int tiles_x, const float* __restrict__ x,
                                            long long x_nstride, int bf_x, const IS* __restrict__ hseg, HTrace ht,
                                            int sumc, int choff_in, float theta, float alpha, int relaxed,
                                            float* __restrict__ partial) {
  constexpr int P = CINP * COUTP;                     // (co, ci) pairs
  constexpr int PPT = P >= NTH ? P / NTH : 1;         // pairs per thread
  constexpr int TPP = P >= NTH ? 1 : NTH / P;         // threads per pair
  __shared__ float ghs[COUTP][TT * TT];
  __shared__ float ss[CINP][TT + 2][TT + 2];
  __shared__ float red[TPP > 1 ? NTH * 9 : 1];
  const int tile = xcd_remap(blockIdx.x, gridDim.x), n = blockIdx.y;
  const int ty0 = (tile / tiles_x) * TT, tx0 = (tile % tiles_x) * TT;
  const int HW = H * W;
  float acc[PPT][9];
#pragma unroll
  for (int k = 0; k < PPT; ++k)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) acc[k][tap] = 0.f;
  const int sub = TPP > 1 ? threadIdx.x / P : 0;      // row subset of this thread
  // staging: this thread's entries of the g_h tile and of the haloed input
  // tile, loaded into registers one frame ahead (all loads of a frame in
  // flight together, while the previous frame is being multiplied)
  constexpr int kG = COUTP * TT * TT, kS = CINP * (TT + 2) * (TT + 2);
  constexpr int kGt = (kG + NTH - 1) / NTH, kSt = (kS + NTH - 1) / NTH;
  // Loads go through buffer resources bounded to the frame's planes, at
  // 32-bit byte offsets fixed for the whole segment; entries outside the
  // image (or past the real channels) get offsets of 2^31 and up, which read
  // 0 -- and 0 stages as 0 (its spike and its bf16 rounding are 0).
  constexpr unsigned ESI = sizeof(IS);
  unsigned goff[kGt], soff[kSt];
#pragma unroll
  for (int k = 0; k < kGt; ++k) {
    const int e = threadIdx.x + NTH * k;
    const int co = e / (TT * TT), r = (e / TT) % TT, cc = e % TT;
    const int y = ty0 + r, xx = tx0 + cc;
    goff[k] = el_off<GS>(e < kG && co < Cout && y < H && xx < W, (unsigned)co * (unsigned)HW + (unsigned)(y * W + xx));
  }
#pragma unroll
  for (int k = 0; k < kSt; ++k) {
    const int e = threadIdx.x + NTH * k;
    const int ci = e / ((TT + 2) * (TT + 2)), r = (e / (TT + 2)) % (TT + 2), cc = e % (TT + 2);
    const int y = ty0 - 1 + r, xx = tx0 - 1 + cc;
    const bool live = e < kS && ci < Cin && y >= 0 && y < H && xx >= 0 && xx < W;
    // x: planar [ci][H][W]; h of the layer below: the pixel-major trace
    const unsigned el = hseg ? (unsigned)(y * W + xx) * (unsigned)ht.cw + (unsigned)ci
                             : (unsigned)ci * (unsigned)HW + (unsigned)(y * W + xx);
    soff[k] = live ? ESI * el : kDeadOff;
  }
  float gpre[kGt], spre[kSt];
  auto fetch = [&](int t) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<GS*>(gh + ((size_t)n * len + t) * Cout * HW), (short)0, (int)((unsigned)sizeof(GS) * Cout * HW),
        0x00020000);
    const void* sb = hseg ? static_cast<const void*>(hseg + ht.base(n, len, t, HW))
                          : static_cast<const void*>(x + (size_t)n * x_nstride + (size_t)t * Cin * HW);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void*>(sb), (short)0, (int)(ESI * (hseg ? (unsigned)ht.cw : (unsigned)Cin) * HW), 0x00020000);
#pragma unroll
    for (int k = 0; k < kGt; ++k) gpre[k] = ld_el<GS>(rg, goff[k], 0);
#pragma unroll
    for (int k = 0; k < kSt; ++k) spre[k] = ld_el<IS>(rs, soff[k], 0);
  };
  fetch(0);
  for (int t = 0; t < len; ++t) {
    __syncthreads();                                   // the previous frame's tiles are consumed
#pragma unroll
    for (int k = 0; k < kGt; ++k) {
      const int e = threadIdx.x + NTH * k;
      if (e < kG) (&ghs[0][0])[e] = gpre[k];
    }
#pragma unroll
    for (int k = 0; k < kSt; ++k) {
      const int e = threadIdx.x + NTH * k;
      if (e < kS) {
        const float v = spre[k];
        (&ss[0][0][0])[e] = hseg ? spike_of(v, theta, alpha, relaxed) : (bf_x ? round_bf16(v) : v);
      }
    }
    if (t + 1 < len) fetch(t + 1);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int pr = (TPP > 1 ? threadIdx.x % P : threadIdx.x + NTH * k);
      const int co = pr / CINP, ci = pr % CINP;
      // rows sub, sub + TPP, ...; along a row the 3x3 input window slides,
      // so each pixel reads one new column of three values
      for (int py = sub; py < TT; py += TPP) {
        const float* r0 = &ss[ci][py][0];
        const float* r1 = &ss[ci][py + 1][0];
        const float* r2 = &ss[ci][py + 2][0];
        const float* gr = &ghs[co][py * TT];
        float a0 = r0[0], a1 = r0[1], b0 = r1[0], b1 = r1[1], c0 = r2[0], c1 = r2[1];
#pragma unroll
        for (int px = 0; px < TT; ++px) {
          const float a2 = r0[px + 2], b2 = r1[px + 2], c2 = r2[px + 2];
          const float gvv = gr[px];
          acc[k][0] = fmaf(gvv, a0, acc[k][0]);
          acc[k][1] = fmaf(gvv, a1, acc[k][1]);
          acc[k][2] = fmaf(gvv, a2, acc[k][2]);
          acc[k][3] = fmaf(gvv, b0, acc[k][3]);
          acc[k][4] = fmaf(gvv, b1, acc[k][4]);
          acc[k][5] = fmaf(gvv, b2, acc[k][5]);
          acc[k][6] = fmaf(gvv, c0, acc[k][6]);
          acc[k][7] = fmaf(gvv, c1, acc[k][7]);
          acc[k][8] = fmaf(gvv, c2, acc[k][8]);
          a0 = a1; a1 = a2; b0 = b1; b1 = b2; c0 = c1; c1 = c2;
        }
      }
    }
  }
  float* out = partial + ((size_t)blockIdx.y * gridDim.x + tile) * P * 9;
  if constexpr (TPP > 1) {
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) red[threadIdx.x * 9 + tap] = acc[0][tap];
    __syncthreads();
    if (threadIdx.x < P) {
      for (int tap = 0; tap < 9; ++tap) {
        float sacc = 0.f;
        for (int s2 = 0; s2 < TPP; ++s2) sacc += red[(s2 * P + threadIdx.x) * 9 + tap];
        out[threadIdx.x * 9 + tap] += sacc;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < PPT; ++k)
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) out[(threadIdx.x + NTH * k) * 9 + tap] += acc[k][tap];
  }
}

// Weight gradient of a 16 -> 16 conv fed by hard spikes, on the bf16 matrix
// pipe.  Per tap, dW[co][ci] = sum_p g_h[co][p] s[ci][p + tap] is a 16 x 16
// product over pixels: g_h as the A operand (rows co), the shifted spikes as
// B (columns ci), 32 pixels per MFMA.  Spikes are exact in bf16 and g_h is
// split exactly into three bf16 parts (h = bf16(g), m = bf16(g - h),
// l = g - h - m), so every product is exact and the sums accumulate in FP32.
// Per frame the tile's g_h parts and its spikes, in three copies shifted by
// the tap column (16-byte operand reads), are staged in LDS from registers
// that were loaded during the previous frame's products; wave w takes pixel
// rows 4w .. 4w+3, and the four waves' partials are added in wave order at
// the end (fixed association: reproducible).  BF16 nets (B16) store g_h in
// bf16 already: one part, a third of the products.
constexpr int kGspBytes = 3 * 16 * TT * TT * 2;          // g_h parts [part][co][pixel]
constexpr int kSsbBytes = 3 * 16 * (TT + 2) * TT * 2;    // spikes [dx][ci][row][col]
// spike staging: (haloed pixel, 8-channel half) vectors of the pixel-major trace
constexpr int kSsVec = 2 * (TT + 2) * (TT + 2);
constexpr int kSsPerThread = (kSsVec + NTH - 1) / NTH;
__device__ inline uint16_t bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

template <bool B16>
__global__ __launch_bounds__(NTH) void k_dw_mfma(const typename Store<B16>::G* __restrict__ gh, int Cout, int Cin,
                                                 int len, int H, int W, int tiles_x,
                                                 const typename Store<B16>::H* __restrict__ hseg, HTrace ht,
                                                 int sumc, int choff_in, float theta, float* __restrict__ partial) {
  using HS = typename Store<B16>::H;
  using GS = typename Store<B16>::G;
  constexpr int NP = B16 ? 1 : 3;                      // bf16 parts of g_h
  __shared__ __attribute__((aligned(16))) char lds[kGspBytes + kSsbBytes];
  uint16_t* const gsp = reinterpret_cast<uint16_t*>(lds);
  uint16_t* const ssb = reinterpret_cast<uint16_t*>(lds + kGspBytes);
  const int tile = xcd_remap(blockIdx.x, gridDim.x), n = blockIdx.y;
  const int ty0 = (tile / tiles_x) * TT, tx0 = (tile % tiles_x) * TT;
  const int HW = H * W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  // staging: this thread's g_h pixel (all 16 channels) and spike-tile entries
  const int gy = ty0 + threadIdx.x / TT, gx = tx0 + threadIdx.x % TT;
  // loads through buffer resources bounded to the frame's planes, at 32-bit
  // byte offsets fixed for the segment; entries outside the image or past
  // the real channels sit at 2^31 and up and read 0 (whose spike is 0)
  constexpr unsigned ESG = sizeof(GS), ESH = sizeof(HS);
  const unsigned goff = el_off<GS>(gy < H && gx < W, (unsigned)(gy * W + gx));
  // vector v: haloed pixel v / 2, channels 8 (v & 1) .. +7 as two loads
  // of four (consecutive lanes read consecutive memory); channels at or past
  // the trace block's width cw (a multiple of 4, at most 16) read 0.
  unsigned soff[kSsPerThread][2];
#pragma unroll
  for (int k = 0; k < kSsPerThread; ++k) {
    const int v = threadIdx.x + NTH * k, q = v >> 1;
    const int rr = q / (TT + 2), cc = q % (TT + 2);
    const int y = ty0 - 1 + rr, xx = tx0 - 1 + cc;
    const bool in = v < kSsVec && y >= 0 && y < H && xx >= 0 && xx < W;
#pragma unroll
    for (int hq = 0; hq < 2; ++hq) {
      const int c0 = 8 * (v & 1) + 4 * hq;
      soff[k][hq] = el_off<HS>(in && c0 < ht.cw, (unsigned)(y * W + xx) * (unsigned)ht.cw + (unsigned)c0);
    }
  }
  float gr[16], hr[kSsPerThread][8];
  auto fetch = [&](int t) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<GS*>(gh + ((size_t)n * len + t) * Cout * HW), (short)0, (int)(ESG * Cout * HW), 0x00020000);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<HS*>(hseg + ht.base(n, len, t, HW)), (short)0, (int)(ESH * (unsigned)ht.cw * HW), 0x00020000);
#pragma unroll
    for (int co = 0; co < 16; ++co) gr[co] = ld_el<GS>(rg, goff + ESG * co * HW, 0);
#pragma unroll
    for (int k = 0; k < kSsPerThread; ++k) {
      const f4 a = ld4_el<HS>(rs, soff[k][0], 0), b = ld4_el<HS>(rs, soff[k][1], 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        hr[k][i] = a[i];
        hr[k][4 + i] = b[i];
      }
    }
  };
  f4 acc[9];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) acc[tap] = f4{0.f, 0.f, 0.f, 0.f};
  fetch(0);
  for (int t = 0; t < len; ++t) {
    __syncthreads();                                   // the previous frame's operands are consumed
#pragma unroll
    for (int co = 0; co < 16; ++co) {
      const float v = gr[co];
      if constexpr (B16) {
        gsp[co * TT * TT + threadIdx.x] = bf16_bits(v);        // exact: v is a bf16 value
      } else {
        const float h = (float)(__bf16)v, r = v - h, m = (float)(__bf16)r;
        gsp[(0 * 16 + co) * TT * TT + threadIdx.x] = bf16_bits(h);
        gsp[(1 * 16 + co) * TT * TT + threadIdx.x] = bf16_bits(m);
        gsp[(2 * 16 + co) * TT * TT + threadIdx.x] = bf16_bits(r - m);
      }
    }
#pragma unroll
    for (int k = 0; k < kSsPerThread; ++k) {
      const int v = threadIdx.x + NTH * k, q = v >> 1;
      if (v < kSsVec) {
        const int rr = q / (TT + 2), cc = q % (TT + 2);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int ci = 8 * (v & 1) + i;
          const uint16_t b = bf16_bits(spike_of(hr[k][i], theta, 0.f, 0));
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            const int c2 = cc - dx;
            if (c2 >= 0 && c2 < TT) ssb[((dx * 16 + ci) * (TT + 2) + rr) * TT + c2] = b;
          }
        }
      }
    }
    if (t + 1 < len) fetch(t + 1);                     // in flight while this frame multiplies
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      // k-step: pixel rows 4 wave + 2q, +1; lane group g takes 8 pixels of
      // row 4 wave + 2q + g/2 starting at column 8 (g & 1)
      const int row = 4 * wave + 2 * q + (g >> 1), c0 = 8 * (g & 1);
      u4 a[NP];
#pragma unroll
      for (int b = 0; b < NP; ++b) a[b] = *reinterpret_cast<const u4*>(gsp + (b * 16 + j) * TT * TT + row * TT + c0);
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
        const u4 bv = *reinterpret_cast<const u4*>(ssb + ((dx * 16 + j) * (TT + 2) + row + dy) * TT + c0);
#pragma unroll
        for (int b = 0; b < NP; ++b)
          acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a[b]), __builtin_bit_cast(bf8, bv),
                                                            acc[tap], 0, 0, 0);
      }
    }
  }
  // lane (ci = j, g) holds dW[co = 4g + r][ci][tap] of its wave's pixels
  __syncthreads();
  float* rb = reinterpret_cast<float*>(lds);             // waves 1..3: [wave - 1][lane][36]
  if (wave > 0) {
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int r = 0; r < 4; ++r) rb[((wave - 1) * 64 + lane) * 36 + tap * 4 + r] = acc[tap][r];
  }
  __syncthreads();
  if (wave == 0) {
    float* out = partial + ((size_t)blockIdx.y * gridDim.x + tile) * 256 * 9;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[tap][r];
#pragma unroll
        for (int w2 = 0; w2 < 3; ++w2) v += rb[(w2 * 64 + lane) * 36 + tap * 4 + r];
        out[((4 * g + r) * 16 + j) * 9 + tap] += v;
      }
  }
}

// Weight gradient of the input layer of a BF16 net (x of at most 4
// channels, 16 output channels) on the bf16 matrix pipe:
// dW[co][ci][tap] = sum_p g_h[co][p] x[ci][p + tap] is a 16 (co) x 27
// ((ci, tap), two 16-column tiles) product over pixels, g_h (bf16, as
// stored) the A operand and the bf16-rounded x (the operand the forward
// multiplied) the B operand, so every product is exact and the sums
// accumulate in FP32.  Per frame the tile's g_h and its haloed x, in three
// copies shifted by the tap column (16-byte operand reads), are staged in
// LDS from registers loaded during the previous frame's products; wave w
// takes pixel rows 4w .. 4w+3 and the four waves' partials are added in
// wave order at the end.
constexpr int kXsbBytes = 3 * 4 * (TT + 2) * TT * 2;     // x [dx][ci][row][col]
constexpr int kXPerThread = (4 * (TT + 2) * (TT + 2) + NTH - 1) / NTH;
__global__ __launch_bounds__(NTH) void k_dw1_mfma(const __bf16* __restrict__ gh, int Cout, int Cin, int len, int H,
                                                  int W, int tiles_x, const float* __restrict__ x,
                                                  long long x_nstride, float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) char lds[16 * TT * TT * 2 + kXsbBytes];
  uint16_t* const gsp = reinterpret_cast<uint16_t*>(lds);
  uint16_t* const xsb = reinterpret_cast<uint16_t*>(lds + 16 * TT * TT * 2);
  const int tile = xcd_remap(blockIdx.x, gridDim.x), n = blockIdx.y;
  const int ty0 = (tile / tiles_x) * TT, tx0 = (tile % tiles_x) * TT;
  const int HW = H * W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int gy = ty0 + threadIdx.x / TT, gx = tx0 + threadIdx.x % TT;
  const unsigned goff = el_off<__bf16>(gy < H && gx < W, (unsigned)(gy * W + gx));
  unsigned xoff[kXPerThread];
#pragma unroll
  for (int k = 0; k < kXPerThread; ++k) {
    const int e = threadIdx.x + NTH * k;
    const int ci = e / ((TT + 2) * (TT + 2)), rr = (e / (TT + 2)) % (TT + 2), cc = e % (TT + 2);
    const int y = ty0 - 1 + rr, xx = tx0 - 1 + cc;
    xoff[k] = el_off<float>(e < 4 * (TT + 2) * (TT + 2) && ci < Cin && y >= 0 && y < H && xx >= 0 && xx < W,
                            (unsigned)ci * (unsigned)HW + (unsigned)(y * W + xx));
  }
  float gr[16], xr[kXPerThread];
  auto fetch = [&](int t) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<__bf16*>(gh + ((size_t)n * len + t) * Cout * HW), (short)0, (int)(2u * Cout * HW), 0x00020000);
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(x + (size_t)n * x_nstride + (size_t)t * Cin * HW), (short)0, (int)(4u * Cin * HW),
        0x00020000);
#pragma unroll
    for (int co = 0; co < 16; ++co) gr[co] = ld_el<__bf16>(rg, goff + 2u * co * HW, 0);
#pragma unroll
    for (int k = 0; k < kXPerThread; ++k) xr[k] = ld_el<float>(rx, xoff[k], 0);
  };
  // B column j of tile nt: (ci, tap) = ((16 nt + j) / 9, (16 nt + j) % 9);
  // columns 27..31 multiply zeros
  int boff[2];
  bool bcol[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int idx = 16 * nt + j, ci = idx / 9, tap = idx % 9;
    bcol[nt] = idx < 27;
    const int dy = tap / 3, dx = tap % 3;
    boff[nt] = bcol[nt] ? ((dx * 4 + ci) * (TT + 2) + dy) * TT : 0;
  }
  f4 acc[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
  fetch(0);
  for (int t = 0; t < len; ++t) {
    __syncthreads();                                   // the previous frame's operands are consumed
#pragma unroll
    for (int co = 0; co < 16; ++co) gsp[co * TT * TT + threadIdx.x] = bf16_bits(gr[co]);   // exact: bf16 values
#pragma unroll
    for (int k = 0; k < kXPerThread; ++k) {
      const int e = threadIdx.x + NTH * k;
      if (e < 4 * (TT + 2) * (TT + 2)) {
        const int ci = e / ((TT + 2) * (TT + 2)), rr = (e / (TT + 2)) % (TT + 2), cc = e % (TT + 2);
        const uint16_t b = bf16_bits(xr[k]);           // round to nearest: the forward's operand
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int c2 = cc - dx;
          if (c2 >= 0 && c2 < TT) xsb[((dx * 4 + ci) * (TT + 2) + rr) * TT + c2] = b;
        }
      }
    }
    if (t + 1 < len) fetch(t + 1);                     // in flight while this frame multiplies
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      // k-step: pixel rows 4 wave + 2q, +1; lane group g takes 8 pixels of
      // row 4 wave + 2q + g/2 starting at column 8 (g & 1)
      const int row = 4 * wave + 2 * q + (g >> 1), c0 = 8 * (g & 1);
      const u4 a = *reinterpret_cast<const u4*>(gsp + j * TT * TT + row * TT + c0);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        u4 b = u4{0u, 0u, 0u, 0u};
        if (bcol[nt]) b = *reinterpret_cast<const u4*>(xsb + boff[nt] + row * TT + c0);
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b),
                                                          acc[nt], 0, 0, 0);
      }
    }
  }
  // lane (column j, group g) holds dW[co = 4g + r][(ci, tap) = 16 nt + j]
  __syncthreads();
  float* rb = reinterpret_cast<float*>(lds);             // waves 1..3: [wave - 1][lane][8]
  if (wave > 0) {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) rb[((wave - 1) * 64 + lane) * 8 + nt * 4 + r] = acc[nt][r];
  }
  __syncthreads();
  if (wave == 0) {
    float* out = partial + ((size_t)blockIdx.y * gridDim.x + tile) * (4 * 16 * 9);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int idx = 16 * nt + j;
      if (idx < 27) {
        const int ci = idx / 9, tap = idx % 9;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float v = acc[nt][r];
#pragma unroll
          for (int w2 = 0; w2 < 3; ++w2) v += rb[(w2 * 64 + lane) * 8 + nt * 4 + r];
          out[((4 * g + r) * 4 + ci) * 9 + tap] += v;     // [co][ci][tap] with 4 ci slots, as the VALU kernel
        }
      }
    }
  }
}

// acc[e] += sum_b partial[b][e] (e over padded pairs x 9).  A workgroup
// takes 32 consecutive e; each of its 8 b-lanes sums the partials b = lane,
// lane + 8, ... in order, then the 8 lane sums are added in lane order: a
// fixed association, so the result is the same on every run.
constexpr int kRedE = 32, kRedB = 8;
__global__ __launch_bounds__(kRedE * kRedB) void k_dw_reduce(const float* __restrict__ partial, int nblocks,
                                                            int E, float* __restrict__ acc) {
  __shared__ float red[kRedB][kRedE];
  const int el = threadIdx.x % kRedE, bl = threadIdx.x / kRedE;
  const int e = blockIdx.x * kRedE + el;
  float s = 0.f;
  if (e < E) {
    const float* p = partial + e;
#pragma unroll 8
    for (int b = bl; b < nblocks; b += kRedB) s += p[(size_t)b * E];
  }
  red[bl][el] = s;
  __syncthreads();
  if (bl == 0 && e < E) {
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < kRedB; ++k) t += red[k][el];
    acc[e] += t;
  }
}

// grad_w[co][ci][tap] (real layout) from the padded accumulator
__global__ void k_dw_out(const float* __restrict__ acc, int Cout, int Cin, int CINP, float* __restrict__ gw) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= Cout * Cin * 9) return;
  const int tap = e % 9, ci = (e / 9) % Cin, co = e / (9 * Cin);
  gw[e] = acc[(co * CINP + ci) * 9 + tap];
}

struct ConvTArgs {
  const void* gh; int Cout, Cin, len, H, W, tiles_x; const float* wT;
  void* out; long long ons, ots;
  const void* hseg; HTrace ht; int sumc, choff; float* gv; float theta, leak, alpha; int surr, detach;
  int relaxed; float* dw_partial;     // the fused weight gradient of narrow layers
  // the fused input-layer weight gradient (16-wide layer above the input
  // layer): x of the segment, its clip stride, Cin of x, the partial sums
  const float* x1; long long x1_ns; int cin0; float* dw1;
};
template <int CINP, int COUTP, bool B16>
void launch_convT(dim3 g, hipStream_t st, bool adj, const ConvTArgs& a) {
  using HS = typename Store<B16>::H;
  using GS = typename Store<B16>::G;
  const GS* gh = static_cast<const GS*>(a.gh);
  const HS* hseg = static_cast<const HS*>(a.hseg);
  // hidden layers have equal widths, so the matrix-pipe kernel serves 16-wide
  // hidden layers below a 16-wide layer or the output layer
  if constexpr (CINP == 16 && COUTP <= 16) {
    if (adj) {
      if constexpr (COUTP == 16 && !B16) {
        if (a.dw1) {
          hipLaunchKernelGGL((k_convT_mfma<16, B16, true>), g, dim3(NTH), 0, st, gh, a.Cout, a.Cin, a.len, a.H, a.W,
                             a.tiles_x, a.wT, static_cast<GS*>(a.out), hseg, a.ht, a.sumc, a.choff, a.gv, a.theta,
                             a.leak, a.alpha, a.surr, a.detach, a.relaxed, a.dw_partial, a.x1, a.x1_ns, a.cin0, a.dw1);
          return;
        }
      }
      hipLaunchKernelGGL((k_convT_mfma<COUTP, B16>), g, dim3(NTH), 0, st, gh, a.Cout, a.Cin, a.len, a.H, a.W,
                         a.tiles_x, a.wT, static_cast<GS*>(a.out), hseg, a.ht, a.sumc, a.choff, a.gv, a.theta, a.leak,
                         a.alpha, a.surr, a.detach, a.relaxed, a.dw_partial, static_cast<const float*>(nullptr), 0LL,
                         0, static_cast<float*>(nullptr));
      return;
    }
  } else {
    if (adj) {
      hipLaunchKernelGGL((k_convT<CINP, COUTP, true, HS, GS>), g, dim3(NTH), 0, st, gh, a.Cout, a.Cin, a.len, a.H,
                         a.W, a.tiles_x, a.wT, a.out, a.ons, a.ots, hseg, a.ht, a.sumc, a.choff, a.gv, a.theta, a.leak,
                         a.alpha, a.surr, a.detach);
      return;
    }
  }
  hipLaunchKernelGGL((k_convT<CINP, COUTP, false, HS, GS>), g, dim3(NTH), 0, st, gh, a.Cout, a.Cin, a.len, a.H, a.W,
                     a.tiles_x, a.wT, a.out, a.ons, a.ots, hseg, a.ht, a.sumc, a.choff, a.gv, a.theta, a.leak, a.alpha,
                     a.surr, a.detach);
}
template <int CINP, int COUTP, bool B16>
void launch_dw(dim3 g, hipStream_t st, const void* ghv, int Cout, int Cin, int len, int H, int W, int tx,
               const float* x, long long xns, int bfx, const void* hsegv, HTrace ht, int sumc, int choff_in, float theta,
               float alpha, int relaxed, float* partial) {
  using HS = typename Store<B16>::H;
  using GS = typename Store<B16>::G;
  const GS* gh = static_cast<const GS*>(ghv);
  const HS* hseg = static_cast<const HS*>(hsegv);
  if (CINP == 16 && COUTP == 16 && hseg && !relaxed) {   // hard spikes in: bf16 matrix pipe
    hipLaunchKernelGGL(k_dw_mfma<B16>, g, dim3(NTH), 0, st, gh, Cout, Cin, len, H, W, tx, hseg, ht, sumc, choff_in,
                       theta, partial);
    return;
  }
  if constexpr (B16 && CINP == 4 && COUTP == 16) {
    if (!hseg) {                                         // input layer of a BF16 net: bf16 matrix pipe
      hipLaunchKernelGGL(k_dw1_mfma, g, dim3(NTH), 0, st, gh, Cout, Cin, len, H, W, tx, x, xns, partial);
      return;
    }
  }
  if (hseg) {
    hipLaunchKernelGGL((k_dw<CINP, COUTP, HS, GS>), g, dim3(NTH), 0, st, gh, Cout, Cin, len, H, W, tx, x, xns, bfx,
                       hseg, ht, sumc, choff_in, theta, alpha, relaxed, partial);
  } else {
    hipLaunchKernelGGL((k_dw<CINP, COUTP, float, GS>), g, dim3(NTH), 0, st, gh, Cout, Cin, len, H, W, tx, x, xns,
                       bfx, static_cast<const float*>(nullptr), ht, sumc, choff_in, theta, alpha, relaxed, partial);
  }
}

#define EVS_DISPATCH_PAD(CI, CO, CALL)                                   \
  do {                                                                   \
    if (CI == 4 && CO == 2) CALL(4, 2);                                  \
    else if (CI == 4 && CO == 16) CALL(4, 16);                           \
    else if (CI == 4 && CO == 32) CALL(4, 32);                           \
    else if (CI == 16 && CO == 2) CALL(16, 2);                           \
    else if (CI == 16 && CO == 16) CALL(16, 16);                         \
    else if (CI == 16 && CO == 32) CALL(16, 32);                         \
    else if (CI == 32 && CO == 2) CALL(32, 2);                           \
    else if (CI == 32 && CO == 16) CALL(32, 16);                         \
    else CALL(32, 32);                                                   \
  } while (0)

// Planes per frame of the pixel-major segment trace: every hidden layer's
// width rounded up to a multiple of 4, and 4 for the output layer.
int trace_planes(const evs_net& net) {
  int tp = 4;
  for (int l = 1; l < net.n_layers; ++l) tp += (net.ch[l] + 3) & ~3;
  return tp;
}

struct BwdLayout {
  size_t hseg, gv, gh, gh2, partial, acc, wT, lw, total;
  int k, nseg, cmax, tiles_x, tiles_y;
};

BwdLayout layout(const evs_net& net, const evs_clip& c, int k) {
  BwdLayout L{};
  const size_t HW = (size_t)c.H * c.W;
  const int sumc = real_sum_channels(net);
  int cmax = 0, accsum = 0;
  const int tp = trace_planes(net);
  for (int l = 1; l <= net.n_layers; ++l) {
    cmax = net.ch[l] > cmax ? net.ch[l] : cmax;
    const int e = pad_in(net.ch[l - 1]) * pad_out(net.ch[l]) * 9;
    accsum += e;
  }
  L.k = k;
  L.nseg = (c.T + k - 1) / k;
  L.cmax = cmax;
  L.tiles_x = (c.W + TT - 1) / TT;
  L.tiles_y = (c.H + TT - 1) / TT;
  const size_t nblk = (size_t)L.tiles_x * L.tiles_y * c.N;
  // segment potentials and adjoints: fp16 / bf16 for BF16 nets, else float
  const size_t es = net.precision == EVS_BF16 ? 2 : 4;
  size_t o = 0;
  L.hseg = o; o += align256((size_t)c.N * k * tp * HW * es);
  L.gv = o; o += align256((size_t)c.N * sumc * HW * 4);
  L.gh = o; o += align256((size_t)c.N * k * cmax * HW * es);
  L.gh2 = o; o += align256((size_t)c.N * k * cmax * HW * es);
  L.partial = o; o += align256(nblk * accsum * 4);
  L.acc = o; o += align256((size_t)accsum * 4);
  L.wT = o; o += align256((size_t)accsum * 4);
  // the layer-by-layer recompute's own buffers (shapes without fused kernels)
  L.lw = o; o += fused_shape(net) ? 0 : align256(layerwise_workspace_bytes(net, c.N, c.H, c.W));
  L.total = o;
  return L;
}

}  // namespace

size_t backward_workspace_bytes(const evs_net& net, const evs_clip& clip, int ckpt_every) {
  if (net.input != EVS_INPUT_DIRECT || validate_clip(net, clip, false) != EVS_OK || ckpt_every < 1) return (size_t)-1;
  return layout(net, clip, ckpt_every < clip.T ? ckpt_every : clip.T).total;
}

// The segment loop of the backward (see the top of this file); B16: the
// storage of BF16 nets (Store<true>).
template <bool B16>
int run_backward(const evs_net& net, const void* packed, const evs_clip& clip, const float* ckpt, int ckpt_every,
                 int k, const BwdLayout& Lo, int nseg_ck, const float* grad_s, float* const* grad_w, float* grad_x,
                 float* grad_v, void* ws, int32_t* status, hipStream_t st) {
  using HS = typename Store<B16>::H;
  using GS = typename Store<B16>::G;
  int rc = 0;
  char* w8 = reinterpret_cast<char*>(ws);
  HS* hseg = reinterpret_cast<HS*>(w8 + Lo.hseg);
  float* gv = reinterpret_cast<float*>(w8 + Lo.gv);
  // g_h of layer l and of the layer below, swapped after each layer
  GS* ghb[2] = {reinterpret_cast<GS*>(w8 + Lo.gh), reinterpret_cast<GS*>(w8 + Lo.gh2)};
  float* partial = reinterpret_cast<float*>(w8 + Lo.partial);
  float* acc = reinterpret_cast<float*>(w8 + Lo.acc);
  float* wT = reinterpret_cast<float*>(w8 + Lo.wT);
  const int N = clip.N, T = clip.T, H = clip.H, W = clip.W, L = net.n_layers;
  const long long HW = (long long)H * W;
  const int sumc = real_sum_channels(net);
  const int cin0 = net.ch[0], cout = net.ch[L];
  const bool bf = net.precision == EVS_BF16;
  const FwdNetArgs na = make_net_args(net, packed);
  const float* wbase = reinterpret_cast<const float*>(packed);
  int choff[kMaxLayers + 1] = {};
  for (int l = 1; l < L; ++l) choff[l] = choff[l - 1] + net.ch[l];   // choff[l-1] = offset of layer l
  // the layers' blocks in the pixel-major segment trace: ht[l - 1] is layer l
  const int tpf = trace_planes(net);
  HTrace ht[kMaxLayers];
  for (int l = 1, o = 0; l <= L; ++l) {
    const int cw = l == L ? 4 : (net.ch[l] + 3) & ~3;
    ht[l - 1] = HTrace{tpf, o, cw};
    o += cw;
  }
  int accofs[kMaxLayers + 1] = {};
  for (int l = 1; l <= L; ++l) accofs[l] = accofs[l - 1] + pad_in(net.ch[l - 1]) * pad_out(net.ch[l]) * 9;

  if ((rc = zero_f32(gv, (size_t)N * sumc * HW, st))) return rc;
  if ((rc = zero_f32(acc, (size_t)accofs[L], st))) return rc;
  // per-workgroup dW partial sums of every layer, [layer][block][E_l],
  // accumulated over the segments and reduced once at the end
  const size_t nblk = (size_t)Lo.tiles_x * Lo.tiles_y * N;
  if ((rc = zero_f32(partial, nblk * accofs[L], st))) return rc;
  for (int l = 1; l <= L; ++l) {
    const int CI = pad_in(net.ch[l - 1]), CO = pad_out(net.ch[l]);
    hipLaunchKernelGGL(k_pack_wT, dim3((9 * CI * CO + 255) / 256), dim3(256), 0, st, wbase + na.wofs[l - 1],
                       net.ch[l], net.ch[l - 1], CI, CO, bf ? 1 : 0, wT + accofs[l - 1]);
    EVS_HIP(hipGetLastError());
  }
  const bool fused = fused_shape(net);
  const int tile = fused ? choose_tile(net, H, W, N) : -1;
  int th = 0, tw = 0;
  if (fused) {
    forward_tile_dims(net, tile, &th, &tw);
    if (th == 0) return fail(EVS_EUNSUPPORTED, "backward: no forward kernel for this network");
  }

  for (int s = Lo.nseg - 1; s >= 0; --s) {
    const int t0 = s * k;
    const int len = (t0 + k <= T ? k : T - t0);
    // 1. recompute the segment's potentials from its checkpoint (the forward
    // stored one state every ckpt_every frames)
    if (t0 % ckpt_every != 0) return fail(EVS_EINVAL, "backward: segment start is not a checkpoint");
    if (!fused) {
      LwClip lc{};
      lc.N = N; lc.T = len; lc.H = H; lc.W = W;
      lc.x = clip.x + (size_t)t0 * cin0 * HW;
      lc.x_nstride = (long long)T * cin0 * HW;
      lc.v_in = ckpt + (size_t)(t0 / ckpt_every) * sumc * HW;
      lc.vin_nstride = (long long)nseg_ck * sumc * HW;
      lc.rtrace = hseg;
      lc.rt_f16 = B16 ? 1 : 0;
      lc.rt_nstride = (long long)len * tpf * HW;
      if ((rc = layerwise_forward(net, wbase, lc, w8 + Lo.lw, st))) return rc;
    } else {
      FwdClipArgs ca{};
      ca.x = clip.x + (size_t)t0 * cin0 * HW;
      ca.x_nstride = (long long)T * cin0 * HW;
      // checkpoint index: the forward stored one state every ckpt_every frames
      ca.v_in = ckpt + (size_t)(t0 / ckpt_every) * sumc * HW;
      ca.vin_nstride = (long long)nseg_ck * sumc * HW;
      ca.h_trace = reinterpret_cast<float*>(hseg);
      ca.trace_f16 = B16 ? 1 : 0;
      ca.trace_pm = 1;
      ca.trace_nstride = (long long)len * tpf * HW;
      ca.tb_y0 = 0; ca.tb_x0 = 0; ca.tb_h = H; ca.tb_w = W;
      ca.N = N; ca.T = len; ca.H = H; ca.W = W;
      ca.tiles_x = (W + tw - 1) / tw;
      ca.tiles_y = (H + th - 1) / th;
      if ((rc = launch_forward(net, na, ca, tile, st))) return rc;
    }

    // 2-4. layers L..1: the top layer's adjoint scan reads grad_s; each
    // lower layer's scan runs inside the conv-transpose of the layer above
    {
      const int C = net.ch[L];
      const long long tot = (long long)N * C * HW;
      hipLaunchKernelGGL((k_adjoint<HS, GS>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, hseg, ht[L - 1], sumc,
                         choff[L - 1], C, len, N, (int)HW, grad_s + (size_t)t0 * cout * HW, (long long)T * cout * HW,
                         (long long)cout * HW, ghb[0], gv, net.theta, net.leak, net.surr_alpha, net.surrogate,
                         net.detach_reset, status);
      EVS_HIP(hipGetLastError());
    }
    int cur = 0;
    bool dw1_done = false;
    for (int l = L; l >= 1; --l) {
      const int C = net.ch[l], Cin = net.ch[l - 1];
      GS* gh = ghb[cur];
      // weight gradient partials for this segment (a narrow layer above a
      // 16-wide one forms them inside its conv-transpose), then the
      // fixed-order reduction; then the g_h of the layer below (the
      // conv-transpose and that layer's adjoint scan), or grad_x
      const int CI = pad_in(Cin), CO = pad_out(C);
      const bool fused_dw = (l >= 2 && CI == 16 && CO <= 4) || (l == 1 && dw1_done);
      // FP32 nets: a 16-wide layer 2 over the input layer forms the input
      // layer's weight gradient inside its conv-transpose (BF16 nets keep
      // their separate bf16 kernel, faster than FP32 MFMAs at the fused
      // kernel's lower occupancy)
      const bool fuse_dw1 = !B16 && l == 2 && CI == 16 && CO == 16 && pad_in(net.ch[0]) == 4;
      const dim3 gdw((unsigned)(Lo.tiles_x * Lo.tiles_y), (unsigned)N);
      if (!fused_dw) {
        const HS* hin = l >= 2 ? hseg : nullptr;
        const int choff_in = l >= 2 ? choff[l - 2] : 0;
#define EVS_CALL_DW(A, B)                                                                              \
  launch_dw<A, B, B16>(gdw, st, gh, C, Cin, len, H, W, Lo.tiles_x, clip.x + (size_t)t0 * cin0 * HW,          \
                  (long long)T * cin0 * HW, bf ? 1 : 0, hin, ht[l >= 2 ? l - 2 : 0], sumc, choff_in, net.theta, net.surr_alpha, \
                  net.relaxed ? 1 + net.surrogate : 0, partial + nblk * accofs[l - 1])
        EVS_DISPATCH_PAD(CI, CO, EVS_CALL_DW);
#undef EVS_CALL_DW
        EVS_HIP(hipGetLastError());
      }
      const bool convt = l >= 2 || grad_x;
      if (convt) {
        ConvTArgs a{};
        a.gh = gh; a.Cout = C; a.Cin = Cin; a.len = len; a.H = H; a.W = W; a.tiles_x = Lo.tiles_x;
        a.wT = wT + accofs[l - 1];
        a.theta = net.theta; a.leak = net.leak; a.alpha = net.surr_alpha; a.surr = net.surrogate;
        a.detach = net.detach_reset; a.sumc = sumc;
        a.relaxed = net.relaxed ? 1 + net.surrogate : 0;
        a.dw_partial = partial + nblk * accofs[l - 1];
        if (l >= 2) {
          a.out = ghb[cur ^ 1];
          a.hseg = hseg; a.ht = ht[l - 2]; a.choff = choff[l - 2]; a.gv = gv;
          if (fuse_dw1) {
            a.x1 = clip.x + (size_t)t0 * cin0 * HW;
            a.x1_ns = (long long)T * cin0 * HW;
            a.cin0 = cin0;
            a.dw1 = partial;                           // layer 1's slots: accofs[0] = 0
            if (!grad_x) a.out = nullptr;              // g_h1 only feeds the input gradient
            dw1_done = true;
          }
        } else {
          a.out = grad_x + (size_t)t0 * cin0 * HW;
          a.ons = (long long)T * cin0 * HW;
          a.ots = (long long)cin0 * HW;
        }
        const dim3 gct((unsigned)(Lo.tiles_x * Lo.tiles_y), (unsigned)N);
#define EVS_CALL_CT(A, B) launch_convT<A, B, B16>(gct, st, l >= 2, a)
        EVS_DISPATCH_PAD(CI, CO, EVS_CALL_CT);
#undef EVS_CALL_CT
        EVS_HIP(hipGetLastError());
      }
      if (convt) {
        cur ^= 1;
      }
    }
  }
  // the fixed-order reduction of each layer's partial sums, then outputs
  for (int l = 1; l <= L; ++l) {
    const int E = accofs[l] - accofs[l - 1];
    hipLaunchKernelGGL(k_dw_reduce, dim3((E + kRedE - 1) / kRedE), dim3(kRedE * kRedB), 0, st,
                       partial + nblk * accofs[l - 1], (int)nblk, E, acc + accofs[l - 1]);
    EVS_HIP(hipGetLastError());
  }
  for (int l = 1; l <= L; ++l) {
    const int E = net.ch[l] * net.ch[l - 1] * 9;
    hipLaunchKernelGGL(k_dw_out, dim3((E + 255) / 256), dim3(256), 0, st, acc + accofs[l - 1], net.ch[l],
                       net.ch[l - 1], pad_in(net.ch[l - 1]), grad_w[l - 1]);
    EVS_HIP(hipGetLastError());
  }
  if (grad_v) {
    if ((rc = copy_f32(grad_v, gv, (size_t)N * sumc * HW, st))) return rc;
  }
  return EVS_OK;
}

int backward(const evs_net& net, const void* packed, const evs_clip& clip, const float* ckpt, int ckpt_every,
             const float* grad_s, float* const* grad_w, float* grad_x, float* grad_v, void* ws, size_t ws_bytes,
             int32_t* status, hipStream_t st) {
  int rc = validate_net(&net);
  if (rc) return rc;
  if (net.input != EVS_INPUT_DIRECT)
    return fail(EVS_EUNSUPPORTED, "backward: direct input only (pass the output of evs_logdiff)");
  if ((rc = validate_clip(net, clip, true))) return rc;
  if (!packed || !ckpt || !grad_s || !grad_w) return fail(EVS_EINVAL, "backward: NULL argument");
  if (ckpt_every < 1) return fail(EVS_EINVAL, "backward: ckpt_every must be >= 1");
  if ((reinterpret_cast<uintptr_t>(status) & 3u) != 0) return fail(EVS_EINVAL, "backward: dev_status must be 4-byte aligned");
  for (int l = 0; l < net.n_layers; ++l)
    if (!grad_w[l]) return fail(EVS_EINVAL, "backward: NULL grad_w entry");
  // the gradient kernels address a frame's planes of one layer with 32-bit
  // byte offsets
  if ((size_t)32 * clip.H * clip.W * 4 >= ((size_t)1 << 31))
    return fail(EVS_EUNSUPPORTED, "backward: frame too large (32 x H x W x 4 bytes must stay below 2 GiB)");
  const int k = ckpt_every < clip.T ? ckpt_every : clip.T;
  const BwdLayout Lo = layout(net, clip, k);
  if (!ws || ws_bytes < Lo.total) return fail(EVS_EWORKSPACE, "backward: workspace too small");
  // the checkpoints were written with ceil(T / ckpt_every) segments
  const int nseg_ck = (clip.T + ckpt_every - 1) / ckpt_every;
  if (net.precision == EVS_BF16)
    return run_backward<true>(net, packed, clip, ckpt, ckpt_every, k, Lo, nseg_ck, grad_s, grad_w, grad_x, grad_v, ws,
                              status, st);
  return run_backward<false>(net, packed, clip, ckpt, ckpt_every, k, Lo, nseg_ck, grad_s, grad_w, grad_x, grad_v, ws,
                             status, st);
}

}  // namespace evs
