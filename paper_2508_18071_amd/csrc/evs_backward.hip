// Surrogate-gradient BPTT backward of EvSNet (arXiv 2508.18071, Sec. 3.3,
// Eq. 4), with membrane checkpoints every k frames.
//
// Segments of k frames are visited from the last to the first.  For each:
//   1. the forward kernel recomputes the segment's charged potentials h of
//      every layer from the segment's checkpoint (bit-identical to the
//      original forward: same kernel, same state);
//   2. for layers L..1: a reverse-time adjoint scan per neuron
//          g_h = (G - theta g_v) psi(h) + g_v     (G psi(h) + g_v detached)
//          g_v <- leak * g_h
//      with g_v carried across segment boundaries;
//   3. the weight gradient dW[co][ci][tap] = sum_t,p g_h[co][p] s_in[ci][p+tap]
//      as per-tile partial sums in registers, reduced in a fixed order (no
//      float atomics: results are bitwise reproducible);
//   4. the incoming gradient of the layer below, G = conv_transpose(g_h, W)
//      (grad_x for layer 1).
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

__device__ inline float wq(const float* w, int idx, bool bf) {
  const float v = w[idx];
  return bf ? round_bf16(v) : v;
}

// ---------------------------------------------------------------- adjoint scan
__global__ __launch_bounds__(256) void k_adjoint(const float* __restrict__ hseg, int sumc, int choff, int C,
                                                 int len, int N, int HW, const float* __restrict__ G,
                                                 long long G_nstride, long long G_tstride,
                                                 float* __restrict__ gh, float* __restrict__ gv, float theta,
                                                 float leak, float alpha, int surr, int detach) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long total = (long long)N * C * HW;
  if (idx >= total) return;
  const int p = (int)(idx % HW);
  const int c = (int)((idx / HW) % C);
  const int n = (int)(idx / ((long long)HW * C));
  float* gvp = gv + ((size_t)n * sumc + choff + c) * HW + p;
  float g_v = *gvp;
  for (int t = len - 1; t >= 0; --t) {
    const float h = hseg[(((size_t)n * len + t) * sumc + choff + c) * HW + p];
    const float Gv = G[(size_t)n * G_nstride + (size_t)t * G_tstride + (size_t)c * HW + p];
    const float psi = surrogate(h, theta, alpha, surr);
    const float g_h = detach ? fmaf(Gv, psi, g_v) : fmaf(fmaf(-theta, g_v, Gv), psi, g_v);
    gh[(((size_t)n * len + t) * C + c) * HW + p] = g_h;
    g_v = leak * g_h;
  }
  *gvp = g_v;
}

// ---------------------------------------------------------------- conv transpose
// out[n][t][ci][y][x] = sum_{co,tap} W[co][ci][tap] * gh[n][t][co][y-dy][x-dx]
template <int CINP, int COUTP>
__global__ __launch_bounds__(NTH) void k_convT(const float* __restrict__ gh, int Cout, int Cin, int len,
                                               int H, int W, int tiles_x, const float* __restrict__ w, int bf,
                                               float* __restrict__ out, long long out_nstride,
                                               long long out_tstride) {
  __shared__ float ghs[COUTP][TT + 2][TT + 2];
  __shared__ __attribute__((aligned(16))) float wls[9][COUTP][CINP];
  const int tile = blockIdx.x, t = blockIdx.y, n = blockIdx.z;
  const int ty0 = (tile / tiles_x) * TT, tx0 = (tile % tiles_x) * TT;
  const int HW = H * W;
  const float* g = gh + ((size_t)n * len + t) * Cout * HW;
  for (int e = threadIdx.x; e < COUTP * (TT + 2) * (TT + 2); e += NTH) {
    const int co = e / ((TT + 2) * (TT + 2)), r = (e / (TT + 2)) % (TT + 2), cc = e % (TT + 2);
    const int y = ty0 - 1 + r, x = tx0 - 1 + cc;
    ghs[co][r][cc] = (co < Cout && y >= 0 && y < H && x >= 0 && x < W) ? g[(size_t)co * HW + y * W + x] : 0.f;
  }
  for (int e = threadIdx.x; e < 9 * COUTP * CINP; e += NTH) {
    const int ci = e % CINP, co = (e / CINP) % COUTP, tap = e / (CINP * COUTP);
    wls[tap][co][ci] = (co < Cout && ci < Cin) ? wq(w, (co * Cin + ci) * 9 + tap, bf) : 0.f;
  }
  __syncthreads();
  const int ty = threadIdx.x / TT, tx = threadIdx.x % TT;
  float acc[CINP];
#pragma unroll
  for (int ci = 0; ci < CINP; ++ci) acc[ci] = 0.f;
  for (int co = 0; co < Cout; ++co) {
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      const float gv = ghs[co][ty + 1 - dy][tx + 1 - dx];
#pragma unroll
      for (int ci = 0; ci < CINP; ++ci) acc[ci] = fmaf(wls[tap][co][ci], gv, acc[ci]);
    }
  }
  const int y = ty0 + ty, x = tx0 + tx;
  if (y < H && x < W) {
    float* o = out + (size_t)n * out_nstride + (size_t)t * out_tstride + (size_t)y * W + x;
#pragma unroll
    for (int ci = 0; ci < CINP; ++ci)
      if (ci < Cin) o[(size_t)ci * HW] = acc[ci];
  }
}

// ---------------------------------------------------------------- weight gradient
// Per (tile, clip) workgroup over all frames of the segment: partial
// dW[co][ci][tap] in registers; s_in is x (layer 1) or the spikes of the
// layer below recomputed from its h.
template <int CINP, int COUTP>
__global__ __launch_bounds__(NTH) void k_dw(const float* __restrict__ gh, int Cout, int Cin, int len, int H,
                                            int W, int tiles_x, const float* __restrict__ x,
                                            long long x_nstride, int bf_x, const float* __restrict__ hseg,
                                            int sumc, int choff_in, float theta, float alpha, int relaxed,
                                            float* __restrict__ partial) {
  constexpr int P = CINP * COUTP;                     // (co, ci) pairs
  constexpr int PPT = P >= NTH ? P / NTH : 1;         // pairs per thread
  constexpr int TPP = P >= NTH ? 1 : NTH / P;         // threads per pair
  __shared__ float ghs[COUTP][TT * TT];
  __shared__ float ss[CINP][TT + 2][TT + 2];
  __shared__ float red[TPP > 1 ? NTH * 9 : 1];
  const int tile = blockIdx.x, n = blockIdx.y;
  const int ty0 = (tile / tiles_x) * TT, tx0 = (tile % tiles_x) * TT;
  const int HW = H * W;
  float acc[PPT][9];
#pragma unroll
  for (int k = 0; k < PPT; ++k)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) acc[k][tap] = 0.f;
  const int sub = TPP > 1 ? threadIdx.x / P : 0;      // row subset of this thread
  for (int t = 0; t < len; ++t) {
    __syncthreads();
    const float* g = gh + ((size_t)n * len + t) * Cout * HW;
    for (int e = threadIdx.x; e < COUTP * TT * TT; e += NTH) {
      const int co = e / (TT * TT), r = (e / TT) % TT, cc = e % TT;
      const int y = ty0 + r, xx = tx0 + cc;
      ghs[co][r * TT + cc] = (co < Cout && y < H && xx < W) ? g[(size_t)co * HW + y * W + xx] : 0.f;
    }
    for (int e = threadIdx.x; e < CINP * (TT + 2) * (TT + 2); e += NTH) {
      const int ci = e / ((TT + 2) * (TT + 2)), r = (e / (TT + 2)) % (TT + 2), cc = e % (TT + 2);
      const int y = ty0 - 1 + r, xx = tx0 - 1 + cc;
      float v = 0.f;
      if (ci < Cin && y >= 0 && y < H && xx >= 0 && xx < W) {
        if (hseg) {
          const float h = hseg[(((size_t)n * len + t) * sumc + choff_in + ci) * HW + (size_t)y * W + xx];
          v = spike_of(h, theta, alpha, relaxed);
        } else {
          v = x[(size_t)n * x_nstride + ((size_t)t * Cin + ci) * HW + (size_t)y * W + xx];
          if (bf_x) v = round_bf16(v);
        }
      }
      ss[ci][r][cc] = v;
    }
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
  float* out = partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * P * 9;
  if constexpr (TPP > 1) {
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) red[threadIdx.x * 9 + tap] = acc[0][tap];
    __syncthreads();
    if (threadIdx.x < P) {
      for (int tap = 0; tap < 9; ++tap) {
        float sacc = 0.f;
        for (int s2 = 0; s2 < TPP; ++s2) sacc += red[(s2 * P + threadIdx.x) * 9 + tap];
        out[threadIdx.x * 9 + tap] = sacc;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < PPT; ++k)
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) out[(threadIdx.x + NTH * k) * 9 + tap] = acc[k][tap];
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
// the end (fixed association: reproducible).
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
constexpr int kGspBytes = 3 * 16 * TT * TT * 2;          // g_h parts [part][co][pixel]
constexpr int kSsbBytes = 3 * 16 * (TT + 2) * TT * 2;    // spikes [dx][ci][row][col]
constexpr int kSsPerThread = (16 * (TT + 2) * (TT + 2) + NTH - 1) / NTH;
__device__ inline uint16_t bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

__global__ __launch_bounds__(NTH) void k_dw_mfma(const float* __restrict__ gh, int Cout, int Cin, int len, int H,
                                                 int W, int tiles_x, const float* __restrict__ hseg, int sumc,
                                                 int choff_in, float theta, float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) char lds[kGspBytes + kSsbBytes];
  uint16_t* const gsp = reinterpret_cast<uint16_t*>(lds);
  uint16_t* const ssb = reinterpret_cast<uint16_t*>(lds + kGspBytes);
  const int tile = blockIdx.x, n = blockIdx.y;
  const int ty0 = (tile / tiles_x) * TT, tx0 = (tile % tiles_x) * TT;
  const int HW = H * W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  // staging: this thread's g_h pixel (all 16 channels) and spike-tile entries
  const int gy = ty0 + threadIdx.x / TT, gx = tx0 + threadIdx.x % TT;
  const bool gin = gy < H && gx < W;
  float gr[16], hr[kSsPerThread];
  auto fetch = [&](int t) __attribute__((always_inline)) {
    const float* gf = gh + ((size_t)n * len + t) * Cout * HW + (size_t)gy * W + gx;
#pragma unroll
    for (int co = 0; co < 16; ++co) gr[co] = (co < Cout && gin) ? gf[(size_t)co * HW] : 0.f;
#pragma unroll
    for (int k = 0; k < kSsPerThread; ++k) {
      const int e = threadIdx.x + NTH * k;
      const int ci = e / ((TT + 2) * (TT + 2)), rr = (e / (TT + 2)) % (TT + 2), cc = e % (TT + 2);
      const int y = ty0 - 1 + rr, xx = tx0 - 1 + cc;
      const bool in = e < 16 * (TT + 2) * (TT + 2) && ci < Cin && y >= 0 && y < H && xx >= 0 && xx < W;
      // out-of-image entries hold a value whose spike is 0
      hr[k] = in ? hseg[(((size_t)n * len + t) * sumc + choff_in + ci) * HW + (size_t)y * W + xx] : 0.f;
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
      const float h = (float)(__bf16)v, r = v - h, m = (float)(__bf16)r;
      gsp[(0 * 16 + co) * TT * TT + threadIdx.x] = bf16_bits(h);
      gsp[(1 * 16 + co) * TT * TT + threadIdx.x] = bf16_bits(m);
      gsp[(2 * 16 + co) * TT * TT + threadIdx.x] = bf16_bits(r - m);
    }
#pragma unroll
    for (int k = 0; k < kSsPerThread; ++k) {
      const int e = threadIdx.x + NTH * k;
      if (e < 16 * (TT + 2) * (TT + 2)) {
        const int ci = e / ((TT + 2) * (TT + 2)), rr = (e / (TT + 2)) % (TT + 2), cc = e % (TT + 2);
        const uint16_t b = bf16_bits(spike_of(hr[k], theta, 0.f, 0));
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int c2 = cc - dx;
          if (c2 >= 0 && c2 < TT) ssb[((dx * 16 + ci) * (TT + 2) + rr) * TT + c2] = b;
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
      u4 a[3];
#pragma unroll
      for (int b = 0; b < 3; ++b) a[b] = *reinterpret_cast<const u4*>(gsp + (b * 16 + j) * TT * TT + row * TT + c0);
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
        const u4 bv = *reinterpret_cast<const u4*>(ssb + ((dx * 16 + j) * (TT + 2) + row + dy) * TT + c0);
#pragma unroll
        for (int b = 0; b < 3; ++b)
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
    float* out = partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 256 * 9;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[tap][r];
#pragma unroll
        for (int w2 = 0; w2 < 3; ++w2) v += rb[(w2 * 64 + lane) * 36 + tap * 4 + r];
        out[((4 * g + r) * 16 + j) * 9 + tap] = v;
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

template <int CINP, int COUTP>
void launch_convT(dim3 g, hipStream_t st, const float* gh, int Cout, int Cin, int len, int H, int W, int tx,
                  const float* w, int bf, float* out, long long ons, long long ots) {
  hipLaunchKernelGGL((k_convT<CINP, COUTP>), g, dim3(NTH), 0, st, gh, Cout, Cin, len, H, W, tx, w, bf, out, ons,
                     ots);
}
template <int CINP, int COUTP>
void launch_dw(dim3 g, hipStream_t st, const float* gh, int Cout, int Cin, int len, int H, int W, int tx,
               const float* x, long long xns, int bfx, const float* hseg, int sumc, int choff_in, float theta,
               float alpha, int relaxed, float* partial) {
  if (CINP == 16 && COUTP == 16 && hseg && !relaxed) {   // hard spikes in: bf16 matrix pipe
    hipLaunchKernelGGL(k_dw_mfma, g, dim3(NTH), 0, st, gh, Cout, Cin, len, H, W, tx, hseg, sumc, choff_in, theta,
                       partial);
    return;
  }
  hipLaunchKernelGGL((k_dw<CINP, COUTP>), g, dim3(NTH), 0, st, gh, Cout, Cin, len, H, W, tx, x, xns, bfx, hseg,
                     sumc, choff_in, theta, alpha, relaxed, partial);
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

struct BwdLayout {
  size_t hseg, gv, gh, ga, gb, partial, acc, total;
  int k, nseg, cmax, tiles_x, tiles_y;
};

BwdLayout layout(const evs_net& net, const evs_clip& c, int k) {
  BwdLayout L{};
  const size_t HW = (size_t)c.H * c.W;
  const int sumc = real_sum_channels(net);
  int cmax = 0, emax = 0, accsum = 0;
  for (int l = 1; l <= net.n_layers; ++l) {
    cmax = net.ch[l] > cmax ? net.ch[l] : cmax;
    const int e = pad_in(net.ch[l - 1]) * pad_out(net.ch[l]) * 9;
    emax = e > emax ? e : emax;
    accsum += e;
  }
  L.k = k;
  L.nseg = (c.T + k - 1) / k;
  L.cmax = cmax;
  L.tiles_x = (c.W + TT - 1) / TT;
  L.tiles_y = (c.H + TT - 1) / TT;
  const size_t nblk = (size_t)L.tiles_x * L.tiles_y * c.N;
  size_t o = 0;
  L.hseg = o; o += align256((size_t)c.N * k * sumc * HW * 4);
  L.gv = o; o += align256((size_t)c.N * sumc * HW * 4);
  L.gh = o; o += align256((size_t)c.N * k * cmax * HW * 4);
  L.ga = o; o += align256((size_t)c.N * k * cmax * HW * 4);
  L.gb = o; o += align256((size_t)c.N * k * cmax * HW * 4);
  L.partial = o; o += align256(nblk * emax * 4);
  L.acc = o; o += align256((size_t)accsum * 4);
  L.total = o;
  return L;
}

}  // namespace

size_t backward_workspace_bytes(const evs_net& net, const evs_clip& clip, int ckpt_every) {
  if (net.input != EVS_INPUT_DIRECT || validate_clip(net, clip, false) != EVS_OK || ckpt_every < 1) return (size_t)-1;
  return layout(net, clip, ckpt_every < clip.T ? ckpt_every : clip.T).total;
}

int backward(const evs_net& net, const void* packed, const evs_clip& clip, const float* ckpt, int ckpt_every,
             const float* grad_s, float* const* grad_w, float* grad_x, float* grad_v, void* ws, size_t ws_bytes,
             hipStream_t st) {
  int rc = validate_net(&net);
  if (rc) return rc;
  if (net.input != EVS_INPUT_DIRECT)
    return fail(EVS_EUNSUPPORTED, "backward: direct input only (pass the output of evs_logdiff)");
  if ((rc = validate_clip(net, clip, true))) return rc;
  if (!packed || !ckpt || !grad_s || !grad_w) return fail(EVS_EINVAL, "backward: NULL argument");
  if (ckpt_every < 1) return fail(EVS_EINVAL, "backward: ckpt_every must be >= 1");
  for (int l = 0; l < net.n_layers; ++l)
    if (!grad_w[l]) return fail(EVS_EINVAL, "backward: NULL grad_w entry");
  const int k = ckpt_every < clip.T ? ckpt_every : clip.T;
  const BwdLayout Lo = layout(net, clip, k);
  if (!ws || ws_bytes < Lo.total) return fail(EVS_EWORKSPACE, "backward: workspace too small");
  // the checkpoints were written with ceil(T / ckpt_every) segments
  const int nseg_ck = (clip.T + ckpt_every - 1) / ckpt_every;
  char* w8 = reinterpret_cast<char*>(ws);
  float* hseg = reinterpret_cast<float*>(w8 + Lo.hseg);
  float* gv = reinterpret_cast<float*>(w8 + Lo.gv);
  float* gh = reinterpret_cast<float*>(w8 + Lo.gh);
  float* Gbuf[2] = {reinterpret_cast<float*>(w8 + Lo.ga), reinterpret_cast<float*>(w8 + Lo.gb)};
  float* partial = reinterpret_cast<float*>(w8 + Lo.partial);
  float* acc = reinterpret_cast<float*>(w8 + Lo.acc);
  const int N = clip.N, T = clip.T, H = clip.H, W = clip.W, L = net.n_layers;
  const long long HW = (long long)H * W;
  const int sumc = real_sum_channels(net);
  const int cin0 = net.ch[0], cout = net.ch[L];
  const bool bf = net.precision == EVS_BF16;
  const FwdNetArgs na = make_net_args(net, packed);
  const float* wbase = reinterpret_cast<const float*>(packed);
  int choff[4] = {0, 0, 0, 0};
  for (int l = 1; l < L; ++l) choff[l] = choff[l - 1] + net.ch[l];   // choff[l-1] = offset of layer l
  int accofs[4] = {0, 0, 0, 0};
  for (int l = 1; l <= L; ++l) accofs[l] = accofs[l - 1] + pad_in(net.ch[l - 1]) * pad_out(net.ch[l]) * 9;

  if ((rc = zero_f32(gv, (size_t)N * sumc * HW, st))) return rc;
  if ((rc = zero_f32(acc, (size_t)accofs[L], st))) return rc;
  const int tile = choose_tile(net, H, W);
  int th = 0, tw = 0;
  forward_tile_dims(net, tile, &th, &tw);
  if (th == 0) return fail(EVS_EUNSUPPORTED, "backward: no forward kernel for this network");
  const dim3 gconv((unsigned)(Lo.tiles_x * Lo.tiles_y), 1, (unsigned)N);

  for (int s = Lo.nseg - 1; s >= 0; --s) {
    const int t0 = s * k;
    const int len = (t0 + k <= T ? k : T - t0);
    // 1. recompute the segment's potentials from its checkpoint
    FwdClipArgs ca{};
    ca.x = clip.x + (size_t)t0 * cin0 * HW;
    ca.x_nstride = (long long)T * cin0 * HW;
    // checkpoint index: the forward stored one state every ckpt_every frames
    if (t0 % ckpt_every != 0) return fail(EVS_EINVAL, "backward: segment start is not a checkpoint");
    ca.v_in = ckpt + (size_t)(t0 / ckpt_every) * sumc * HW;
    ca.vin_nstride = (long long)nseg_ck * sumc * HW;
    ca.h_trace = hseg;
    ca.trace_nstride = (long long)len * sumc * HW;
    ca.tb_y0 = 0; ca.tb_x0 = 0; ca.tb_h = H; ca.tb_w = W;
    ca.N = N; ca.T = len; ca.H = H; ca.W = W;
    ca.tiles_x = (W + tw - 1) / tw;
    ca.tiles_y = (H + th - 1) / th;
    if ((rc = launch_forward(net, na, ca, tile, st))) return rc;

    // 2-4. layers L..1
    const float* G = grad_s + (size_t)t0 * cout * HW;
    long long G_ns = (long long)T * cout * HW, G_ts = (long long)cout * HW;
    int gsel = 0;
    for (int l = L; l >= 1; --l) {
      const int C = net.ch[l], Cin = net.ch[l - 1];
      const long long tot = (long long)N * C * HW;
      hipLaunchKernelGGL(k_adjoint, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, hseg, sumc,
                         choff[l - 1], C, len, N, (int)HW, G, G_ns, G_ts, gh, gv, net.theta, net.leak,
                         net.surr_alpha, net.surrogate, net.detach_reset);
      EVS_HIP(hipGetLastError());
      // weight gradient partials for this segment, then fixed-order reduction
      const int CI = pad_in(Cin), CO = pad_out(C);
      const dim3 gdw((unsigned)(Lo.tiles_x * Lo.tiles_y), (unsigned)N);
      const float* hin = l >= 2 ? hseg : nullptr;
      const int choff_in = l >= 2 ? choff[l - 2] : 0;
#define EVS_CALL_DW(A, B)                                                                              \
  launch_dw<A, B>(gdw, st, gh, C, Cin, len, H, W, Lo.tiles_x, clip.x + (size_t)t0 * cin0 * HW,          \
                  (long long)T * cin0 * HW, bf ? 1 : 0, hin, sumc, choff_in, net.theta, net.surr_alpha, \
                  net.relaxed ? 1 + net.surrogate : 0, partial)
      EVS_DISPATCH_PAD(CI, CO, EVS_CALL_DW);
#undef EVS_CALL_DW
      EVS_HIP(hipGetLastError());
      const int E = CI * CO * 9;
      hipLaunchKernelGGL(k_dw_reduce, dim3((E + kRedE - 1) / kRedE), dim3(kRedE * kRedB), 0, st, partial,
                         Lo.tiles_x * Lo.tiles_y * N, E, acc + accofs[l - 1]);
      EVS_HIP(hipGetLastError());
      // gradient for the layer below (or the input)
      if (l >= 2 || grad_x) {
        float* out;
        long long ons, ots;
        if (l >= 2) {
          out = Gbuf[gsel];
          ons = (long long)len * Cin * HW;
          ots = (long long)Cin * HW;
        } else {
          out = grad_x + (size_t)t0 * cin0 * HW;
          ons = (long long)T * cin0 * HW;
          ots = (long long)cin0 * HW;
        }
        const dim3 gct((unsigned)(Lo.tiles_x * Lo.tiles_y), (unsigned)len, (unsigned)N);
        const float* wl = wbase + na.wofs[l - 1];
#define EVS_CALL_CT(A, B) launch_convT<A, B>(gct, st, gh, C, Cin, len, H, W, Lo.tiles_x, wl, bf ? 1 : 0, out, ons, ots)
        EVS_DISPATCH_PAD(CI, CO, EVS_CALL_CT);
#undef EVS_CALL_CT
        EVS_HIP(hipGetLastError());
        if (l >= 2) {
          G = out;
          G_ns = ons;
          G_ts = ots;
          gsel ^= 1;
        }
      }
    }
  }
  // outputs
  for (int l = 1; l <= L; ++l) {
    const int E = net.ch[l] * net.ch[l - 1] * 9;
    hipLaunchKernelGGL(k_dw_out, dim3((E + 255) / 256), dim3(256), 0, st, acc + accofs[l - 1], net.ch[l],
                       net.ch[l - 1], pad_in(net.ch[l - 1]), grad_w[l - 1]);
    EVS_HIP(hipGetLastError());
  }
  if (grad_v) {
    if ((rc = copy_f32(grad_v, gv, (size_t)N * sumc * HW, st))) return rc;
  }
  (void)gconv;
  return EVS_OK;
}

}  // namespace evs
