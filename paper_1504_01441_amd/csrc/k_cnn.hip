// k_cnn.hip -- the learned displacement proposal (an extension beyond the
// paper: a small CNN predicts each level-0 tile's displacement so that the
// Sec. 2.2 search only scans a window around it). Inference and training run
// on the matrix cores: every convolution is an implicit GEMM on
// v_mfma_f32_16x16x16_bf16 (bf16 operands, fp32 accumulation).
//
// Network (per tile): x [16][16][4] -> conv3x3 s1 -> 32 ch [16][16] -> conv s2
// -> [8][8] -> conv s1 -> [8][8] -> conv s2 -> [4][4] -> linear 512 -> 3,
// ReLU after every convolution, activations rounded to bf16; outputs
// (dx / 8, dy / 8, confidence logit). On the device, activations are NHWC
// (32 channels innermost) so that an MFMA operand is one 8-byte load.
//
// MFMA 16x16x16 operand layout (lane l, r = l % 16, g = l / 16, j = 0..3):
//   A[r][4g + j],  B[4g + j][r],  D[4g + j][r].
//
//  k_cnn_pack     fp32 master parameters -> bf16 weight layouts for the kernels
//  k_cnn_input    tile pairs -> network input: the tiles' 2x2 sums and the
//                 64 x 64 windows' 4x4 sums (bf16), for listed tiles
//  k_cnn_fwd      four samples per workgroup at a time, four waves per sample
//                 (each a quarter of every layer's output tiles), weights
//                 shared in LDS;
//                 inference writes the proposal (window centre, fallback
//                 flag), training writes the activations and outputs
//  k_cnn_loss     loss and output gradient per sample
//  k_cnn_bwd      per-sample back-propagation through the ReLUs and the
//                 transposed convolutions (activation gradients)
//  k_cnn_wgrad    weight and bias gradients of one layer, per block of samples
//  k_cnn_head_grad  head gradients
//  k_cnn_adamw    sums the per-block gradients and applies AdamW (fp32)
#include "lnr_internal.h"

namespace lnr {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CH = 32;
constexpr int kWave = 64;
constexpr int kFwdWaves = 16;     // forward workgroup: 4 samples at a time,
constexpr int kFwdGroupWaves = 4;  // four waves per sample

constexpr int C1 = 4;              // input channels
constexpr int kIn = C1 * 256;       // input values per sample

// flat parameter vector: W1[32][4][3][3] b1 W2[32][32][3][3] b2 W3 b3 W4 b4
// Wh[3][512] bh[3]
constexpr int kOffW[4] = {0, 1184, 10432, 19680};
constexpr int kOffB[4] = {1152, 10400, 19648, 28896};
constexpr int kOffWh = 28928, kOffBh = 30464, kNParam = 30467;

// packed bf16 weights: W1p[32 co][48 k] (k = tap * 4 + ci, zero from 36),
// Wp[l][32 co][9 tap][32 ci] and the transposes WT[l][32 ci][9 tap][32 co]
constexpr int kK1 = 48;
constexpr int kW1p = CH * kK1;
constexpr int kWp = CH * 9 * CH;
constexpr int kPacked = kW1p + 3 * kWp + 3 * kWp;

// per-sample stored activations (bf16, NHWC): x, a1, a2, a3, a4
constexpr int kActX = 0, kActA1 = kIn, kActA2 = kActA1 + 8192, kActA3 = kActA2 + 2048,
              kActA4 = kActA3 + 2048, kActN = kActA4 + 512;
// per-sample activation gradients after the ReLU (bf16, channel-major [c][p])
constexpr int kDz1 = 0, kDz2 = 8192, kDz3 = kDz2 + 2048, kDz4 = kDz3 + 2048,
              kDzN = kDz4 + 512;

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ inline bf16x4 ld4(const uint16_t* p) { return *reinterpret_cast<const bf16x4*>(p); }

__global__ __launch_bounds__(256) void k_cnn_pack(const float* __restrict__ P,
                                                  uint16_t* __restrict__ pk) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < kW1p) {
    const int co = i / kK1, k = i % kK1;
    float v = 0.f;
    if (k < 9 * C1) {
      const int tap = k / C1, ci = k % C1;
      v = P[kOffW[0] + (co * C1 + ci) * 9 + tap];
    }
    pk[i] = f2bf(v);
    return;
  }
  int j = i - kW1p;
  if (j >= 6 * kWp) return;
  const bool tr = j >= 3 * kWp;
  if (tr) j -= 3 * kWp;
  const int l = 1 + j / kWp, e = j % kWp;
  int co, tap, ci;
  if (!tr) { co = e / (9 * CH); tap = (e / CH) % 9; ci = e % CH; }
  else { ci = e / (9 * CH); tap = (e / CH) % 9; co = e % CH; }
  pk[i] = f2bf(P[kOffW[l] + (co * CH + ci) * 9 + tap]);
}

// Network inputs: sample i is tile tiles[i] (tile i without a list), i below
// *count (or n). The 64 x 64 windows of both images around the tile (16 px
// on every side; rows and columns outside the image repeat the edge) are
// staged in workgroup memory; channels 0, 1 are the 2x2 sums of the central
// 32 x 32 tile, channels 2, 3 the 4x4 sums of the window, each value
// bf16((s - mid) / scale), exact before the one rounding.
__global__ __launch_bounds__(256) void k_cnn_input(const uint8_t* __restrict__ ref,
                                                   const uint8_t* __restrict__ wrp, int w, int h,
                                                   int ntx, const int32_t* __restrict__ tiles,
                                                   const int* __restrict__ count, int n,
                                                   uint16_t* __restrict__ x) {
  __shared__ uint32_t win[2][64][16];
  const int i = blockIdx.x;
  const int m = count ? *count : n;
  if (i >= m) return;
  const int t = tiles ? tiles[i] : i;
  const int x0 = (t % ntx) * 32 - 16, y0 = (t / ntx) * 32 - 16;
  for (int k = threadIdx.x; k < 2 * 64 * 16; k += 256) {
    const int c = k >> 10, r = (k >> 4) & 63, d = k & 15;
    const uint8_t* img = c ? wrp : ref;
    const int yy = min(max(y0 + r, 0), h - 1);
    const uint8_t* row = img + (size_t)yy * w;
    const int xs = x0 + 4 * d;
    const int off = (int)(reinterpret_cast<uintptr_t>(row + xs) & 3u);
    uint32_t v = 0;
    if (xs >= 0 && (xs - off) + 8 <= w) {
      const uint8_t* base = row + xs - off;  // aligned
      const uint32_t lo = *reinterpret_cast<const uint32_t*>(base);
      const uint32_t hi = *reinterpret_cast<const uint32_t*>(base + 4);
      v = __builtin_amdgcn_alignbyte(hi, lo, off);
    } else {
      for (int b = 0; b < 4; ++b)
        v |= (uint32_t)row[min(max(xs + b, 0), w - 1)] << (8 * b);
    }
    win[c][r][d] = v;
  }
  __syncthreads();
  uint16_t* xo = x + (size_t)i * kIn;
  const uint8_t* wb = reinterpret_cast<const uint8_t*>(win);
  for (int k = threadIdx.x; k < kIn; k += 256) {
    const int c = k >> 8, yi = (k >> 4) & 15, xj = k & 15;
    const int img = c & 1;
    float v;
    if (c < 2) {
      const uint8_t* p0 = wb + (img * 64 + 16 + 2 * yi) * 64 + 16 + 2 * xj;
      const int s = p0[0] + p0[1] + p0[64] + p0[65];
      v = (float)(s - 510) * (1.f / 512.f);
    } else {
      uint32_t s = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        s = __builtin_amdgcn_udot4(win[img][4 * yi + u][xj], 0x01010101u, s, false);
      v = (float)((int)s - 2040) * (1.f / 2048.f);
    }
    xo[k] = f2bf(v);
  }
}

// The forward layers, each computed by the four waves of a sample (part):
// conv1 (2 -> 32, stride 1; K = 18 (tap, ci) padded to 32) four of its 16
// position tiles per wave, the 32 -> 32 layers (3x3, pad 1, stride S, NHWC
// bf16 in / out, W [co][tap][ci]) one position tile per wave, and the last
// layer's two channel halves on parts 0 and 1. Every output element sums its
// MFMA products in (tap, channel half) order.
// In LDS a position's 32 channels take kPS elements (80 bytes) and a weight
// row [tap][ci] kWS elements (592 bytes): the padding spreads the 16 rows of
// an MFMA operand over the banks (unpadded, activation reads conflict ~6-way
// and weight reads 4-way).
constexpr int kPS = 40;
constexpr int kWS = 9 * CH + 8;

__device__ void conv1_fwd_part(const uint16_t* in, const uint16_t* W1p, const float* bias,
                               uint16_t* out, int lane, int part) {
  // K = (tap, ci) = tap * 4 + ci over three steps of 16: step ks covers taps
  // 4 ks .. 4 ks + 3, lane group g one tap's four channels (one 8-byte load)
  const int r = lane & 15, g = lane >> 4;
  const int mt0 = 4 * part;
  const bf16x4 zero = {0, 0, 0, 0};
  f32x4 acc[4][2];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u][0] = acc[u][1] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < 3; ++ks) {
    const int tap = 4 * ks + g;
    const bf16x4 b0 = ld4(W1p + r * kK1 + ks * 16 + g * 4);
    const bf16x4 b1 = ld4(W1p + (16 + r) * kK1 + ks * 16 + g * 4);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int m = (mt0 + u) * 16 + r, oy = m >> 4, ox = m & 15;
      const int iy = oy + tap / 3 - 1, ix = ox + tap % 3 - 1;
      const bool ok = tap < 9 && iy >= 0 && iy < 16 && ix >= 0 && ix < 16;
      const bf16x4 a = ok ? ld4(in + (iy * 16 + ix) * C1) : zero;
      acc[u][0] = mfma(a, b0, acc[u][0]);
      acc[u][1] = mfma(a, b1, acc[u][1]);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int p = (mt0 + u) * 16 + g * 4 + j;
      out[p * kPS + r] = f2bf(fmaxf(acc[u][0][j] + bias[r], 0.f));
      out[p * kPS + 16 + r] = f2bf(fmaxf(acc[u][1][j] + bias[16 + r], 0.f));
    }
}

template <int HIN, int HOUT, int S>
__device__ void conv_fwd_part(const uint16_t* in, const uint16_t* W, const float* bias,
                              uint16_t* out, int lane, int part) {
  const int r = lane & 15, g = lane >> 4;
  constexpr int MT = HOUT * HOUT / 16;
  static_assert(MT == 4 || MT == 1, "position tiles per sample");
  // MT == 4: position tile `part`, both channel halves; MT == 1: channel half
  // `part` of the single position tile (parts 2, 3 idle)
  if (MT == 1 && part >= 2) return;
  const int mt = MT == 4 ? part : 0;
  const int n0 = MT == 4 ? 0 : part, n1 = MT == 4 ? 2 : part + 1;
  const bf16x4 zero = {0, 0, 0, 0};
  f32x4 acc[2] = {(f32x4){0.f, 0.f, 0.f, 0.f}, (f32x4){0.f, 0.f, 0.f, 0.f}};
  const int m = mt * 16 + r, oy = m / HOUT, ox = m % HOUT;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
    const bool ok = iy >= 0 && iy < HIN && ix >= 0 && ix < HIN;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int ci = half * 16 + g * 4;
      const bf16x4 a = ok ? ld4(in + (iy * HIN + ix) * kPS + ci) : zero;
      for (int nt = n0; nt < n1; ++nt) {
        const bf16x4 b = ld4(W + (nt * 16 + r) * kWS + tap * CH + ci);
        acc[nt - n0] = mfma(a, b, acc[nt - n0]);
      }
    }
  }
  for (int nt = n0; nt < n1; ++nt)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int p = mt * 16 + g * 4 + j;
      out[p * kPS + nt * 16 + r] = f2bf(fmaxf(acc[nt - n0][j] + bias[nt * 16 + r], 0.f));
    }
}

struct ProposalOut {
  int32_t* centre;    // [ntiles][2] window centre (null: not wanted)
  uint8_t* fallback;  // [ntiles] 1: exhaustive search
  int clampc;         // |centre| <= clampc
  float conf_logit;   // window search when the logit is >= this
  const int32_t* tiles;  // sample -> tile (null: sample s is tile s)
  const int* count;      // samples (device; null: the launch's n)
  int* lists;            // window tiles [0, ntiles), fallback tiles [ntiles, 2 ntiles)
  int* counts;           // [2] entries of the two lists
  int ntiles;
};

// LDS: packed weights (W1p, then W2..W4 with padded rows) and biases, shared
// by the workgroup's 16 waves; then per sample in flight a 256-position and a
// 64-position activation buffer (x -> a1 -> a2 -> a3 -> a4 ping-pong). The
// head's weights are read from global memory.
constexpr int kFwdLdsWeights = (kW1p + 3 * CH * kWS) * 2 + 4 * CH * 4;
constexpr int kFwdBufA = 256 * kPS, kFwdBufB = 64 * kPS;  // elements
constexpr int kFwdLdsSample = (kFwdBufA + kFwdBufB) * 2;
constexpr int kFwdSamples = kFwdWaves / kFwdGroupWaves;
constexpr int kFwdLds = kFwdLdsWeights + kFwdSamples * kFwdLdsSample;
static_assert(kFwdLds <= 160 * 1024, "forward workgroup LDS");

template <bool TRAIN>
__global__ __launch_bounds__(kFwdWaves * kWave) void k_cnn_fwd(
    const uint16_t* __restrict__ pk, const float* __restrict__ P, const uint16_t* __restrict__ x,
    int n, float* __restrict__ out, uint16_t* __restrict__ acts, ProposalOut po) {
  extern __shared__ __align__(16) uint8_t sm[];
  if (po.count) n = *po.count;
  uint16_t* sW1 = reinterpret_cast<uint16_t*>(sm);
  uint16_t* sW = sW1 + kW1p;  // [3][32 co][kWS]: [9 tap][32 ci] + padding
  float* sb = reinterpret_cast<float*>(sW + 3 * CH * kWS);  // [4][32]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = wave / kFwdGroupWaves, part = wave % kFwdGroupWaves;
  const int gt = part * kWave + lane;  // thread index within the sample's group
  constexpr int GT = kFwdGroupWaves * kWave;
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(pk);
    uint32_t* dst = reinterpret_cast<uint32_t*>(sm);
    for (int i = tid; i < kW1p / 2; i += blockDim.x) dst[i] = src[i];
    // W2..W4 rows (96 rows of 144 dwords) into the padded rows
    uint32_t* dw = reinterpret_cast<uint32_t*>(sW);
    const uint32_t* sw = src + kW1p / 2;
    for (int i = tid; i < 3 * CH * (9 * CH / 2); i += blockDim.x) {
      const int row = i / (9 * CH / 2), q = i % (9 * CH / 2);
      dw[row * (kWS / 2) + q] = sw[i];
    }
    for (int i = tid; i < 4 * CH; i += blockDim.x) sb[i] = P[kOffB[i / CH] + i % CH];
  }
  uint16_t* bufA = reinterpret_cast<uint16_t*>(sm + kFwdLdsWeights + grp * kFwdLdsSample);
  uint16_t* bufB = bufA + kFwdBufA;
  // every group runs the same number of rounds (the barriers are block-wide);
  // a group past the last sample idles through its round
  for (int s0 = blockIdx.x * kFwdSamples; s0 < n; s0 += gridDim.x * kFwdSamples) {
    const int s = s0 + grp;
    const bool act = s < n;
    __syncthreads();  // weights loaded / previous round's buffers free
    if (act) {
      // x: NCHW [4][16][16] -> NHWC [16][16][4] in bufB
      const uint16_t* xs = x + (size_t)s * kIn;
      for (int i = gt; i < 256; i += GT)
#pragma unroll
        for (int c = 0; c < C1; ++c) bufB[C1 * i + c] = xs[c * 256 + i];
    }
    __syncthreads();
    if (act) {
      if (TRAIN)
        for (int i = gt; i < kIn; i += GT) acts[(size_t)s * kActN + kActX + i] = bufB[i];
      conv1_fwd_part(bufB, sW1, sb, bufA, lane, part);  // a1 -> bufA
    }
    __syncthreads();
    if (act) conv_fwd_part<16, 8, 2>(bufA, sW, sb + CH, bufB, lane, part);  // a2 -> bufB
    __syncthreads();
    if (act) {
      if (TRAIN) {  // stored unpadded: position * 32 + channel
        uint16_t* a = acts + (size_t)s * kActN;
        for (int i = gt; i < 8192; i += GT) a[kActA1 + i] = bufA[(i >> 5) * kPS + (i & 31)];
        for (int i = gt; i < 2048; i += GT) a[kActA2 + i] = bufB[(i >> 5) * kPS + (i & 31)];
      }
    }
    __syncthreads();  // a1 copied out before a3 overwrites it
    if (act) conv_fwd_part<8, 8, 1>(bufB, sW + CH * kWS, sb + 2 * CH, bufA, lane, part);  // a3 -> bufA
    __syncthreads();
    if (act) conv_fwd_part<8, 4, 2>(bufA, sW + 2 * CH * kWS, sb + 3 * CH, bufB, lane, part);  // a4 -> bufB
    __syncthreads();
    if (act && TRAIN) {
      uint16_t* a = acts + (size_t)s * kActN;
      for (int i = gt; i < 2048; i += GT) a[kActA3 + i] = bufA[(i >> 5) * kPS + (i & 31)];
      for (int i = gt; i < 512; i += GT) a[kActA4 + i] = bufB[(i >> 5) * kPS + (i & 31)];
    }
    if (act && part == 0) {
      // head (fp32): f = p * 32 + c, eight features per lane
      float o[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int f = lane * 8 + k;
        const float a = bf2f(bufB[(f >> 5) * kPS + (f & 31)]);
#pragma unroll
        for (int j = 0; j < 3; ++j) o[j] += P[kOffWh + j * 512 + f] * a;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) o[j] += __shfl_xor(o[j], off);
      if (lane == 0) {
        const float o0 = o[0] + P[kOffBh], o1 = o[1] + P[kOffBh + 1], o2 = o[2] + P[kOffBh + 2];
        if (out) {
          out[(size_t)s * 3] = o0;
          out[(size_t)s * 3 + 1] = o1;
          out[(size_t)s * 3 + 2] = o2;
        }
        if (po.centre) {
          // window centre: prediction rounded half up, kept inside the search range
          int cx = (int)floorf(8.f * o0 + 0.5f), cy = (int)floorf(8.f * o1 + 0.5f);
          cx = min(max(cx, -po.clampc), po.clampc);
          cy = min(max(cy, -po.clampc), po.clampc);
          const int t = po.tiles ? po.tiles[s] : s;
          const int fb = o2 >= po.conf_logit ? 0 : 1;
          po.centre[2 * t] = cx;
          po.centre[2 * t + 1] = cy;
          po.fallback[t] = (uint8_t)fb;
          if (po.lists) po.lists[fb * po.ntiles + atomicAdd(&po.counts[fb], 1)] = t;
        }
      }
    }
  }
}

// loss and output gradient (the soft target is held constant)
__global__ __launch_bounds__(256) void k_cnn_loss(const float* __restrict__ o,
                                                  const int32_t* __restrict__ lab, int n,
                                                  float* __restrict__ dO,
                                                  float* __restrict__ loss) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  const float ex = 8.f * o[3 * s] - (float)lab[2 * s];
  const float ey = 8.f * o[3 * s + 1] - (float)lab[2 * s + 1];
  const float z = o[3 * s + 2];
  const float q = 1.f / (1.f + expf(-4.f * (2.5f - fmaxf(fabsf(ex), fabsf(ey)))));
  const float inv = 1.f / (float)n;
  dO[3 * s] = 8.f * fminf(fmaxf(ex, -1.f), 1.f) * inv;
  dO[3 * s + 1] = 8.f * fminf(fmaxf(ey, -1.f), 1.f) * inv;
  dO[3 * s + 2] = (1.f / (1.f + expf(-z)) - q) * inv;
  if (loss) {
    auto hub = [](float e) { return fabsf(e) <= 1.f ? 0.5f * e * e : fabsf(e) - 0.5f; };
    loss[s] = hub(ex) + hub(ey) + fmaxf(z, 0.f) - q * z + log1pf(expf(-fabsf(z)));
  }
}

// da_in = transposed conv of dz (NHWC [HOUT^2][32]) with W (WT [ci][tap][co]);
// dz_in = bf16(da_in where a_in > 0), to LDS (NHWC) and global ([ci][q])
template <int HIN, int HOUT, int S>
__device__ void conv_bwd_data(const uint16_t* dz, const uint16_t* WT,
                              const uint16_t* __restrict__ a_in /*global NHWC*/,
                              uint16_t* dz_in, uint16_t* __restrict__ dz_in_g, int lane) {
  const int r = lane & 15, g = lane >> 4;
  constexpr int MT = HIN * HIN / 16;
  const bf16x4 zero = {0, 0, 0, 0};
  for (int mt = 0; mt < MT; ++mt) {
    const int q = mt * 16 + r, qy = q / HIN, qx = q % HIN;
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ty = qy + 1 - tap / 3, tx = qx + 1 - tap % 3;
      const int oy = ty / S, ox = tx / S;
      const bool ok = ty >= 0 && tx >= 0 && ty % S == 0 && tx % S == 0 && oy < HOUT && ox < HOUT;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int co = half * 16 + g * 4;
        const bf16x4 a = ok ? ld4(dz + (oy * HOUT + ox) * CH + co) : zero;
        const bf16x4 b0 = ld4(WT + (r * 9 + tap) * CH + co);
        const bf16x4 b1 = ld4(WT + ((16 + r) * 9 + tap) * CH + co);
        acc0 = mfma(a, b0, acc0);
        acc1 = mfma(a, b1, acc1);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int p = mt * 16 + g * 4 + j;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int ci = h * 16 + r;
        const float d = h ? acc1[j] : acc0[j];
        const uint16_t v = a_in[p * CH + ci] != 0 && bf2f(a_in[p * CH + ci]) > 0.f ? f2bf(d) : 0;
        dz_in[p * CH + ci] = v;
        dz_in_g[ci * HIN * HIN + p] = v;
      }
    }
  }
}

constexpr int kBwdLdsWeights = 3 * kWp * 2 + 3 * 512 * 4;
constexpr int kBwdLdsWave = (8192 + 2048 + 2048) * 2;
constexpr int kBwdWaves = 4;
constexpr int kBwdLds = kBwdLdsWeights + kBwdWaves * kBwdLdsWave;

__global__ __launch_bounds__(kBwdWaves * kWave) void k_cnn_bwd(
    const uint16_t* __restrict__ pk, const float* __restrict__ P,
    const uint16_t* __restrict__ acts, const float* __restrict__ dO, int n,
    uint16_t* __restrict__ dzs) {
  extern __shared__ __align__(16) uint8_t sm[];
  uint16_t* sWT = reinterpret_cast<uint16_t*>(sm);  // [3][32 ci][9][32 co]
  float* sWh = reinterpret_cast<float*>(sWT + 3 * kWp);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(pk + kW1p + 3 * kWp);
    uint32_t* dst = reinterpret_cast<uint32_t*>(sm);
    for (int i = tid; i < 3 * kWp / 2; i += blockDim.x) dst[i] = src[i];
    for (int i = tid; i < 3 * 512; i += blockDim.x) sWh[i] = P[kOffWh + i];
  }
  __syncthreads();
  uint16_t* bufA = reinterpret_cast<uint16_t*>(sm + kBwdLdsWeights + wave * kBwdLdsWave);
  uint16_t* bufB = bufA + 8192;
  uint16_t* bufC = bufB + 2048;
  for (int s = blockIdx.x * kBwdWaves + wave; s < n; s += gridDim.x * kBwdWaves) {
    const uint16_t* a = acts + (size_t)s * kActN;
    uint16_t* dz = dzs + (size_t)s * kDzN;
    const float d0 = dO[3 * s], d1 = dO[3 * s + 1], d2 = dO[3 * s + 2];
    // through the head and the last ReLU: dz4 (NHWC in bufB, [c][p] global)
    for (int f = lane; f < 512; f += kWave) {
      const float da = sWh[f] * d0 + sWh[512 + f] * d1 + sWh[1024 + f] * d2;
      const uint16_t av = a[kActA4 + f];
      const uint16_t v = av != 0 && bf2f(av) > 0.f ? f2bf(da) : 0;
      bufB[f] = v;
      dz[kDz4 + (f % CH) * 16 + f / CH] = v;
    }
    conv_bwd_data<8, 4, 2>(bufB, sWT + 2 * kWp, a + kActA3, bufC, dz + kDz3, lane);
    conv_bwd_data<8, 8, 1>(bufC, sWT + kWp, a + kActA2, bufB, dz + kDz2, lane);
    conv_bwd_data<16, 8, 2>(bufB, sWT, a + kActA1, bufA, dz + kDz1, lane);
  }
}

// Weight and bias gradients of layer L (1..4) over the samples of this block:
// dW[co][tap][ci] = sum_{s,p} dz[s][co][p] a_in[s][in(p, tap)][ci]
// (M = co, N = (tap, ci), K = (s, p)), written to part[block] in the master
// layout.
template <int L>
__global__ __launch_bounds__(256) void k_cnn_wgrad(const uint16_t* __restrict__ acts,
                                                   const uint16_t* __restrict__ dzs, int n,
                                                   int per_block, float* __restrict__ part) {
  constexpr int CIN = L == 1 ? C1 : CH;
  constexpr int HIN = L <= 2 ? 16 : 8;
  constexpr int HOUT = L == 1 ? 16 : (L == 4 ? 4 : 8);
  constexpr int S = (L == 2 || L == 4) ? 2 : 1;
  constexpr int NP = HOUT * HOUT;
  constexpr int NN = 9 * CIN;                 // 18 or 288
  constexpr int NT = (NN + 15) / 16;          // N tiles
  constexpr int NTW = (NT + 3) / 4;           // per wave
  constexpr int AIN = L == 1 ? kActX : (L == 2 ? kActA1 : (L == 3 ? kActA2 : kActA3));
  constexpr int DZ = L == 1 ? kDz1 : (L == 2 ? kDz2 : (L == 3 ? kDz3 : kDz4));
  __shared__ float bsum[8][CH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int s0 = blockIdx.x * per_block, s1 = min(n, s0 + per_block);
  f32x4 acc[2][NTW];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int t = 0; t < NTW; ++t) acc[m][t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (int s = s0; s < s1; ++s) {
    const uint16_t* dz = dzs + (size_t)s * kDzN + DZ;
    const uint16_t* ain = acts + (size_t)s * kActN + AIN;
    for (int k0 = 0; k0 < NP; k0 += 16) {
      const int p0 = k0 + g * 4;
      const bf16x4 a0 = ld4(dz + r * NP + p0);
      const bf16x4 a1 = ld4(dz + (16 + r) * NP + p0);
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        const int nt = wave + 4 * t;
        if (nt >= NT) continue;
        const int nn = nt * 16 + r;
        bf16x4 b = {0, 0, 0, 0};
        if (nn < NN) {
          const int tap = nn / CIN, ci = nn % CIN;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int p = p0 + j, oy = p / HOUT, ox = p % HOUT;
            const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
            if (iy >= 0 && iy < HIN && ix >= 0 && ix < HIN)
              b[j] = (short)ain[(iy * HIN + ix) * CIN + ci];
          }
        }
        acc[0][t] = mfma(a0, b, acc[0][t]);
        acc[1][t] = mfma(a1, b, acc[1][t]);
      }
    }
  }
  float* out = part + (size_t)blockIdx.x * kNParam;
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    const int nt = wave + 4 * t;
    const int nn = nt * 16 + r;
    if (nt >= NT || nn >= NN) continue;
    const int tap = nn / CIN, ci = nn % CIN;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int co = m * 16 + g * 4 + j;
        out[kOffW[L - 1] + (co * CIN + ci) * 9 + tap] = acc[m][t][j];
      }
  }
  // bias gradient: 8 position groups per channel
  {
    const int co = tid & 31, grp = tid >> 5;
    float sacc = 0.f;
    for (int s = s0; s < s1; ++s) {
      const uint16_t* dz = dzs + (size_t)s * kDzN + DZ + co * NP;
      for (int p = grp; p < NP; p += 8) sacc += bf2f(dz[p]);
    }
    bsum[grp][co] = sacc;
    __syncthreads();
    if (tid < CH) {
      float b = 0.f;
      for (int q = 0; q < 8; ++q) b += bsum[q][tid];
      out[kOffB[L - 1] + tid] = b;
    }
  }
}

__global__ __launch_bounds__(256) void k_cnn_head_grad(const uint16_t* __restrict__ acts,
                                                       const float* __restrict__ dO, int n,
                                                       int per_block, float* __restrict__ part) {
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * per_block, s1 = min(n, s0 + per_block);
  float* out = part + (size_t)blockIdx.x * kNParam;
  for (int f = tid; f < 512; f += 256) {
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
    for (int s = s0; s < s1; ++s) {
      const float a = bf2f(acts[(size_t)s * kActN + kActA4 + f]);
      g0 += dO[3 * s] * a;
      g1 += dO[3 * s + 1] * a;
      g2 += dO[3 * s + 2] * a;
    }
    out[kOffWh + f] = g0;
    out[kOffWh + 512 + f] = g1;
    out[kOffWh + 1024 + f] = g2;
  }
  if (tid < 3) {
    float b = 0.f;
    for (int s = s0; s < s1; ++s) b += dO[3 * s + tid];
    out[kOffBh + tid] = b;
  }
}

struct AdamArgs {
  float lr, b1, b2, eps, wd, c1, c2;  // c1 = 1 - b1^t, c2 = 1 - b2^t
};

__global__ __launch_bounds__(256) void k_cnn_adamw(const float* __restrict__ part, int nblk,
                                                   float* __restrict__ P, float* __restrict__ m,
                                                   float* __restrict__ v, AdamArgs a,
                                                   float* __restrict__ grad_out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kNParam) return;
  float g = 0.f;
  for (int b = 0; b < nblk; ++b) g += part[(size_t)b * kNParam + i];
  if (grad_out) grad_out[i] = g;
  if (a.lr == 0.f && a.wd == 0.f) return;  // gradient only
  const float mi = a.b1 * m[i] + (1.f - a.b1) * g;
  const float vi = a.b2 * v[i] + (1.f - a.b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / a.c1, vh = vi / a.c2;
  P[i] = P[i] - a.lr * (mh / (sqrtf(vh) + a.eps) + a.wd * P[i]);
}

}  // namespace

int cnn_param_count() { return kNParam; }
size_t cnn_packed_elems() { return kPacked; }
size_t cnn_act_elems() { return kActN; }
size_t cnn_dz_elems() { return kDzN; }
size_t cnn_input_elems() { return kIn; }

hipError_t launch_cnn_pack(const float* params, uint16_t* packed, hipStream_t st) {
  LNR_LAUNCH(k_cnn_pack, dim3((kPacked + 255) / 256), dim3(256), 0, st, params, packed);
  return hipGetLastError();
}

hipError_t launch_cnn_input(const uint8_t* ref, const uint8_t* warped, int w, int h, int ntx,
                            int nty, const int32_t* tiles, const int* count, uint16_t* x,
                            hipStream_t st) {
  if (ntx * nty == 0) return hipSuccess;
  LNR_LAUNCH(k_cnn_input, dim3(ntx * nty), dim3(256), 0, st, ref, warped, w, h, ntx, tiles,
             count, ntx * nty, x);
  return hipGetLastError();
}

// one workgroup per CU at most (each loads the weights once), looping over
// the samples four at a time
static int fwd_blocks(int n) {
  int b = (n + kFwdSamples - 1) / kFwdSamples;
  return b < 256 ? (b < 1 ? 1 : b) : 256;
}

hipError_t launch_cnn_forward(const uint16_t* packed, const float* params, const uint16_t* x,
                              int n, float* out, uint16_t* acts, int32_t* centre,
                              uint8_t* fallback, int clampc, float conf_logit, hipStream_t st,
                              const int32_t* tiles, const int* count, int* lists, int* counts) {
  if (n <= 0) return hipSuccess;
  ProposalOut po{centre, fallback, clampc, conf_logit, tiles, count, lists, counts, n};
  hipError_t e;
  if (acts) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cnn_fwd<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kFwdLds);
    if (e != hipSuccess) return e;
    LNR_LAUNCH(k_cnn_fwd<true>, dim3(fwd_blocks(n)), dim3(kFwdWaves * kWave), kFwdLds, st,
               packed, params, x, n, out, acts, po);
  } else {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cnn_fwd<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kFwdLds);
    if (e != hipSuccess) return e;
    LNR_LAUNCH(k_cnn_fwd<false>, dim3(fwd_blocks(n)), dim3(kFwdWaves * kWave), kFwdLds, st,
               packed, params, x, n, out, acts, po);
  }
  return hipGetLastError();
}

int cnn_grad_blocks(int n, int* per_block) {
  const int pb = 64;
  *per_block = pb;
  return (n + pb - 1) / pb;
}

hipError_t launch_cnn_backward(const uint16_t* packed, const float* params,
                               const uint16_t* acts, const float* out, const int32_t* labels,
                               int n, float* dO, float* loss, uint16_t* dzs, float* part,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  LNR_LAUNCH(k_cnn_loss, dim3((n + 255) / 256), dim3(256), 0, st, out, labels, n, dO, loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cnn_bwd),
                          hipFuncAttributeMaxDynamicSharedMemorySize, kBwdLds);
  if (e != hipSuccess) return e;
  LNR_LAUNCH(k_cnn_bwd, dim3(fwd_blocks(n)), dim3(kBwdWaves * kWave), kBwdLds, st, packed, params,
             acts, dO, n, dzs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int pb = 0;
  const int nb = cnn_grad_blocks(n, &pb);
  LNR_LAUNCH(k_cnn_wgrad<1>, dim3(nb), dim3(256), 0, st, acts, dzs, n, pb, part);
  LNR_LAUNCH(k_cnn_wgrad<2>, dim3(nb), dim3(256), 0, st, acts, dzs, n, pb, part);
  LNR_LAUNCH(k_cnn_wgrad<3>, dim3(nb), dim3(256), 0, st, acts, dzs, n, pb, part);
  LNR_LAUNCH(k_cnn_wgrad<4>, dim3(nb), dim3(256), 0, st, acts, dzs, n, pb, part);
  LNR_LAUNCH(k_cnn_head_grad, dim3(nb), dim3(256), 0, st, acts, dO, n, pb, part);
  return hipGetLastError();
}

hipError_t launch_cnn_adamw(const float* part, int nblk, float* params, float* m, float* v,
                            float lr, float wd, int step, float* grad_out, hipStream_t st) {
  AdamArgs a;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  a.wd = wd;
  a.c1 = (float)(1.0 - pow(0.9, step));
  a.c2 = (float)(1.0 - pow(0.999, step));
  LNR_LAUNCH(k_cnn_adamw, dim3((kNParam + 255) / 256), dim3(256), 0, st, part, nblk, params, m,
             v, a, grad_out);
  return hipGetLastError();
}

}  // namespace lnr
