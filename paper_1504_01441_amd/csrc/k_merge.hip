// k_merge.hip -- error-tolerant exposure fusion (paper Sec. 2.5): Mertens et
// al.'s contrast, saturation and well-exposedness weights, times the SSIM
// between the equalised reference and each warped frame (Wang et al.:
// Gaussian window, five filterings), blended with Laplacian pyramids.
//
//  k_ssim:    4 output rows x (256 - 2r) columns per block: the vertical
//             Gaussian sums of each input column are built in registers, the
//             horizontal ones from LDS, two output columns per thread. The
//             sums (x, y, xy, x^2 + y^2) are double precision: SSIM divides
//             covariance errors by sx^2 + sy^2 + C2 (~1e-3 in flat regions)
//             and the fusion weights amplify them again.
//  k_weights: per pixel, every frame's C * S * E (* max(SSIM, 0)) + 1e-12,
//             normalised over the frames; threads walk down columns so that
//             the Laplacian's rows are read once, and take the left and right
//             neighbours from the adjacent lanes.
//  k_reduce:  REDUCE ([1 4 6 4 1]/16 separable, clamped, even samples) of
//             every weight and image plane of one level, through LDS.
//  k_blend:   from the top level down, R_l = sum_k W_k,l (G_k,l - E(G_k,l+1))
//             + E(R_l+1), E the EXPAND rule, on 64x16 tiles whose coarse
//             neighbourhoods are staged (and row-expanded) in LDS; level 0
//             goes to the output. Small levels use k_blend_px instead (one
//             thread per pixel and channel, samples read directly).
#include "lnr_internal.h"

namespace lnr {
namespace {

struct FramePtrs {
  const float* img[16];
  const float* ssim[16];
  float* wout[16];
};

constexpr int kMaxMaps = 64;
constexpr int kSsimMaxR = 8, kSsimTH = 4;

// normalised Gaussian window taps g[0 .. 2r]
struct SsimWin {
  double g[2 * kSsimMaxR + 1];
};

// One block: kSsimTH output rows by 256 - 2R output columns. SSIM needs the
// Gaussian sums of x, y, xy and of x^2 + y^2 (only the sum of the two
// variances enters it), accumulated in double precision: SSIM divides
// covariance errors by sx^2 + sy^2 + C2 (~1e-3 in flat regions) and the
// fusion weights amplify them again near SSIM = 0, so float sums of
// E[x^2] - E[x]^2 are not accurate enough there.
//  1. vertical: thread t owns input column ox - R + t (clamped) and reads its
//     kSsimTH + 2R rows straight from global memory (a wave reads 64
//     consecutive floats per row); each row's values and products are
//     scattered into the kSsimTH outputs they belong to, all in registers;
//  2. the vertical sums go to LDS; thread t takes output columns 2t and 2t+1
//     of half the tile's rows, reading the shared window as aligned pairs of
//     doubles (16-byte LDS reads, half the reads of one column per thread).
template <int R>
__global__ __launch_bounds__(256) void k_ssim(const float* __restrict__ a,
                                              const float* __restrict__ b, int W, int H,
                                              SsimWin win, double c1, double c2,
                                              float* __restrict__ out) {
  constexpr int TW = 256 - 2 * R, NR = kSsimTH + 2 * R, NS = 4;
  static_assert(kSsimTH % 2 == 0, "two row halves");
  __shared__ double2 vs[NS][kSsimTH][128];  // column pairs of the vertical sums
  int bx, by;
  xcd_block(gridDim.x, gridDim.y, bx, by);
  const int tid = threadIdx.x;
  const int ox = bx * TW, oy = by * kSsimTH;
  {
    const int gx = min(max(ox - R + tid, 0), W - 1);
    float pa[NR], pb[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {  // every load in flight before the sums
      const size_t o = (size_t)min(max(oy - R + i, 0), H - 1) * W + gx;
      pa[i] = a[o];
      pb[i] = b[o];
    }
    double acc[kSsimTH][NS];
#pragma unroll
    for (int o = 0; o < kSsimTH; ++o)
#pragma unroll
      for (int t = 0; t < NS; ++t) acc[o][t] = 0.0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const double p = pa[i], q = pb[i];
      const double ss = p * p + q * q, pq = p * q;
#pragma unroll
      for (int o = 0; o < kSsimTH; ++o) {
        const int k = i - o;  // tap of input row oy - R + i for output row oy + o
        if (k < 0 || k > 2 * R) continue;
        const double wd = win.g[k];
        acc[o][0] += wd * p;
        acc[o][1] += wd * q;
        acc[o][2] += wd * ss;
        acc[o][3] += wd * pq;
      }
    }
    double* vd = reinterpret_cast<double*>(vs);
#pragma unroll
    for (int o = 0; o < kSsimTH; ++o)
#pragma unroll
      for (int t = 0; t < NS; ++t) vd[(t * kSsimTH + o) * 256 + tid] = acc[o][t];
  }
  __syncthreads();
  const int pr = tid & 127, half = tid >> 7;  // column pair, row half
  const int gx = ox + 2 * pr;
  if (2 * pr >= TW || gx >= W) return;
  const bool two = 2 * pr + 1 < TW && gx + 1 < W;
#pragma unroll
  for (int oo = 0; oo < kSsimTH / 2; ++oo) {
    const int o = half * (kSsimTH / 2) + oo;
    const int gy = oy + o;
    if (gy >= H) break;
    double s0[NS] = {0.0, 0.0, 0.0, 0.0}, s1[NS] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m <= R; ++m) {  // inputs 2pr + 2m and 2pr + 2m + 1
      const double wl = win.g[2 * m];
      const double wr = 2 * m + 1 <= 2 * R ? win.g[2 * m + 1] : 0.0;
      const double wp = m > 0 ? win.g[2 * m - 1] : 0.0;
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const double2 v = vs[t][o][pr + m];
        // output 2pr takes taps 2m (v.x) and 2m + 1 (v.y); output 2pr + 1
        // takes taps 2m - 1 (v.x) and 2m (v.y)
        s0[t] += wl * v.x;
        if (2 * m + 1 <= 2 * R) s0[t] += wr * v.y;
        if (m > 0) s1[t] += wp * v.x;
        s1[t] += wl * v.y;
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (c == 1 && !two) break;
      const double* sv = c ? s1 : s0;
      const double m1 = sv[0], m2 = sv[1];
      const double vxy = sv[2] - m1 * m1 - m2 * m2, cxy = sv[3] - m1 * m2;
      out[(size_t)gy * W + gx + c] = (float)(((2.0 * m1 * m2 + c1) * (2.0 * cxy + c2)) /
                                             ((m1 * m1 + m2 * m2 + c1) * (vxy + c2)));
    }
  }
}

__device__ inline double grey_of(int ch, float r, float g, float b) {
  return ch == 3 ? (0.299 * (double)r + 0.587 * (double)g) + 0.114 * (double)b : (double)r;
}

// C * S * E (* max(SSIM, 0)) of one frame at one pixel, from the grey values
// of the pixel (gc) and its four neighbours, and the pixel's colour. Contrast
// and saturation are differences of nearly equal values in flat regions, and
// the normalised weights divide by their sum, which can be ~1e-12 there: they
// are evaluated in double precision.
__device__ inline double raw_weight(int ch, double gu, double gl, double gr, double gd,
                                    double gc, float R, float G, float B, bool warped,
                                    float ssim, float two_se2) {
  const double C = fabs(gu + gl + gr + gd - 4.0 * gc);
  double S = 1.0;
  float e;
  if (ch == 3) {
    const double r = R, g = G, b = B;
    const double mu = (r + g + b) * (1.0 / 3.0);
    const double var = ((r - mu) * (r - mu) + (g - mu) * (g - mu) + (b - mu) * (b - mu)) * (1.0 / 3.0);
    S = (double)sqrtf((float)var);  // the cancelling differences are in double
    e = (float)((r - 0.5) * (r - 0.5) + (g - 0.5) * (g - 0.5) + (b - 0.5) * (b - 0.5));
  } else {
    e = (float)(((double)R - 0.5) * ((double)R - 0.5));
  }
  double wt = C * S * (double)expf(-e / two_se2);
  if (warped) wt *= fmax((double)ssim, 0.0);
  return wt + 1e-12;
}

constexpr int kWeightRows = 8;
constexpr int kWeightCols = 62;  // output columns per wave (lanes 1..62)

// Each thread walks down kWeightRows rows of one column: the grey values of
// the rows above, at and below the pixel stay in registers, so every colour
// sample is fetched from memory once. A wave covers 62 columns and two halo
// lanes (0 and 63, clamped at the image border like the pixels' own
// neighbours); the left and right neighbours' grey values come from the
// adjacent lanes by shuffle. The samples of the next row are loaded before
// the current row's weights are formed and stored, so one row's loads are
// always in flight.
template <int NMAX>
__global__ __launch_bounds__(256) void k_weights(FramePtrs f, int n, int ch, int W, int H,
                                                 int ref, float two_se2) {
  int bx, by;
  xcd_block(gridDim.x, gridDim.y, bx, by);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = (bx * 4 + wave) * kWeightCols + lane - 1;
  const int xc = min(max(x, 0), W - 1);
  const bool writes = lane >= 1 && lane <= kWeightCols && x < W;
  const int lsrc = lane > 0 ? lane - 1 : 0, rsrc = lane < 63 ? lane + 1 : 63;
  const int y0 = by * kWeightRows, y1 = min(y0 + kWeightRows, H);
  const size_t plane = (size_t)W * H;
  auto ld = [&](const float* I, size_t o, float& r, float& g, float& b) {
    r = I[o];
    g = ch == 3 ? I[plane + o] : 0.f;
    b = ch == 3 ? I[2 * plane + o] : 0.f;
  };
  // samples of row y: d* the row below, s the SSIM
  float dr[NMAX], dg[NMAX], db[NMAX], sv[NMAX];
  auto fetch = [&](int y) {  // y < H
    const size_t od = (size_t)min(y + 1, H - 1) * W + xc;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
      if (k >= n) continue;
      ld(f.img[k], od, dr[k], dg[k], db[k]);
      sv[k] = k != ref ? f.ssim[k][(size_t)y * W + xc] : 0.f;
    }
  };
  double gu[NMAX], gc[NMAX];
  float cr[NMAX], cg[NMAX], cb[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    if (k >= n) continue;
    float r, g, b;
    ld(f.img[k], (size_t)max(y0 - 1, 0) * W + xc, r, g, b);
    gu[k] = grey_of(ch, r, g, b);
    ld(f.img[k], (size_t)y0 * W + xc, cr[k], cg[k], cb[k]);
    gc[k] = grey_of(ch, cr[k], cg[k], cb[k]);
  }
  // stacks of up to 4 frames keep the next row's samples in flight; larger
  // ones (whose samples would not fit the registers) load each frame's
  // samples where they are used
  constexpr bool kAhead = NMAX <= 4;
  if constexpr (kAhead) fetch(y0);
  for (int y = y0; y < y1; ++y) {
    const size_t o = (size_t)y * W + xc;
    float Dr[NMAX], Dg[NMAX], Db[NMAX], S[NMAX];
    if constexpr (kAhead) {
#pragma unroll
      for (int k = 0; k < NMAX; ++k) {
        Dr[k] = dr[k]; Dg[k] = dg[k]; Db[k] = db[k];
        S[k] = sv[k];
      }
      if (y + 1 < y1) fetch(y + 1);
    }
    // the raw weights keep 24-bit relative precision as floats once the
    // cancelling differences inside them were taken in double precision
    float wk[NMAX];
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
      if (k >= n) continue;
      if constexpr (!kAhead) {
        ld(f.img[k], (size_t)min(y + 1, H - 1) * W + xc, Dr[k], Dg[k], Db[k]);
        S[k] = k != ref ? f.ssim[k][o] : 0.f;
      }
      const bool warped = k != ref;
      const double gd = grey_of(ch, Dr[k], Dg[k], Db[k]);
      const double gl = __shfl(gc[k], lsrc), gr = __shfl(gc[k], rsrc);
      wk[k] = (float)raw_weight(ch, gu[k], gl, gr, gd, gc[k], cr[k], cg[k], cb[k], warped, S[k],
                                two_se2);
      sum += (double)wk[k];
      gu[k] = gc[k];
      gc[k] = gd;
      cr[k] = Dr[k]; cg[k] = Dg[k]; cb[k] = Db[k];
    }
    if (writes) {
#pragma unroll
      for (int k = 0; k < NMAX; ++k) {
        if (k >= n) continue;
        f.wout[k][o] = (float)((double)wk[k] / sum);
      }
    }
  }
}

// Irradiance map of the registered frames, one pixel per thread and every
// channel: each frame's value over its relative exposure, averaged with the
// hat weight min(v, 1 - v) (0 at black and saturation), non-reference
// frames' weights times max(SSIM, 0); the reference's value where every
// weight is 0.
struct IrrPtrs {
  const float* img[16];
  const float* ssim[16];
  float rel[16];  // exposure relative to the reference
};

__device__ inline float hat_weight(float v) {
  const float a = v < 1.f - v ? v : 1.f - v;
  return a > 0.f ? a : 0.f;
}

template <int NMAX>
__global__ __launch_bounds__(256) void k_irradiance(IrrPtrs f, int n, int ch, int ref,
                                                    long long npix, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= npix) return;
  float s[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    s[k] = 1.f;
    if (k < n && k != ref) {
      const float q = f.ssim[k][i];
      s[k] = q > 0.f ? q : 0.f;
    }
  }
  for (int c = 0; c < ch; ++c) {
    const long long o = (long long)c * npix + i;
    float v[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) v[k] = k < n ? f.img[k][o] : 0.f;  // all loads in flight
    float sw = 0.f, se = 0.f;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
      if (k >= n) continue;
      const float wk = hat_weight(v[k]) * s[k];
      sw += wk;
      se += wk * (v[k] / f.rel[k]);
    }
    out[o] = sw > 0.f ? se / sw : f.img[ref][o];
  }
}

struct MapPtrs {
  const float* in[kMaxMaps];
  float* out[kMaxMaps];
};

constexpr int kRedTW = 128, kRedTH = 8;

__global__ __launch_bounds__(256) void k_reduce(MapPtrs m, int w, int h, int w2, int h2) {
  __shared__ float src[2 * kRedTH + 3][2 * kRedTW + 3];
  __shared__ float hb[2 * kRedTH + 3][kRedTW];
  const float kf[5] = {1.f / 16, 4.f / 16, 6.f / 16, 4.f / 16, 1.f / 16};
  const float* in = m.in[blockIdx.z];
  float* out = m.out[blockIdx.z];
  const int ox = blockIdx.x * kRedTW, oy = blockIdx.y * kRedTH;
  constexpr int rows = 2 * kRedTH + 3, cols = 2 * kRedTW + 3;
  constexpr int per = (rows * cols + 255) / 256;
  float v[per];
#pragma unroll
  for (int q = 0; q < per; ++q) {  // all loads in flight before the LDS stores
    const int i = threadIdx.x + 256 * q;
    const int yy = i / cols, xx = i % cols;
    const int gy = min(max(2 * oy - 2 + yy, 0), h - 1), gx = min(max(2 * ox - 2 + xx, 0), w - 1);
    v[q] = i < rows * cols ? in[(size_t)gy * w + gx] : 0.f;
  }
#pragma unroll
  for (int q = 0; q < per; ++q) {
    const int i = threadIdx.x + 256 * q;
    if (i < rows * cols) src[i / cols][i % cols] = v[q];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < rows * kRedTW; i += 256) {
    const int yy = i / kRedTW, xx = i % kRedTW;
    float s = 0.f;
    for (int k = 0; k < 5; ++k) s += kf[k] * src[yy][2 * xx + k];
    hb[yy][xx] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kRedTH * kRedTW; i += 256) {
    const int yy = i / kRedTW, xx = i % kRedTW;
    const int gy = oy + yy, gx = ox + xx;
    if (gy >= h2 || gx >= w2) continue;
    float s = 0.f;
    for (int k = 0; k < 5; ++k) s += kf[k] * hb[2 * yy + k][xx];
    out[(size_t)gy * w2 + gx] = s;
  }
}

struct BlendPtrs {
  const float* w[16];        // normalised weights at level l
  const float* g[16][3];     // image planes at level l
  const float* gc[16][3];    // image planes at level l + 1
  const float* rc[3];        // collapsed result at level l + 1
  float* out[3];             // collapsed result at level l
};

constexpr int kBW = 64, kBH = 16;                 // fine output tile
constexpr size_t kBlendPxMax = 1 << 18;           // levels up to this size: k_blend_px
constexpr int kCW = kBW / 2 + 2, kCH = kBH / 2 + 2;  // coarse tile with its EXPAND halo

// One 64 x 16 tile of level l, channels [c0, c0 + cg):
//   R_l = sum_k W_k (G_k - E(G_k,l+1)) + E(R_l+1).
// EXPAND (even 2i: (c[i-1] + 6 c[i] + c[i+1]) / 8, odd 2i+1: (c[i] + c[i+1]) / 2,
// clamped coarse indices; rows first, then columns) reads the coarse planes
// from LDS tiles (kCH x kCW, clamped at load) loaded once per block; each
// thread expands the coarse rows it needs in registers. Each thread owns one
// column of the tile (4 rows), or four pixels of a row, and reads each weight
// once.
// EXPAND at fine column 2 (li + cx0) + (xeven ? 0 : 1) of one staged row
__device__ inline float ex_row(const float* row, int li, bool xeven) {
  return xeven ? (row[li - 1] + 6.f * row[li] + row[li + 1]) / 8.f
               : (row[li] + row[li + 1]) / 2.f;
}

__device__ inline float expand_tile(const float* t, int li, bool xeven, int lj, bool yeven) {
  const float m = ex_row(t + lj * kCW, li, xeven), p = ex_row(t + (lj + 1) * kCW, li, xeven);
  if (yeven) {
    const float a = ex_row(t + (lj - 1) * kCW, li, xeven);
    return (a + 6.f * m + p) / 8.f;
  }
  return (m + p) / 2.f;
}

// the four fine columns from the even one of coarse index li (li, li + 1)
__device__ inline float4 ex_row4(const float* row, int li) {
  const float a = row[li - 1], m = row[li], p = row[li + 1], q = row[li + 2];
  return make_float4((a + 6.f * m + p) / 8.f, (m + p) / 2.f, (m + 6.f * p + q) / 8.f,
                     (p + q) / 2.f);
}

__device__ inline float4 expand_tile4(const float* t, int li, int lj, bool yeven) {
  const float4 m = ex_row4(t + lj * kCW, li), p = ex_row4(t + (lj + 1) * kCW, li);
  if (yeven) {
    const float4 a = ex_row4(t + (lj - 1) * kCW, li);
    return make_float4((a.x + 6.f * m.x + p.x) / 8.f, (a.y + 6.f * m.y + p.y) / 8.f,
                       (a.z + 6.f * m.z + p.z) / 8.f, (a.w + 6.f * m.w + p.w) / 8.f);
  }
  return make_float4((m.x + p.x) / 2.f, (m.y + p.y) / 2.f, (m.z + p.z) / 2.f, (m.w + p.w) / 2.f);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_blend(BlendPtrs b, int n, int c0, int cg, int w, int h,
                                               int cw, int chh, int top, int vec) {
  extern __shared__ float sm[];
  const int tid = threadIdx.x;
  int bx, by;
  xcd_block(gridDim.x, gridDim.y, bx, by);
  const int ox = bx * kBW, oy = by * kBH;
  const int cx0 = (ox >> 1) - 1, cy0 = (oy >> 1) - 1;
  const int nm = top ? 0 : (n + 1) * cg;  // plane m = cc (n + 1) + k, k = n: R
  float* ct = sm;                         // [nm][kCH][kCW] coarse tiles
  if (!top) {
    const int ntot = nm * kCH * kCW;
    for (int i0 = tid; i0 < ntot; i0 += 12 * 256) {  // twelve loads in flight per thread
      float v[12];
#pragma unroll
      for (int u = 0; u < 12; ++u) {
        const int i = i0 + 256 * u;
        v[u] = 0.f;
        if (i < ntot) {
          const int m = i / (kCH * kCW), r = (i / kCW) % kCH, q = i % kCW;
          const int cc = m / (n + 1), k = m % (n + 1);
          const float* src = k < n ? b.gc[k][c0 + cc] : b.rc[c0 + cc];
          const int gy = min(max(cy0 + r, 0), chh - 1), gx = min(max(cx0 + q, 0), cw - 1);
          v[u] = src[(size_t)gy * cw + gx];
        }
      }
#pragma unroll
      for (int u = 0; u < 12; ++u)
        if (i0 + 256 * u < ntot) ct[i0 + 256 * u] = v[u];
    }
    __syncthreads();
  }
  if (vec) {
    // rows of 16-byte aligned planes, width a multiple of 4: a thread owns four
    // consecutive pixels of one row (float4 loads and stores)
    const int xq = 4 * (tid & 15), y = oy + (tid >> 4);
    const int x = ox + xq;
    if (x >= w || y >= h) return;
    const size_t o = (size_t)y * w + x;
    const int li = (x >> 1) - cx0, lj = (y >> 1) - cy0;  // local coarse indices
    const bool even = (y & 1) == 0;
    float4 acc[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) acc[cc] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int k = 0; k < n; ++k) {
      const float4 wv = *reinterpret_cast<const float4*>(b.w[k] + o);
      float4 gv[3];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        gv[cc] = cc < cg ? *reinterpret_cast<const float4*>(b.g[k][c0 + cc] + o)
                         : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        if (cc >= cg) break;
        const float4 e = top ? make_float4(0.f, 0.f, 0.f, 0.f)
                             : expand_tile4(ct + (cc * (n + 1) + k) * kCH * kCW, li, lj, even);
        acc[cc].x += wv.x * (gv[cc].x - e.x);
        acc[cc].y += wv.y * (gv[cc].y - e.y);
        acc[cc].z += wv.z * (gv[cc].z - e.z);
        acc[cc].w += wv.w * (gv[cc].w - e.w);
      }
    }
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      if (cc >= cg) break;
      float4 v = acc[cc];
      if (!top) {
        const float4 e = expand_tile4(ct + (cc * (n + 1) + n) * kCH * kCW, li, lj, even);
        v.x += e.x; v.y += e.y; v.z += e.z; v.w += e.w;
      }
      *reinterpret_cast<float4*>(b.out[c0 + cc] + o) = v;
    }
    return;
  }
  // thread = one column of the tile (lanes are consecutive pixels), 4 rows
  const int fx = tid & 63, fy0 = tid >> 6;
  const int x = ox + fx;
  if (x >= w) return;
  const int li = (x >> 1) - cx0;
  const bool xeven = (x & 1) == 0;
  float acc[3][4];
  for (int cc = 0; cc < cg; ++cc)
    for (int q = 0; q < 4; ++q) acc[cc][q] = 0.f;
  for (int k = 0; k < n; ++k) {
    // this frame's weights and image values first (16 loads in flight)
    float wv[4], gv[3][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int y = oy + fy0 + 4 * q;
      wv[q] = y < h ? b.w[k][(size_t)y * w + x] : 0.f;
    }
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int y = oy + fy0 + 4 * q;
        gv[cc][q] = cc < cg && y < h ? b.g[k][c0 + cc][(size_t)y * w + x] : 0.f;
      }
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      if (cc >= cg) break;
      const float* t = ct + (cc * (n + 1) + k) * kCH * kCW;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int y = oy + fy0 + 4 * q;
        if (y >= h) break;
        const float e = top ? 0.f : expand_tile(t, li, xeven, (y >> 1) - cy0, (y & 1) == 0);
        acc[cc][q] += wv[q] * (gv[cc][q] - e);
      }
    }
  }
  for (int cc = 0; cc < cg; ++cc) {
    const float* t = ct + (cc * (n + 1) + n) * kCH * kCW;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int y = oy + fy0 + 4 * q;
      if (y >= h) break;
      const float v =
          top ? acc[cc][q] : acc[cc][q] + expand_tile(t, li, xeven, (y >> 1) - cy0, (y & 1) == 0);
      b.out[c0 + cc][(size_t)y * w + x] = v;
    }
  }
}

// A pixel of EXPAND(c) at (x, y) of the finer level: rows of the coarse plane
// (cw x chh, clamped indices) expanded along x first, then along y, with the
// arithmetic of k_blend's LDS path.
__device__ inline float expand_px(const float* __restrict__ c, int cw, int chh, int x, int y) {
  const int i = x >> 1, j = y >> 1;
  const int xa = max(i - 1, 0), xm = min(i, cw - 1), xp = min(i + 1, cw - 1);
  float rv[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float* row = c + (size_t)min(max(j - 1 + q, 0), chh - 1) * cw;
    const float a = row[xa], m = row[xm], p = row[xp];
    rv[q] = (x & 1) == 0 ? (a + 6.f * m + p) / 8.f : (m + p) / 2.f;
  }
  return (y & 1) == 0 ? (rv[0] + 6.f * rv[1] + rv[2]) / 8.f : (rv[1] + rv[2]) / 2.f;
}

// Small levels: one thread per pixel and channel (blockIdx.y), every sample
// read straight from memory (all in flight together) instead of staged
// tiles, which leave too few workgroups to hide their latency.
__global__ __launch_bounds__(256) void k_blend_px(BlendPtrs b, int n, int w, int h, int cw,
                                                  int chh, int top) {
  const int pix = blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
  if (pix >= w * h) return;
  const int x = pix % w, y = pix / w;
  float acc = 0.f;
  for (int k = 0; k < n; ++k) {
    const float wv = b.w[k][pix], gv = b.g[k][c][pix];
    const float e = top ? 0.f : expand_px(b.gc[k][c], cw, chh, x, y);
    acc += wv * (gv - e);
  }
  if (!top) acc += expand_px(b.rc[c], cw, chh, x, y);
  b.out[c][pix] = acc;
}

}  // namespace

int merge_levels(int W, int H) {
  const int m = W < H ? W : H;
  int k = 0;
  while ((8ll << (k + 1)) <= m) ++k;
  return 1 + k;
}

// elements of one plane's pyramid levels 1..L-1
size_t merge_pyr_elems(int W, int H, int levels) {
  size_t tot = 0;
  int w = W, h = H;
  for (int l = 1; l < levels; ++l) {
    w = (w + 1) / 2;
    h = (h + 1) / 2;
    tot += (size_t)w * h;
  }
  return tot;
}

// SSIM of every frame but the reference against the reference, into
// ssim + k * W * H
hipError_t launch_ssim_maps(int n, int W, int H, const float* const* yeqs, int ref_index,
                            const lnr_params& p, float* ssim, hipStream_t st) {
  const size_t N = (size_t)W * H;
  hipError_t e;
  for (int k = 0; k < n; ++k) {
    if (k == ref_index) continue;
    const int r = p.ssim_radius;
    SsimWin win;
    double gs = 0.0;
    for (int j = -r; j <= r; ++j) {
      win.g[j + r] = exp(-(double)(j * j) / (2.0 * p.ssim_sigma * p.ssim_sigma));
      gs += win.g[j + r];
    }
    for (int j = 0; j <= 2 * r; ++j) win.g[j] /= gs;
    const int tw = 256 - 2 * r;
    dim3 g((W + tw - 1) / tw, (H + kSsimTH - 1) / kSsimTH);
    const float* ya = yeqs[ref_index];
    const float* yb = yeqs[k];
    float* so = ssim + (size_t)k * N;
    switch (r) {
#define SSIM_CASE(R_)                                                                          \
  case R_:                                                                                     \
    LNR_LAUNCH(k_ssim<R_>, g, dim3(256), 0, st, ya, yb, W, H, win, p.ssim_c1, p.ssim_c2, so); \
    break;
      SSIM_CASE(1) SSIM_CASE(2) SSIM_CASE(3) SSIM_CASE(4)
      SSIM_CASE(5) SSIM_CASE(6) SSIM_CASE(7) SSIM_CASE(8)
#undef SSIM_CASE
      default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_merge(int n, int ch, int W, int H, const float* const* imgs,
                        const float* const* yeqs, int ref_index, const lnr_params& p,
                        const MergeBufs& bufs, float* out, hipStream_t st) {
  const int L = merge_levels(W, H);
  const size_t N = (size_t)W * H;
  const size_t tot = merge_pyr_elems(W, H, L);
  int lw[32], lh[32];
  size_t loff[33];
  lw[0] = W; lh[0] = H; loff[0] = 0; loff[1] = 0;
  for (int l = 1; l < L; ++l) {
    lw[l] = (lw[l - 1] + 1) / 2;
    lh[l] = (lh[l - 1] + 1) / 2;
    loff[l + 1] = loff[l] + (size_t)lw[l] * lh[l];
  }
  hipError_t e;
  FramePtrs fp;
  for (int k = 0; k < n; ++k) {
    fp.img[k] = imgs[k];
    fp.ssim[k] = bufs.ssim + (size_t)k * N;
    fp.wout[k] = bufs.w0 + (size_t)k * N;
  }
  if ((e = launch_ssim_maps(n, W, H, yeqs, ref_index, p, bufs.ssim, st)) != hipSuccess) return e;
  {
    const dim3 g((W + 4 * kWeightCols - 1) / (4 * kWeightCols),
                 (H + kWeightRows - 1) / kWeightRows);
    const float two_se2 = (float)(2.0 * p.sigma_e * p.sigma_e);
    if (n <= 2)
      LNR_LAUNCH(k_weights<2>, g, dim3(256), 0, st, fp, n, ch, W, H, ref_index, two_se2);
    else if (n <= 4)
      LNR_LAUNCH(k_weights<4>, g, dim3(256), 0, st, fp, n, ch, W, H, ref_index, two_se2);
    else if (n <= 8)
      LNR_LAUNCH(k_weights<8>, g, dim3(256), 0, st, fp, n, ch, W, H, ref_index, two_se2);
    else
      LNR_LAUNCH(k_weights<16>, g, dim3(256), 0, st, fp, n, ch, W, H, ref_index, two_se2);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // Gaussian pyramids of every weight and image plane
  const int maps = n * (ch + 1);
  auto plane_ptr = [&](int z, int l) -> float* {
    const int k = z / (ch + 1), q = z % (ch + 1);
    if (l == 0)
      return q == 0 ? bufs.w0 + (size_t)k * N : const_cast<float*>(imgs[k]) + (size_t)(q - 1) * N;
    return bufs.pyr + (size_t)z * tot + loff[l];
  };
  for (int l = 1; l < L; ++l) {
    MapPtrs mp;
    for (int z = 0; z < maps; ++z) {
      mp.in[z] = plane_ptr(z, l - 1);
      mp.out[z] = plane_ptr(z, l);
    }
    dim3 g((lw[l] + kRedTW - 1) / kRedTW, (lh[l] + kRedTH - 1) / kRedTH, maps);
    LNR_LAUNCH(k_reduce, g, dim3(256), 0, st, mp, lw[l - 1], lh[l - 1], lw[l], lh[l]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // blend + collapse, top level first
  for (int l = L - 1; l >= 0; --l) {
    BlendPtrs bp;
    for (int k = 0; k < n; ++k) {
      bp.w[k] = plane_ptr(k * (ch + 1), l);
      for (int c = 0; c < ch; ++c) {
        bp.g[k][c] = plane_ptr(k * (ch + 1) + 1 + c, l);
        bp.gc[k][c] = l + 1 < L ? plane_ptr(k * (ch + 1) + 1 + c, l + 1) : nullptr;
      }
    }
    for (int c = 0; c < ch; ++c) {
      bp.rc[c] = l + 1 < L ? bufs.acc + (size_t)c * tot + loff[l + 1] : nullptr;
      bp.out[c] = l == 0 ? out + (size_t)c * N : bufs.acc + (size_t)c * tot + loff[l];
    }
    const int cw = l + 1 < L ? lw[l + 1] : 1, chh = l + 1 < L ? lh[l + 1] : 1;
    const int top = l + 1 == L ? 1 : 0;
    const size_t per_plane = (size_t)kCH * kCW * sizeof(float);
    int cg = ch;  // channels per launch, so that the coarse tiles fit in 64 KB of LDS
    while (cg > 1 && (size_t)(n + 1) * cg * per_plane > 64 * 1024) --cg;
    if ((size_t)(n + 1) * per_plane > 64 * 1024) {  // stacks of more than 15 frames
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_blend),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)((n + 1) * per_plane));
      if (e != hipSuccess) return e;
    }
    if ((size_t)lw[l] * lh[l] <= kBlendPxMax) {
      LNR_LAUNCH(k_blend_px, dim3((lw[l] * lh[l] + 255) / 256, ch), dim3(256), 0, st, bp, n,
                 lw[l], lh[l], cw, chh, top);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      continue;
    }
    for (int c0 = 0; c0 < ch; c0 += cg) {
      const int g = min(cg, ch - c0);
      const size_t lds = top ? 0 : (size_t)(n + 1) * g * per_plane;
      // float4 path: width a multiple of 4 and every plane 16-byte aligned
      bool vec = lw[l] % 4 == 0;
      auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
      for (int k = 0; k < n && vec; ++k) {
        vec = vec && al(bp.w[k]);
        for (int c = c0; c < c0 + g; ++c) vec = vec && al(bp.g[k][c]);
      }
      for (int c = c0; c < c0 + g; ++c) vec = vec && al(bp.out[c]);
      LNR_LAUNCH(k_blend, dim3((lw[l] + kBW - 1) / kBW, (lh[l] + kBH - 1) / kBH), dim3(256),
                 lds, st, bp, n, c0, g, lw[l], lh[l], cw, chh, top, vec ? 1 : 0);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_irradiance(int n, int ch, int W, int H, const float* const* imgs,
                             const float* const* yeqs, const float* rel, int ref_index,
                             const lnr_params& p, float* ssim, float* out, hipStream_t st) {
  hipError_t e;
  if ((e = launch_ssim_maps(n, W, H, yeqs, ref_index, p, ssim, st)) != hipSuccess) return e;
  const long long N = (long long)W * H;
  IrrPtrs f;
  for (int k = 0; k < 16; ++k) {
    f.img[k] = k < n ? imgs[k] : nullptr;
    f.ssim[k] = k < n && k != ref_index ? ssim + (size_t)k * N : nullptr;
    f.rel[k] = k < n ? rel[k] : 1.f;
  }
  const dim3 g((unsigned)((N + 255) / 256));
  if (n <= 2)
    LNR_LAUNCH(k_irradiance<2>, g, dim3(256), 0, st, f, n, ch, ref_index, N, out);
  else if (n <= 4)
    LNR_LAUNCH(k_irradiance<4>, g, dim3(256), 0, st, f, n, ch, ref_index, N, out);
  else if (n <= 8)
    LNR_LAUNCH(k_irradiance<8>, g, dim3(256), 0, st, f, n, ch, ref_index, N, out);
  else
    LNR_LAUNCH(k_irradiance<16>, g, dim3(256), 0, st, f, n, ch, ref_index, N, out);
  return hipGetLastError();
}

}  // namespace lnr
