// k_merge.hip -- error-tolerant exposure fusion (paper Sec. 2.5): Mertens et
// al.'s contrast, saturation and well-exposedness weights, times the SSIM
// between the equalised reference and each warped frame (Wang et al.:
// Gaussian window, five filterings), blended with Laplacian pyramids.
//
//  k_ssim:    32x16 output tile; the two luma maps (+ halo) are staged in LDS,
//             the five horizontal Gaussian sums are kept in LDS, then the
//             vertical sums give SSIM. The sums are double precision: SSIM
//             divides covariance errors by sx^2 + sy^2 + C2 (~1e-3 in flat
//             regions) and the fusion weights amplify them again.
//  k_weights: per pixel, every frame's C * S * E (* max(SSIM, 0)) + 1e-12,
//             normalised over the frames.
//  k_reduce:  REDUCE ([1 4 6 4 1]/16 separable, clamped, even samples) of
//             every weight and image plane of one level, through LDS.
//  k_blend:   from the top level down, R_l = sum_k W_k,l (G_k,l - E(G_k,l+1))
//             + E(R_l+1), E the EXPAND rule, on 64x16 tiles whose coarse
//             neighbourhoods are staged (and row-expanded) in LDS; level 0
//             goes to the output.
#include "lnr_internal.h"

namespace lnr {
namespace {

struct FramePtrs {
  const float* img[16];
  const float* ssim[16];
  float* wout[16];
};

constexpr int kMaxMaps = 64;
constexpr int kSsimTW = 32, kSsimTH = 16, kSsimMaxR = 8;

// The five Gaussian sums (x, y, x^2, y^2, xy) are accumulated in double
// precision: SSIM divides covariance errors by sx^2 + sy^2 + C2 (~1e-3 in flat
// regions) and the fusion weights amplify them again near SSIM = 0, so float
// sums of E[x^2] - E[x]^2 are not accurate enough there.
__global__ __launch_bounds__(256) void k_ssim(const float* __restrict__ a,
                                              const float* __restrict__ b, int W, int H, int r,
                                              double sigma, double c1, double c2,
                                              float* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int rows = kSsimTH + 2 * r, cols = kSsimTW + 2 * r;
  const int n5 = rows * kSsimTW;
  double* hv = reinterpret_cast<double*>(smem);                  // [5][rows][TW]
  float* sa = reinterpret_cast<float*>(hv + 5 * n5);            // [rows][cols]
  float* sb = sa + rows * cols;
  __shared__ double gw[2 * kSsimMaxR + 1];
  if (tid == 0) {
    double g[2 * kSsimMaxR + 1], s = 0;
    for (int k = -r; k <= r; ++k) {
      g[k + r] = exp(-(double)(k * k) / (2.0 * sigma * sigma));
      s += g[k + r];
    }
    for (int k = 0; k <= 2 * r; ++k) gw[k] = g[k] / s;
  }
  int bx, by;
  xcd_block(gridDim.x, gridDim.y, bx, by);
  const int ox = bx * kSsimTW, oy = by * kSsimTH;
#pragma unroll 4
  for (int i = tid; i < rows * cols; i += 256) {
    const int yy = i / cols, xx = i % cols;
    const int gy = min(max(oy + yy - r, 0), H - 1), gx = min(max(ox + xx - r, 0), W - 1);
    sa[i] = a[(size_t)gy * W + gx];
    sb[i] = b[(size_t)gy * W + gx];
  }
  __syncthreads();
  for (int i = tid; i < n5; i += 256) {
    const int yy = i / kSsimTW, xx = i % kSsimTW;
    double m1 = 0, m2 = 0, s11 = 0, s22 = 0, s12 = 0;
    const float* ra = sa + yy * cols + xx;
    const float* rb = sb + yy * cols + xx;
    for (int k = 0; k <= 2 * r; ++k) {
      const double p = ra[k], q = rb[k], wd = gw[k];
      m1 += wd * p;
      m2 += wd * q;
      s11 += wd * (p * p);
      s22 += wd * (q * q);
      s12 += wd * (p * q);
    }
    hv[i] = m1; hv[n5 + i] = m2; hv[2 * n5 + i] = s11; hv[3 * n5 + i] = s22; hv[4 * n5 + i] = s12;
  }
  __syncthreads();
  // vertical sums: a thread owns two consecutive output rows of one column,
  // so 2r + 2 horizontal sums serve both
  {
    const int xx = tid % kSsimTW, yy = 2 * (tid / kSsimTW);  // rows yy, yy + 1
    double acc[2][5];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int t = 0; t < 5; ++t) acc[q][t] = 0.0;
    for (int k = 0; k <= 2 * r + 1; ++k) {
      const int j = (yy + k) * kSsimTW + xx;
      double hvv[5];
#pragma unroll
      for (int t = 0; t < 5; ++t) hvv[t] = hv[t * n5 + j];
      if (k <= 2 * r) {
        const double wd = gw[k];
#pragma unroll
        for (int t = 0; t < 5; ++t) acc[0][t] += wd * hvv[t];
      }
      if (k >= 1) {
        const double wd = gw[k - 1];
#pragma unroll
        for (int t = 0; t < 5; ++t) acc[1][t] += wd * hvv[t];
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int gy = oy + yy + q, gx = ox + xx;
      if (gy >= H || gx >= W) continue;
      const double m1 = acc[q][0], m2 = acc[q][1];
      const double vx = acc[q][2] - m1 * m1, vy = acc[q][3] - m2 * m2, cxy = acc[q][4] - m1 * m2;
      out[(size_t)gy * W + gx] = (float)(((2.0 * m1 * m2 + c1) * (2.0 * cxy + c2)) /
                                         ((m1 * m1 + m2 * m2 + c1) * (vx + vy + c2)));
    }
  }
}

__device__ inline double grey_at(const float* I, int ch, size_t plane, size_t o) {
  return ch == 3 ? (0.299 * (double)I[o] + 0.587 * (double)I[plane + o]) + 0.114 * (double)I[2 * plane + o]
                 : (double)I[o];
}

// C * S * E (* max(SSIM, 0)) of frame k at one pixel. Contrast and saturation
// are differences of nearly equal values in flat regions, and the normalised
// weights divide by their sum, which can be ~1e-12 there: they are evaluated
// in double precision.
__device__ inline double raw_weight(const FramePtrs& f, int k, int ch, int ref, size_t plane,
                                    size_t o, size_t oU, size_t oL, size_t oR, size_t oD,
                                    float two_se2) {
  const float* I = f.img[k];
  const double lap = grey_at(I, ch, plane, oU) + grey_at(I, ch, plane, oL) +
                     grey_at(I, ch, plane, oR) + grey_at(I, ch, plane, oD) -
                     4.0 * grey_at(I, ch, plane, o);
  const double C = fabs(lap);
  double S = 1.0;
  float e;
  if (ch == 3) {
    const double R = I[o], G = I[plane + o], B = I[2 * plane + o];
    const double mu = (R + G + B) * (1.0 / 3.0);
    const double var = ((R - mu) * (R - mu) + (G - mu) * (G - mu) + (B - mu) * (B - mu)) * (1.0 / 3.0);
    S = (double)sqrtf((float)var);  // the cancelling differences are in double
    e = (float)((R - 0.5) * (R - 0.5) + (G - 0.5) * (G - 0.5) + (B - 0.5) * (B - 0.5));
  } else {
    e = (float)((I[o] - 0.5) * (I[o] - 0.5));
  }
  double wt = C * S * (double)expf(-e / two_se2);
  if (k != ref) wt *= fmax((double)f.ssim[k][o], 0.0);
  return wt + 1e-12;
}

__global__ __launch_bounds__(256) void k_weights(FramePtrs f, int n, int ch, int W, int H,
                                                 int ref, float two_se2) {
  int bx, y;
  xcd_block(gridDim.x, gridDim.y, bx, y);  // rows y - 1, y, y + 1 in one L2
  const int x = bx * blockDim.x + threadIdx.x;
  if (x >= W) return;
  const size_t plane = (size_t)W * H, o = (size_t)y * W + x;
  const size_t oU = (size_t)max(y - 1, 0) * W + x, oD = (size_t)min(y + 1, H - 1) * W + x;
  const size_t oL = (size_t)y * W + max(x - 1, 0), oR = (size_t)y * W + min(x + 1, W - 1);
  // the raw weights keep 24-bit relative precision as floats once the
  // cancelling differences inside them were taken in double precision
  float wk[16];  // n <= 16; kept in registers (every index is a constant)
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    wk[k] = k < n ? (float)raw_weight(f, k, ch, ref, plane, o, oU, oL, oR, oD, two_se2) : 0.f;
    sum += (double)wk[k];
  }
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < n) f.wout[k][o] = (float)((double)wk[k] / sum);
}

struct MapPtrs {
  const float* in[kMaxMaps];
  float* out[kMaxMaps];
};

constexpr int kRedTW = 64, kRedTH = 8;

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
constexpr int kCW = kBW / 2 + 2, kCH = kBH / 2 + 2;  // coarse tile with its EXPAND halo

// One 64 x 16 tile of level l, channels [c0, c0 + cg):
//   R_l = sum_k W_k (G_k - E(G_k,l+1)) + E(R_l+1).
// EXPAND (even 2i: (c[i-1] + 6 c[i] + c[i+1]) / 8, odd 2i+1: (c[i] + c[i+1]) / 2,
// clamped coarse indices; rows first, then columns) reads the coarse planes
// from LDS tiles loaded once per block and expanded along x in LDS. Each
// thread owns one column of the tile (4 rows) and reads each weight once.
__device__ inline float expand_col(const float* col, int lj, bool even) {
  return even ? (col[(lj - 1) * kBW] + 6.f * col[lj * kBW] + col[(lj + 1) * kBW]) / 8.f
              : (col[lj * kBW] + col[(lj + 1) * kBW]) / 2.f;
}

__device__ inline float4 expand_col4(const float* col, int lj, bool even) {
  const float4 m = *reinterpret_cast<const float4*>(col + lj * kBW);
  const float4 p = *reinterpret_cast<const float4*>(col + (lj + 1) * kBW);
  if (even) {
    const float4 a = *reinterpret_cast<const float4*>(col + (lj - 1) * kBW);
    return make_float4((a.x + 6.f * m.x + p.x) / 8.f, (a.y + 6.f * m.y + p.y) / 8.f,
                       (a.z + 6.f * m.z + p.z) / 8.f, (a.w + 6.f * m.w + p.w) / 8.f);
  }
  return make_float4((m.x + p.x) / 2.f, (m.y + p.y) / 2.f, (m.z + p.z) / 2.f, (m.w + p.w) / 2.f);
}

__global__ __launch_bounds__(256) void k_blend(BlendPtrs b, int n, int c0, int cg, int w, int h,
                                               int cw, int chh, int top, int vec) {
  extern __shared__ float sm[];
  const int tid = threadIdx.x;
  int bx, by;
  xcd_block(gridDim.x, gridDim.y, bx, by);
  const int ox = bx * kBW, oy = by * kBH;
  const int cx0 = (ox >> 1) - 1, cy0 = (oy >> 1) - 1;
  const int nm = top ? 0 : (n + 1) * cg;  // plane m = cc (n + 1) + k, k = n: R
  float* ct = sm;                         // [nm][kCH][kCW] coarse tiles
  float* rx = sm + nm * kCH * kCW;        // [nm][kCH][kBW] expanded along x
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
    for (int i = tid; i < nm * kCH * kBW; i += 256) {
      const int m = i / (kCH * kBW), r = (i / kBW) % kCH, fx = i % kBW;
      const float* row = ct + (m * kCH + r) * kCW;
      const int li = ((ox + fx) >> 1) - cx0;  // local index of coarse i
      rx[i] = ((ox + fx) & 1) == 0 ? (row[li - 1] + 6.f * row[li] + row[li + 1]) / 8.f
                                    : (row[li] + row[li + 1]) / 2.f;
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
    const int lj = (y >> 1) - cy0;
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
                             : expand_col4(rx + (cc * (n + 1) + k) * kCH * kBW + xq, lj, even);
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
        const float4 e = expand_col4(rx + (cc * (n + 1) + n) * kCH * kBW + xq, lj, even);
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
      const float* col = rx + (cc * (n + 1) + k) * kCH * kBW + fx;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int y = oy + fy0 + 4 * q;
        if (y >= h) break;
        const float e = top ? 0.f : expand_col(col, (y >> 1) - cy0, (y & 1) == 0);
        acc[cc][q] += wv[q] * (gv[cc][q] - e);
      }
    }
  }
  for (int cc = 0; cc < cg; ++cc) {
    const float* col = rx + (cc * (n + 1) + n) * kCH * kBW + fx;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int y = oy + fy0 + 4 * q;
      if (y >= h) break;
      const float v = top ? acc[cc][q] : acc[cc][q] + expand_col(col, (y >> 1) - cy0, (y & 1) == 0);
      b.out[c0 + cc][(size_t)y * w + x] = v;
    }
  }
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
  // SSIM of every warped frame against the reference
  FramePtrs fp;
  for (int k = 0; k < n; ++k) {
    fp.img[k] = imgs[k];
    fp.ssim[k] = bufs.ssim + (size_t)k * N;
    fp.wout[k] = bufs.w0 + (size_t)k * N;
    if (k == ref_index) continue;
    dim3 g((W + kSsimTW - 1) / kSsimTW, (H + kSsimTH - 1) / kSsimTH);
    const int r = p.ssim_radius, rows = kSsimTH + 2 * r, cols = kSsimTW + 2 * r;
    const size_t lds = (size_t)rows * kSsimTW * 5 * 8 + (size_t)rows * cols * 8;
    LNR_LAUNCH(k_ssim, g, dim3(256), lds, st, yeqs[ref_index], yeqs[k], W, H,
                       p.ssim_radius, p.ssim_sigma, p.ssim_c1, p.ssim_c2,
                       bufs.ssim + (size_t)k * N);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  LNR_LAUNCH(k_weights, dim3((W + 255) / 256, H), dim3(256), 0, st, fp, n, ch, W, H,
                     ref_index, (float)(2.0 * p.sigma_e * p.sigma_e));
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
    const size_t per_plane = (size_t)kCH * (kCW + kBW) * sizeof(float);
    int cg = ch;  // channels per launch, so that the coarse tiles fit in 64 KB of LDS
    while (cg > 1 && (size_t)(n + 1) * cg * per_plane > 64 * 1024) --cg;
    if ((size_t)(n + 1) * per_plane > 64 * 1024) {  // stacks of more than 15 frames
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_blend),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)((n + 1) * per_plane));
      if (e != hipSuccess) return e;
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

}  // namespace lnr
