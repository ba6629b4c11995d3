// k_equalize.hip -- exposure normalisation (histogram equalisation, applied to
// every input before matching: paper Sec. 3 opening) and the matching pyramid
// (Sec. 2.2 / 2.6: up to 5 levels, 2x2 box mean rounded half up).
//
// k_hist: LDS histograms (16 copies; a wave per row, two rows per wave, 32-bit
// loads), one global atomic add per bin per block.
// k_lut_pyr: each block rebuilds the 256-entry LUT from the histogram (wave
// prefix sums), equalises a 64x64 block of Y and writes pyramid levels 1..L-1
// of that block from LDS, so the pyramid costs no extra pass over HBM; the
// reference's block is also written column-major for the propagation.
#include "lnr_internal.h"

namespace lnr {
namespace {

constexpr int kHistRows = 8;  // rows per block, two per wave

constexpr int kCopies = 16, kCopyStride = 257;  // odd stride: copies hit different banks

__global__ __launch_bounds__(256) void k_hist(const uint8_t* __restrict__ y0, int s0,
                                              const uint8_t* __restrict__ y1, int s1, int W,
                                              int H, uint32_t* __restrict__ hist) {
  // neighbouring pixels share values, so lanes spread their LDS atomics over
  // 16 copies of the bins
  __shared__ uint32_t bins[kCopies * kCopyStride];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < kCopies * kCopyStride; i += 256) bins[i] = 0;
  __syncthreads();
  const uint8_t* img = blockIdx.y ? y1 : y0;
  const int stride = blockIdx.y ? s1 : s0;
  uint32_t* mine = bins + (lane & (kCopies - 1)) * kCopyStride;
  for (int row = blockIdx.x * kHistRows + wave; row < min(H, (blockIdx.x + 1) * kHistRows);
       row += 4) {
    // the row as aligned 32-bit words plus unaligned head and tail bytes
    const uint8_t* p = img + (size_t)row * stride;
    const int head = min(W, (int)((4 - ((uintptr_t)p & 3)) & 3));
    const int nw = (W - head) >> 2;
    const int tail = W - head - 4 * nw;
    if (lane < head) atomicAdd(&mine[p[lane]], 1u);
    if (lane < tail) atomicAdd(&mine[p[head + 4 * nw + lane]], 1u);
    const uint32_t* pw = reinterpret_cast<const uint32_t*>(p + head);
    for (int i0 = lane; i0 < nw; i0 += 64 * 4) {
      uint32_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = pw[min(i0 + 64 * u, nw - 1)];  // in bounds, used if < nw
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + 64 * u < nw) {
          atomicAdd(&mine[v[u] & 255u], 1u);
          atomicAdd(&mine[(v[u] >> 8) & 255u], 1u);
          atomicAdd(&mine[(v[u] >> 16) & 255u], 1u);
          atomicAdd(&mine[v[u] >> 24], 1u);
        }
    }
  }
  __syncthreads();
  uint32_t s = 0;
  for (int c = 0; c < kCopies; ++c) s += bins[c * kCopyStride + tid];
  if (s) atomicAdd(&hist[blockIdx.y * 256 + tid], s);
}

// LUT[v] = round-half-up(255 (cdf[v] - cdf_min) / (n - cdf_min)), cdf_min the
// cdf at the first occupied bin; identity when the image has one value. The
// cdf is a wave scan per 64 bins plus the wave totals.
__device__ void build_lut(const uint32_t* __restrict__ hist, uint8_t* lut) {
  __shared__ uint32_t wsum[4];
  __shared__ int wfirst[4];
  const int v = threadIdx.x, lane = v & 63, wave = v >> 6;
  const uint32_t h = hist[v];
  uint32_t incl = h;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  const unsigned long long occ = __ballot(h != 0u);
  if (lane == 63) {
    wsum[wave] = incl;
    wfirst[wave] = occ ? wave * 64 + __ffsll((long long)occ) - 1 : 256;
  }
  __syncthreads();
  uint32_t before = 0, n = 0;
  int first = 256;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    before += q < wave ? wsum[q] : 0u;
    n += wsum[q];
    first = min(first, wfirst[q]);
  }
  const uint32_t cdf = before + incl;
  const int64_t c0 = first < 256 ? (int64_t)hist[first] : 0;  // cdf at the first occupied bin
  int64_t num = (int64_t)cdf - c0;
  if (num < 0) num = 0;
  const int64_t den = (int64_t)n - c0;
  lut[v] = den == 0 ? (uint8_t)v : (uint8_t)((2 * 255 * num + den) / (2 * den));
  __syncthreads();
}

struct LevelGeom {
  int w[kMaxLevels], h[kMaxLevels];
  long long off[kMaxLevels];
  int levels;
};

__global__ __launch_bounds__(256) void k_lut_pyr(const uint8_t* __restrict__ y0, int s0,
                                                 const uint8_t* __restrict__ y1, int s1,
                                                 const uint32_t* __restrict__ hist,
                                                 LevelGeom g, uint8_t* __restrict__ pyr0,
                                                 uint8_t* __restrict__ pyr1,
                                                 uint8_t* __restrict__ lut_out,
                                                 uint8_t* __restrict__ out0,
                                                 uint8_t* __restrict__ out1,
                                                 uint8_t* __restrict__ gt0, int hp) {
  __shared__ uint8_t lut[256];
  __shared__ uint8_t tileA[64 * 64];
  __shared__ uint8_t tileB[32 * 32];
  const int f = blockIdx.z, tid = threadIdx.x;
  build_lut(hist + f * 256, lut);
  if (lut_out && blockIdx.x == 0 && blockIdx.y == 0) lut_out[f * 256 + tid] = lut[tid];
  const uint8_t* img = f ? y1 : y0;
  const int stride = f ? s1 : s0;
  uint8_t* pyr = f ? pyr1 : pyr0;
  uint8_t* cpy = f ? out1 : out0;  // optional second copy of level 0
  const int bx = blockIdx.x * 64, by = blockIdx.y * 64;
  const int W = g.w[0], H = g.h[0];
  // level 0: 64 x 64 block, four 4-byte groups per thread (one 32-bit load
  // and store each where the row allows, all loads in flight first)
  uint32_t raw[4];
  bool wide[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = tid + 256 * u;
    const int r = i >> 4, c4 = (i & 15) * 4;
    const int y = min(by + r, H - 1), x = bx + c4;
    const uint8_t* src = img + (size_t)y * stride + x;
    wide[u] = x + 4 <= W && ((reinterpret_cast<uintptr_t>(src) & 3u) == 0);
    raw[u] = 0u;
    if (wide[u]) {
      raw[u] = *reinterpret_cast<const uint32_t*>(src);
    } else {
      for (int k = 0; k < 4; ++k)
        if (x + k < W) raw[u] |= (uint32_t)src[k] << (8 * k);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = tid + 256 * u;
    const int r = i >> 4, c4 = (i & 15) * 4;
    const int y = by + r, x = bx + c4;
    uint32_t packed = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (x + k < W) packed |= (uint32_t)lut[(raw[u] >> (8 * k)) & 255u] << (8 * k);
    if (y < H) {
      for (int c = 0; c < 2; ++c) {
        uint8_t* dst = c == 0 ? pyr + g.off[0] + (size_t)y * W + x
                              : (cpy ? cpy + (size_t)y * W + x : nullptr);
        if (!dst) break;
        if (wide[u] && ((reinterpret_cast<uintptr_t>(dst) & 3u) == 0)) {
          *reinterpret_cast<uint32_t*>(dst) = packed;
        } else {
          for (int k = 0; k < 4; ++k)
            if (x + k < W) dst[k] = (uint8_t)(packed >> (8 * k));
        }
      }
    } else {
      packed = 0;
    }
    *reinterpret_cast<uint32_t*>(&tileA[r * 64 + c4]) = packed;
  }
  __syncthreads();
  if (f == 0 && gt0) store_tile_columns(tileA, bx, by, W, hp, gt0);
  // levels 1.. from the block in LDS; level l of this block covers
  // [bx >> l, (bx >> l) + (64 >> l)) and only pixels inside the level are kept.
  uint8_t* cur = tileA;
  uint8_t* nxt = tileB;
  int side = 64;
  for (int l = 1; l < g.levels; ++l) {
    const int ns = side >> 1;
    const int ox = bx >> l, oy = by >> l;
    for (int i = tid; i < ns * ns; i += 256) {
      const int r = i / ns, c = i % ns;
      const int s = cur[(2 * r) * side + 2 * c] + cur[(2 * r) * side + 2 * c + 1] +
                    cur[(2 * r + 1) * side + 2 * c] + cur[(2 * r + 1) * side + 2 * c + 1];
      const uint8_t val = (uint8_t)((s + 2) >> 2);
      nxt[r * ns + c] = val;
      const int x = ox + c, y = oy + r;
      if (x < g.w[l] && y < g.h[l]) pyr[g.off[l] + (size_t)y * g.w[l] + x] = val;
    }
    __syncthreads();
    uint8_t* t = cur;  // both buffers hold any level from 32 x 32 down
    cur = nxt;
    nxt = t;
    side = ns;
  }
}

// Metering decision (Sec. 2.1) from a 256-bin luma histogram: the pixels
// below `dark`, and 2, 3 or 4 stops by their share of npix (compared in
// double precision). One wave.
__global__ __launch_bounds__(64) void k_meter(const uint32_t* __restrict__ hist, int dark,
                                              float frac3, float frac4, long long npix,
                                              int32_t* __restrict__ out) {
  const int lane = threadIdx.x;
  unsigned long long c = 0;
  for (int v = lane; v < 256; v += 64)
    if (v < dark) c += hist[v];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (lane == 0) {
    const double n = (double)npix;
    out[0] = (double)c <= (double)frac3 * n ? 2 : ((double)c <= (double)frac4 * n ? 3 : 4);
    out[1] = (int32_t)c;
  }
}

}  // namespace

hipError_t launch_meter(const uint32_t* hist, int dark, float frac3, float frac4,
                        long long npix, int32_t* out, hipStream_t st) {
  LNR_LAUNCH(k_meter, dim3(1), dim3(64), 0, st, hist, dark, frac3, frac4, npix, out);
  return hipGetLastError();
}

hipError_t launch_hist(const uint8_t* y0, int s0, const uint8_t* y1, int s1, int W, int H,
                       uint32_t* hist, int nframes, hipStream_t st) {
  dim3 grid((H + kHistRows - 1) / kHistRows, nframes);
  LNR_LAUNCH(k_hist, grid, dim3(256), 0, st, y0, s0, y1, s1, W, H, hist);
  return hipGetLastError();
}

hipError_t launch_lut_pyr(const uint8_t* y0, int s0, const uint8_t* y1, int s1,
                          const uint32_t* hist, const Geometry& geo, uint8_t* pyr0,
                          uint8_t* pyr1, uint8_t* lut_out, int nframes, hipStream_t st,
                          uint8_t* out0, uint8_t* out1, uint8_t* gt0) {
  LevelGeom g;
  g.levels = geo.levels;
  for (int l = 0; l < kMaxLevels; ++l) {
    g.w[l] = l < geo.levels ? geo.lv[l].w : 0;
    g.h[l] = l < geo.levels ? geo.lv[l].h : 0;
    g.off[l] = l < geo.levels ? (long long)geo.lv[l].pix_off : 0;
  }
  dim3 grid((geo.W + 63) / 64, (geo.H + 63) / 64, nframes);
  LNR_LAUNCH(k_lut_pyr, grid, dim3(256), 0, st, y0, s0, y1, s1, hist, g, pyr0, pyr1,
                     lut_out, out0, out1, gt0, dt_guide_stride(geo.H));
  return hipGetLastError();
}

}  // namespace lnr
