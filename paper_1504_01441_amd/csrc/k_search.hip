// k_search.hip -- the matcher of paper Sec. 2.2 on one pyramid level.
//
// k_warp_q8: the source level warped by the previous level's homography
// (Eq. 3, evaluated as a resampling). Sample positions are computed in double
// precision in a fixed operation order, rounded half up to 1/256 px, and
// blended with integer Q16 weights, so the result is exact integers.
//
// k_search: one workgroup per full tile.
//  1. The tile's reference region (every candidate's quadrants and patch) is
//     staged in LDS; 4 threads per candidate sum its quadrants (Eq. 1), Eq. 2
//     gates, and an LDS atomicMax on (C << 8 | 255 - index) picks the first
//     largest cornerness.
//  2. The warped source window around the corner (patch + 2R) is staged in
//     LDS, 0 outside the image.
//  3. Thread (dy, strip) scores KX consecutive dx. The SSD is computed exactly
//     as  sum r^2 + sum w^2 - 2 sum r w : the cross term uses v_dot4_u32_u8 on
//     the packed patch rows against window dwords realigned with
//     v_alignbyte_b32 (about 0.5 VALU instructions per pixel-candidate); the
//     window energies are column sums of LDS row energies (also v_dot4).
//  Staging reads aligned dwords (realigned in registers), several in flight
//  per thread: the kernel's latency, not its arithmetic, bounds the coarse
//  levels, which have few tiles. The region, its row sums and the window
//  share one dynamic allocation sized for the parameters (about 14 KB at
//  level 0), so that ten 3-wave workgroups fit on a CU.
//  4. The argmin key (ssd << 32 | (|dx|+|dy|) << 16 | (dy+R) << 8 | (dx+R)) is
//     reduced with wave shuffles and LDS; equal keys cannot occur, so the
//     result does not depend on the reduction order.
// With `Hlit` (Eq. 3 taken literally) the window is the unwarped source
// around q = round(Hp x) for the tile's corner x, Hp the pixel homography of
// the previous level; ties are ordered on the offset from q and the result
// is the absolute displacement q + d - x.
#include "lnr_device.h"
#include "lnr_internal.h"

namespace lnr {
namespace {

constexpr int KX = 8;        // candidates per thread (consecutive dx)
constexpr int NW = 6;        // patch row dwords (2P+1 <= 24)

__device__ inline long long q8(double s) {
  double q = floor(s * 256.0 + 0.5);
  if (!(q > -1073741824.0)) q = -1073741824.0;
  if (q > 1073741824.0) q = 1073741824.0;
  return (long long)q;
}

__device__ inline uint32_t warp_px(const uint8_t* __restrict__ src, int w, int h,
                                   const double* hp, int x, int y) {
  const double X = (double)x, Y = (double)y;
  const double den = (hp[6] * X + hp[7] * Y) + hp[8];
  const double sx = ((hp[0] * X + hp[1] * Y) + hp[2]) / den;
  const double sy = ((hp[3] * X + hp[4] * Y) + hp[5]) / den;
  const long long QX = q8(sx), QY = q8(sy);
  const long long ix = QX >> 8, iy = QY >> 8;
  const uint32_t fx = (uint32_t)(QX & 255), fy = (uint32_t)(QY & 255);
  const int x0 = (int)(ix < 0 ? 0 : (ix > w - 1 ? w - 1 : ix));
  const int x1 = (int)(ix + 1 < 0 ? 0 : (ix + 1 > w - 1 ? w - 1 : ix + 1));
  const int y0 = (int)(iy < 0 ? 0 : (iy > h - 1 ? h - 1 : iy));
  const int y1 = (int)(iy + 1 < 0 ? 0 : (iy + 1 > h - 1 ? h - 1 : iy + 1));
  const uint32_t p00 = src[(size_t)y0 * w + x0], p10 = src[(size_t)y0 * w + x1];
  const uint32_t p01 = src[(size_t)y1 * w + x0], p11 = src[(size_t)y1 * w + x1];
  const uint32_t acc = (256 - fx) * (256 - fy) * p00 + fx * (256 - fy) * p10 +
                       (256 - fx) * fy * p01 + fx * fy * p11;
  return (acc + 32768u) >> 16;
}

// Four consecutive pixels per thread, one 32-bit store when the row allows it.
// Block (0, 0) also clears the level's valid-match bits vbz[0, nwords) and
// least-squares sums (the search that follows fills the bits).
__global__ __launch_bounds__(256) void k_warp_q8(const uint8_t* __restrict__ src, int w, int h,
                                                 const double* __restrict__ Hn,
                                                 uint8_t* __restrict__ out,
                                                 unsigned long long* __restrict__ vbz, int nwords,
                                                 long long* __restrict__ sums) {
  if (vbz && blockIdx.x == 0 && blockIdx.y == 0) {
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) vbz[i] = 0ull;
    if (threadIdx.x < 24) sums[threadIdx.x] = 0;
  }
  const int x = 4 * (blockIdx.x * blockDim.x + threadIdx.x), y = blockIdx.y;
  if (x >= w) return;
  // every thread forms the pixel homography itself (uniform, no barrier)
  double hp[9];
  pixel_homography(Hn, w, h, hp);
  uint8_t* row = out + (size_t)y * w;
  if (x + 4 <= w && ((reinterpret_cast<uintptr_t>(row + x) & 3u) == 0)) {
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) v |= warp_px(src, w, h, hp, x + k, y) << (8 * k);
    *reinterpret_cast<uint32_t*>(row + x) = v;
  } else {
    for (int k = 0; k < 4 && x + k < w; ++k) row[x + k] = (uint8_t)warp_px(src, w, h, hp, x + k, y);
  }
}

// Copy rows [y0, y0 + nrows) x bytes [x0, x0 + 4 * ndw) of an 8-bit image
// into LDS (row stride `ldst`), 0 outside the image. Interior dwords are read
// as two aligned dwords realigned with v_alignbyte_b32, unrolled so that
// several loads are in flight per thread.
__device__ inline void stage_rows(const uint8_t* __restrict__ img, int w, int h, int x0, int y0,
                                  int nrows, int ndw, uint8_t* dst, int ldst, int tid, int nt) {
  const int total = nrows * ndw;
#pragma unroll 4
  for (int i = tid; i < total; i += nt) {
    const int r = i / ndw, j = i % ndw;
    const int gy = y0 + r, gx = x0 + 4 * j;
    uint32_t v = 0;
    if (gy >= 0 && gy < h) {
      const uint8_t* row = img + (size_t)gy * w;
      const uintptr_t addr = reinterpret_cast<uintptr_t>(row + gx);
      const int off = (int)(addr & 3u);
      const uint8_t* base = row + gx - off;  // aligned
      if (gx >= 0 && (gx - off) + 8 <= w) {
        const uint32_t lo = *reinterpret_cast<const uint32_t*>(base);
        const uint32_t hi = *reinterpret_cast<const uint32_t*>(base + 4);
        v = __builtin_amdgcn_alignbyte(hi, lo, off);
      } else {
        for (int b = 0; b < 4; ++b) {
          const int xx = gx + b;
          if (xx >= 0 && xx < w) v |= (uint32_t)row[xx] << (8 * b);
        }
      }
    }
    *reinterpret_cast<uint32_t*>(dst + r * ldst + 4 * j) = v;
  }
}

struct SearchShape {
  int R, nstrips, nthreads;
  int split;     // patch rows split over this many thread groups (partial SSDs summed in LDS)
  int NR;        // window rows = 2P + 2R + 1
  int wrow;      // window row stride in bytes (an odd number of dwords)
  int ncand;     // 2R + 1
  // workgroup memory, sized for these parameters: the reference region
  // (rows of rs bytes), the quadrant row sums, then the window
  int rs, off_hsum, off_win;
};

// nearest integer of a predicted source coordinate (half up), clamped far
// outside any image (NaN too)
__device__ inline int round_pred(double s) {
  double q = floor(s + 0.5);
  if (!(q > -1048576.0)) q = -1048576.0;
  if (q > 1048576.0) q = 1048576.0;
  return (int)q;
}

__device__ inline unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long u = __shfl_xor(v, o);
    v = u < v ? u : v;
  }
  return v;
}

__global__ __launch_bounds__(1024) void k_search(const uint8_t* __restrict__ ref,
                                                 const uint8_t* __restrict__ wimg, int w, int h,
                                                 SearchCfg c, SearchShape sh, int ntx,
                                                 int32_t* __restrict__ corner_xy,
                                                 int32_t* __restrict__ disp,
                                                 uint32_t* __restrict__ ssd_out,
                                                 uint8_t* __restrict__ flags,
                                                 const int32_t* __restrict__ centre,
                                                 const uint8_t* __restrict__ mode, int want,
                                                 unsigned long long* __restrict__ vb,
                                                 const double* __restrict__ Hlit) {
  extern __shared__ __align__(16) uint8_t dyn[];
  uint8_t* reg = dyn;
  uint32_t* hsum = reinterpret_cast<uint32_t*>(dyn + sh.off_hsum);
  __shared__ uint32_t qsum[4 * 49];
  __shared__ uint32_t best_key;
  __shared__ uint32_t refp[(2 * kMaxPatchR + 1) * NW];
  __shared__ uint32_t er_sum;
  __shared__ unsigned long long wmin[16];

  const int tid = threadIdx.x, nt = blockDim.x;
  const int tile = blockIdx.x;
  // with a proposal, each tile is searched by the launch of its mode only
  if (mode && mode[tile] != want) return;
  int cdx = centre ? centre[2 * tile] : 0, cdy = centre ? centre[2 * tile + 1] : 0;
  const int tx = tile % ntx, ty = tile / ntx;
  const int ext = c.K * c.g + (c.r > c.P ? c.r : c.P);
  const int side = 2 * ext + 1;
  const int cx0 = tx * c.S + c.S / 2, cy0 = ty * c.S + c.S / 2;
  const int rx0 = cx0 - ext, ry0 = cy0 - ext;

  // 1. corners (Eq. 1-2) ----------------------------------------------------
  // the region lies inside the tile; dword-aligned loads realigned in registers
  stage_rows(ref, w, h, rx0, ry0, side, (side + 3) / 4, reg, sh.rs, tid, nt);
  if (tid == 0) { best_key = 0u; er_sum = 0u; }
  __syncthreads();
  const int nc1 = 2 * c.K + 1, ncand = nc1 * nc1;
  // Quadrant sums as separable box sums: horizontal r-pixel sums for every
  // region row and every quadrant x-origin (left origin px - r and right
  // origin px of each candidate column a), then r-row vertical sums.
  {
    const uint32_t* rdw = reinterpret_cast<const uint32_t*>(reg);
    const int nrow = 2 * (c.K * c.g + c.r);       // rows spanned by the quadrants
    const int yo = ext - c.K * c.g - c.r;          // first such region row
    const int nxo = 2 * nc1;
    const int nd = (c.r + 3) >> 2;
    for (int i = tid; i < nrow * nxo; i += nt) {
      const int row = i / nxo, xo = i % nxo;
      const int a = xo >> 1;
      const int X0 = ext + c.g * (a - c.K) - ((xo & 1) ? 0 : c.r);
      const uint32_t* rp = rdw + (yo + row) * (sh.rs / 4) + (X0 >> 2);
      const int rsh = X0 & 3;
      uint32_t s = 0;
      for (int m = 0; m < nd; ++m) {
        const int nb = c.r - 4 * m;
        const uint32_t mask = nb >= 4 ? 0xffffffffu : ((1u << (8 * nb)) - 1u);
        const uint32_t d = __builtin_amdgcn_alignbyte(rp[m + 1], rp[m], rsh) & mask;
        s = __builtin_amdgcn_udot4(d, 0x01010101u, s, false);
      }
      hsum[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < 4 * ncand; i += nt) {
      const int ci = i >> 2, q = i & 3;
      const int a = ci % nc1, b = ci / nc1;
      // quadrants in cyclic order TL, TR, BR, BL
      const int xo = 2 * a + ((q == 0 || q == 3) ? 0 : 1);
      const int r0 = c.g * b + ((q <= 1) ? 0 : c.r);   // first row, relative to yo
      uint32_t s = 0;
      for (int yy = 0; yy < c.r; ++yy) s += hsum[(r0 + yy) * nxo + xo];
      qsum[i] = s;
    }
  }
  __syncthreads();
  for (int ci = tid; ci < ncand; ci += nt) {
    uint32_t C = 0, mn = 0xffffffffu;
    for (int j = 0; j < 4; ++j) {
      const int d = (int)qsum[4 * ci + ((j + 1) & 3)] - (int)qsum[4 * ci + j];
      const uint32_t ad = (uint32_t)(d < 0 ? -d : d);
      C += ad;
      mn = ad < mn ? ad : mn;
    }
    if (mn > (uint32_t)c.thr) atomicMax(&best_key, (C << 8) | (uint32_t)(255 - ci));
  }
  __syncthreads();
  const uint32_t bk = best_key;
  if (bk == 0u) {
    if (tid == 0) {
      corner_xy[2 * tile] = -1;
      corner_xy[2 * tile + 1] = -1;
      disp[2 * tile] = 0;
      disp[2 * tile + 1] = 0;
      ssd_out[tile] = 0;
      flags[tile] = 0;
    }
    return;
  }
  const int bci = 255 - (int)(bk & 255u);
  const int ba = bci % nc1 - c.K, bb = bci / nc1 - c.K;
  const int px = cx0 + c.g * ba, py = cy0 + c.g * bb;  // corner, level coordinates
  const int prx = ext + c.g * ba, pry = ext + c.g * bb;  // corner, region coordinates
  if (Hlit) {  // every thread predicts the corner's source position itself
    double hp[9];
    pixel_homography(Hlit, w, h, hp);
    const double X = (double)px, Y = (double)py;
    const double den = (hp[6] * X + hp[7] * Y) + hp[8];
    const double sx = ((hp[0] * X + hp[1] * Y) + hp[2]) / den;
    const double sy = ((hp[3] * X + hp[4] * Y) + hp[5]) / den;
    cdx = round_pred(sx) - px;
    cdy = round_pred(sy) - py;
  }

  // 2. packed reference patch and the warped window ------------------------
  const int P = c.P, PW = 2 * P + 1, R = sh.R;
  for (int i = tid; i < PW * NW; i += nt) {
    const int row = i / NW, dw = i % NW;
    uint32_t v = 0;
    for (int k = 0; k < 4; ++k) {
      const int col = dw * 4 + k;
      if (col < PW) v |= (uint32_t)reg[(pry - P + row) * sh.rs + prx - P + col] << (8 * k);
    }
    refp[i] = v;
  }
  uint8_t* win = dyn + sh.off_win;
  uint32_t* rowsq = reinterpret_cast<uint32_t*>(win + sh.NR * sh.wrow);
  const int wx0 = px + cdx - P - R, wy0 = py + cdy - P - R;
  stage_rows(wimg, w, h, wx0, wy0, sh.NR, sh.wrow / 4, win, sh.wrow, tid, nt);
  __syncthreads();
  // patch energy and window row energies rowsq[y][k] = sum_c win[y][k + c]^2,
  // from realigned dwords with v_dot4 (bytes past the patch width masked off)
  {
    uint32_t part = 0;
    for (int i = tid; i < PW * NW; i += nt) part = __builtin_amdgcn_udot4(refp[i], refp[i], part, false);
    if (part) atomicAdd(&er_sum, part);
  }
  {
    const uint32_t* wdw = reinterpret_cast<const uint32_t*>(win);
    const int rowdw = sh.wrow >> 2;
    for (int i = tid; i < sh.NR * sh.ncand; i += nt) {
      const int yy = i / sh.ncand, k = i % sh.ncand;
      const uint32_t* rp = wdw + yy * rowdw + (k >> 2);
      const int rsh = k & 3;
      uint32_t s2 = 0;
#pragma unroll
      for (int m = 0; m < NW; ++m) {
        const int nb = PW - 4 * m;
        const uint32_t mask = nb >= 4 ? 0xffffffffu : (nb <= 0 ? 0u : ((1u << (8 * nb)) - 1u));
        const uint32_t d = __builtin_amdgcn_alignbyte(rp[m + 1], rp[m], rsh) & mask;
        s2 = __builtin_amdgcn_udot4(d, d, s2, false);
      }
      rowsq[i] = s2;
    }
  }
  __syncthreads();

  // 3. SSD of KX candidates per thread (over a group of patch rows) -------
  unsigned long long key = ~0ull;
  const int base_threads = sh.ncand * sh.nstrips;
  const int ncp = sh.nstrips * KX;  // padded candidates per row
  uint32_t* tot = rowsq + sh.NR * sh.ncand + KX;  // [2][ncand][ncp] when split > 1
  if (sh.split > 1) {
    for (int i = tid; i < 2 * sh.ncand * ncp; i += nt) tot[i] = 0u;
    __syncthreads();
  }
  const int grp = tid / base_threads, rem = tid % base_threads;
  const int j = rem / sh.nstrips, s = rem % sh.nstrips;  // dy index, strip
  uint32_t acc[KX], ew[KX];
#pragma unroll
  for (int k = 0; k < KX; ++k) { acc[k] = 0; ew[k] = 0; }
  if (tid < sh.nthreads) {
    const uint32_t* wdw = reinterpret_cast<const uint32_t*>(win);
    const int rowdw = sh.wrow >> 2;
    const int i0 = grp * PW / sh.split, i1 = (grp + 1) * PW / sh.split;
    for (int i = i0; i < i1; ++i) {
      const uint32_t* wr = wdw + (j + i) * rowdw + s * (KX / 4);
      uint32_t wv[KX / 4 + NW + 1];
#pragma unroll
      for (int m = 0; m < KX / 4 + NW + 1; ++m) wv[m] = wr[m];
      uint32_t rr[NW];
#pragma unroll
      for (int m = 0; m < NW; ++m) rr[m] = refp[i * NW + m];
      uint32_t sft[4][KX / 4 + NW];
#pragma unroll
      for (int m = 0; m < KX / 4 + NW; ++m) {
        sft[0][m] = wv[m];
        sft[1][m] = __builtin_amdgcn_alignbyte(wv[m + 1], wv[m], 1);
        sft[2][m] = __builtin_amdgcn_alignbyte(wv[m + 1], wv[m], 2);
        sft[3][m] = __builtin_amdgcn_alignbyte(wv[m + 1], wv[m], 3);
      }
#pragma unroll
      for (int k = 0; k < KX; ++k) {
        const int q = k >> 2, rsh = k & 3;
#pragma unroll
        for (int m = 0; m < NW; ++m)
          acc[k] = __builtin_amdgcn_udot4(sft[rsh][q + m], rr[m], acc[k], false);
      }
      // window energy of the KX candidates: column sums of the row energies
      const uint32_t* rq = rowsq + (j + i) * sh.ncand + s * KX;
#pragma unroll
      for (int k = 0; k < KX; ++k) ew[k] += (s * KX + k < sh.ncand) ? rq[k] : 0u;
    }
    if (sh.split > 1) {  // exact integer partial sums: any order gives the same totals
#pragma unroll
      for (int k = 0; k < KX; ++k) {
        atomicAdd(&tot[j * ncp + s * KX + k], acc[k]);
        atomicAdd(&tot[sh.ncand * ncp + j * ncp + s * KX + k], ew[k]);
      }
    }
  }
  if (sh.split > 1) {
    __syncthreads();
    if (tid < base_threads)
#pragma unroll
      for (int k = 0; k < KX; ++k) {
        acc[k] = tot[j * ncp + s * KX + k];
        ew[k] = tot[sh.ncand * ncp + j * ncp + s * KX + k];
      }
  }
  if (tid < base_threads) {
    const uint32_t er = er_sum;
#pragma unroll
    for (int k = 0; k < KX; ++k) {
      const int dxi = s * KX + k;
      if (dxi >= sh.ncand) continue;
      const int dx = dxi - R + cdx, dy = j - R + cdy;
      if (px + dx - P < 0 || px + dx + P > w - 1 || py + dy - P < 0 || py + dy + P > h - 1)
        continue;
      const uint32_t ssd = er + ew[k] - 2u * acc[k];
      // ties on the absolute displacement, or on the offset from the
      // predicted position when the window is centred on a prediction
      const int kx = Hlit ? dxi - R : dx, ky = Hlit ? j - R : dy;
      const uint32_t l1 = (uint32_t)((kx < 0 ? -kx : kx) + (ky < 0 ? -ky : ky));
      // (ssd, |dx| + |dy|, dy, dx), displacements biased by 64 (|d| <= 64)
      const unsigned long long kk = ((unsigned long long)ssd << 32) |
                                    ((unsigned long long)l1 << 16) |
                                    ((unsigned long long)(ky + 64) << 8) |
                                    (unsigned long long)(kx + 64);
      key = kk < key ? kk : key;
    }
  }
  // 4. argmin ---------------------------------------------------------------
  key = wave_min_u64(key);
  if ((tid & 63) == 0) wmin[tid >> 6] = key;
  __syncthreads();
  if (tid == 0) {
    unsigned long long b = ~0ull;
    for (int i = 0; i < (nt + 63) / 64; ++i) b = wmin[i] < b ? wmin[i] : b;
    corner_xy[2 * tile] = px;
    corner_xy[2 * tile + 1] = py;
    if (b == ~0ull) {
      disp[2 * tile] = 0;
      disp[2 * tile + 1] = 0;
      ssd_out[tile] = 0;
      flags[tile] = (uint8_t)(1 | (mode && want ? 16 : 0));
    } else {
      disp[2 * tile] = (int)(b & 255ull) - 64 + (Hlit ? cdx : 0);
      disp[2 * tile + 1] = (int)((b >> 8) & 255ull) - 64 + (Hlit ? cdy : 0);
      ssd_out[tile] = (uint32_t)(b >> 32);
      flags[tile] = (uint8_t)(3 | (mode && want ? 16 : 0));
      if (vb) atomicOr(vb + (tile >> 6), 1ull << (tile & 63));
    }
  }
}

// A random 8-bit texture (every tile has corners): the search autotuner's input.
__global__ __launch_bounds__(256) void k_texture(uint8_t* __restrict__ p, int n, uint32_t seed) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  uint32_t z = (uint32_t)i * 0x9E3779B1u ^ seed;
  z = (z ^ (z >> 15)) * 0x2C1B3C6Du;
  z = (z ^ (z >> 12)) * 0x297A2D39u;
  p[i] = (uint8_t)(z ^ (z >> 15));
}

}  // namespace

hipError_t launch_warp_q8(const uint8_t* src, int w, int h, const double* Hn, uint8_t* out,
                          hipStream_t st, const WeedBufs* wb, int nwords) {
  dim3 grid((w + 1023) / 1024, h);
  LNR_LAUNCH(k_warp_q8, grid, dim3(256), 0, st, src, w, h, Hn, out, wb ? wb->vb : nullptr,
             nwords, wb ? wb->sums : nullptr);
  return hipGetLastError();
}

int search_split_candidates(int R, const SearchCfg& c, int* out, int max) {
  const int ncand = 2 * R + 1, base = ncand * ((ncand + KX - 1) / KX);
  int n = 0;
  for (int s = 1; s <= 7 && s <= 2 * c.P + 1 && n < max; ++s)
    if (base * s <= 1024) out[n++] = s;
  return n;
}

hipError_t launch_texture(uint8_t* p, int n, uint32_t seed, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  LNR_LAUNCH(k_texture, dim3((n + 255) / 256), dim3(256), 0, st, p, n, seed);
  return hipGetLastError();
}

hipError_t launch_search(const uint8_t* ref, const uint8_t* wimg, int w, int h, int R,
                         const SearchCfg& c, int ntx, int nty, int32_t* corner_xy,
                         int32_t* disp, uint32_t* ssd, uint8_t* flags, hipStream_t st,
                         const int32_t* centre, const uint8_t* mode, int want,
                         unsigned long long* vb, int split, const double* Hlit) {
  if (ntx * nty == 0) return hipSuccess;
  SearchShape sh;
  sh.R = R;
  sh.ncand = 2 * R + 1;
  sh.nstrips = (sh.ncand + KX - 1) / KX;
  const int base = sh.ncand * sh.nstrips;
  if (split > 0) {  // a tuned split (the results do not depend on it)
    sh.split = split;
  } else {
    // when the level has too few candidate threads to fill the chip (coarse
    // levels, small windows), split the patch rows so that a tile keeps about
    // 256 threads busy
    sh.split = (long long)ntx * nty * base >= 262144 ? 1 : (256 + base / 2) / base;
  }
  if (sh.split < 1) sh.split = 1;
  if (sh.split > 7) sh.split = 7;
  if (sh.split > 2 * c.P + 1) sh.split = 2 * c.P + 1;
  while (sh.split > 1 && base * sh.split > 1024) --sh.split;
  sh.nthreads = base * sh.split;
  sh.NR = 2 * c.P + 2 * R + 1;
  // bytes read per row: the last strip's (KX/4 + NW + 1) dwords
  const int need = (sh.nstrips * KX) + 4 * (NW + 1);
  // an odd number of dwords per row: the threads of a wave read rows
  // (j + i) at dword offsets 2 s, which an even stride maps onto the same banks
  sh.wrow = (need + 3) / 4 * 4;
  if ((sh.wrow / 4) % 2 == 0) sh.wrow += 4;
  int block = (sh.nthreads + 63) / 64 * 64;
  if (block < 64) block = 64;
  // the reference region: side rows of rs bytes, rs covering the realigned
  // dword reads of the quadrant sums (up to 6 bytes past a row's end) and one
  // spare row after the last; the quadrant row sums: 2 (K g + r) rows of
  // 2 (2K + 1) words
  const int ext = c.K * c.g + (c.r > c.P ? c.r : c.P);
  const int side = 2 * ext + 1;
  sh.rs = (side + 8 + 3) / 4 * 4;
  const int hsum_words = 2 * (c.K * c.g + c.r) * 2 * (2 * c.K + 1);
  sh.off_hsum = (sh.rs * (side + 1) + 15) / 16 * 16;
  sh.off_win = (sh.off_hsum + hsum_words * 4 + 15) / 16 * 16;
  // (+ KX words: the last strip's padded candidates read past the last row;
  // + the partial-sum totals when the rows are split)
  const size_t lds = (size_t)sh.off_win + (size_t)sh.NR * sh.wrow +
                     (size_t)sh.NR * sh.ncand * 4 + KX * 4 +
                     (sh.split > 1 ? (size_t)2 * sh.ncand * sh.nstrips * KX * 4 : 0);
  LNR_LAUNCH(k_search, dim3(ntx * nty), dim3(block), lds, st, ref, wimg, w, h, c, sh,
                     ntx, corner_xy, disp, ssd, flags, centre, mode, want, vb, Hlit);
  return hipGetLastError();
}

}  // namespace lnr
