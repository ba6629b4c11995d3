// k_search.hip -- the matcher of paper Sec. 2.2 on one pyramid level.
//
// k_warp_q8: the source level warped by the previous level's homography
// (Eq. 3, evaluated as a resampling). Sample positions are computed in double
// precision in a fixed operation order, rounded half up to 1/256 px, and
// blended with integer Q16 weights, so the result is exact integers.
//
// k_search<KX, ROLE, MB>: one workgroup per full tile of one pair's level (ROLE
// names the launch for profiles: coarse levels, level 0, stage calls and
// autotuner trials; only the coarse-level kernel carries the on-the-fly warp
// of the window, whose registers would cost the others occupancy).
// k_search_work<KX, VISIT, WARP, MB>: one workgroup per item of a
// work list: the tiles of several pairs' levels (a SearchJob table; batches),
// or a device list of tile indices (the learned proposal's window and
// fallback tiles); VISIT kVisitCornersOnly runs the corner phase alone and
// appends each cornered tile to a list.
// k_warp_jobs: k_warp_q8 over the rows of several pairs' levels.
//  1. The tile's reference region (every candidate's quadrants and patch) is
//     staged in LDS; 4 threads per candidate sum its quadrants (Eq. 1), Eq. 2
//     gates, and an LDS atomicMax on (C << 8 | 255 - index) picks the first
//     largest cornerness.
//  2. The warped source window around the corner (patch + 2R) is staged in
//     LDS, 0 outside the image.
//  3. The SSD is computed exactly as  sum r^2 + sum w^2 - 2 sum r w. KX 8 or
//     12: thread (dy, strip) scores KX consecutive dx, the cross term with
//     v_dot4 on the packed patch rows against window dwords realigned with
//     v_alignbyte_b32 (about 0.45 VALU instructions per pixel-candidate).
//     KX 0: the cross terms on the matrix cores (v_mfma_i32_16x16x64_i8,
//     window rows times the Toeplitz matrix of a patch row; MB: at most that
//     many blocks of 16 candidates), computed first, into registers, so that
//     the energies can reuse the patch rows' and the window's memory. The
//     window energies are vertical box sums (sliding, once per tile) of LDS
//     row energies (also v_dot4).
//  Staging reads aligned dwords (realigned in registers), several in flight
//  per thread: the kernel's latency, not its arithmetic, bounds the coarse
//  levels, which have few tiles. The region, its row sums, the window and
//  the energies share one dynamic allocation sized for the parameters (about
//  14 KB for the radius-16 matrix-core tile), so that ten 3-wave workgroups
//  fit on a CU.
//  4. The argmin key (ssd << 32 | (|dx|+|dy|) << 16 | (dy+R) << 8 | (dx+R)) is
//     reduced with wave shuffles and LDS; equal keys cannot occur, so the
//     result does not depend on the reduction order.
// With `Hlit` (Eq. 3 taken literally) the window is the unwarped source
// around q = round(Hp x) for the tile's corner x, Hp the pixel homography of
// the previous level; ties are ordered on the offset from q and the result
// is the absolute displacement q + d - x.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "lnr_device.h"
#include "lnr_internal.h"

namespace lnr {
namespace {

constexpr int NW = 6;        // patch row dwords (2P+1 <= 24)
constexpr int kMaxNB = 5;    // blocks of 16 candidates per axis (2R + 1 <= 65)

__device__ inline long long q8(double s) {
  double q = floor(s * 256.0 + 0.5);
  if (!(q > -1073741824.0)) q = -1073741824.0;
  if (q > 1073741824.0) q = 1073741824.0;
  return (long long)q;
}

// The Q8 sample of output pixel (x, y): the four clamped taps and the Q8
// fractions.
struct Q8Tap {
  int x0, x1, y0, y1;
  uint32_t fx, fy;
};

__device__ inline Q8Tap warp_tap(const double* hp, int w, int h, int x, int y) {
  const double X = (double)x, Y = (double)y;
  const double den = (hp[6] * X + hp[7] * Y) + hp[8];
  const double sx = ((hp[0] * X + hp[1] * Y) + hp[2]) / den;
  const double sy = ((hp[3] * X + hp[4] * Y) + hp[5]) / den;
  const long long QX = q8(sx), QY = q8(sy);
  const long long ix = QX >> 8, iy = QY >> 8;
  Q8Tap t;
  t.fx = (uint32_t)(QX & 255);
  t.fy = (uint32_t)(QY & 255);
  t.x0 = (int)(ix < 0 ? 0 : (ix > w - 1 ? w - 1 : ix));
  t.x1 = (int)(ix + 1 < 0 ? 0 : (ix + 1 > w - 1 ? w - 1 : ix + 1));
  t.y0 = (int)(iy < 0 ? 0 : (iy > h - 1 ? h - 1 : iy));
  t.y1 = (int)(iy + 1 < 0 ? 0 : (iy + 1 > h - 1 ? h - 1 : iy + 1));
  return t;
}

__device__ inline uint32_t blend_q8(uint32_t p00, uint32_t p10, uint32_t p01, uint32_t p11,
                                    uint32_t fx, uint32_t fy) {
  const uint32_t acc = (256 - fx) * (256 - fy) * p00 + fx * (256 - fy) * p10 +
                       (256 - fx) * fy * p01 + fx * fy * p11;
  return (acc + 32768u) >> 16;
}

__device__ inline uint32_t warp_px(const uint8_t* __restrict__ src, int w, int h,
                                   const double* hp, int x, int y) {
  const Q8Tap t = warp_tap(hp, w, h, x, y);
  return blend_q8(src[(size_t)t.y0 * w + t.x0], src[(size_t)t.y0 * w + t.x1],
                  src[(size_t)t.y1 * w + t.x0], src[(size_t)t.y1 * w + t.x1], t.fx, t.fy);
}

// Four consecutive pixels per thread, one 32-bit store when the row allows it.
// Block (0, 0) also clears the level's valid-match bits vbz[0, nwords) and
// least-squares sums (the search that follows fills the bits).
__global__ __launch_bounds__(256) void k_warp_q8(const uint8_t* __restrict__ src, int w, int h,
                                                 const double* __restrict__ Hn,
                                                 uint8_t* __restrict__ out,
                                                 unsigned long long* __restrict__ vbz, int nwords,
                                                 long long* __restrict__ sums,
                                                 int* __restrict__ zint, int nzint) {
  if (vbz && blockIdx.x == 0 && blockIdx.y == 0) {
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) vbz[i] = 0ull;
    if (threadIdx.x < 24) sums[threadIdx.x] = 0;
    if (threadIdx.x < nzint) zint[threadIdx.x] = 0;
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

// k_warp_q8 for a table of jobs: block b covers run b % nxb (1024 pixels) of
// row b / nxb of all the jobs' levels (job j owns rows [row0[j], row0[j + 1])).
// The first row's first run of each job clears that job's weeding bits and sums.
__global__ __launch_bounds__(256) void k_warp_jobs(const WarpJob* __restrict__ jobs,
                                                   const int* __restrict__ row0, int njobs,
                                                   int nxb) {
  const int gy = blockIdx.x / nxb, bx = blockIdx.x % nxb;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (__builtin_amdgcn_readfirstlane(row0[mid]) <= gy) lo = mid;
    else hi = mid - 1;
  }
  const WarpJob J = jobs[lo];
  const int y = gy - __builtin_amdgcn_readfirstlane(row0[lo]);
  if (y == 0 && bx == 0) {
    for (int i = threadIdx.x; i < J.nwords; i += blockDim.x) J.vb[i] = 0ull;
    if (threadIdx.x < 24) J.sums[threadIdx.x] = 0;
  }
  const int x = 4 * (bx * blockDim.x + threadIdx.x);
  if (x >= J.w) return;
  double hp[9];
  pixel_homography(J.Hn, J.w, J.h, hp);
  uint8_t* row = J.out + (size_t)y * J.w;
  if (x + 4 <= J.w && ((reinterpret_cast<uintptr_t>(row + x) & 3u) == 0)) {
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) v |= warp_px(J.src, J.w, J.h, hp, x + k, y) << (8 * k);
    *reinterpret_cast<uint32_t*>(row + x) = v;
  } else {
    for (int k = 0; k < 4 && x + k < J.w; ++k)
      row[x + k] = (uint8_t)warp_px(J.src, J.w, J.h, hp, x + k, y);
  }
}

// Copy rows [y0, y0 + nrows) x bytes [x0, x0 + 4 * ndw) of an 8-bit image
// into LDS (row stride `ldst`), 0 outside the image. Interior dwords are read
// as two aligned dwords realigned with v_alignbyte_b32, unrolled so that
// several loads are in flight per thread.
__device__ inline void stage_rows(const uint8_t* __restrict__ img, int w, int h, int x0, int y0,
                                  int nrows, int ndw, uint8_t* dst, int ldst, int tid, int nt,
                                  uint32_t flip = 0u) {
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
    *reinterpret_cast<uint32_t*>(dst + r * ldst + 4 * j) = v ^ flip;
  }
}

// stage_rows with between() run once by every thread while its first batch
// of loads (four dwords) is in flight, before their LDS stores.
template <typename F>
__device__ inline void stage_rows_around(const uint8_t* __restrict__ img, int w, int h, int x0,
                                         int y0, int nrows, int ndw, uint8_t* dst, int ldst,
                                         int tid, int nt, uint32_t flip, F&& between) {
  const int total = nrows * ndw;
  bool pending = true;
  for (int i0 = tid; i0 < total; i0 += 4 * nt) {
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * nt;
      v[u] = 0;
      if (i >= total) continue;
      const int r = i / ndw, j = i % ndw;
      const int gy = y0 + r, gx = x0 + 4 * j;
      if (gy >= 0 && gy < h) {
        const uint8_t* row = img + (size_t)gy * w;
        const uintptr_t addr = reinterpret_cast<uintptr_t>(row + gx);
        const int off = (int)(addr & 3u);
        const uint8_t* base = row + gx - off;  // aligned
        if (gx >= 0 && (gx - off) + 8 <= w) {
          const uint32_t lo = *reinterpret_cast<const uint32_t*>(base);
          const uint32_t hi = *reinterpret_cast<const uint32_t*>(base + 4);
          v[u] = __builtin_amdgcn_alignbyte(hi, lo, off);
        } else {
          for (int b = 0; b < 4; ++b) {
            const int xx = gx + b;
            if (xx >= 0 && xx < w) v[u] |= (uint32_t)row[xx] << (8 * b);
          }
        }
      }
    }
    if (pending) {
      between();
      pending = false;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * nt;
      if (i < total) {
        const int r = i / ndw, j = i % ndw;
        *reinterpret_cast<uint32_t*>(dst + r * ldst + 4 * j) = v[u] ^ flip;
      }
    }
  }
  if (pending) between();
}

// The window rows [y0, y0 + nrows) x bytes [x0, x0 + 4 * ndw) of the level
// warped on the fly: each pixel inside the level is warp_px of the unwarped
// source (the value k_warp_q8 stores there), 0 outside, as stage_rows reads
// the stored warped level; every byte XOR flip. Four pixels per thread at a
// time: their sample positions first, then all sixteen taps in flight, then
// the blends.
__device__ inline void stage_warped(const uint8_t* __restrict__ src, int w, int h,
                                    const double* hp, int x0, int y0, int nrows, int ndw,
                                    uint8_t* dst, int ldst, int tid, int nt, uint32_t flip) {
  constexpr int U = 4;
  const int total = nrows * ndw * 4;
  for (int i0 = tid; i0 < total; i0 += U * nt) {
    Q8Tap t[U];
    bool in[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * nt;
      const int r = i / (4 * ndw), b = i % (4 * ndw);
      const int gy = y0 + r, gx = x0 + b;
      in[u] = i < total && gy >= 0 && gy < h && gx >= 0 && gx < w;
      t[u] = warp_tap(hp, w, h, in[u] ? gx : 0, in[u] ? gy : 0);
    }
    uint32_t p[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint8_t* r0 = src + (size_t)t[u].y0 * w;
      const uint8_t* r1 = src + (size_t)t[u].y1 * w;
      p[u][0] = r0[t[u].x0];
      p[u][1] = r0[t[u].x1];
      p[u][2] = r1[t[u].x0];
      p[u][3] = r1[t[u].x1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * nt;
      if (i >= total) break;
      const int r = i / (4 * ndw), b = i % (4 * ndw);
      const uint32_t v = in[u] ? blend_q8(p[u][0], p[u][1], p[u][2], p[u][3], t[u].fx, t[u].fy)
                               : 0u;
      dst[r * ldst + b] = (uint8_t)(v ^ flip);
    }
  }
}

struct SearchShape {
  int R, nstrips, nthreads;
  int split;     // patch rows split over this many thread groups (partial SSDs summed in LDS)
  int NR;        // window rows = 2P + 2R + 1
  int wrow;      // window row stride in bytes
  int stage_dw;  // dwords staged per window row
  int ncand;     // 2R + 1
  // matrix-core cross terms: candidate blocks of 16 (dy and dx), 64-byte
  // chunks of a window row, the patch rows' zero padding (bytes, before the
  // patch) and their length (dwords)
  int NB, KC, padB, LB;
  // workgroup memory, sized for these parameters. 8 or 12 candidates per
  // lane: the reference region (rows of rs bytes), the quadrant row sums,
  // then the window, its row energies, the split totals, the window
  // energies. Matrix cores (the cross terms come first, into registers): the
  // window, then the reference region, the quadrant row sums and the padded
  // patch rows; the row energies then take the place of the region, the
  // sums and the patch rows, the window energies that of the window, and
  // the split totals follow. off_cend: the end of the corner phase's memory.
  int rs, off_reg, off_hsum, off_cend, off_win, off_rowsq, off_tot, off_colE, off_pb;
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

// Workgroup state shared by the phases of one tile visit.
struct TileShared {
  uint32_t qsum[4 * 49];
  uint32_t best_key;
  uint32_t refp[(2 * kMaxPatchR + 1) * NW];
  uint32_t er_sum;
  unsigned long long wmin[16];
};

typedef int v4i __attribute__((ext_vector_type(4)));

// Cross terms of one wave over patch rows [i0, i1) (see search_tile): ar is
// the wave's first A row, pr0 its first padded patch dword; every row's
// loads are issued before its NBT matrix products.
template <int NBT>
__device__ inline void cross_mfma(const uint8_t* ar, const uint32_t* pr0, int LB, int bs,
                                  int wrow, int i0, int i1, v4i* acc) {
#pragma unroll 2
  for (int i = i0; i < i1; ++i) {
    const uint32_t* pr = pr0 + i * LB;
    const uint32_t e0 = pr[0], e1 = pr[1], e2 = pr[2], e3 = pr[3], e4 = pr[4];
    const uint8_t* ai = ar + i * wrow;
    v4i A[NBT];
#pragma unroll
    for (int mb = 0; mb < NBT; ++mb) A[mb] = *reinterpret_cast<const v4i*>(ai + 16 * mb * wrow);
    const v4i B = v4i{(int)__builtin_amdgcn_alignbyte(e1, e0, bs),
                      (int)__builtin_amdgcn_alignbyte(e2, e1, bs),
                      (int)__builtin_amdgcn_alignbyte(e3, e2, bs),
                      (int)__builtin_amdgcn_alignbyte(e4, e3, bs)};
#pragma unroll
    for (int mb = 0; mb < NBT; ++mb)
      acc[mb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mb], B, acc[mb], 0, 0, 0);
  }
}

// Dword dw of patch row `row` packed from the staged region (pixel - 128 as
// a signed byte; 0 past the patch width PW): the patch's first pixel is at
// region row r0, column c0.
__device__ inline uint32_t patch_dword(const uint8_t* reg, int rs, int r0, int c0, int PW,
                                       int row, int dw) {
  const uint8_t* p = reg + (r0 + row) * rs + c0;
  uint32_t v = 0;
  for (int k = 0; k < 4; ++k) {
    const int col = dw * 4 + k;
    if (col < PW) v |= (uint32_t)(p[col] ^ 0x80u) << (8 * k);
  }
  return v;
}

// One tile of one job, by the whole workgroup (every branch below that
// skips the rest of the tile is uniform over the workgroup).
//  list / count (kVisitCornersOnly): the cornered tile's global index gidx is
//  appended to list.
template <int KX, bool WARP, int MB>
__device__ void search_tile(const SearchJob& J, int tile, int gidx, const SearchCfg& c,
                            const SearchShape& sh, int visit, int want, int* list, int* count,
                            uint8_t* dyn, TileShared& S) {
  uint8_t* reg = dyn + sh.off_reg;
  uint32_t* hsum = reinterpret_cast<uint32_t*>(dyn + sh.off_hsum);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int w = J.w, h = J.h;
  int cdx = J.centre ? J.centre[2 * tile] : 0, cdy = J.centre ? J.centre[2 * tile + 1] : 0;
  const int tx = tile % J.ntx, ty = tile / J.ntx;
  const int ext = c.K * c.g + (c.r > c.P ? c.r : c.P);
  const int cx0 = tx * c.S + c.S / 2, cy0 = ty * c.S + c.S / 2;
  int px, py;  // corner, level coordinates
  int pr0 = 0, pc0 = 0;  // the patch's first row and column in the staged region

  if (visit == kVisitKnownCorner) {
    px = J.corner_xy[2 * tile];
    py = J.corner_xy[2 * tile + 1];
    if (tid == 0) S.er_sum = 0u;
    // the patch around the known corner
    const int P = c.P, PW = 2 * P + 1;
    stage_rows(J.ref, w, h, px - P, py - P, PW, (PW + 3) / 4, reg, sh.rs, tid, nt);
    __syncthreads();
    for (int i = tid; i < PW * NW; i += nt) S.refp[i] = patch_dword(reg, sh.rs, 0, 0, PW, i / NW, i % NW);
  } else {
    // 1. corners (Eq. 1-2) --------------------------------------------------
    // the region lies inside the tile; dword-aligned loads realigned in registers
    const int side = 2 * ext + 1;
    const int rx0 = cx0 - ext, ry0 = cy0 - ext;
    stage_rows(J.ref, w, h, rx0, ry0, side, (side + 3) / 4, reg, sh.rs, tid, nt);
    if (tid == 0) { S.best_key = 0u; S.er_sum = 0u; }
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
        S.qsum[i] = s;
      }
    }
    __syncthreads();
    for (int ci = tid; ci < ncand; ci += nt) {
      uint32_t C = 0, mn = 0xffffffffu;
      for (int j = 0; j < 4; ++j) {
        const int d = (int)S.qsum[4 * ci + ((j + 1) & 3)] - (int)S.qsum[4 * ci + j];
        const uint32_t ad = (uint32_t)(d < 0 ? -d : d);
        C += ad;
        mn = ad < mn ? ad : mn;
      }
      if (mn > (uint32_t)c.thr) atomicMax(&S.best_key, (C << 8) | (uint32_t)(255 - ci));
    }
    __syncthreads();
    const uint32_t bk = S.best_key;
    if (bk == 0u) {
      if (tid == 0) {
        J.corner_xy[2 * tile] = -1;
        J.corner_xy[2 * tile + 1] = -1;
        J.disp[2 * tile] = 0;
        J.disp[2 * tile + 1] = 0;
        J.ssd[tile] = 0;
        J.flags[tile] = 0;
      }
      return;
    }
    const int bci = 255 - (int)(bk & 255u);
    const int ba = bci % nc1 - c.K, bb = bci / nc1 - c.K;
    px = cx0 + c.g * ba;
    py = cy0 + c.g * bb;
    if (visit == kVisitCornersOnly) {
      if (tid == 0) {
        J.corner_xy[2 * tile] = px;
        J.corner_xy[2 * tile + 1] = py;
        J.flags[tile] = 1;
        if (list) list[atomicAdd(count, 1)] = gidx;
      }
      return;
    }
    const int prx = ext + c.g * ba, pry = ext + c.g * bb;  // corner, region coordinates
    // packed reference patch, centred (pixel - 128 as a signed byte; 0 past
    // the patch width)
    const int P = c.P, PW = 2 * P + 1;
    pr0 = pry - P;
    pc0 = prx - P;
    for (int i = tid; i < PW * NW; i += nt)
      S.refp[i] = patch_dword(reg, sh.rs, pr0, pc0, PW, i / NW, i % NW);
  }
  if (J.Hlit) {  // every thread predicts the corner's source position itself
    double hp[9];
    pixel_homography(J.Hlit, w, h, hp);
    const double X = (double)px, Y = (double)py;
    const double den = (hp[6] * X + hp[7] * Y) + hp[8];
    const double sx = ((hp[0] * X + hp[1] * Y) + hp[2]) / den;
    const double sy = ((hp[3] * X + hp[4] * Y) + hp[5]) / den;
    cdx = round_pred(sx) - px;
    cdy = round_pred(sy) - py;
  }

  // 2. the searched window ---------------------------------------------------
  const int P = c.P, PW = 2 * P + 1, R = sh.R;
  // Window and patch are held centred (pixel - 128 as a signed byte; a pixel
  // outside the image is 0, i.e. -128): r - w is unchanged, so the SSD is
  // sum r'^2 + sum w'^2 - 2 sum r'w' exactly, and the cross term fits the
  // signed 8-bit dot products and matrix-core operands.
  uint8_t* win = dyn + sh.off_win;
  uint32_t* rowsq = reinterpret_cast<uint32_t*>(dyn + sh.off_rowsq);
  const int wx0 = px + cdx - P - R, wy0 = py + cdy - P - R;
  const int ncp = KX == 0 ? sh.ncand : sh.nstrips * KX;  // candidates per row of tot
  uint32_t* tot = reinterpret_cast<uint32_t*>(dyn + sh.off_tot);  // split partial sums
  // the patch rows with zero padding for the matrix-core operands: dword d
  // of row i holds patch dword d - padB / 4 (0 outside the patch), packed
  // again from the staged region (the packed patch written above by other
  // waves is not read before the next barrier); the split totals lie past
  // every other buffer here and are cleared now
  auto pack_patch = [&]() {
    if constexpr (KX == 0) {
      uint32_t* pb = reinterpret_cast<uint32_t*>(dyn + sh.off_pb);
      const int d0 = sh.padB >> 2;
      for (int q = tid; q < PW * sh.LB; q += nt) {
        const int i = q / sh.LB, d = q - i * sh.LB - d0;
        pb[q] = (d >= 0 && d < NW) ? patch_dword(reg, sh.rs, pr0, pc0, PW, i, d) : 0u;
      }
      if (sh.split > 1)
        for (int i = tid; i < sh.ncand * sh.ncand; i += nt) tot[i] = 0u;
    }
  };
  // (without WARP the job has no Hwarp: the launchers check it)
  if (WARP && J.Hwarp) {
    double hp[9];
    pixel_homography(J.Hwarp, w, h, hp);
    stage_warped(J.wimg, w, h, hp, wx0, wy0, sh.NR, sh.stage_dw, win, sh.wrow, tid, nt, 0x80u);
    pack_patch();
  } else {
    // (the patch rows are packed while the window's first loads are in flight)
    stage_rows_around(J.wimg, w, h, wx0, wy0, sh.NR, sh.stage_dw, win, sh.wrow, tid, nt,
                      0x80808080u, pack_patch);
  }
  __syncthreads();
  // patch energy (summed over each wave first: one LDS atomic per wave)
  {
    uint32_t part = 0;
    for (int i = tid; i < PW * NW; i += nt)
      part = (uint32_t)__builtin_amdgcn_sdot4((int)S.refp[i], (int)S.refp[i], (int)part, false);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if ((tid & 63) == 0 && part) atomicAdd(&S.er_sum, part);
  }
  // matrix-core lane roles: wave (group msp, dx block mnb), lane (r16, cg)
  const int lane = tid & 63, mwave = tid >> 6;
  const int mnb = mwave % sh.NB, msp = mwave / sh.NB;
  const int r16 = lane & 15, cg = lane >> 4;
  v4i acc[MB > 0 ? MB : 1];
  if constexpr (KX == 0) {
    // 3. cross terms on the matrix cores. For patch row i the cross term of
    // every candidate is a product of two small matrices,
    //   X[dy][dx] += sum_x win[i + dy][x] * pat[i][x - dx],
    // the window rows i .. i + 16 NB - 1 (A: 16 dy x 64 columns) times the
    // Toeplitz matrix of patch row i (B: 64 columns x 16 dx, zero where
    // x - dx falls outside the patch): v_mfma_i32_16x16x64_i8, exact in
    // int32. Wave (group msp, dx block mnb) accumulates the NB dy blocks of
    // its dx block over its group's patch rows; lane (r, g) supplies A row
    // dy = 16 mb + r, B column dx = 16 nb + r and bytes 16 g .. 16 g + 15 of
    // each 64-byte chunk, and receives X[16 mb + 4 g + t][16 nb + r]. The
    // products come before the energies, which then reuse the patch rows'
    // and the window's memory.
    const uint32_t* pb = reinterpret_cast<const uint32_t*>(dyn + sh.off_pb);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = v4i{0, 0, 0, 0};
    const int i0 = msp * PW / sh.split, i1 = (msp + 1) * PW / sh.split;
    for (int kc = 0; kc < sh.KC; ++kc) {
      // B bytes: patch row i at columns x - dx, x = 64 kc + 16 g + 0..15,
      // i.e. bytes qb .. qb + 15 of the padded row (qb >= 1)
      const int qb = 64 * kc + 16 * cg - (16 * mnb + r16) + sh.padB;
      const uint8_t* ar = win + r16 * sh.wrow + 64 * kc + 16 * cg;
      const uint32_t* pr0 = pb + (qb >> 2);
      if constexpr (MB <= 3) {
        switch (sh.NB) {
          case 1: cross_mfma<1>(ar, pr0, sh.LB, qb & 3, sh.wrow, i0, i1, acc); break;
          case 2: cross_mfma<2>(ar, pr0, sh.LB, qb & 3, sh.wrow, i0, i1, acc); break;
          default: cross_mfma<3>(ar, pr0, sh.LB, qb & 3, sh.wrow, i0, i1, acc); break;
        }
      } else {
        switch (sh.NB) {
          case 4: cross_mfma<4>(ar, pr0, sh.LB, qb & 3, sh.wrow, i0, i1, acc); break;
          default: cross_mfma<5>(ar, pr0, sh.LB, qb & 3, sh.wrow, i0, i1, acc); break;
        }
      }
    }
    if (sh.split > 1) {  // exact integer partial sums: any order gives the same totals
      const int dxi = 16 * mnb + r16;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int j = 16 * mb + 4 * cg + t;
          if (mb < sh.NB && j < sh.ncand && dxi < sh.ncand)
            atomicAdd(&tot[j * ncp + dxi], (uint32_t)acc[mb][t]);
        }
    }
    __syncthreads();  // (the row energies below overwrite the patch rows)
  }
  // window row energies rowsq[y][k] = sum_c win[y][k + c]^2, from realigned
  // dwords with v_dot4 (bytes past the patch width masked off)
  // (a thread per run of 8 candidates of a window row: the first sum from
  // dwords, then sliding by one pixel four candidates at a time, from the
  // dword holding the pixels that leave and the realigned dword holding those
  // that enter; exact in integers. The step is written as (b - a)(b + a):
  // hipcc folds e + b*b - a*a on two bytes into one v_dot4_u32_u8 of the
  // packed pair, which adds a*a instead of subtracting it. A run's first
  // dwords may reach a few bytes past the row: those bytes are masked off.)
  {
    constexpr int CH = 8;
    const uint32_t* wdw = reinterpret_cast<const uint32_t*>(win);
    const int rowdw = sh.wrow >> 2;
    const int nch = (sh.ncand + CH - 1) / CH;
    for (int it = tid; it < sh.NR * nch; it += nt) {
      const int yy = it / nch, c0 = (it - yy * nch) * CH;
      const uint32_t* rp = wdw + yy * rowdw;
      uint32_t e = 0;
#pragma unroll
      for (int m = 0; m < NW; ++m) {
        const int nb = PW - 4 * m;
        const uint32_t mask = nb >= 4 ? 0xffffffffu : (nb <= 0 ? 0u : ((1u << (8 * nb)) - 1u));
        const int d = (int)(rp[(c0 >> 2) + m] & mask);
        e = (uint32_t)__builtin_amdgcn_sdot4(d, d, (int)e, false);
      }
      uint32_t* out = rowsq + yy * sh.ncand;
      out[c0] = e;
      const int cend = min(c0 + CH, sh.ncand);
      // candidate k + 1 = candidate k - pixel k + pixel k + PW
#pragma unroll
      for (int g = 0; g < CH / 4; ++g) {
        const int k0 = c0 + 4 * g;
        if (k0 + 1 >= cend) break;
        const uint32_t A = rp[k0 >> 2];
        const int bq = (k0 + PW) >> 2;
        const uint32_t B = __builtin_amdgcn_alignbyte(rp[bq + 1], rp[bq], (k0 + PW) & 3);
        uint32_t v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int a = (int)(int8_t)(A >> (8 * q)), b = (int)(int8_t)(B >> (8 * q));
          e += (uint32_t)((b - a) * (b + a));
          v[q] = e;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (k0 + q + 1 < cend) out[k0 + q + 1] = v[q];
      }
    }
  }
  __syncthreads();
  // (matrix cores: the window energies overwrite the window)
  uint32_t* colE = reinterpret_cast<uint32_t*>(dyn + sh.off_colE);  // [ncand][ncand]
  // window energies: vertical box sums of the row energies, sliding over
  // runs of 7 candidate rows per column
  {
    const int nch = (sh.ncand + 6) / 7;
    for (int it = tid; it < sh.ncand * nch; it += nt) {
      const int dxi = it % sh.ncand, ch = it / sh.ncand;
      const int y0 = ch * 7, y1 = min(y0 + 7, sh.ncand);
      uint32_t e = 0;
      for (int i = 0; i < PW; ++i) e += rowsq[(y0 + i) * sh.ncand + dxi];
      colE[y0 * sh.ncand + dxi] = e;
      for (int y = y0 + 1; y < y1; ++y) {
        e += rowsq[(y - 1 + PW) * sh.ncand + dxi] - rowsq[(y - 1) * sh.ncand + dxi];
        colE[y * sh.ncand + dxi] = e;
      }
    }
  }
  if constexpr (KX != 0)
    if (sh.split > 1)
      for (int i = tid; i < sh.ncand * ncp; i += nt) tot[i] = 0u;
  __syncthreads();

  unsigned long long key = ~0ull;
  const uint32_t er = S.er_sum;
  // candidate (dy index j, dx index dxi) with cross term x: its key, if its
  // patch lies inside the level
  auto score = [&](int j, int dxi, uint32_t x) {
    const int dx = dxi - R + cdx, dy = j - R + cdy;
    if (px + dx - P < 0 || px + dx + P > w - 1 || py + dy - P < 0 || py + dy + P > h - 1) return;
    // exact modulo 2^32, and the SSD itself is below 2^32
    const uint32_t ssd = er + colE[j * sh.ncand + dxi] - 2u * x;
    // ties on the absolute displacement, or on the offset from the
    // predicted position when the window is centred on a prediction
    const int kx = J.Hlit ? dxi - R : dx, ky = J.Hlit ? j - R : dy;
    const uint32_t l1 = (uint32_t)((kx < 0 ? -kx : kx) + (ky < 0 ? -ky : ky));
    // (ssd, |dx| + |dy|, dy, dx), displacements biased by 64 (|d| <= 64)
    const unsigned long long kk = ((unsigned long long)ssd << 32) |
                                  ((unsigned long long)l1 << 16) |
                                  ((unsigned long long)(ky + 64) << 8) |
                                  (unsigned long long)(kx + 64);
    key = kk < key ? kk : key;
  };

  if constexpr (KX == 0) {
    const int dxi = 16 * mnb + r16;
    if (msp == 0 && dxi < sh.ncand) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int j = 16 * mb + 4 * cg + t;
          if (mb >= sh.NB || j >= sh.ncand) continue;
          score(j, dxi, sh.split > 1 ? tot[j * ncp + dxi] : (uint32_t)acc[mb][t]);
        }
    }
  } else {
    // 3. cross terms of KX candidates per thread (over a group of patch
    // rows), signed 8-bit dot products of the centred bytes
    const int base_threads = sh.ncand * sh.nstrips;
    const int grp = tid / base_threads, rem = tid % base_threads;
    const int j = rem / sh.nstrips, s = rem % sh.nstrips;  // dy index, strip
    uint32_t acc[KX];
#pragma unroll
    for (int k = 0; k < KX; ++k) acc[k] = 0;
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
        for (int m = 0; m < NW; ++m) rr[m] = S.refp[i * NW + m];
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
            acc[k] = (uint32_t)__builtin_amdgcn_sdot4((int)sft[rsh][q + m], (int)rr[m],
                                                       (int)acc[k], false);
        }
      }
      if (sh.split > 1)  // exact integer partial sums: any order gives the same totals
#pragma unroll
        for (int k = 0; k < KX; ++k) atomicAdd(&tot[j * ncp + s * KX + k], acc[k]);
    }
    if (sh.split > 1) {
      __syncthreads();
      if (tid < base_threads)
#pragma unroll
        for (int k = 0; k < KX; ++k) acc[k] = tot[j * ncp + s * KX + k];
    }
    if (tid < base_threads) {
#pragma unroll
      for (int k = 0; k < KX; ++k) {
        const int dxi = s * KX + k;
        if (dxi < sh.ncand) score(j, dxi, acc[k]);
      }
    }
  }
  // 4. argmin -------------------------------------------------------------------
  key = wave_min_u64(key);
  if ((tid & 63) == 0) S.wmin[tid >> 6] = key;
  __syncthreads();
  if (tid == 0) {
    unsigned long long b = ~0ull;
    for (int i = 0; i < (nt + 63) / 64; ++i) b = S.wmin[i] < b ? S.wmin[i] : b;
    const uint8_t fb = (uint8_t)(want ? 16 : 0);
    J.corner_xy[2 * tile] = px;
    J.corner_xy[2 * tile + 1] = py;
    if (b == ~0ull) {
      J.disp[2 * tile] = 0;
      J.disp[2 * tile + 1] = 0;
      J.ssd[tile] = 0;
      J.flags[tile] = (uint8_t)(1 | fb);
    } else {
      J.disp[2 * tile] = (int)(b & 255ull) - 64 + (J.Hlit ? cdx : 0);
      J.disp[2 * tile + 1] = (int)((b >> 8) & 255ull) - 64 + (J.Hlit ? cdy : 0);
      J.ssd[tile] = (uint32_t)(b >> 32);
      J.flags[tile] = (uint8_t)(3 | fb);
      if (J.vb) atomicOr(J.vb + (tile >> 6), 1ull << (tile & 63));
    }
  }
}

// One workgroup per tile of one job. ROLE names the launch only.
template <int KX, int ROLE, int MB>
__global__ __launch_bounds__(1024) void k_search(SearchJob J, SearchCfg c, SearchShape sh,
                                                 const uint8_t* __restrict__ mode, int want) {
  extern __shared__ __align__(16) uint8_t dyn[];
  __shared__ TileShared S;
  const int tile = blockIdx.x;
  // with a proposal, each tile is searched by the launch of its mode only
  if (mode && mode[tile] != want) return;
  search_tile<KX, ROLE == kRoleCoarse, MB>(J, tile, tile, c, sh, kVisitSearchAll, mode ? want : 0,
                                       nullptr, nullptr, dyn,
                  S);
}

// One workgroup per item of the work: item i of [0, n) is global tile i (or
// list[i] when the work has a list, n = *count; the grid covers the largest
// possible n and the workgroups past it return at once); the job is the last
// one whose first tile is <= the global tile. (Persistent workgroups looping
// over the items, fetched by an atomic counter, were measured slower on the
// 5 MP pair's level 0: 96 us against 82 us.)
template <int KX, int VISIT, bool WARP, int MB>
__global__ __launch_bounds__(1024) void k_search_work(SearchJob one,
                                                      const SearchJob* __restrict__ jobs,
                                                      SearchWork wk, SearchCfg c,
                                                      SearchShape sh, int want) {
  extern __shared__ __align__(16) uint8_t dyn[];
  __shared__ TileShared S;
  const int n = wk.list ? *wk.count : wk.ntotal;
  const int i = blockIdx.x;
  if (i >= n) return;
  // uniform over the workgroup: kept in scalar registers
  const int g = __builtin_amdgcn_readfirstlane(wk.list ? wk.list[i] : i);
  if (!jobs) {  // one job, given by value
    search_tile<KX, WARP, MB>(one, g, g, c, sh, VISIT, want, wk.out_list, wk.out_count, dyn, S);
    return;
  }
  int lo = 0, hi = wk.njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (__builtin_amdgcn_readfirstlane(wk.first[mid]) <= g) lo = mid;
    else hi = mid - 1;
  }
  const SearchJob J = jobs[lo];
  search_tile<KX, WARP, MB>(J, g - __builtin_amdgcn_readfirstlane(wk.first[lo]), g, c, sh, VISIT,
                        want,
                  wk.out_list, wk.out_count, dyn, S);
}

// Ordered lists of one level's tiles from their flags, by one workgroup (a
// per-tile append to a shared counter serialises: about 12 ns per tile).
// Without `mode`: lists[0, n) = the cornered tiles (flag bit 0), counts[0].
// With `mode`: lists[n, 2n) = the cornered tiles of mode 0 (window search),
// lists[2n, 3n) = those of any other mode (exhaustive fallback), counts[1]
// and counts[2]. Tiles appear in ascending order. Thread i owns a run of
// consecutive tiles; the runs' counts are scanned within each wave, then
// over the waves. (Runs loaded at once as membership bits, or rounds of
// 1024 tiles ranked by ballots, measured slower: the kernel's few loads per
// thread are not its cost.)
__global__ __launch_bounds__(1024) void k_tile_lists(const uint8_t* __restrict__ flags,
                                                     const uint8_t* __restrict__ mode, int n,
                                                     int* __restrict__ lists,
                                                     int* __restrict__ counts) {
  __shared__ int wsum[2][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int per = (n + 1023) / 1024;
  const int t0 = min(tid * per, n), t1 = min(t0 + per, n);
  auto in_a = [&](int t) { return (flags[t] & 1) && (!mode || mode[t] == 0); };
  auto in_b = [&](int t) { return (flags[t] & 1) && mode && mode[t] != 0; };
  int c0 = 0, c1 = 0;
  for (int t = t0; t < t1; ++t) {
    c0 += in_a(t);
    c1 += in_b(t);
  }
  int s0 = c0, s1 = c1;  // inclusive scans over the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u0 = __shfl_up(s0, o), u1 = __shfl_up(s1, o);
    if (lane >= o) {
      s0 += u0;
      s1 += u1;
    }
  }
  if (lane == 63) {
    wsum[0][wv] = s0;
    wsum[1][wv] = s1;
  }
  __syncthreads();
  int b0 = 0, b1 = 0;
  for (int w = 0; w < wv; ++w) {
    b0 += wsum[0][w];
    b1 += wsum[1][w];
  }
  int p0 = b0 + s0 - c0, p1 = b1 + s1 - c1;  // this run's first entries
  int* la = mode ? lists + n : lists;
  int* lb = lists + 2 * n;
  for (int t = t0; t < t1; ++t) {
    if (in_a(t)) la[p0++] = t;
    else if (in_b(t)) lb[p1++] = t;
  }
  if (tid == 1023) {  // the last run ends both lists
    if (mode) {
      counts[1] = b0 + s0;
      counts[2] = b1 + s1;
    } else {
      counts[0] = b0 + s0;
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

// Most distinct dwords that one bank serves for the SSD loop's first window
// read, over the half-waves of a workgroup, at row stride d dwords.
int bank_degree(int d, int ncand, int nstrips, int split, int KX, int rows_per_grp) {
  const int base = ncand * nstrips, nthr = base * split;
  int deg = 0;
  for (int h0 = 0; h0 < nthr; h0 += 32) {
    int addr[32], n = 0;
    for (int t = h0; t < h0 + 32 && t < nthr; ++t) {
      const int grp = t / base, rem = t % base;
      addr[n++] = (rem / nstrips + grp * rows_per_grp) * d + (rem % nstrips) * (KX / 4);
    }
    std::sort(addr, addr + n);
    const int u = (int)(std::unique(addr, addr + n) - addr);
    int per_bank[32] = {0};
    for (int k = 0; k < u; ++k) deg = std::max(deg, ++per_bank[addr[k] % 32]);
  }
  return deg;
}

int window_stride(int d0, int ncand, int nstrips, int split, int KX, int rows_per_grp) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int, int, int>, int> memo;
  const auto key = std::make_tuple(d0, ncand, nstrips, split, KX, rows_per_grp);
  std::lock_guard<std::mutex> lk(mu);
  auto it = memo.find(key);
  if (it != memo.end()) return it->second;
  int best = d0, best_deg = 1 << 30;
  for (int d = d0; d < d0 + 8; ++d) {  // at most 28 bytes more per row
    const int deg = bank_degree(d, ncand, nstrips, split, KX, rows_per_grp);
    if (deg < best_deg) { best_deg = deg; best = d; }
  }
  memo[key] = best;
  return best;
}

SearchShape make_shape(int R, const SearchCfg& c, int split, long long ntiles, int KX,
                       size_t* lds, int* block) {
  SearchShape sh{};
  sh.R = R;
  sh.ncand = 2 * R + 1;
  const int PW = 2 * c.P + 1;
  // threads of one patch-row group: a lane per (dy, strip of KX dx), or a
  // wave per block of 16 dx (matrix cores)
  sh.NB = (sh.ncand + 15) / 16;
  sh.nstrips = KX == 0 ? 0 : (sh.ncand + KX - 1) / KX;
  const int base = KX == 0 ? 64 * sh.NB : sh.ncand * sh.nstrips;
  if (split > 0) {  // a tuned split (the results do not depend on it)
    sh.split = split;
  } else {
    // when the level has too few candidate threads to fill the chip (coarse
    // levels, small windows), split the patch rows so that a tile keeps about
    // 256 threads busy
    sh.split = ntiles * base >= 262144 ? 1 : (256 + base / 2) / base;
  }
  if (sh.split < 1) sh.split = 1;
  if (sh.split > 7) sh.split = 7;
  if (sh.split > PW) sh.split = PW;
  while (sh.split > 1 && base * sh.split > 1024) --sh.split;
  sh.nthreads = base * sh.split;
  sh.NR = 2 * c.P + 2 * R + 1;
  int nrows = sh.NR;  // window rows held
  if (KX == 0) {
    // A reads 64-byte chunks of rows up to i + 16 NB - 1 (the rows and
    // columns past the window only meet zero B entries or unused outputs)
    const int wc = sh.ncand - 1 + PW;
    sh.KC = (wc + 63) / 64;
    sh.wrow = 64 * sh.KC + 16;  // 16-byte aligned rows, shifted by 4 banks
    sh.stage_dw = (wc + 3) / 4;
    nrows = std::max(sh.NR, 16 * sh.NB + PW - 1);
    sh.padB = 16 * sh.NB;
    sh.LB = 16 * sh.KC + 4 * sh.NB + 1;
  } else {
    // bytes read per row: the last strip's (KX/4 + NW + 1) dwords
    const int need = (sh.nstrips * KX) + 4 * (NW + 1);
    // The row stride: the lanes of a wave read window rows (j + i) at dword
    // offsets (KX / 4) s; of the strides that hold a row (and up to 7 dwords
    // more), the one whose half-waves (32 lanes, 32 banks) hit a bank with the
    // fewest distinct dwords (then the shortest)
    sh.wrow = 4 * window_stride((need + 3) / 4, sh.ncand, sh.nstrips, sh.split, KX,
                                PW / sh.split);
    sh.stage_dw = sh.wrow / 4;
  }
  int b = (sh.nthreads + 63) / 64 * 64;
  if (b < 64) b = 64;
  *block = b;
  // the reference region: side rows of rs bytes, rs covering the realigned
  // dword reads of the quadrant sums (up to 6 bytes past a row's end) and one
  // spare row after the last; the quadrant row sums: 2 (K g + r) rows of
  // 2 (2K + 1) words
  const int ext = c.K * c.g + (c.r > c.P ? c.r : c.P);
  const int side = 2 * ext + 1;
  sh.rs = (side + 8 + 3) / 4 * 4;
  const int hsum_words = 2 * (c.K * c.g + c.r) * 2 * (2 * c.K + 1);
  auto a16 = [](int x) { return (x + 15) / 16 * 16; };
  const int reg_bytes = sh.rs * (side + 1);
  const int tot_bytes = sh.split > 1 ? sh.ncand * (KX == 0 ? sh.ncand : sh.nstrips * KX) * 4 : 0;
  if (KX != 0) {
    // region, row sums, window, row energies (+ KX words: the last strip's
    // padded candidates read past the last row), split totals, window
    // energies
    sh.off_reg = 0;
    sh.off_hsum = a16(reg_bytes);
    sh.off_cend = sh.off_hsum + hsum_words * 4;
    sh.off_win = a16(sh.off_cend);
    sh.off_rowsq = sh.off_win + nrows * sh.wrow;
    sh.off_tot = sh.off_rowsq + (sh.NR * sh.ncand + KX) * 4;
    sh.off_colE = sh.off_tot + tot_bytes;
    sh.off_pb = a16(sh.off_colE + sh.ncand * sh.ncand * 4);  // (no patch rows)
    *lds = (size_t)sh.off_pb;
  } else {
    // window (later its energies), region, row sums, padded patch rows (the
    // three later the row energies), split totals; the products read whole
    // 16-row blocks past the window, i.e. into the buffers after it, for
    // outputs that are never used
    sh.off_win = 0;
    sh.off_colE = 0;
    sh.off_reg = a16(std::max(sh.NR * sh.wrow, sh.ncand * sh.ncand * 4));
    sh.off_hsum = a16(sh.off_reg + reg_bytes);
    sh.off_cend = sh.off_hsum + hsum_words * 4;
    sh.off_pb = a16(sh.off_cend);
    sh.off_rowsq = sh.off_reg;
    sh.off_tot = a16(std::max(sh.off_pb + PW * sh.LB * 4, sh.off_rowsq + sh.NR * sh.ncand * 4));
    *lds = (size_t)std::max(sh.off_tot + tot_bytes, nrows * sh.wrow);
  }
  return sh;
}

}  // namespace

hipError_t launch_warp_q8(const uint8_t* src, int w, int h, const double* Hn, uint8_t* out,
                          hipStream_t st, const WeedBufs* wb, int nwords, int* zint, int nzint) {
  dim3 grid((w + 1023) / 1024, h);
  LNR_LAUNCH(k_warp_q8, grid, dim3(256), 0, st, src, w, h, Hn, out, wb ? wb->vb : nullptr,
             nwords, wb ? wb->sums : nullptr, zint, zint ? nzint : 0);
  return hipGetLastError();
}

hipError_t launch_warp_jobs(const WarpJob* jobs, const int* row0, int njobs, int rows,
                            int wmax, hipStream_t st) {
  if (njobs < 1 || rows < 1) return hipSuccess;
  const int nxb = (wmax + 1023) / 1024;
  LNR_LAUNCH(k_warp_jobs, dim3(nxb * rows), dim3(256), 0, st, jobs, row0, njobs, nxb);
  return hipGetLastError();
}

bool search_shape_fits(int R, const SearchCfg& c, int code) {
  const int split = code & kSearchSplitMask;
  if (split < 1 || split > 7 || split > 2 * c.P + 1 || search_threads(R, code) > 1024) return false;
  size_t lds = 0;
  int block = 0;
  make_shape(R, c, split, 1, shape_kx(code, 8), &lds, &block);
  return lds + sizeof(TileShared) <= 65536;
}

int search_split_candidates(int R, const SearchCfg& c, int* out, int max) {
  int n = 0;
  for (const int code : {0, kSearchKx12, kSearchMfma})
    for (int s = 1; s <= 7 && n < max; ++s)
      if (search_shape_fits(R, c, s | code)) out[n++] = s | code;
  return n;
}

hipError_t launch_tile_lists(const uint8_t* flags, const uint8_t* mode, int n, int* lists,
                             int* counts, hipStream_t st) {
  LNR_LAUNCH(k_tile_lists, dim3(1), dim3(1024), 0, st, flags, mode, n, lists, counts);
  return hipGetLastError();
}

hipError_t launch_texture(uint8_t* p, int n, uint32_t seed, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  LNR_LAUNCH(k_texture, dim3((n + 255) / 256), dim3(256), 0, st, p, n, seed);
  return hipGetLastError();
}

template <int KX, int MB>
hipError_t launch_search_kx(const SearchJob& J, int ntiles, const SearchCfg& c,
                            const SearchShape& sh, int role, int block, size_t lds,
                            hipStream_t st, const uint8_t* mode, int want) {
  switch (role) {
    case kRoleCoarse:
      LNR_LAUNCH((k_search<KX, kRoleCoarse, MB>), dim3(ntiles), dim3(block), lds, st, J, c, sh, mode,
                 want);
      break;
    case kRoleLevel0:
      LNR_LAUNCH((k_search<KX, kRoleLevel0, MB>), dim3(ntiles), dim3(block), lds, st, J, c, sh, mode,
                 want);
      break;
    case kRoleTrial:
      LNR_LAUNCH((k_search<KX, kRoleTrial, MB>), dim3(ntiles), dim3(block), lds, st, J, c, sh, mode,
                 want);
      break;
    default:
      LNR_LAUNCH((k_search<KX, kRoleStage, MB>), dim3(ntiles), dim3(block), lds, st, J, c, sh, mode,
                 want);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_search(const SearchJob& J, int nty, int R, const SearchCfg& c, int role,
                         hipStream_t st, const uint8_t* mode, int want, int split) {
  const int ntiles = J.ntx * nty;
  if (ntiles == 0) return hipSuccess;
  if (J.Hwarp && role != kRoleCoarse) return hipErrorInvalidValue;  // no warp in that kernel
  // a tuned choice: the split (1..7), plus kSearchKx12 (12 candidates per
  // lane) or kSearchMfma (matrix-core cross terms)
  const int kx = shape_kx(split, 8);
  // (a shape that does not fit these patch and corner parameters: the
  // automatic split)
  if (split && !search_shape_fits(R, c, split)) split &= ~kSearchSplitMask;
  size_t lds = 0;
  int block = 0;
  const SearchShape sh = make_shape(R, c, split & kSearchSplitMask, ntiles, kx, &lds, &block);
  switch (kx) {
    case 0:  // (matrix-core operands held for at most 3 or 5 blocks of 16 candidates)
      return sh.NB <= 3
                 ? launch_search_kx<0, 3>(J, ntiles, c, sh, role, block, lds, st, mode, want)
                 : launch_search_kx<0, kMaxNB>(J, ntiles, c, sh, role, block, lds, st, mode, want);
    case 12: return launch_search_kx<12, 0>(J, ntiles, c, sh, role, block, lds, st, mode, want);
    default: return launch_search_kx<8, 0>(J, ntiles, c, sh, role, block, lds, st, mode, want);
  }
}

template <int KX, int MB>
hipError_t launch_work_kx(const SearchJob& one, const SearchJob* jobs, const SearchWork& wk,
                          const SearchCfg& c, const SearchShape& sh, int visit, int want,
                          bool warp, int grid, int block, size_t lds, hipStream_t st) {
  switch (visit) {
    case kVisitCornersOnly:
      LNR_LAUNCH((k_search_work<KX, kVisitCornersOnly, false, MB>), dim3(grid), dim3(block), lds, st,
                 one, jobs, wk, c, sh, want);
      break;
    case kVisitKnownCorner:
      LNR_LAUNCH((k_search_work<KX, kVisitKnownCorner, false, MB>), dim3(grid), dim3(block), lds, st,
                 one, jobs, wk, c, sh, want);
      break;
    default:
      if (warp)
        LNR_LAUNCH((k_search_work<KX, kVisitSearchAll, true, MB>), dim3(grid), dim3(block), lds, st,
                   one, jobs, wk, c, sh, want);
      else
        LNR_LAUNCH((k_search_work<KX, kVisitSearchAll, false, MB>), dim3(grid), dim3(block), lds, st,
                   one, jobs, wk, c, sh, want);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_search_work(const SearchJob* jobs, const SearchWork& wk, int R,
                              const SearchCfg& c, int visit, int want, int split, int kx,
                              int grid, hipStream_t st, const SearchJob* one, bool warp) {
  if (grid < 1) return hipSuccess;
  // a single job with a warp needs the kernel that carries it
  if (one && one->Hwarp && !(warp && visit == kVisitSearchAll)) return hipErrorInvalidValue;
  kx = shape_kx(split, kx);  // flags in a tuned shape code take precedence
  if ((split & kSearchSplitMask) && !search_shape_fits(R, c, split)) split = 0;
  split &= kSearchSplitMask;
  if (kx != 0 && kx != 8 && kx != 12) return hipErrorInvalidValue;
  if (!jobs && !one) return hipErrorInvalidValue;
  size_t lds = 0;
  int block = 0;
  const SearchShape sh = make_shape(R, c, split, grid, kx, &lds, &block);
  // the corner phase uses only the reference region and its row sums
  if (visit == kVisitCornersOnly) lds = (size_t)sh.off_cend;
  const SearchJob none{};
  const SearchJob& J = one ? *one : none;
  switch (kx) {
    case 0:
      return sh.NB <= 3 ? launch_work_kx<0, 3>(J, jobs, wk, c, sh, visit, want, warp, grid, block,
                                               lds, st)
                        : launch_work_kx<0, kMaxNB>(J, jobs, wk, c, sh, visit, want, warp, grid,
                                                    block, lds, st);
    case 12:
      return launch_work_kx<12, 0>(J, jobs, wk, c, sh, visit, want, warp, grid, block, lds, st);
    default:
      return launch_work_kx<8, 0>(J, jobs, wk, c, sh, visit, want, warp, grid, block, lds, st);
  }
}

}  // namespace lnr
