// lnr_internal.h -- declarations shared by the HIP sources of liblnr (GPU path
// only). Kernels are launched through the host functions declared here; each
// returns hipSuccess or the launch error.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lnr.h"

namespace lnr {

// Optional per-kernel timing: while a traced API call runs on this thread,
// every kernel launch is bracketed by a TraceScope that records a HIP event
// pair on the launch stream. Without tracing it does nothing.
struct TraceScope {
  TraceScope(const char* name, hipStream_t st);
  ~TraceScope();
  int slot = -1;
  hipStream_t stream = nullptr;
};

#define LNR_LAUNCH(kernel, grid, block, lds, st, ...)                    \
  do {                                                                    \
    ::lnr::TraceScope lnr_ts_(#kernel, st);                               \
    hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);        \
  } while (0)

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// For kernels whose neighbouring blocks read overlapping rows, this maps the
// dispatch index so that each XCD walks one contiguous band of the grid (in
// raster order), keeping the shared rows in one L2.
__device__ inline void xcd_block(int gx, int gy, int& bx, int& by) {
  const int nb = gx * gy, b = blockIdx.x + gx * blockIdx.y, full = nb / 8 * 8;
  const int j = b < full ? (b % 8) * (nb / 8) + b / 8 : b;
  bx = j % gx;
  by = j / gx;
}

constexpr int kMaxLevels = 5;
constexpr int kMaxRadius = 32;
constexpr int kMaxPatchR = 11;   // patch rows fit in 6 dwords
constexpr int kWeedWave = 64;

struct Level {
  int w, h;          // level size
  int ntx, nty;      // full tiles
  int tile_off;      // first tile of this level in the per-tile arrays
  size_t pix_off;    // offset of this level in a pyramid buffer
};

struct Geometry {
  int W, H, levels, tiles_total;
  Level lv[kMaxLevels];
  size_t pyr_bytes;  // bytes of one 8-bit pyramid (all levels)
};

// search-kernel constants derived from lnr_params
struct SearchCfg {
  int S, P, g, K, r;
  int thr;           // corner_t * r * r
};

// ---- equalisation + pyramid (k_equalize.hip)
hipError_t launch_hist(const uint8_t* y0, int s0, const uint8_t* y1, int s1, int W, int H,
                       uint32_t* hist /*[nframes][256]*/, int nframes, hipStream_t st);
// the metering decision from a luma histogram: out[0] = stops, out[1] = the
// pixels below dark
hipError_t launch_meter(const uint32_t* hist, int dark, float frac3, float frac4,
                        long long npix, int32_t* out, hipStream_t st);
// out0 / out1 (optional): second copies of the equalised level 0;
// gt0 (optional): column-major copy of frame 0's equalised level 0, column x
// at gt0 + x * dt_guide_stride(H) (the propagation's column-pass guide)
hipError_t launch_lut_pyr(const uint8_t* y0, int s0, const uint8_t* y1, int s1,
                          const uint32_t* hist, const Geometry& g, uint8_t* pyr0,
                          uint8_t* pyr1, uint8_t* lut_out, int nframes, hipStream_t st,
                          uint8_t* out0 = nullptr, uint8_t* out1 = nullptr,
                          uint8_t* gt0 = nullptr);

// ---- warp + search (k_search.hip)
struct WeedBufs;
// wb (optional): the level's weeding buffers, whose valid-match bits and
// least-squares sums the warp clears and the search then fills
// zint: nzint (<= 256) counters to clear as well (the learned path's lists)
hipError_t launch_warp_q8(const uint8_t* src, int w, int h, const double* Hn, uint8_t* out,
                          hipStream_t st, const WeedBufs* wb = nullptr, int nwords = 0,
                          int* zint = nullptr, int nzint = 0);
// One level of one pair for the search: the equalised reference level and
// the searched source level (dense w x h), the level's full tiles (ntx
// across) and their outputs.
struct SearchJob {
  const uint8_t* ref;
  const uint8_t* wimg;      // warped source level, or the unwarped one with Hlit
  int w, h, ntx;
  int32_t* corner_xy;       // [tiles][2]
  int32_t* disp;            // [tiles][2]
  uint32_t* ssd;            // [tiles]
  uint8_t* flags;           // [tiles]
  const int32_t* centre;    // [tiles][2] window centres of the learned proposal, or null
  unsigned long long* vb;   // valid-match bits set by the search, or null
  const double* Hlit;       // previous level's homography (unwarped search), or null
  const double* Hwarp;      // previous level's homography: the window is the
                            // unwarped level wimg warped by it on the fly, or null
};
// The tiles one work-list launch visits: global tile g of job j is
// first[j] + tile; all of [0, ntotal) or the *count entries of list.
struct SearchWork {
  const int* first;         // [njobs + 1] (device)
  int njobs;
  const int* list;          // global tile indices (device), or null
  const int* count;         // entries of list (device)
  int ntotal;
  int* out_list;            // corner visits: cornered tiles appended here (device)
  int* out_count;
};
// a tuned search shape: the patch-row split (1..7), plus kSearchKx12 when
// the lanes score 12 consecutive candidates instead of 8, or kSearchMfma
// when the cross terms run on the matrix cores (a wave per 16 dx)
constexpr int kSearchKx12 = 16, kSearchMfma = 32, kSearchSplitMask = 7;
// candidates per lane of a shape code (0: matrix cores), dflt without flags
inline int shape_kx(int code, int dflt) {
  return (code & kSearchMfma) ? 0 : (code & kSearchKx12) ? 12 : dflt;
}
// threads of one workgroup for radius R and a shape code with a split
inline int search_threads(int R, int code) {
  const int ncand = 2 * R + 1, kx = shape_kx(code, 8), split = code & kSearchSplitMask;
  const int base = kx == 0 ? 64 * ((ncand + 15) / 16) : ncand * ((ncand + kx - 1) / kx);
  return base * split;
}
// names of single-job search launches (profiles tell the levels apart)
constexpr int kRoleCoarse = 0, kRoleLevel0 = 1, kRoleTrial = 2, kRoleStage = 3;
// tile visits of the work-list search
constexpr int kVisitSearchAll = 0, kVisitCornersOnly = 1, kVisitKnownCorner = 2;
// one workgroup per tile of J (mode/want: only the tiles whose mode is want);
// split: 0 (a rule on the level size) or a tuned shape
// k_warp_q8 over several pairs' levels (batches): job j's rows are the grid
// rows [row0[j], row0[j + 1]) (device tables), rows = row0[njobs]
struct WarpJob {
  const uint8_t* src;       // source level (dense w x h)
  int w, h, nwords;
  const double* Hn;         // the previous level's homography
  uint8_t* out;             // warped level
  unsigned long long* vb;   // the level's weeding bits and sums, cleared here
  long long* sums;
};
hipError_t launch_warp_jobs(const WarpJob* jobs, const int* row0, int njobs, int rows,
                            int wmax, hipStream_t st);
// (a job with Hwarp only with role kRoleCoarse)
hipError_t launch_search(const SearchJob& J, int nty, int R, const SearchCfg& c, int role,
                         hipStream_t st, const uint8_t* mode = nullptr, int want = 0,
                         int split = 0);
// `grid` workgroups, one per item of the work (at least the number of items);
// kx: candidates per lane (8 or 12); jobs null: the single job `one` (by
// value), whose tiles the work's items are; warp: the jobs may warp their
// windows on the fly (Hwarp; only with kVisitSearchAll)
hipError_t launch_search_work(const SearchJob* jobs, const SearchWork& wk, int R,
                              const SearchCfg& c, int visit, int want, int split, int kx,
                              int grid, hipStream_t st, const SearchJob* one = nullptr,
                              bool warp = false);

// search shapes that launch_search accepts for radius R (splits of the patch
// rows over thread groups, with 8 or 12 candidates per lane or the matrix
// cores: at most 1024 threads and 64 KB of workgroup memory); and a random
// 8-bit texture for timing the search
bool search_shape_fits(int R, const SearchCfg& c, int code);
int search_split_candidates(int R, const SearchCfg& c, int* out, int max);
hipError_t launch_texture(uint8_t* p, int n, uint32_t seed, hipStream_t st);

// ---- weeding + level homography (k_weed.hip)
struct WeedBufs {
  int32_t* nmatch;          // [1] valid matches of the level
  double* G;                // [iters][8] hypothesis homographies
  int32_t* cnt;             // [iters] inlier counts (-1: hypothesis unusable)
  unsigned long long* bal;  // [ceil(ntiles/64)][iters] inlier bitmask rows
  unsigned long long* vb;   // [ceil(ntiles/64)] valid-match bits, tile order
  long long* sums;          // [23] least-squares sums of the level fit
};
// one level of one pair for the weeding and level fit
struct WeedJob {
  const int32_t* cxy;
  const int32_t* disp;
  uint8_t* flags;
  int ntiles, w, h, words;
  WeedBufs b;
  const double* Hprev;  // H^{l+1} (kept when the fit fails)
  const double* Hbase;  // the map G is composed on (H^{l+1}, or the identity)
  double* Hout;
  int32_t* counts;
  // cleared by the solve for the next level's search (null: nothing)
  unsigned long long* clear_vb;
  int clear_words;
};
// the weeding kernels over a device table of jobs (the search set the
// valid-match bits and the warp cleared the sums); max_tiles: the largest
// job's tiles
hipError_t launch_weed_jobs(const WeedJob* jobs, int njobs, int max_tiles, int level,
                            const lnr_params& p, hipStream_t st);
// clear_words > 0: the solve then clears the first clear_words valid-match
// words and the sums, for the next level's search
hipError_t launch_weed_fit(const int32_t* corner_xy, const int32_t* disp, uint8_t* flags,
                           int ntiles, int w, int h, int level, const lnr_params& p,
                           const double* H_prev, double* H_out, int32_t* counts,
                           const WeedBufs& b, hipStream_t st, bool vb_ready = false,
                           const double* H_base = nullptr, int clear_words = 0);

// ---- domain-transform propagation (k_dt.hip)
// Kernel shapes: rows of SEG pixels per thread in NT-thread blocks; columns as
// NCOL columns x NSEG segments of L rows per block. Only the instantiated
// combinations are valid (dt_shape_valid).
struct DtShape {
  int seg, nt;         // row kernel
  int l, ncol, nseg;   // column kernel
};
DtShape dt_default_shape(int W, int H);
bool dt_shape_valid(const DtShape& s, int W, int H);
int dt_shape_candidates(int W, int H, DtShape* out, int max);
// The propagation's working maps: one 12-byte record per pixel (the three
// maps), so that a column pass reads whole runs of neighbouring columns.
// The propagation maps (12 bytes per pixel) and, 256-byte aligned after
// them, one flag byte per row (padded so that 8-row loads stay inside).
inline size_t dt_rowflag_offset(int W, int H) {
  return ((size_t)W * H * 12 + 255) / 256 * 256;
}
inline size_t dt_maps_bytes(int W, int H) {
  return dt_rowflag_offset(W, H) + ((size_t)H + 64 + 255) / 256 * 256;
}
// The column pass reads the guide column-major: column x at x * stride, the
// rows padded to a multiple of 64 plus one more 64-row block (so that a
// segment's aligned load never leaves the column).
inline int dt_guide_stride(int H) { return ((H + 63) / 64 + 1) * 64; }
inline size_t dt_guide_t_bytes(int W, int H) { return (size_t)W * dt_guide_stride(H); }
// guide_t: dt_guide_t_bytes(W, H) of workspace; filled here from guide
// unless guide_t_ready (k_lut_pyr wrote it)
hipError_t launch_flow(const int32_t* corner_xy, const int32_t* disp, const uint8_t* flags,
                       int ntx, int nty, int tile, const uint8_t* guide, uint8_t* guide_t,
                       int W, int H, const lnr_params& p, void* maps /*[H][W] records*/,
                       double* coef /*[iters][256]*/, float* flow, float* ntilde,
                       hipStream_t st, const DtShape* shape = nullptr, bool coef_ready = false,
                       bool guide_t_ready = false);
// Column-major copy of a 64 x 64 byte tile held in LDS (row r at tile + 64 r,
// rows past the image zero): column bx + c gets rows [by, by + 64) at
// gt + (bx + c) * hp + by. Called by all 256 threads of a block.
__device__ inline void store_tile_columns(const uint8_t* tile, int bx, int by, int W, int hp,
                                          uint8_t* __restrict__ gt) {
  const int c = threadIdx.x >> 2, q = threadIdx.x & 3;
  if (bx + c >= W) return;
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) v |= (uint32_t)tile[(16 * q + 4 * k + b) * 64 + c] << (8 * b);
    w[k] = v;
  }
  *reinterpret_cast<uint4*>(gt + (size_t)(bx + c) * hp + by + 16 * q) =
      make_uint4(w[0], w[1], w[2], w[3]);
}
// the propagation's coefficient tables (coef [iters][256]); the first block
// also clears zero[0, nzero) and sets ident (optional) to the 3x3 identity
hipError_t launch_dt_coef(const lnr_params& p, double* coef, uint32_t* zero, int nzero,
                          double* ident, hipStream_t st, unsigned long long* zero64 = nullptr,
                          int nzero64 = 0, long long* sums = nullptr);

// ---- backward warp (k_warp.hip)
// Chroma of a 4:2:0 frame: U at u[(y/2) su + (x/2) cs], V likewise (I420: two
// planes, cs = 1; NV12: one interleaved plane, v = u + 1, cs = 2); u null for
// luma-only frames.
struct Chroma {
  const uint8_t* u = nullptr;
  const uint8_t* v = nullptr;
  int su = 0, sv = 0, cs = 1;
};
hipError_t launch_backward_warp(const uint8_t* y, int sy, const Chroma& c, const uint8_t* yeq,
                                int W, int H, const double* Hn, const float* flow, float* image,
                                float* yeq_w, hipStream_t st);
// RGB of a frame plus, optionally, an 8-bit plane yin mapped to [0, 1] in yout
hipError_t launch_frame_rgb_unit(const uint8_t* y, int sy, const Chroma& c, int W, int H,
                                 float* image, const uint8_t* yin, float* yout, hipStream_t st);

// ---- merge (k_merge.hip)
struct MergeBufs {
  float* ssim;     // [n][H][W] SSIM maps (reference slot unused)
  float* w0;       // [n][H][W] normalised weights (pyramid level 0)
  float* pyr;      // [n (ch + 1)][levels 1..L-1] weight and image pyramids
  float* acc;      // [ch][levels 1..L-1] collapsed result
};
size_t merge_pyr_elems(int W, int H, int levels);
int merge_levels(int W, int H);
hipError_t launch_merge(int n, int ch, int W, int H, const float* const* imgs,
                        const float* const* yeqs, int ref_index, const lnr_params& p,
                        const MergeBufs& b, float* out, hipStream_t st);
// HDR irradiance map (reference units) of n frames with exposures rel[k]
// relative to the reference; ssim: n * W * H floats of scratch
hipError_t launch_irradiance(int n, int ch, int W, int H, const float* const* imgs,
                             const float* const* yeqs, const float* rel, int ref_index,
                             const lnr_params& p, float* ssim, float* out, hipStream_t st);

// ---- learned displacement proposal (k_cnn.hip)
int cnn_param_count();
size_t cnn_packed_elems();   // bf16 packed weights
size_t cnn_act_elems();      // stored activations per sample (bf16)
size_t cnn_dz_elems();       // activation gradients per sample (bf16)
size_t cnn_input_elems();    // network input values per tile (bf16)
int cnn_grad_blocks(int n, int* per_block);
hipError_t launch_cnn_pack(const float* params, uint16_t* packed, hipStream_t st);
// network inputs x[i] of tile tiles[i] (tile i without a list), i below
// *count (without it, every tile)
hipError_t launch_cnn_input(const uint8_t* ref, const uint8_t* warped, int w, int h, int ntx,
                            int nty, const int32_t* tiles, const int* count, uint16_t* x,
                            hipStream_t st);
// the cornered tiles of flags[0, n) in order (lists[0 ..], counts[0]), or
// with `mode` those of mode 0 (lists[n ..], counts[1]) and the others
// (lists[2n ..], counts[2])
hipError_t launch_tile_lists(const uint8_t* flags, const uint8_t* mode, int n, int* lists,
                             int* counts, hipStream_t st);
// inference (centre != null) or training forward of n samples; with `count`
// (device) only the first *count samples (n is then the most there can be),
// sample s being tile tiles[s]; with `lists`, each tile is appended to the
// window list (lists[0 ..]) or the fallback list (lists[n ..]), counts[2]
hipError_t launch_cnn_forward(const uint16_t* packed, const float* params, const uint16_t* x,
                              int n, float* out, uint16_t* acts, int32_t* centre,
                              uint8_t* fallback, int clampc, float conf_logit, hipStream_t st,
                              const int32_t* tiles = nullptr, const int* count = nullptr,
                              int* lists = nullptr, int* counts = nullptr);
hipError_t launch_cnn_backward(const uint16_t* packed, const float* params,
                               const uint16_t* acts, const float* out, const int32_t* labels,
                               int n, float* dO, float* loss, uint16_t* dzs, float* part,
                               hipStream_t st);
hipError_t launch_cnn_adamw(const float* part, int nblk, float* params, float* m, float* v,
                            float lr, float wd, int step, float* grad_out, hipStream_t st);

}  // namespace lnr
