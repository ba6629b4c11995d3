/*
 * lnr.h -- C ABI of the MI355X (gfx950) implementation of locally non-rigid
 * HDR registration and deghosted merging (Gallo, Troccoli, Hu, Pulli, Kautz:
 * "Locally Non-rigid Registration for Mobile HDR Photography").
 *
 * Conventions (all entry points):
 *  - Every image, table and output pointer is a DEVICE pointer on the
 *    context's GPU, allocated and owned by the caller. The library owns only
 *    its context and an internal workspace, which grows on first use of a
 *    larger shape (hipMalloc) and is freed by lnr_destroy.
 *  - `stream` is a hipStream_t passed as void* (0 = the null stream). All work
 *    is enqueued on it asynchronously; no entry point synchronises the device
 *    except lnr_create / lnr_destroy.
 *  - Errors return a negative lnr_status before anything is enqueued
 *    (invalid arguments, unsupported sizes) or after a failed HIP call;
 *    lnr_last_error() gives a message. No entry point aborts or throws.
 *  - Images are row-major 8-bit planes with a byte stride per row; I420 frames
 *    carry full-size Y and half-size U, V (even width and height). Float
 *    outputs are dense planar [c][H][W].
 *  - Level l of the matching pyramid has size (W >> l) x (H >> l) (floor
 *    halving), up to 5 levels, none with a side below min_level_dim
 *    (paper Sec. 2.6). Per-tile arrays hold every level's full tiles, level
 *    by level, each level in raster order; lnr_query_sizes gives the offsets.
 *  - Calls that share one context must not overlap: a context's workspace is
 *    reused by every call on it.
 */
#ifndef LNR_H
#define LNR_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LNR_OK = 0,
  LNR_E_ARG = -1,          /* null pointer, bad size, mismatched frames */
  LNR_E_UNSUPPORTED = -2,  /* parameter outside the supported range     */
  LNR_E_TOO_SMALL = -3,    /* image smaller than one tile               */
  LNR_E_HIP = -4,          /* a HIP runtime call failed                  */
  LNR_E_NOMEM = -5,        /* workspace allocation failed               */
  LNR_E_CAPTURE = -6,      /* the workspace would have to grow while the
                              stream is being captured into a graph     */
  LNR_E_WEIGHTS = -7       /* network file unreadable, of another format
                              or size, or holding non-finite values     */
} lnr_status;

typedef enum { LNR_Y8 = 0, LNR_I420 = 1, LNR_NV12 = 2 } lnr_format;

typedef struct {
  int32_t width, height;
  int32_t format;            /* lnr_format                                      */
  int32_t reserved;
  const uint8_t* plane[3];   /* Y, U, V (device); U, V null for LNR_Y8; for
                                LNR_NV12 plane[1] holds U and V interleaved
                                (U first, W bytes per row, H/2 rows) and
                                plane[2] is unused                             */
  int32_t stride[3];         /* bytes per row of each plane                     */
  float exposure;            /* relative exposure; the shortest is the reference */
} lnr_frame;

/* Method parameters. lnr_default_params() fills the paper's constants
 * (Sec. 2.6: 5 levels, 100 px, 21x21 patches, radius 10, grid 1/16 of the
 * tile, sigma_s 400) and the documented readings for what the paper leaves
 * open. Supported ranges are checked by every entry point. */
typedef struct {
  int32_t tile;            /* S: tile side, 16..64, multiple of 4              */
  int32_t patch_r;         /* P: patch (2P+1)^2, 1..11                          */
  int32_t corner_step;     /* g: candidate spacing                              */
  int32_t corner_half;     /* K: candidates at centre + g*[-K,K]^2, K <= 3      */
  int32_t quad_r;          /* r: quadrant side of Eq. 1-2                       */
  int32_t corner_t;        /* T of Eq. 2 (mean DN; compared on sums as T*r*r)   */
  int32_t max_levels;      /* 1..5                                              */
  int32_t min_level_dim;   /* smallest side of a coarse level                   */
  int32_t radius_coarse;   /* search radius on levels >= 1, <= 32               */
  int32_t radius0;         /* search radius on level 0, <= 32                   */
  int32_t weed_iters;      /* weeding iterations (Sec. 2.3), 1..65536           */
  int32_t weed_delta_min;  /* delta = max(min, ceil(pct * N / 100))  (Eq. 5)    */
  int32_t weed_delta_pct;
  int32_t dt_iters;        /* domain-transform iterations, 1..8                 */
  double weed_eps;         /* inlier radius in level pixels                     */
  double sigma_s;          /* spatial sigma of the propagation (Sec. 2.6: 400)  */
  double sigma_r;          /* range sigma on the [0,1] guide                    */
  double n_min;            /* F = P~/N~ only where N~ > n_min (Sec. 2.4)         */
  double ssim_sigma;       /* SSIM Gaussian window sigma                         */
  int32_t ssim_radius;     /* SSIM window radius, 1..8                          */
  int32_t search_frame;    /* 0: each level searches the source warped by the
                              previous level's homography; 1: Eq. 3 as
                              printed: each level searches the unwarped
                              source around round(Hp x), fits its
                              homography to those absolute matches, and the
                              absolute level-0 flow is propagated (the
                              source is sampled at x + F(x); warped0 is not
                              written). 1 with learned = 1 is rejected   */
  double ssim_c1, ssim_c2; /* SSIM stabilisers                                   */
  double sigma_e;          /* Mertens well-exposedness sigma                     */
  uint64_t seed;           /* weeding sampler seed                               */
  /* learned displacement proposal (an extension beyond the paper): with
   * learned = 1 the level-0 search of Sec. 2.2 scans only centre + [-window_r,
   * window_r]^2 per tile, the centre being the context's network prediction,
   * and falls back to the exhaustive radius0 search where the network's
   * confidence is below conf_min. Needs lnr_proposal_set() first and tile 32. */
  int32_t learned;         /* 0: plain method (default), 1: learned proposal    */
  int32_t window_r;        /* window radius, 0..radius0 (default 2)             */
  double conf_min;         /* confidence threshold in [0, 1] (default 0.5): 0
                              windows every cornered tile, 1 searches every
                              tile exhaustively (the plain method's result) */
} lnr_params;

typedef struct {
  int32_t levels;          /* matching pyramid levels                          */
  int32_t tiles_total;     /* per-tile array length (all levels)               */
  int32_t tile_off[6];     /* level l's tiles are [tile_off[l], tile_off[l+1]) */
  int32_t level_w[5], level_h[5];
  int32_t channels;        /* 3 for I420 (RGB output), 1 for Y8 (grey)         */
  int32_t blend_levels;    /* Laplacian-pyramid levels of the merge            */
} lnr_sizes;

/* Outputs of one registration (device pointers, caller-owned). Pointers
 * marked optional may be null. Per-tile flags: 1 corner found, 2 valid
 * match, 4 kept by the weeding filter (Eq. 5), 8 used for the level fit,
 * 16 exhaustive fallback taken (learned proposal only). */
typedef struct {
  int32_t* corner_xy;      /* [tiles_total][2] corner pixel, -1 if none        */
  int32_t* disp;           /* [tiles_total][2] integer displacement d          */
  uint32_t* ssd;           /* [tiles_total] SSD at the argmin                  */
  uint8_t* flags;          /* [tiles_total]                                    */
  int32_t* counts;         /* [5][4] per level: N valid, fit count,
                              best-consensus count, best iteration             */
  double* H;               /* [levels+1][9] normalised-frame homographies:
                              H[l] for l < levels, H[levels] = initial (I)     */
  uint8_t* yeq_ref;        /* [H][W] equalised reference Y                     */
  uint8_t* yeq_src;        /* [H][W] equalised source Y (optional)             */
  uint8_t* warped0;        /* [H][W] level-0 source warped by H[1] (optional)  */
  float* flow;             /* [2][H][W] residual flow F (Sec. 2.4)             */
  float* ntilde;           /* [H][W] filtered N (optional)                     */
  float* image;            /* [channels][H][W] warped source in [0, 1]         */
  float* yeq_warped;       /* [H][W] warped source Y_eq / 255                  */
} lnr_registration;

typedef struct lnr_ctx lnr_ctx;

/* Create a context on HIP device `device`. */
lnr_status lnr_create(lnr_ctx** ctx, int32_t device);
void lnr_destroy(lnr_ctx* ctx);
const char* lnr_last_error(const lnr_ctx* ctx);
void lnr_default_params(lnr_params* p);
/* Sizes of every output for a width x height frame of `format`. */
lnr_status lnr_query_sizes(int32_t width, int32_t height, int32_t format,
                           const lnr_params* p, lnr_sizes* out);

/* Register `src` to `ref` (paper Sec. 2.2 - 2.4): equalise both, estimate the
 * pyramid homographies (matcher + weeding per level), search level 0, weed,
 * propagate the kept matches to a dense residual flow, and warp the source
 * backwards. Both frames must share size and format. Only kernel launches are
 * enqueued (no host round trip, no memset), so the call can be captured into
 * a graph once a call of the same size has sized the workspace outside the
 * capture; otherwise it returns LNR_E_CAPTURE. */
lnr_status lnr_register_pair(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                             const lnr_params* p, lnr_registration* out, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lnr_register_pair
 * with the same arguments, results and kernels, but its scratch (pyramids,
 * warped level, weeding buffers, propagation maps, network inputs) comes from
 * a fixed device array of LNR_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends, instead of the context's
 * workspace. It calls no allocating routine and never grows anything: a job
 * that needs more scratch (a 5 MP pair needs about 85 MB; much larger frames do
 * not fit) returns LNR_E_NOMEM before any launch. Every call on one GPU,
 * from any context, uses that GPU's one array, so such calls must not
 * overlap in time (calls on different streams race); the kernels clear what
 * must start at zero, so a call does not depend on the previous contents.
 * Tracing (lnr_trace_enable) does not apply to it. */
#define LNR_NOALLOC_SCRATCH_BYTES ((uint64_t)96 << 20)
lnr_status lnr_register_pair_noalloc(lnr_ctx* ctx, const lnr_frame* ref, const lnr_frame* src,
                                     const lnr_params* p, lnr_registration* out, void* stream);

/* Register an n-frame stack (paper Sec. 2: n - 1 registrations): the
 * reference is the frame with the smallest exposure (Sec. 2.1; lowest index
 * on ties), written to *ref_index; outs[k] receives the registration of the
 * k-th non-reference frame, in frame order. When the exposures are not known
 * (not every one positive and finite) the darkest frame is the reference:
 * the lowest mean luma (lowest index on ties); that case reads the frames'
 * histograms back and waits for `stream` once. All frames must share size
 * and format. */
lnr_status lnr_register_stack(lnr_ctx* ctx, const lnr_frame* frames, int32_t n,
                              const lnr_params* p, lnr_registration* outs,
                              int32_t* ref_index, void* stream);

/* Error-tolerant exposure fusion (paper Sec. 2.5): Mertens et al.'s contrast,
 * saturation and well-exposedness weights times the SSIM between the
 * equalised reference and each warped frame, blended with Laplacian
 * pyramids. regs[k] is the registration of the k-th non-reference frame (as
 * produced by lnr_register_stack); out is [channels][H][W] float. */
lnr_status lnr_merge(lnr_ctx* ctx, const lnr_frame* frames, int32_t n, int32_t ref_index,
                     const lnr_registration* regs, const lnr_params* p, float* out,
                     void* stream);
/* HDR irradiance map of the registered frames, the paper's alternative output
 * in its quality comparison (Sec. 3.1), in place of the fusion: per channel
 * the average of value / (exposure / reference exposure) weighted by
 * min(v, 1 - v) (0 at black and saturation), non-reference weights times
 * max(SSIM, 0) against the reference as in Sec. 2.5; the reference's value
 * where every weight is 0. Arguments as lnr_merge; out [ch][H][W] fp32 in
 * the reference's units (1 = the reference's white). Every exposure must be
 * positive and finite (LNR_E_ARG). */
lnr_status lnr_merge_irradiance(lnr_ctx* ctx, const lnr_frame* frames, int32_t n,
                                int32_t ref_index, const lnr_registration* regs,
                                const lnr_params* p, float* out, void* stream);

/* ---- stage entry points: one stage on caller-given inputs (used to check
 * each kernel on exactly the inputs the oracle sees). -------------------- */

/* Histogram equalisation (Sec. 3 opening) of one 8-bit plane: lut[256] and
 * out[h][w] (dense). */
lnr_status lnr_stage_equalize(lnr_ctx* ctx, const uint8_t* img, int32_t w, int32_t h,
                              int32_t stride, uint8_t* lut, uint8_t* out, void* stream);
/* Metering of the second exposure (Sec. 2.1): the first frame is exposed to
 * the right; the second is 2, 3 or 4 stops brighter the more under-exposed
 * pixels the first has. y: the first frame's 8-bit luma (device, w x h,
 * row stride). A pixel is under-exposed below `dark`; with n of the w h
 * pixels under-exposed the choice is 2 stops when n <= frac3 w h, 3 when
 * n <= frac4 w h, else 4 (the thresholds are readings; defaults 16, 0.05,
 * 0.20). Writes out[0] = stops and out[1] = n (device int32[2]). */
lnr_status lnr_meter(lnr_ctx* ctx, const uint8_t* y, int32_t w, int32_t h, int32_t stride,
                     int32_t dark, float frac3, float frac4, int32_t* out, void* stream);
/* Q8 bilinear warp of a level image through the normalised homography
 * H[9] (device, double), Eq. 3 frame (Sec. 2.2). */
lnr_status lnr_stage_warp_q8(lnr_ctx* ctx, const uint8_t* src, int32_t w, int32_t h,
                             const double* H, uint8_t* out, void* stream);
/* Corners (Eq. 1-2) on `ref` and SSD search (Sec. 2.2) in `warped` with
 * radius R, for every full tile: corner_xy, disp, ssd, flags (bits 1, 2). */
lnr_status lnr_stage_search(lnr_ctx* ctx, const uint8_t* ref, const uint8_t* warped,
                            int32_t w, int32_t h, int32_t R, const lnr_params* p,
                            int32_t* corner_xy, int32_t* disp, uint32_t* ssd,
                            uint8_t* flags, void* stream);
/* Weeding (Sec. 2.3, Eq. 5) and level homography (Sec. 2.2) over the tiles of
 * one level (flags bit 2 = valid match): sets flags bits 4 and 8, writes
 * counts[4] and H_out[9] = H_prev o G. */
lnr_status lnr_stage_weed_fit(lnr_ctx* ctx, const int32_t* corner_xy, const int32_t* disp,
                              uint8_t* flags, int32_t ntiles, int32_t w, int32_t h,
                              int32_t level, const lnr_params* p, const double* H_prev,
                              double* H_out, int32_t* counts, void* stream);
/* Sparse-to-dense flow (Sec. 2.4, Eq. 6-7) from the level-0 tiles with flags
 * bit 4, guided by `guide` (dense [h][w]): flow [2][h][w], ntilde (optional). */
lnr_status lnr_stage_flow(lnr_ctx* ctx, const int32_t* corner_xy, const int32_t* disp,
                          const uint8_t* flags, int32_t ntiles, const uint8_t* guide,
                          int32_t w, int32_t h, const lnr_params* p, float* flow,
                          float* ntilde, void* stream);
/* Backward warp of `src` through H[9] (device, normalised, level 0) and the
 * flow: image [channels][h][w] in [0, 1] and the warped yeq / 255. */
lnr_status lnr_stage_backward_warp(lnr_ctx* ctx, const lnr_frame* src, const uint8_t* yeq,
                                   const double* H, const float* flow, float* image,
                                   float* yeq_warped, void* stream);
/* The merge's conversion of an unwarped frame (the reference, Sec. 2.5):
 * image [channels][h][w] = BT.601 full-range RGB of f in [0, 1] (Y8: Y / 255;
 * 4:2:0 chroma by pixel repetition), the same conversion the backward warp
 * applies to its samples; with yeq (device, [h][w] 8-bit, may be null),
 * yeq_out = yeq / 255. All pointers device; LNR_E_ARG on a bad frame or a
 * null image (or yeq given without yeq_out). */
lnr_status lnr_stage_frame_rgb(lnr_ctx* ctx, const lnr_frame* f, const uint8_t* yeq,
                               float* image, float* yeq_out, void* stream);
/* Deghosted merge (Sec. 2.5) of n float images [ch][h][w] in [0, 1] with
 * their equalised luma maps yeqs[k] ([h][w], in [0, 1]); frame ref_index
 * gets no SSIM weight. imgs and yeqs are device pointers held in host arrays. */
lnr_status lnr_stage_merge(lnr_ctx* ctx, int32_t n, int32_t ch, int32_t w, int32_t h,
                           const float* const* imgs, const float* const* yeqs,
                           int32_t ref_index, const lnr_params* p, float* out, void* stream);
/* The irradiance map of lnr_merge_irradiance from n float images and luma
 * maps as lnr_stage_merge takes them; exposures: n positive values (host). */
lnr_status lnr_stage_irradiance(lnr_ctx* ctx, int32_t n, int32_t ch, int32_t w, int32_t h,
                                const float* const* imgs, const float* const* yeqs,
                                const float* exposures, int32_t ref_index, const lnr_params* p,
                                float* out, void* stream);

/* ---- batches: several pairs of any sizes in one call (streams, graphs,
 * autotuning; no new method). -------------------------------------------- */
#define LNR_BATCH_GRAPH 1     /* capture the batch as one HIP graph, cached per
                                 (inputs, outputs, parameters), and launch it */
#define LNR_BATCH_AUTOTUNE 2  /* on the first call of a batch shape, time 1, 2,
                                 4 and 8 concurrent streams and keep the fastest */
/* Register n pairs (refs[i], srcs[i]) -> outs[i], each exactly as
 * lnr_register_pair would. The pairs are spread over concurrent streams
 * (longest first, each to the least-loaded stream), each with its own
 * workspace slot; the call's stream waits for all of them. Graph mode needs
 * the same pointers again to reuse a capture. */
lnr_status lnr_register_batch(lnr_ctx* ctx, const lnr_frame* refs, const lnr_frame* srcs,
                              int32_t n, const lnr_params* p, lnr_registration* outs,
                              int32_t flags, void* stream);
/* Time every domain-transform kernel shape that covers w x h (Sec. 2.4 pass;
 * results do not depend on the shape) and use the fastest for that size from
 * then on. shape_out[5] (optional): rows per thread, row block, rows per
 * column segment, columns per block, segments per column. Synchronises. */
lnr_status lnr_autotune_flow(lnr_ctx* ctx, int32_t w, int32_t h, const lnr_params* p,
                             int32_t* shape_out, void* stream);
/* Use one propagation kernel shape (five values, in the order of
 * lnr_autotune_flow's shape_out) for w x h from now on, in place of the
 * default or tuned one: for reproducible configurations. LNR_E_UNSUPPORTED
 * unless it is one of the shapes lnr_flow_shapes lists for w x h. */
lnr_status lnr_set_flow_shape(lnr_ctx* ctx, int32_t w, int32_t h, const int32_t* shape);
/* The propagation shapes that cover w x h (host only): writes up to max of
 * them to shapes[5 * i ...] (may be null) and returns how many there are. */
int32_t lnr_flow_shapes(int32_t w, int32_t h, int32_t* shapes, int32_t max);
/* Time every workgroup shape of the matcher's search (Sec. 2.2: how many
 * thread groups share a tile's patch rows, and whether the SSD cross terms
 * run as 8-bit dot products with each lane scoring 8 or 12 consecutive
 * candidates, or on the matrix cores) at each pyramid level of a w x h pair,
 * on a synthetic texture, and use the fastest for those level sizes and
 * radii from then on (results do not depend on it). splits_out[5]
 * (optional): the choice per level, the split (1..7) plus 16 where 12
 * candidates per lane or 32 where the matrix cores were faster, 0 past the
 * last level. Synchronises. */
lnr_status lnr_autotune_search(lnr_ctx* ctx, int32_t w, int32_t h, const lnr_params* p,
                               int32_t* splits_out, void* stream);
/* Pin the search shape (as lnr_autotune_search reports it: a split 1..7,
 * plus 16 for 12 candidates per lane or 32 for the matrix cores) for pyramid
 * levels of level_w x level_h searched at `radius` (host only; LNR_E_ARG
 * for a shape the search does not have, or one that needs more than 1024
 * threads or 64 KB of workgroup memory with the default parameters; with
 * other patch and corner parameters a shape that does not fit falls back to
 * the automatic one). Results do not depend on it. lnr_stage_search and
 * lnr_stage_search_window use the shape pinned or tuned for their size and
 * radius. */
lnr_status lnr_set_search_shape(lnr_ctx* ctx, int32_t level_w, int32_t level_h, int32_t radius,
                                int32_t shape);

/* ---- learned displacement proposal (an extension beyond the paper; it
 * narrows the Sec. 2.2 search). The network: per level-0 tile of 32 x 32 the
 * input x[4][16][16]: channels 0, 1 the tile of the reference and of the
 * warped source (2 x 2 sums s mapped to bf16((s - 510) / 512)); channels 2,
 * 3 the 64 x 64 windows around the tile (16 px on every side, edge pixels
 * repeated outside the image; 4 x 4 sums s mapped to bf16((s - 2040) /
 * 2048)), so that displacements across the whole search range are in view;
 * four 3x3 convolutions to 32 channels (strides 1, 2, 1, 2, padding 1, ReLU,
 * activations rounded to bf16), a linear head 512 -> 3.
 * Outputs o: predicted displacement (8 o[0], 8 o[1]) and confidence logit
 * o[2]. Parameters: one fp32 vector of LNR_PROPOSAL_PARAMS values, in order
 * W1[32][4][3][3] b1[32] W2[32][32][3][3] b2 W3 b3 W4 b4 Wh[3][512] bh[3]
 * (head feature f = (y * 4 + x) * 32 + c). The context owns one network and
 * its AdamW state; the calls below run on the GPU (bf16 matrix cores, fp32
 * accumulation). ------------------------------------------------------------ */
#define LNR_PROPOSAL_PARAMS 30467

/* Load the network parameters params[LNR_PROPOSAL_PARAMS] (device, fp32)
 * into the context and reset the AdamW moments and step count. */
lnr_status lnr_proposal_set(lnr_ctx* ctx, const float* params, void* stream);
/* Copy the context's parameters to params[LNR_PROPOSAL_PARAMS] (device). */
lnr_status lnr_proposal_get(lnr_ctx* ctx, float* params, void* stream);
/* Network file (host path; little-endian): the 4 bytes "LNRP", uint32
 * version 1, uint32 parameter count (LNR_PROPOSAL_PARAMS), uint32 0, then
 * the fp32 parameters in the order above. lnr_proposal_save writes the
 * context's network (LNR_E_ARG without one; LNR_E_WEIGHTS when the file
 * cannot be written); it waits for `stream`. lnr_proposal_load reads a file,
 * checks its header, size and that every value is finite (LNR_E_WEIGHTS
 * otherwise, before the context's network is touched), then loads it as
 * lnr_proposal_set does; it waits for the host-to-device copy. */
lnr_status lnr_proposal_save(lnr_ctx* ctx, const char* path, void* stream);
lnr_status lnr_proposal_load(lnr_ctx* ctx, const char* path, void* stream);
/* Training checkpoint (host path; little-endian): "LNRK", uint32 version 1,
 * uint32 parameter count, uint32 AdamW step count, uint64 `counter`, then the
 * fp32 parameters, first moments and second moments (each in the order
 * above). `counter` is the caller's position in its data order (the training
 * pipeline stores its global step), returned by the load, so that training
 * resumed from a checkpoint repeats the uninterrupted run bit for bit.
 * Save: LNR_E_ARG without a network, LNR_E_WEIGHTS when the file cannot be
 * written; waits for `stream`. Load: header, size, finite values and
 * non-negative second moments are checked (LNR_E_WEIGHTS otherwise, before
 * the context's network is touched); then parameters, moments and step count
 * replace the context's; waits for the copy. */
lnr_status lnr_proposal_checkpoint_save(lnr_ctx* ctx, const char* path, uint64_t counter,
                                        void* stream);
lnr_status lnr_proposal_checkpoint_load(lnr_ctx* ctx, const char* path, uint64_t* counter,
                                        void* stream);
/* Network inputs of every full 32 x 32 tile of two dense [h][w] 8-bit
 * images (raster tile order): x[ntiles][4][16][16], bf16 bit patterns. */
lnr_status lnr_proposal_inputs(lnr_ctx* ctx, const uint8_t* ref, const uint8_t* warped,
                               int32_t w, int32_t h, uint16_t* x, void* stream);
/* Inference on n inputs (device bf16 [n][4][16][16]): out[n][3] (device). */
lnr_status lnr_proposal_forward(lnr_ctx* ctx, const uint16_t* x, int32_t n, float* out,
                                void* stream);
/* One training step on a batch: forward, loss (Huber on 8 o[0] - label_x and
 * 8 o[1] - label_y, plus the logistic loss of o[2] against the soft target
 * q = sigmoid(4 (2.5 - max |pred - label|)) held constant: "the rounded
 * prediction lies within 2 px"), back-propagation and AdamW
 * (beta 0.9 / 0.999, eps 1e-8, decoupled decay wd). labels[n][2] (device
 * int32). Optional outputs: loss[n] per sample, grad[LNR_PROPOSAL_PARAMS]
 * the batch gradient. lr = 0 and wd = 0 leaves the parameters unchanged. */
lnr_status lnr_proposal_train_step(lnr_ctx* ctx, const uint16_t* x, const int32_t* labels,
                                   int32_t n, float lr, float wd, float* loss, float* grad,
                                   void* stream);
/* The Sec. 2.2 search of lnr_stage_search restricted, per tile t, to the
 * displacements centre[t] + [-R, R]^2 (centre [ntiles][2], device int32,
 * |centre| + R <= 32). */
lnr_status lnr_stage_search_window(lnr_ctx* ctx, const uint8_t* ref, const uint8_t* warped,
                                   int32_t w, int32_t h, int32_t R, const int32_t* centre,
                                   const lnr_params* p, int32_t* corner_xy, int32_t* disp,
                                   uint32_t* ssd, uint8_t* flags, void* stream);

/* ---- timing: optional per-kernel GPU timing with HIP events recorded on the
 * call's stream around every kernel launch of the calls that follow (off by
 * default; adds one event pair per launch). -------------------------------- */
typedef struct {
  char name[32];      /* kernel name, e.g. "k_search"                        */
  int32_t count;      /* launches timed since the last reset                 */
  int32_t reserved;
  double ms_total;    /* summed event-to-event time of those launches        */
} lnr_trace_entry;

/* Enable (on != 0) or disable timing, and discard what was recorded. */
lnr_status lnr_trace_enable(lnr_ctx* ctx, int32_t on);
/* Wait for the recorded events, write up to `max` entries (one per kernel
 * name, in first-launch order) and return how many there are (or < 0). */
int32_t lnr_trace_read(lnr_ctx* ctx, lnr_trace_entry* out, int32_t max);

#ifdef __cplusplus
}
#endif
#endif
