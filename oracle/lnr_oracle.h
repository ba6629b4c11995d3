/*
 * lnr_oracle.h -- plain, slow CPU oracle for locally non-rigid HDR
 * registration (Gallo, Troccoli, Hu, Pulli, Kautz: "Locally Non-rigid
 * Registration for Mobile HDR Photography").
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it. It shares no source with the GPU
 * path: every stage is written here again, as plain loops, in double
 * precision wherever the method uses real numbers, directly from the paper's
 * description (section / equation cited per function) and the readings of
 * the paper listed in the design notes.
 *
 * Images are row-major, tightly packed unless a stride is given. Tile data is
 * per tile in raster order. "Level" 0 is full resolution.
 */
#ifndef LNR_ORACLE_H
#define LNR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t tile;          /* tile size S (pixels, every level)                 */
  int32_t patch_r;       /* SSD patch half-size P: (2P+1)^2 patch (Sec. 2.6)  */
  int32_t corner_step;   /* candidate grid spacing g = S/16 (Sec. 2.6)        */
  int32_t corner_half;   /* candidates at centre + g*{-K..K}^2                */
  int32_t quad_r;        /* quadrant side r for the means of Eq. 1-2          */
  int32_t corner_t;      /* T of Eq. 2 in DN (compared as sums: T*r*r)        */
  int32_t max_levels;    /* pyramid levels, at most 5 (Sec. 2.6)              */
  int32_t min_level_dim; /* no level below 100 px (Sec. 2.6)                  */
  int32_t radius_coarse; /* search radius on levels >= 1 (Sec. 2.6: 10)       */
  int32_t radius0;       /* search radius on level 0                          */
  int32_t weed_iters;    /* weeding iterations (Sec. 2.3)                     */
  int32_t weed_delta_min;/* delta = max(min, ceil(pct*N/100)) (Eq. 5)         */
  int32_t weed_delta_pct;
  int32_t dt_iters;      /* domain-transform RF iterations                    */
  double weed_eps;       /* inlier radius (level pixels)                      */
  double sigma_s;        /* 400 (Sec. 2.6)                                    */
  double sigma_r;        /* range sigma on the [0,1] guide                    */
  double n_min;          /* flow defined where filtered N > n_min (Sec. 2.4)  */
  double ssim_sigma;     /* SSIM Gaussian window (Wang et al.)                */
  int32_t ssim_radius;
  int32_t search_frame;  /* 0: search the source warped by H^{l+1}; 1: Eq. 3 as
                            printed, around round(H^{l+1} x) in the unwarped
                            source, matches and flow absolute               */
  double ssim_c1, ssim_c2;
  double sigma_e;        /* Mertens well-exposedness sigma                    */
  uint64_t seed;         /* weeding sampler seed                              */
} lo_params;

/* Registration outputs of one pair. Per-tile arrays span all levels: level l's
 * tiles start at tile_off[l] (tile_off has max_levels+1 entries). */
typedef struct {
  int32_t levels;
  int32_t tile_off[6];
  int32_t *corner_x, *corner_y;   /* corner pixel (level coords), -1 if none */
  int32_t *dx, *dy;               /* integer displacement                     */
  uint32_t *ssd;                  /* SSD at the argmin                        */
  uint8_t *flags;                 /* 1 corner, 2 valid, 4 in M, 8 fit set     */
  int32_t *n_valid, *n_inliers;   /* per level: N, matches used for the fit   */
  int32_t *best_iter;             /* per level: best-consensus iteration      */
  double *H;                      /* (levels+1) x 9: H[l], H[levels] = init   */
  uint8_t *yeq_ref, *yeq_src;     /* W*H equalised Y                          */
  uint8_t *warped0;               /* W*H level-0 source warped by H[1]        */
  double *flow_u, *flow_v;        /* W*H residual flow                        */
  double *ntilde;                 /* W*H filtered N (for masking)             */
  double *rgb;                    /* ch*W*H warped source in [0,1]            */
  double *yeq_warped;             /* W*H warped source Y_eq / 255             */
} lo_registration;

void lo_default_params(lo_params* p);
int  lo_num_levels(int w, int h, const lo_params* p);

/* Sec. 3: histogram equalisation */
void lo_histogram(const uint8_t* img, int w, int h, int stride, uint32_t hist[256]);
void lo_equalize_lut(const uint32_t hist[256], uint8_t lut[256]);
void lo_apply_lut(const uint8_t* img, int w, int h, int stride, const uint8_t lut[256],
                  uint8_t* out);
/* Sec. 2.2 / 2.6: next pyramid level (floor(w/2) x floor(h/2)) */
void lo_downsample(const uint8_t* in, int w, int h, uint8_t* out);
/* Sec. 2.2, Eq. 1-2: one corner per tile (or none) */
void lo_corners(const uint8_t* img, int w, int h, const lo_params* p,
                int32_t* cx, int32_t* cy, uint8_t* has);
/* Sec. 2.2, Eq. 3: normalised-frame homography -> level pixel homography */
void lo_pixel_homography(const double H[9], int w, int h, double Hp[9]);
/* global homography warp of a level image (Q8 bilinear, clamp to edge) */
void lo_warp_q8(const uint8_t* src, int w, int h, const double Hp[9], uint8_t* out);
/* Sec. 2.2: SSD patch search around each corner */
void lo_search(const uint8_t* ref, const uint8_t* wimg, int w, int h, const lo_params* p,
               int R, const int32_t* cx, const int32_t* cy, const uint8_t* has,
               int32_t* dx, int32_t* dy, uint32_t* ssd, uint8_t* valid);
/* Sec. 2.2, Eq. 3 as printed: the same search, in the unwarped source around
 * the predicted position q = round(Hp x) of each corner (Hp: the previous
 * level's pixel homography); dx, dy receive the absolute displacement
 * q + d - x, the tie order applies to d */
void lo_search_unwarped(const uint8_t* ref, const uint8_t* src, int w, int h,
                        const lo_params* p, int R, const double Hp[9], const int32_t* cx,
                        const int32_t* cy, const uint8_t* has, int32_t* dx, int32_t* dy,
                        uint32_t* ssd, uint8_t* valid);
/* Sec. 2.3, Eq. 5: union-of-inliers filter over iterations [it0, it1).
 * inM is OR-ed (not cleared), so chunks can be merged by repeated calls.
 * best_count / best_iter: the largest inlier count and its iteration (lowest
 * index on ties; -1 if no hypothesis was fitted). Returns N (valid matches). */
int  lo_weed(int ntiles, const int32_t* cx, const int32_t* cy, const int32_t* dx,
             const int32_t* dy, const uint8_t* valid, int w, int h, int level,
             const lo_params* p, int it0, int it1, uint8_t* inM, int32_t* best_count,
             int32_t* best_iter);
/* delta of Eq. 5 for N valid matches */
int  lo_weed_delta(int n, const lo_params* p);
/* inlier set (per tile) of weeding iteration `it`; returns its size or -1 */
int  lo_hypothesis_inliers(int ntiles, const int32_t* cx, const int32_t* cy, const int32_t* dx,
                           const int32_t* dy, const uint8_t* valid, int w, int h, int level,
                           const lo_params* p, int it, uint8_t* sel);
/* 4-point homography (exposed for tests): rows from src (sx,sy) -> dst (tx,ty).
 * Returns 0 if singular. */
int  lo_fit4(const double sx[4], const double sy[4], const double tx[4],
             const double ty[4], double g[9]);
/* Sec. 2.2: level homography, least squares over the selected matches;
 * returns the number selected */
int  lo_fit_level(int ntiles, const int32_t* cx, const int32_t* cy, const int32_t* dx,
                  const int32_t* dy, const uint8_t* sel, int w, int h,
                  const double Hprev[9], double Hout[9]);
/* the same fit when the matches are absolute (paper-literal search): the
 * level homography is the fitted map itself; Hprev is kept on failure */
int  lo_fit_level_absolute(int ntiles, const int32_t* cx, const int32_t* cy,
                           const int32_t* dx, const int32_t* dy, const uint8_t* sel, int w,
                           int h, const double Hprev[9], double Hout[9]);
/* Sec. 2.4, Eq. 6-7: edge-aware sparse-to-dense flow */
void lo_sparse_to_dense(int ntiles, const int32_t* cx, const int32_t* cy, const int32_t* dx,
                        const int32_t* dy, const uint8_t* inM, const uint8_t* guide,
                        int w, int h, const lo_params* p, double* fu, double* fv,
                        double* ntilde);
/* backward warp of the source through H[1] and the flow */
void lo_backward_warp(const uint8_t* y, const uint8_t* u, const uint8_t* v,
                      const uint8_t* yeq, int w, int h, const double Hp[9],
                      const double* fu, const double* fv, double* rgb, double* yeq_w);
/* reference frame to [0,1] RGB (or grey for Y8, u == NULL) */
void lo_frame_to_rgb(const uint8_t* y, const uint8_t* u, const uint8_t* v, int w, int h,
                     double* rgb);
/* Sec. 2.5: SSIM map (Wang et al.) */
void lo_ssim(const double* a, const double* b, int w, int h, const lo_params* p, double* out);
/* Sec. 2.5: normalised fusion weights (Mertens et al. x SSIM) */
void lo_fusion_weights(int n, int ch, int w, int h, const double* const* imgs,
                       const double* const* ssim, const lo_params* p, double* const* wout);
/* Sec. 2.5: multiresolution blend of n images with normalised weights */
int  lo_num_blend_levels(int w, int h);
/* the blend's pyramid steps: REDUCE of a w x h plane to ceil(w/2) x ceil(h/2),
 * and EXPAND of a cw x chh plane to the finer w x h */
void lo_reduce(const double* in, int w, int h, double* out);
void lo_expand(const double* c, int cw, int chh, int w, int h, double* out);
void lo_blend(int n, int ch, int w, int h, const double* const* imgs,
              const double* const* weights, double* out);
/* Sec. 2.1: reference of an n-frame stack (shortest exposure; without known
 * exposures the lowest mean luma), lowest index on ties */
int  lo_pick_reference(int n, const float* exposure, const uint8_t* const* ys, int w, int h,
                       int stride);
/* whole pair (Sec. 2.2 - 2.4 + warp) */
int  lo_register_pair(const uint8_t* ref_y, const uint8_t* src_y, const uint8_t* src_u,
                      const uint8_t* src_v, int w, int h, const lo_params* p,
                      const double* H_init, lo_registration* out);
/* deghosted merge (Sec. 2.5) of n frames; imgs/yeqs as produced above */
int  lo_merge(int n, int ch, int w, int h, const double* const* imgs,
              const double* const* yeqs, int ref_index, const lo_params* p, double* out);
/* the fusion weights' sum per pixel before normalisation (its conditioning) */
int  lo_fusion_weight_sum(int n, int ch, int w, int h, const double* const* imgs,
                          const double* const* yeqs, int ref_index, const lo_params* p,
                          double* out);
/* Metering of the second exposure (Sec. 2.1; thresholds: readings, see
 * lnr_oracle.c): 2, 3 or 4 stops; *n_dark receives the under-exposed count */
int  lo_meter(const uint8_t* y, int w, int h, int stride, int dark, float frac3, float frac4,
              long long* n_dark);
/* HDR irradiance map of the registered frames (the paper's comparison output,
 * Sec. 3.1; formula: reading, see lnr_oracle.c); exposures[k] > 0 */
double lo_hat_weight(double v);
int  lo_irradiance(int n, int ch, int w, int h, const double* const* imgs,
                   const double* const* yeqs, const double* exposures, int ref_index,
                   const lo_params* p, double* out);

/* ---- learned displacement proposal (proposal_oracle.c; an extension, not
 * part of the paper: it narrows the search of Sec. 2.2) ---------------------- */
double lo_bf16(double v);
int    lo_cnn_param_count(void);
void   lo_cnn_tile_input(const uint8_t* ref, const uint8_t* warped, int w, int h, int x0,
                         int y0, double* x /* [4][16][16] */);
void   lo_cnn_forward(const double* params, const double* x, int n, int rnd, double* out);
double lo_cnn_loss_grad(const double* params, const double* x, const int32_t* label, int n,
                        int rnd, double* grad);
void   lo_adamw(double* w, double* m, double* v, const double* g, int n, int t, double lr,
                double b1, double b2, double eps, double wd);
void   lo_search_window(const uint8_t* ref, const uint8_t* wimg, int w, int h,
                        const lo_params* p, int R, const int32_t* ccx, const int32_t* ccy,
                        const int32_t* cx, const int32_t* cy, const uint8_t* has, int32_t* dx,
                        int32_t* dy, uint32_t* ssd, uint8_t* valid);

#ifdef __cplusplus
}
#endif
#endif
