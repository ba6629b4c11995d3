/*
 * lnr_oracle.c -- plain CPU oracle (test infrastructure; see lnr_oracle.h).
 *
 * Written for readability against the paper, not for speed: every stage is a
 * direct loop over its definition. Real-valued stages run in double
 * precision. Compiled with -ffp-contract=off so that the double-precision
 * steps whose results are rounded to integers (warp coordinates, weeding
 * inlier tests, homography fits) use one rounding per operation, in the order
 * written here.
 */
#include "lnr_oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }
static int iclamp(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

void lo_default_params(lo_params* p) {
  memset(p, 0, sizeof(*p));
  p->tile = 32;
  p->patch_r = 10;        /* 21x21 patches (Sec. 2.6) */
  p->corner_step = 2;     /* 1/16 of the tile (Sec. 2.6) */
  p->corner_half = 2;
  p->quad_r = 10;
  p->corner_t = 2;
  p->max_levels = 5;      /* Sec. 2.6 */
  p->min_level_dim = 100; /* Sec. 2.6 */
  p->radius_coarse = 10;  /* Sec. 2.6 */
  p->radius0 = 16;
  p->weed_iters = 1024;
  p->weed_delta_min = 8;
  p->weed_delta_pct = 2;
  p->dt_iters = 3;
  p->weed_eps = 2.0;
  p->sigma_s = 400.0;     /* Sec. 2.6 */
  p->sigma_r = 1.0;
  p->n_min = 1e-30;
  p->ssim_sigma = 1.5;
  p->ssim_radius = 5;
  p->ssim_c1 = 0.01 * 0.01;
  p->ssim_c2 = 0.03 * 0.03;
  p->sigma_e = 0.2;
  p->seed = 0x1504014410ull;
}

/* Sec. 2.6: up to max_levels levels; stop before a level whose width or
 * height would fall below min_level_dim. Each level halves (floor) the last. */
int lo_num_levels(int w, int h, const lo_params* p) {
  int levels = 1;
  while (levels < p->max_levels) {
    int w2 = w / 2, h2 = h / 2;
    if (imin(w2, h2) < p->min_level_dim) break;
    w = w2;
    h = h2;
    ++levels;
  }
  return levels;
}

/* ---------------------------------------------------------------------------
 * Sec. 3 (opening): every input is histogram-equalised before matching.
 * LUT[v] = round-half-up(255 * (cdf[v] - cdf_min) / (n - cdf_min)), where
 * cdf_min is the cdf at the first occupied bin (the classic definition).
 * ------------------------------------------------------------------------- */
void lo_histogram(const uint8_t* img, int w, int h, int stride, uint32_t hist[256]) {
  memset(hist, 0, 256 * sizeof(uint32_t));
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) hist[img[(size_t)y * stride + x]]++;
}

void lo_equalize_lut(const uint32_t hist[256], uint8_t lut[256]) {
  int64_t cdf[256];
  int64_t acc = 0;
  for (int v = 0; v < 256; ++v) { acc += hist[v]; cdf[v] = acc; }
  int64_t n = acc, c0 = 0;
  for (int v = 0; v < 256; ++v)
    if (hist[v]) { c0 = cdf[v]; break; }
  for (int v = 0; v < 256; ++v) {
    if (n == c0) { lut[v] = (uint8_t)v; continue; }
    int64_t num = cdf[v] - c0;
    if (num < 0) num = 0;
    int64_t den = n - c0;
    lut[v] = (uint8_t)((2 * 255 * num + den) / (2 * den));
  }
}

void lo_apply_lut(const uint8_t* img, int w, int h, int stride, const uint8_t lut[256],
                  uint8_t* out) {
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) out[(size_t)y * w + x] = lut[img[(size_t)y * stride + x]];
}

/* Sec. 2.2 pyramid: 2x2 box mean, rounded half up. */
void lo_downsample(const uint8_t* in, int w, int h, uint8_t* out) {
  int w2 = w / 2, h2 = h / 2;
  for (int j = 0; j < h2; ++j)
    for (int i = 0; i < w2; ++i) {
      int s = in[(size_t)(2 * j) * w + 2 * i] + in[(size_t)(2 * j) * w + 2 * i + 1] +
              in[(size_t)(2 * j + 1) * w + 2 * i] + in[(size_t)(2 * j + 1) * w + 2 * i + 1];
      out[(size_t)j * w2 + i] = (uint8_t)((s + 2) >> 2);
    }
}

/* ---------------------------------------------------------------------------
 * Sec. 2.2, Eq. 1-2 (cornerness and minimum activity).
 * Quadrants around p, taken in cyclic order TL, TR, BR, BL so that
 * consecutive entries are contiguous quadrants; mu_j is the quadrant mean.
 * C(p) = sum_j |mu_{j+1} - mu_j|; p qualifies iff min_j |mu_{j+1}-mu_j| > T.
 * Means share the divisor r*r, so both are evaluated on integer sums, with
 * the threshold T*r*r. Candidates: tile centre + g*(a, b), a, b in [-K, K],
 * visited b-major then a; the first qualifying candidate with the largest C
 * wins. A tile with no qualifying candidate has no corner.
 * ------------------------------------------------------------------------- */
static int64_t box_sum(const uint8_t* img, int w, int x0, int y0, int x1, int y1) {
  int64_t s = 0;
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x) s += img[(size_t)y * w + x];
  return s;
}

void lo_corners(const uint8_t* img, int w, int h, const lo_params* p,
                int32_t* cx, int32_t* cy, uint8_t* has) {
  const int S = p->tile, r = p->quad_r, K = p->corner_half, g = p->corner_step;
  const int64_t thr = (int64_t)p->corner_t * r * r;
  const int ntx = w / S, nty = h / S;
  for (int ty = 0; ty < nty; ++ty)
    for (int tx = 0; tx < ntx; ++tx) {
      int t = ty * ntx + tx;
      int64_t bestC = -1;
      int bx = -1, by = -1;
      for (int b = -K; b <= K; ++b)
        for (int a = -K; a <= K; ++a) {
          int x = tx * S + S / 2 + g * a, y = ty * S + S / 2 + g * b;
          int64_t q[4];
          q[0] = box_sum(img, w, x - r, y - r, x, y);     /* top-left     */
          q[1] = box_sum(img, w, x, y - r, x + r, y);     /* top-right    */
          q[2] = box_sum(img, w, x, y, x + r, y + r);     /* bottom-right */
          q[3] = box_sum(img, w, x - r, y, x, y + r);     /* bottom-left  */
          int64_t C = 0, mn = -1;
          for (int j = 0; j < 4; ++j) {
            int64_t d = q[(j + 1) % 4] - q[j];
            if (d < 0) d = -d;
            C += d;
            if (mn < 0 || d < mn) mn = d;
          }
          if (mn > thr && C > bestC) { bestC = C; bx = x; by = y; }
        }
      has[t] = bestC >= 0;
      cx[t] = bx;
      cy[t] = by;
    }
}

/* ---------------------------------------------------------------------------
 * Sec. 2.2, Eq. 3: homographies act on normalised coordinates with the origin
 * at the image centre, x in [-1, 1], y in [-h/w, h/w]:
 *     xn = (2x - (w-1)) / w,   yn = (2y - (h-1)) / w.
 * In homogeneous form xn ~ C [x y 1]^T with C = [[2,0,-(w-1)],[0,2,-(h-1)],[0,0,w]]
 * and [x y 1]^T ~ B xn with B = [[w,0,w-1],[0,w,h-1],[0,0,2]] (B C = 2w I),
 * so the level pixel homography is Hp = B (H C) (scale is irrelevant).
 * ------------------------------------------------------------------------- */
static void mat3_mul(const double a[9], const double b[9], double out[9]) {
  double t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = a[3 * i + 0] * b[0 + j];
      s = s + a[3 * i + 1] * b[3 + j];
      s = s + a[3 * i + 2] * b[6 + j];
      t[3 * i + j] = s;
    }
  memcpy(out, t, sizeof(t));
}

void lo_pixel_homography(const double H[9], int w, int h, double Hp[9]) {
  const double B[9] = {(double)w, 0, (double)(w - 1), 0, (double)w, (double)(h - 1), 0, 0, 2};
  const double C[9] = {2, 0, (double)(-(w - 1)), 0, 2, (double)(-(h - 1)), 0, 0, (double)w};
  double T[9];
  mat3_mul(H, C, T);
  mat3_mul(B, T, Hp);
}

/* Map (X, Y) through a 3x3 homography; fixed operation order. */
static void apply_h(const double m[9], double X, double Y, double* sx, double* sy) {
  double den = (m[6] * X + m[7] * Y) + m[8];
  *sx = ((m[0] * X + m[1] * Y) + m[2]) / den;
  *sy = ((m[3] * X + m[4] * Y) + m[5]) / den;
}

/* Warped source W(x) = Src(Hp x) for the search (Eq. 3 evaluated as a
 * resampling). The sample position is quantised to 1/256 px with
 * round-half-up, taps are clamped to the image, and the 8-bit result is the
 * rounded Q16 bilinear blend. */
static int64_t q8_coord(double s) {
  double q = floor(s * 256.0 + 0.5);
  if (!(q > -1073741824.0)) q = -1073741824.0; /* also maps NaN */
  if (q > 1073741824.0) q = 1073741824.0;
  return (int64_t)q;
}

void lo_warp_q8(const uint8_t* src, int w, int h, const double Hp[9], uint8_t* out) {
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      double sx, sy;
      apply_h(Hp, (double)x, (double)y, &sx, &sy);
      int64_t X = q8_coord(sx), Y = q8_coord(sy);
      int64_t ix = X >> 8, iy = Y >> 8; /* floor */
      int fx = (int)(X & 255), fy = (int)(Y & 255);
      int x0 = (int)(ix < 0 ? 0 : (ix > w - 1 ? w - 1 : ix));
      int x1 = (int)(ix + 1 < 0 ? 0 : (ix + 1 > w - 1 ? w - 1 : ix + 1));
      int y0 = (int)(iy < 0 ? 0 : (iy > h - 1 ? h - 1 : iy));
      int y1 = (int)(iy + 1 < 0 ? 0 : (iy + 1 > h - 1 ? h - 1 : iy + 1));
      uint32_t p00 = src[(size_t)y0 * w + x0], p10 = src[(size_t)y0 * w + x1];
      uint32_t p01 = src[(size_t)y1 * w + x0], p11 = src[(size_t)y1 * w + x1];
      uint32_t acc = (uint32_t)((256 - fx) * (256 - fy)) * p00 + (uint32_t)(fx * (256 - fy)) * p10 +
                     (uint32_t)((256 - fx) * fy) * p01 + (uint32_t)(fx * fy) * p11;
      out[(size_t)y * w + x] = (uint8_t)((acc + 32768u) >> 16);
    }
}

/* ---------------------------------------------------------------------------
 * Sec. 2.2: for each reference corner p, the displacement d in [-R, R]^2
 * minimising the SSD between the (2P+1)^2 patch at p in the reference and the
 * patch at p + d in the warped source. Candidates whose patch leaves the
 * image are skipped. Ties: smallest SSD, then smallest |dx|+|dy|, then
 * smallest dy, then smallest dx.
 * ------------------------------------------------------------------------- */
void lo_search(const uint8_t* ref, const uint8_t* wimg, int w, int h, const lo_params* p,
               int R, const int32_t* cx, const int32_t* cy, const uint8_t* has,
               int32_t* dx, int32_t* dy, uint32_t* ssd, uint8_t* valid) {
  const int S = p->tile, P = p->patch_r;
  const int ntiles = (w / S) * (h / S);
  for (int t = 0; t < ntiles; ++t) {
    valid[t] = 0;
    dx[t] = 0;
    dy[t] = 0;
    ssd[t] = 0;
    if (!has[t]) continue;
    int px = cx[t], py = cy[t];
    int found = 0;
    uint32_t bs = 0;
    int bl = 0, bdx = 0, bdy = 0;
    for (int ddy = -R; ddy <= R; ++ddy)
      for (int ddx = -R; ddx <= R; ++ddx) {
        if (px + ddx - P < 0 || px + ddx + P > w - 1) continue;
        if (py + ddy - P < 0 || py + ddy + P > h - 1) continue;
        uint32_t s = 0;
        for (int j = -P; j <= P; ++j)
          for (int i = -P; i <= P; ++i) {
            int a = ref[(size_t)(py + j) * w + (px + i)];
            int b = wimg[(size_t)(py + ddy + j) * w + (px + ddx + i)];
            s += (uint32_t)((a - b) * (a - b));
          }
        int l1 = abs(ddx) + abs(ddy);
        int better = !found || s < bs || (s == bs && (l1 < bl || (l1 == bl && (ddy < bdy ||
                     (ddy == bdy && ddx < bdx)))));
        if (better) { found = 1; bs = s; bl = l1; bdx = ddx; bdy = ddy; }
      }
    if (found) { valid[t] = 1; dx[t] = bdx; dy[t] = bdy; ssd[t] = bs; }
  }
}

/* Sec. 2.2 with Eq. 3 taken as printed: the previous level's homography
 * predicts where each reference corner x lies in the *unwarped* source,
 * q = (floor(sx + 0.5), floor(sy + 0.5)) with (sx, sy) = Hp x, and the SSD
 * search runs over q + d, d in [-R, R]^2, against the unwarped source. Same
 * patch, skip rule and tie order (on d) as lo_search; the match is the
 * absolute correspondence x -> q + d, stored as dx, dy = q + d - x. */
static int32_t round_pred(double s) {
  double q = floor(s + 0.5);
  if (!(q > -1048576.0)) q = -1048576.0; /* also maps NaN */
  if (q > 1048576.0) q = 1048576.0;
  return (int32_t)q;
}

void lo_search_unwarped(const uint8_t* ref, const uint8_t* src, int w, int h,
                        const lo_params* p, int R, const double Hp[9], const int32_t* cx,
                        const int32_t* cy, const uint8_t* has, int32_t* dx, int32_t* dy,
                        uint32_t* ssd, uint8_t* valid) {
  const int S = p->tile, P = p->patch_r;
  const int ntiles = (w / S) * (h / S);
  for (int t = 0; t < ntiles; ++t) {
    valid[t] = 0;
    dx[t] = 0;
    dy[t] = 0;
    ssd[t] = 0;
    if (!has[t]) continue;
    const int px = cx[t], py = cy[t];
    double sx, sy;
    apply_h(Hp, (double)px, (double)py, &sx, &sy);
    const int qx = round_pred(sx), qy = round_pred(sy);
    int found = 0;
    uint32_t bs = 0;
    int bl = 0, bdx = 0, bdy = 0;
    for (int ddy = -R; ddy <= R; ++ddy)
      for (int ddx = -R; ddx <= R; ++ddx) {
        const int sx0 = qx + ddx, sy0 = qy + ddy;  /* candidate centre in the source */
        if (sx0 - P < 0 || sx0 + P > w - 1 || sy0 - P < 0 || sy0 + P > h - 1) continue;
        uint32_t s = 0;
        for (int j = -P; j <= P; ++j)
          for (int i = -P; i <= P; ++i) {
            int a = ref[(size_t)(py + j) * w + (px + i)];
            int b = src[(size_t)(sy0 + j) * w + (sx0 + i)];
            s += (uint32_t)((a - b) * (a - b));
          }
        int l1 = abs(ddx) + abs(ddy);
        int better = !found || s < bs || (s == bs && (l1 < bl || (l1 == bl && (ddy < bdy ||
                     (ddy == bdy && ddx < bdx)))));
        if (better) { found = 1; bs = s; bl = l1; bdx = ddx; bdy = ddy; }
      }
    if (found) {
      valid[t] = 1;
      dx[t] = qx + bdx - px;
      dy[t] = qy + bdy - py;
      ssd[t] = bs;
    }
  }
}

/* ---------------------------------------------------------------------------
 * Dense 8x8 linear solve, Gaussian elimination with partial pivoting (first
 * largest |pivot|), rows updated as a[r][j] - f * a[c][j]; a pivot below
 * 1e-12 in magnitude (or NaN) means singular.
 * ------------------------------------------------------------------------- */
static int solve8(double a[8][9], double hsol[8]) {
  for (int c = 0; c < 8; ++c) {
    int piv = c;
    double best = fabs(a[c][c]);
    for (int r = c + 1; r < 8; ++r) {
      double v = fabs(a[r][c]);
      if (v > best) { best = v; piv = r; }
    }
    if (!(best >= 1e-12)) return 0;
    if (piv != c)
      for (int j = 0; j < 9; ++j) { double t = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = t; }
    for (int r = c + 1; r < 8; ++r) {
      double f = a[r][c] / a[c][c];
      for (int j = c; j < 9; ++j) a[r][j] = a[r][j] - f * a[c][j];
    }
  }
  for (int c = 7; c >= 0; --c) {
    double s = a[c][8];
    for (int j = c + 1; j < 8; ++j) s = s - a[c][j] * hsol[j];
    hsol[c] = s / a[c][c];
  }
  return 1;
}

/* Four correspondences (s -> t), h33 = 1: for each,
 *   [sx sy 1 0 0 0 -sx*tx -sy*tx] h = tx,  [0 0 0 sx sy 1 -sx*ty -sy*ty] h = ty. */
int lo_fit4(const double sx[4], const double sy[4], const double tx[4], const double ty[4],
            double g[9]) {
  double a[8][9];
  for (int k = 0; k < 4; ++k) {
    double* r0 = a[2 * k];
    double* r1 = a[2 * k + 1];
    r0[0] = sx[k]; r0[1] = sy[k]; r0[2] = 1; r0[3] = 0; r0[4] = 0; r0[5] = 0;
    r0[6] = -(sx[k] * tx[k]); r0[7] = -(sy[k] * tx[k]); r0[8] = tx[k];
    r1[0] = 0; r1[1] = 0; r1[2] = 0; r1[3] = sx[k]; r1[4] = sy[k]; r1[5] = 1;
    r1[6] = -(sx[k] * ty[k]); r1[7] = -(sy[k] * ty[k]); r1[8] = ty[k];
  }
  double hs[8];
  if (!solve8(a, hs)) return 0;
  for (int i = 0; i < 8; ++i) g[i] = hs[i];
  g[8] = 1.0;
  return 1;
}

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the counter-based sampler
 * of the weeding filter. */
static uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* ---------------------------------------------------------------------------
 * Sec. 2.3, Eq. 5: the weeding filter. Matches (valid tiles, raster order)
 * are indexed k = 0..N-1. Iteration i draws four distinct indices (draw t of
 * iteration i uses splitmix64((seed ^ level<<56) + 16 i + t) scaled to
 * [0, N); repeats are redrawn, at most 16 draws), fits a homography H^i that
 * maps each sampled match from the source side (p + d) to the reference side
 * (p), and collects the inliers I^i = {k : |H^i(p_k + d_k) - p_k|^2 < eps^2}.
 * If |I^i| > delta then M = M u I^i. Coordinates are level pixels minus
 * (w/2, h/2) (integer division). Because M only grows by unions, any
 * partition of the iteration range gives the same M (the paper's note that
 * n threads of 1/n iterations equal one run). The iteration with the most
 * inliers (lowest index on ties) is also reported: it seeds the level
 * homography below.
 * ------------------------------------------------------------------------- */
typedef struct {
  int N, delta;
  int* idx_of;
  double *sx, *sy, *tx, *ty;
} match_set;

static void match_set_init(match_set* m, int ntiles, const int32_t* cx, const int32_t* cy,
                           const int32_t* dx, const int32_t* dy, const uint8_t* valid, int w,
                           int h, const lo_params* p) {
  int N = 0;
  for (int t = 0; t < ntiles; ++t) N += valid[t] ? 1 : 0;
  m->N = N;
  m->delta = imax(p->weed_delta_min, (N * p->weed_delta_pct + 99) / 100);
  m->idx_of = (int*)malloc(sizeof(int) * (size_t)(N + 1));
  m->sx = (double*)malloc(sizeof(double) * (size_t)(N + 1) * 4);
  m->sy = m->sx + (N + 1);
  m->tx = m->sx + 2 * (size_t)(N + 1);
  m->ty = m->sx + 3 * (size_t)(N + 1);
  const int ox = w / 2, oy = h / 2;
  int k = 0;
  for (int t = 0; t < ntiles; ++t)
    if (valid[t]) {
      m->idx_of[k] = t;
      m->sx[k] = (double)(cx[t] + dx[t] - ox);
      m->sy[k] = (double)(cy[t] + dy[t] - oy);
      m->tx[k] = (double)(cx[t] - ox);
      m->ty[k] = (double)(cy[t] - oy);
      ++k;
    }
}

static void match_set_free(match_set* m) {
  free(m->sx);
  free(m->idx_of);
}

/* Draw and fit hypothesis `it`; on success fill inl[0..N) and return the count,
 * else return -1. */
static int hypothesis(const match_set* m, int level, int it, const lo_params* p, double g[9],
                      uint8_t* inl) {
  const int N = m->N;
  const uint64_t base = p->seed ^ ((uint64_t)(uint32_t)level << 56);
  int pick[4], np = 0;
  for (int t = 0; t < 16 && np < 4; ++t) {
    uint64_t u = splitmix64(base + (uint64_t)it * 16u + (uint64_t)t);
    int id = (int)(((u >> 32) * (uint64_t)N) >> 32);
    int dup = 0;
    for (int q = 0; q < np; ++q) dup |= pick[q] == id;
    if (!dup) pick[np++] = id;
  }
  if (np < 4) return -1;
  double s4x[4], s4y[4], t4x[4], t4y[4];
  for (int q = 0; q < 4; ++q) {
    s4x[q] = m->sx[pick[q]]; s4y[q] = m->sy[pick[q]];
    t4x[q] = m->tx[pick[q]]; t4y[q] = m->ty[pick[q]];
  }
  if (!lo_fit4(s4x, s4y, t4x, t4y, g)) return -1;
  const double eps2 = p->weed_eps * p->weed_eps;
  int cnt = 0;
  for (int q = 0; q < N; ++q) {
    double den = (g[6] * m->sx[q] + g[7] * m->sy[q]) + 1.0;
    double gx = ((g[0] * m->sx[q] + g[1] * m->sy[q]) + g[2]) / den;
    double gy = ((g[3] * m->sx[q] + g[4] * m->sy[q]) + g[5]) / den;
    double ex = gx - m->tx[q], ey = gy - m->ty[q];
    double e2 = ex * ex + ey * ey;
    inl[q] = e2 < eps2;
    cnt += inl[q];
  }
  return cnt;
}

int lo_weed(int ntiles, const int32_t* cx, const int32_t* cy, const int32_t* dx,
            const int32_t* dy, const uint8_t* valid, int w, int h, int level,
            const lo_params* p, int it0, int it1, uint8_t* inM, int32_t* best_count,
            int32_t* best_iter) {
  match_set m;
  match_set_init(&m, ntiles, cx, cy, dx, dy, valid, w, h, p);
  int bc = -1, bi = -1;
  if (m.N >= 4) {
    uint8_t* inl = (uint8_t*)malloc((size_t)m.N);
    double g[9];
    for (int it = it0; it < it1; ++it) {
      int cnt = hypothesis(&m, level, it, p, g, inl);
      if (cnt < 0) continue;
      if (cnt > bc) { bc = cnt; bi = it; }
      if (cnt > m.delta)
        for (int q = 0; q < m.N; ++q)
          if (inl[q]) inM[m.idx_of[q]] = 1;
    }
    free(inl);
  }
  if (best_count) *best_count = bc;
  if (best_iter) *best_iter = bi;
  int N = m.N;
  match_set_free(&m);
  return N;
}

int lo_weed_delta(int n, const lo_params* p) {
  return imax(p->weed_delta_min, (n * p->weed_delta_pct + 99) / 100);
}

int lo_hypothesis_inliers(int ntiles, const int32_t* cx, const int32_t* cy, const int32_t* dx,
                          const int32_t* dy, const uint8_t* valid, int w, int h, int level,
                          const lo_params* p, int it, uint8_t* sel) {
  match_set m;
  match_set_init(&m, ntiles, cx, cy, dx, dy, valid, w, h, p);
  memset(sel, 0, (size_t)ntiles);
  int cnt = -1;
  if (m.N >= 4) {
    uint8_t* inl = (uint8_t*)malloc((size_t)m.N);
    double g[9];
    cnt = hypothesis(&m, level, it, p, g, inl);
    if (cnt >= 0)
      for (int q = 0; q < m.N; ++q)
        if (inl[q]) sel[m.idx_of[q]] = 1;
    free(inl);
  }
  match_set_free(&m);
  return cnt;
}

/* ---------------------------------------------------------------------------
 * Sec. 2.2: the level homography, from the level's corners and matches:
 * the least-squares DLT (h33 = 1) of G: p -> p + d over a selected set of
 * matches (in the pipeline: the inliers of the weeding iteration with the
 * largest consensus, provided it exceeds delta), composed on the previous
 * level's homography, H^l = H^{l+1} o G^l.
 * The normal equations are summed exactly in 64-bit integers over centred
 * integer coordinates (x - w/2, y - h/2), then scaled by powers of two
 * (exact) for conditioning, solved as above, and G moved to the normalised
 * frame: with xn ~ Pm xc, Pm = [[2,0,ox],[0,2,oy],[0,0,w]],
 * ox = 2(w/2) - (w-1), Gn = Pm Gc Qm, Qm = [[w,0,-ox],[0,w,-oy],[0,0,2]].
 * Fewer than 4 matches, a singular system or a degenerate product keeps H^{l+1}.
 * ------------------------------------------------------------------------- */
/* Hbase: the map the fitted G is composed on (H^{l+1}, or the identity when
 * the matches are absolute); Hprev is the result when the fit fails. */
static int fit_level(int ntiles, const int32_t* cx, const int32_t* cy, const int32_t* dx,
                     const int32_t* dy, const uint8_t* sel, int w, int h,
                     const double Hprev[9], const double Hbase[9], double Hout[9]) {
  const int ox = w / 2, oy = h / 2;
  int64_t ata[8][8], atb[8];
  memset(ata, 0, sizeof(ata));
  memset(atb, 0, sizeof(atb));
  int m = 0;
  for (int t = 0; t < ntiles; ++t) {
    if (!sel[t]) continue;
    int64_t x = cx[t] - ox, y = cy[t] - oy;
    int64_t u = x + dx[t], v = y + dy[t];
    int64_t r1[8] = {x, y, 1, 0, 0, 0, -x * u, -y * u};
    int64_t r2[8] = {0, 0, 0, x, y, 1, -x * v, -y * v};
    for (int i = 0; i < 8; ++i) {
      for (int j = 0; j < 8; ++j) ata[i][j] += r1[i] * r1[j] + r2[i] * r2[j];
      atb[i] += r1[i] * u + r2[i] * v;
    }
    ++m;
  }
  memcpy(Hout, Hprev, 9 * sizeof(double));
  if (m < 4) return m;
  int k = 0;
  while ((1 << k) < imax(imax(ox, oy), 1)) ++k;
  static const int deg[8] = {1, 1, 0, 1, 1, 0, 2, 2};
  double a[8][9];
  for (int i = 0; i < 8; ++i) {
    for (int j = 0; j < 8; ++j) a[i][j] = ldexp((double)ata[i][j], -k * (deg[i] + deg[j]));
    a[i][8] = ldexp((double)atb[i], -k * (deg[i] + 1));
  }
  double hs[8];
  if (!solve8(a, hs)) return m;
  double Gc[9];
  for (int i = 0; i < 8; ++i) Gc[i] = ldexp(hs[i], k * (1 - deg[i]));
  Gc[8] = 1.0;
  const double pox = (double)(2 * ox - (w - 1)), poy = (double)(2 * oy - (h - 1));
  const double Pm[9] = {2, 0, pox, 0, 2, poy, 0, 0, (double)w};
  const double Qm[9] = {(double)w, 0, -pox, 0, (double)w, -poy, 0, 0, 2};
  double T1[9], T2[9], T3[9];
  mat3_mul(Pm, Gc, T1);
  mat3_mul(T1, Qm, T2);
  mat3_mul(Hbase, T2, T3);
  double d = T3[8];
  double Hn[9];
  int ok = d != 0.0;
  for (int i = 0; i < 9 && ok; ++i) {
    Hn[i] = T3[i] / d;
    ok = isfinite(Hn[i]);
  }
  if (ok) memcpy(Hout, Hn, sizeof(Hn));
  return m;
}

int lo_fit_level(int ntiles, const int32_t* cx, const int32_t* cy, const int32_t* dx,
                 const int32_t* dy, const uint8_t* sel, int w, int h,
                 const double Hprev[9], double Hout[9]) {
  return fit_level(ntiles, cx, cy, dx, dy, sel, w, h, Hprev, Hprev, Hout);
}

int lo_fit_level_absolute(int ntiles, const int32_t* cx, const int32_t* cy,
                          const int32_t* dx, const int32_t* dy, const uint8_t* sel, int w,
                          int h, const double Hprev[9], double Hout[9]) {
  static const double I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  return fit_level(ntiles, cx, cy, dx, dy, sel, w, h, Hprev, I3, Hout);
}

/* ---------------------------------------------------------------------------
 * Sec. 2.4, Eq. 6-7: sparse maps P_u, P_v (the match displacement at each
 * kept corner pixel, 0 elsewhere) and N (1 at kept corners), cross-bilateral
 * filtered with the domain transform's recursive filter (Gastal & Oliveira
 * 2011) guided by the equalised reference I = Y_eq / 255: for iteration
 * i = 1..n, sigma_i = sigma_s sqrt(3) 2^(n-i) / sqrt(4^n - 1), a_i =
 * exp(-sqrt(2)/sigma_i), and along each row then each column,
 *   causal:      J[x] = J[x] + a_i^d(x) (J[x-1] - J[x]),  x increasing,
 *   anti-causal: J[x] = J[x] + a_i^d(x+1) (J[x+1] - J[x]), x decreasing,
 * with d(x) = 1 + (sigma_s/sigma_r) |I[x] - I[x-1]|. The flow is
 * F = (P~_u / N~, P~_v / N~) where N~ > n_min, else 0.
 * ------------------------------------------------------------------------- */
static void rf_line(double* a, double* b, double* c, const uint8_t* g, int n, ptrdiff_t st,
                    ptrdiff_t gst, double ai, double ratio) {
  for (int x = 1; x < n; ++x) {
    double diff = fabs((double)g[x * gst] / 255.0 - (double)g[(x - 1) * gst] / 255.0);
    double cf = pow(ai, 1.0 + ratio * diff);
    a[x * st] = a[x * st] + cf * (a[(x - 1) * st] - a[x * st]);
    b[x * st] = b[x * st] + cf * (b[(x - 1) * st] - b[x * st]);
    c[x * st] = c[x * st] + cf * (c[(x - 1) * st] - c[x * st]);
  }
  for (int x = n - 2; x >= 0; --x) {
    double diff = fabs((double)g[(x + 1) * gst] / 255.0 - (double)g[x * gst] / 255.0);
    double cf = pow(ai, 1.0 + ratio * diff);
    a[x * st] = a[x * st] + cf * (a[(x + 1) * st] - a[x * st]);
    b[x * st] = b[x * st] + cf * (b[(x + 1) * st] - b[x * st]);
    c[x * st] = c[x * st] + cf * (c[(x + 1) * st] - c[x * st]);
  }
}

void lo_sparse_to_dense(int ntiles, const int32_t* cx, const int32_t* cy, const int32_t* dx,
                        const int32_t* dy, const uint8_t* inM, const uint8_t* guide,
                        int w, int h, const lo_params* p, double* fu, double* fv,
                        double* ntilde) {
  size_t n = (size_t)w * h;
  double* pu = (double*)calloc(n, sizeof(double));
  double* pv = (double*)calloc(n, sizeof(double));
  double* nn = (double*)calloc(n, sizeof(double));
  for (int t = 0; t < ntiles; ++t)
    if (inM[t]) {
      size_t o = (size_t)cy[t] * w + cx[t];
      pu[o] = dx[t];
      pv[o] = dy[t];
      nn[o] = 1.0;
    }
  const int iters = p->dt_iters;
  const double ratio = p->sigma_s / p->sigma_r;
  for (int i = 1; i <= iters; ++i) {
    double sig = p->sigma_s * sqrt(3.0) * pow(2.0, iters - i) / sqrt(pow(4.0, iters) - 1.0);
    double ai = exp(-sqrt(2.0) / sig);
    for (int y = 0; y < h; ++y) {
      size_t o = (size_t)y * w;
      rf_line(pu + o, pv + o, nn + o, guide + o, w, 1, 1, ai, ratio);
    }
    for (int x = 0; x < w; ++x)
      rf_line(pu + x, pv + x, nn + x, guide + x, h, w, w, ai, ratio);
  }
  for (size_t o = 0; o < n; ++o) {
    if (nn[o] > p->n_min) { fu[o] = pu[o] / nn[o]; fv[o] = pv[o] / nn[o]; }
    else { fu[o] = 0.0; fv[o] = 0.0; }
    if (ntilde) ntilde[o] = nn[o];
  }
  free(pu);
  free(pv);
  free(nn);
}

/* ---------------------------------------------------------------------------
 * Backward warp of the source to the reference (Sec. 2.1: the goal is to warp
 * the source to the reference): sample position m(x) = Hp(x + F(x)),
 * bilinear with clamp to edge; 4:2:0 chroma is upsampled by pixel repetition
 * (tap (X, Y) reads chroma (X>>1, Y>>1)). Output RGB (BT.601 full range) in
 * [0, 1], or grey Y/255 for a luma-only frame, plus the warped Y_eq / 255.
 * ------------------------------------------------------------------------- */
static void yuv_to_rgb(double Y, double U, double V, double* r, double* g, double* b) {
  double up = U - 128.0, vp = V - 128.0;
  *r = (Y + 1.402 * vp) / 255.0;
  *g = (Y - 0.344136 * up - 0.714136 * vp) / 255.0;
  *b = (Y + 1.772 * up) / 255.0;
}

void lo_backward_warp(const uint8_t* y, const uint8_t* u, const uint8_t* v,
                      const uint8_t* yeq, int w, int h, const double Hp[9],
                      const double* fu, const double* fv, double* rgb, double* yeq_w) {
  const size_t n = (size_t)w * h;
  const int cw = w / 2;
  for (int py = 0; py < h; ++py)
    for (int px = 0; px < w; ++px) {
      size_t o = (size_t)py * w + px;
      double sx, sy;
      apply_h(Hp, (double)px + fu[o], (double)py + fv[o], &sx, &sy);
      if (!(sx >= -1.0)) sx = -1.0;
      if (sx > (double)w) sx = (double)w;
      if (!(sy >= -1.0)) sy = -1.0;
      if (sy > (double)h) sy = (double)h;
      double fx0 = floor(sx), fy0 = floor(sy);
      double ax = sx - fx0, ay = sy - fy0;
      int ix = (int)fx0, iy = (int)fy0;
      int x0 = iclamp(ix, 0, w - 1), x1 = iclamp(ix + 1, 0, w - 1);
      int y0 = iclamp(iy, 0, h - 1), y1 = iclamp(iy + 1, 0, h - 1);
#define BIL(P, I00, I10, I01, I11) \
  ((1.0 - ay) * ((1.0 - ax) * (double)(P)[I00] + ax * (double)(P)[I10]) + \
   ay * ((1.0 - ax) * (double)(P)[I01] + ax * (double)(P)[I11]))
      double Yv = BIL(y, (size_t)y0 * w + x0, (size_t)y0 * w + x1, (size_t)y1 * w + x0,
                      (size_t)y1 * w + x1);
      yeq_w[o] = BIL(yeq, (size_t)y0 * w + x0, (size_t)y0 * w + x1, (size_t)y1 * w + x0,
                     (size_t)y1 * w + x1) / 255.0;
      if (!u) {
        rgb[o] = Yv / 255.0;
        continue;
      }
      size_t c00 = (size_t)(y0 >> 1) * cw + (x0 >> 1), c10 = (size_t)(y0 >> 1) * cw + (x1 >> 1);
      size_t c01 = (size_t)(y1 >> 1) * cw + (x0 >> 1), c11 = (size_t)(y1 >> 1) * cw + (x1 >> 1);
      double Uv = BIL(u, c00, c10, c01, c11), Vv = BIL(v, c00, c10, c01, c11);
#undef BIL
      yuv_to_rgb(Yv, Uv, Vv, &rgb[o], &rgb[n + o], &rgb[2 * n + o]);
    }
}

void lo_frame_to_rgb(const uint8_t* y, const uint8_t* u, const uint8_t* v, int w, int h,
                     double* rgb) {
  const size_t n = (size_t)w * h;
  const int cw = w / 2;
  for (int py = 0; py < h; ++py)
    for (int px = 0; px < w; ++px) {
      size_t o = (size_t)py * w + px;
      if (!u) { rgb[o] = y[o] / 255.0; continue; }
      size_t c = (size_t)(py >> 1) * cw + (px >> 1);
      yuv_to_rgb(y[o], u[c], v[c], &rgb[o], &rgb[n + o], &rgb[2 * n + o]);
    }
}

/* ---------------------------------------------------------------------------
 * Sec. 2.5: SSIM (Wang et al. 2004) with an 11x11 Gaussian window
 * (sigma 1.5, normalised, borders clamped), computed from five Gaussian
 * filterings (x, y, x^2, y^2, xy):
 *   SSIM = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2)).
 * ------------------------------------------------------------------------- */
static void gauss_sep(const double* in, int w, int h, const double* g, int r, double* tmp,
                      double* out) {
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      double s = 0;
      for (int k = -r; k <= r; ++k) s += g[k + r] * in[(size_t)y * w + iclamp(x + k, 0, w - 1)];
      tmp[(size_t)y * w + x] = s;
    }
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      double s = 0;
      for (int k = -r; k <= r; ++k) s += g[k + r] * tmp[(size_t)iclamp(y + k, 0, h - 1) * w + x];
      out[(size_t)y * w + x] = s;
    }
}

void lo_ssim(const double* a, const double* b, int w, int h, const lo_params* p, double* out) {
  const int r = p->ssim_radius;
  double* g = (double*)malloc(sizeof(double) * (size_t)(2 * r + 1));
  double gs = 0;
  for (int k = -r; k <= r; ++k) {
    g[k + r] = exp(-(double)(k * k) / (2.0 * p->ssim_sigma * p->ssim_sigma));
    gs += g[k + r];
  }
  for (int k = 0; k <= 2 * r; ++k) g[k] /= gs;
  size_t n = (size_t)w * h;
  double* buf = (double*)malloc(sizeof(double) * n * 7);
  double *prod = buf, *tmp = buf + n, *ma = buf + 2 * n, *mb = buf + 3 * n, *saa = buf + 4 * n,
         *sbb = buf + 5 * n, *sab = buf + 6 * n;
  gauss_sep(a, w, h, g, r, tmp, ma);
  gauss_sep(b, w, h, g, r, tmp, mb);
  for (size_t o = 0; o < n; ++o) prod[o] = a[o] * a[o];
  gauss_sep(prod, w, h, g, r, tmp, saa);
  for (size_t o = 0; o < n; ++o) prod[o] = b[o] * b[o];
  gauss_sep(prod, w, h, g, r, tmp, sbb);
  for (size_t o = 0; o < n; ++o) prod[o] = a[o] * b[o];
  gauss_sep(prod, w, h, g, r, tmp, sab);
  for (size_t o = 0; o < n; ++o) {
    double mx = ma[o], my = mb[o];
    double vx = saa[o] - mx * mx, vy = sbb[o] - my * my, cxy = sab[o] - mx * my;
    out[o] = ((2 * mx * my + p->ssim_c1) * (2 * cxy + p->ssim_c2)) /
             ((mx * mx + my * my + p->ssim_c1) * (vx + vy + p->ssim_c2));
  }
  free(buf);
  free(g);
}

/* ---------------------------------------------------------------------------
 * Sec. 2.5: exposure fusion weights (Mertens et al. 2007) -- contrast
 * |discrete Laplacian of grey|, saturation (std of R, G, B), well-exposedness
 * prod_c exp(-(c - 0.5)^2 / (2 sigma_e^2)) -- times the fourth, registration
 * quality weight max(SSIM, 0) for every frame that was warped (ssim[k] !=
 * NULL), plus 1e-12, normalised over the frames. Grey = 0.299 R + 0.587 G +
 * 0.114 B; a luma-only stack (ch = 1) has no saturation term.
 * ------------------------------------------------------------------------- */
static void fusion_weights(int n, int ch, int w, int h, const double* const* imgs,
                           const double* const* ssim, const lo_params* p, double* const* wout,
                           double* raw_sum) {
  const size_t np = (size_t)w * h;
  double* grey = (double*)malloc(sizeof(double) * np);
  for (int k = 0; k < n; ++k) {
    const double* I = imgs[k];
    for (size_t o = 0; o < np; ++o)
      grey[o] = ch == 3 ? 0.299 * I[o] + 0.587 * I[np + o] + 0.114 * I[2 * np + o] : I[o];
    for (int y = 0; y < h; ++y)
      for (int x = 0; x < w; ++x) {
        size_t o = (size_t)y * w + x;
        double lap = grey[(size_t)iclamp(y - 1, 0, h - 1) * w + x] +
                     grey[(size_t)y * w + iclamp(x - 1, 0, w - 1)] +
                     grey[(size_t)y * w + iclamp(x + 1, 0, w - 1)] +
                     grey[(size_t)iclamp(y + 1, 0, h - 1) * w + x] - 4.0 * grey[o];
        double C = fabs(lap);
        double S = 1.0, E;
        if (ch == 3) {
          double R = I[o], G = I[np + o], B = I[2 * np + o];
          double mu = (R + G + B) / 3.0;
          S = sqrt(((R - mu) * (R - mu) + (G - mu) * (G - mu) + (B - mu) * (B - mu)) / 3.0);
          double e = (R - 0.5) * (R - 0.5) + (G - 0.5) * (G - 0.5) + (B - 0.5) * (B - 0.5);
          E = exp(-e / (2.0 * p->sigma_e * p->sigma_e));
        } else {
          double e = (I[o] - 0.5) * (I[o] - 0.5);
          E = exp(-e / (2.0 * p->sigma_e * p->sigma_e));
        }
        double Wt = C * S * E;
        if (ssim[k]) Wt *= ssim[k][o] > 0.0 ? ssim[k][o] : 0.0;
        wout[k][o] = Wt + 1e-12;
      }
  }
  for (size_t o = 0; o < np; ++o) {
    double s = 0;
    for (int k = 0; k < n; ++k) s += wout[k][o];
    if (raw_sum) raw_sum[o] = s;
    for (int k = 0; k < n; ++k) wout[k][o] = wout[k][o] / s;
  }
  free(grey);
}

void lo_fusion_weights(int n, int ch, int w, int h, const double* const* imgs,
                       const double* const* ssim, const lo_params* p, double* const* wout) {
  fusion_weights(n, ch, w, h, imgs, ssim, p, wout, NULL);
}

/* The sum of the frames' fusion weights at each pixel before normalisation:
 * where it is tiny the normalised weights divide rounding noise, so two
 * merges of inputs that differ by rounding can differ there. */
int lo_fusion_weight_sum(int n, int ch, int w, int h, const double* const* imgs,
                         const double* const* yeqs, int ref_index, const lo_params* p,
                         double* out) {
  if (n < 1 || ref_index < 0 || ref_index >= n) return -1;
  const size_t np = (size_t)w * h;
  double** ssim = (double**)calloc((size_t)n, sizeof(double*));
  double** wts = (double**)calloc((size_t)n, sizeof(double*));
  for (int k = 0; k < n; ++k) {
    wts[k] = (double*)malloc(sizeof(double) * np);
    if (k != ref_index) {
      ssim[k] = (double*)malloc(sizeof(double) * np);
      lo_ssim(yeqs[ref_index], yeqs[k], w, h, p, ssim[k]);
    }
  }
  fusion_weights(n, ch, w, h, imgs, (const double* const*)ssim, p, wts, out);
  for (int k = 0; k < n; ++k) { free(ssim[k]); free(wts[k]); }
  free(ssim);
  free(wts);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Multiresolution blend (Mertens et al., Burt & Adelson): Gaussian pyramid of
 * each weight map, Laplacian pyramid of each image, per-level weighted sum,
 * collapse. REDUCE: separable [1 4 6 4 1]/16, borders clamped, keep even
 * samples (size ceil(w/2)). EXPAND to the finer size: even output 2i takes
 * (c[i-1] + 6 c[i] + c[i+1]) / 8, odd output 2i+1 takes (c[i] + c[i+1]) / 2,
 * coarse indices clamped. Levels: 1 + floor(log2(min(w, h) / 8)), at least 1.
 * ------------------------------------------------------------------------- */
int lo_num_blend_levels(int w, int h) {
  int m = imin(w, h), k = 0;
  while ((int64_t)8 << (k + 1) <= m) ++k;
  return 1 + k;
}

void lo_reduce(const double* in, int w, int h, double* out) {
  static const double kf[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
  int w2 = (w + 1) / 2, h2 = (h + 1) / 2;
  double* tmp = (double*)malloc(sizeof(double) * (size_t)w2 * h);
  for (int y = 0; y < h; ++y)
    for (int i = 0; i < w2; ++i) {
      double s = 0;
      for (int k = -2; k <= 2; ++k) s += kf[k + 2] * in[(size_t)y * w + iclamp(2 * i + k, 0, w - 1)];
      tmp[(size_t)y * w2 + i] = s;
    }
  for (int j = 0; j < h2; ++j)
    for (int i = 0; i < w2; ++i) {
      double s = 0;
      for (int k = -2; k <= 2; ++k) s += kf[k + 2] * tmp[(size_t)iclamp(2 * j + k, 0, h - 1) * w2 + i];
      out[(size_t)j * w2 + i] = s;
    }
  free(tmp);
}

static double expand1(const double* c, int n, int x) {
  int i = x >> 1;
  if ((x & 1) == 0)
    return (c[iclamp(i - 1, 0, n - 1)] + 6.0 * c[iclamp(i, 0, n - 1)] + c[iclamp(i + 1, 0, n - 1)]) / 8.0;
  return (c[iclamp(i, 0, n - 1)] + c[iclamp(i + 1, 0, n - 1)]) / 2.0;
}

/* coarse (cw x chh) -> fine (w x h): rows first, then columns */
void lo_expand(const double* c, int cw, int chh, int w, int h, double* out) {
  double* tmp = (double*)malloc(sizeof(double) * (size_t)w * chh);
  double* col = (double*)malloc(sizeof(double) * (size_t)chh);
  for (int j = 0; j < chh; ++j)
    for (int x = 0; x < w; ++x) tmp[(size_t)j * w + x] = expand1(c + (size_t)j * cw, cw, x);
  for (int x = 0; x < w; ++x) {
    for (int j = 0; j < chh; ++j) col[j] = tmp[(size_t)j * w + x];
    for (int y = 0; y < h; ++y) out[(size_t)y * w + x] = expand1(col, chh, y);
  }
  free(col);
  free(tmp);
}

void lo_blend(int n, int ch, int w, int h, const double* const* imgs,
              const double* const* weights, double* out) {
  const int L = lo_num_blend_levels(w, h);
  int lw[32], lh[32];
  size_t loff[33];
  lw[0] = w; lh[0] = h; loff[0] = 0;
  for (int l = 0; l < L; ++l) {
    if (l) { lw[l] = (lw[l - 1] + 1) / 2; lh[l] = (lh[l - 1] + 1) / 2; }
    loff[l + 1] = loff[l] + (size_t)lw[l] * lh[l];
  }
  const size_t tot = loff[L];
  double* gw = (double*)malloc(sizeof(double) * tot);    /* weight pyramid of frame k */
  double* gi = (double*)malloc(sizeof(double) * tot);    /* image pyramid of one channel */
  double* acc = (double*)calloc(tot, sizeof(double));    /* blended Laplacian pyramid */
  double* ex = (double*)malloc(sizeof(double) * (size_t)w * h);
  for (int c = 0; c < ch; ++c) {
    memset(acc, 0, sizeof(double) * tot);
    for (int k = 0; k < n; ++k) {
      memcpy(gw, weights[k], sizeof(double) * (size_t)w * h);
      memcpy(gi, imgs[k] + (size_t)c * w * h, sizeof(double) * (size_t)w * h);
      for (int l = 1; l < L; ++l) {
        lo_reduce(gw + loff[l - 1], lw[l - 1], lh[l - 1], gw + loff[l]);
        lo_reduce(gi + loff[l - 1], lw[l - 1], lh[l - 1], gi + loff[l]);
      }
      for (int l = 0; l < L; ++l) {
        size_t np = (size_t)lw[l] * lh[l];
        if (l + 1 < L) lo_expand(gi + loff[l + 1], lw[l + 1], lh[l + 1], lw[l], lh[l], ex);
        for (size_t o = 0; o < np; ++o) {
          double lap = gi[loff[l] + o] - (l + 1 < L ? ex[o] : 0.0);
          acc[loff[l] + o] += gw[loff[l] + o] * lap;
        }
      }
    }
    /* collapse: R_top = B_top, R_l = B_l + EXPAND(R_{l+1}) */
    for (int l = L - 2; l >= 0; --l) {
      lo_expand(acc + loff[l + 1], lw[l + 1], lh[l + 1], lw[l], lh[l], ex);
      size_t np = (size_t)lw[l] * lh[l];
      for (size_t o = 0; o < np; ++o) acc[loff[l] + o] += ex[o];
    }
    memcpy(out + (size_t)c * w * h, acc, sizeof(double) * (size_t)w * h);
  }
  free(ex);
  free(acc);
  free(gi);
  free(gw);
}

int lo_merge(int n, int ch, int w, int h, const double* const* imgs,
             const double* const* yeqs, int ref_index, const lo_params* p, double* out) {
  if (n < 1 || ref_index < 0 || ref_index >= n) return -1;
  const size_t np = (size_t)w * h;
  double** ssim = (double**)calloc((size_t)n, sizeof(double*));
  double** wts = (double**)calloc((size_t)n, sizeof(double*));
  for (int k = 0; k < n; ++k) {
    wts[k] = (double*)malloc(sizeof(double) * np);
    if (k != ref_index) {
      ssim[k] = (double*)malloc(sizeof(double) * np);
      lo_ssim(yeqs[ref_index], yeqs[k], w, h, p, ssim[k]);
    }
  }
  lo_fusion_weights(n, ch, w, h, imgs, (const double* const*)ssim, p, wts);
  lo_blend(n, ch, w, h, imgs, (const double* const*)wts, out);
  for (int k = 0; k < n; ++k) { free(ssim[k]); free(wts[k]); }
  free(ssim);
  free(wts);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Metering (Sec. 2.1): the first frame is exposed to the right, and the
 * second is made 2, 3 or 4 stops brighter the more under-exposed pixels the
 * first has. The paper does not say where the steps fall. Reading: a pixel
 * is under-exposed when its 8-bit luma is below `dark`; with n_dark of the
 * w h pixels under-exposed, the choice is 2 stops when n_dark <= frac3 w h,
 * 3 when n_dark <= frac4 w h, else 4 (the products in double precision).
 * ------------------------------------------------------------------------- */
int lo_meter(const uint8_t* y, int w, int h, int stride, int dark, float frac3, float frac4,
             long long* n_dark) {
  long long n = 0;
  for (int r = 0; r < h; ++r)
    for (int c = 0; c < w; ++c)
      if ((int)y[(size_t)r * stride + c] < dark) ++n;
  if (n_dark) *n_dark = n;
  const double npix = (double)w * (double)h;
  if ((double)n <= (double)frac3 * npix) return 2;
  if ((double)n <= (double)frac4 * npix) return 3;
  return 4;
}

/* ---------------------------------------------------------------------------
 * HDR irradiance map of the registered stack. In its quality comparison
 * (Sec. 3.1) the paper merges the warped frames into an irradiance map
 * (then tonemaps it) instead of running its error-tolerant fusion, without
 * giving the merge's formula. Reading: the frames are linear in irradiance;
 * frame k's value v in [0, 1], divided by its exposure relative to the
 * reference, estimates the irradiance in the reference's units; the
 * estimates are averaged per channel with the hat weight min(v, 1 - v)
 * (0 for black and saturated samples), and each non-reference frame's
 * weight is multiplied by max(SSIM_k, 0) against the reference, the
 * deghosting weight of the fusion (Sec. 2.5). Where every weight is 0 the
 * reference's own value is kept.
 * ------------------------------------------------------------------------- */
double lo_hat_weight(double v) {
  const double a = v < 1.0 - v ? v : 1.0 - v;
  return a > 0.0 ? a : 0.0;
}

int lo_irradiance(int n, int ch, int w, int h, const double* const* imgs,
                  const double* const* yeqs, const double* exposures, int ref_index,
                  const lo_params* p, double* out) {
  if (n < 1 || ref_index < 0 || ref_index >= n) return -1;
  for (int k = 0; k < n; ++k)
    if (!(exposures[k] > 0.0)) return -1;
  const size_t np = (size_t)w * h;
  double** ssim = (double**)calloc((size_t)n, sizeof(double*));
  for (int k = 0; k < n; ++k)
    if (k != ref_index) {
      ssim[k] = (double*)malloc(sizeof(double) * np);
      lo_ssim(yeqs[ref_index], yeqs[k], w, h, p, ssim[k]);
    }
  for (int c = 0; c < ch; ++c)
    for (size_t i = 0; i < np; ++i) {
      double sw = 0.0, se = 0.0;
      for (int k = 0; k < n; ++k) {
        const double v = imgs[k][c * np + i];
        double wk = lo_hat_weight(v);
        if (k != ref_index) wk *= ssim[k][i] > 0.0 ? ssim[k][i] : 0.0;
        const double t = exposures[k] / exposures[ref_index];
        sw += wk;
        se += wk * (v / t);
      }
      out[c * np + i] = sw > 0.0 ? se / sw : imgs[ref_index][c * np + i];
    }
  for (int k = 0; k < n; ++k) free(ssim[k]);
  free(ssim);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Reference frame of a stack (Sec. 2.1, Sec. 2 opening): the shortest exposure,
 * the lowest index on ties. When the exposures are not known (not every one
 * positive and finite), the darkest frame stands in for the shortest: the
 * lowest mean luma, compared as exact integer sums over equal-size frames,
 * the lowest index on ties.
 * ------------------------------------------------------------------------- */
int lo_pick_reference(int n, const float* exposure, const uint8_t* const* ys, int w, int h,
                      int stride) {
  if (n < 1) return -1;
  int known = 1;
  for (int k = 0; k < n; ++k)
    if (!(exposure[k] > 0.0f) || !isfinite(exposure[k])) known = 0;
  int r = 0;
  if (known) {
    for (int k = 1; k < n; ++k)
      if (exposure[k] < exposure[r]) r = k;
    return r;
  }
  int64_t best = -1;
  for (int k = 0; k < n; ++k) {
    int64_t sum = 0;
    for (int y = 0; y < h; ++y)
      for (int x = 0; x < w; ++x) sum += ys[k][(size_t)y * stride + x];
    if (best < 0 || sum < best) { best = sum; r = k; }
  }
  return r;
}

/* ---------------------------------------------------------------------------
 * One registration (Sec. 2.2 - 2.4): equalise both frames, build the
 * pyramids, then from the coarsest level down: corners on the reference,
 * warp the source level by H^{l+1}, SSD search (radius 10 on coarse levels,
 * radius0 on level 0), weeding, level homography. Level 0's kept matches
 * are propagated to a dense residual flow, and the source is warped
 * backwards through H^1 and that flow.
 * With search_frame 1 (Eq. 3 as printed) no level is warped: each level
 * searches the unwarped source around round(H^{l+1} x), the level
 * homography is fitted to those absolute matches directly (H^{l+1} kept when
 * the fit fails), and level 0's absolute displacements are propagated, so
 * the source is sampled at x + F(x) without a homography; warped0 is not
 * written.
 * ------------------------------------------------------------------------- */
int lo_register_pair(const uint8_t* ref_y, const uint8_t* src_y, const uint8_t* src_u,
                     const uint8_t* src_v, int w, int h, const lo_params* p,
                     const double* H_init, lo_registration* out) {
  if (w < 1 || h < 1) return -1;
  const int L = lo_num_levels(w, h, p);
  const int literal = p->search_frame == 1;
  out->levels = L;
  int lw[6], lh[6];
  size_t poff[7];
  lw[0] = w; lh[0] = h; poff[0] = 0;
  out->tile_off[0] = 0;
  for (int l = 0; l < L; ++l) {
    if (l) { lw[l] = lw[l - 1] / 2; lh[l] = lh[l - 1] / 2; }
    poff[l + 1] = poff[l] + (size_t)lw[l] * lh[l];
    out->tile_off[l + 1] = out->tile_off[l] + (lw[l] / p->tile) * (lh[l] / p->tile);
  }
  uint8_t* pyr_ref = (uint8_t*)malloc(poff[L]);
  uint8_t* pyr_src = (uint8_t*)malloc(poff[L]);
  uint8_t* warped = (uint8_t*)malloc((size_t)w * h);
  uint32_t hist[256];
  uint8_t lut[256];
  lo_histogram(ref_y, w, h, w, hist);
  lo_equalize_lut(hist, lut);
  lo_apply_lut(ref_y, w, h, w, lut, pyr_ref);
  lo_histogram(src_y, w, h, w, hist);
  lo_equalize_lut(hist, lut);
  lo_apply_lut(src_y, w, h, w, lut, pyr_src);
  for (int l = 1; l < L; ++l) {
    lo_downsample(pyr_ref + poff[l - 1], lw[l - 1], lh[l - 1], pyr_ref + poff[l]);
    lo_downsample(pyr_src + poff[l - 1], lw[l - 1], lh[l - 1], pyr_src + poff[l]);
  }
  memcpy(out->yeq_ref, pyr_ref, (size_t)w * h);
  memcpy(out->yeq_src, pyr_src, (size_t)w * h);
  static const double I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  memcpy(out->H + 9 * L, H_init ? H_init : I3, 9 * sizeof(double));
  for (int l = L - 1; l >= 0; --l) {
    const int o = out->tile_off[l], nt = out->tile_off[l + 1] - o;
    const int R = l == 0 ? p->radius0 : p->radius_coarse;
    double Hp[9];
    lo_corners(pyr_ref + poff[l], lw[l], lh[l], p, out->corner_x + o, out->corner_y + o,
               out->flags + o);
    lo_pixel_homography(out->H + 9 * (l + 1), lw[l], lh[l], Hp);
    if (!literal) lo_warp_q8(pyr_src + poff[l], lw[l], lh[l], Hp, warped);
    uint8_t* has = (uint8_t*)malloc((size_t)nt + 1);
    uint8_t* valid = (uint8_t*)malloc((size_t)nt + 1);
    uint8_t* inM = (uint8_t*)calloc((size_t)nt + 1, 1);
    memcpy(has, out->flags + o, (size_t)nt);
    if (literal)
      lo_search_unwarped(pyr_ref + poff[l], pyr_src + poff[l], lw[l], lh[l], p, R, Hp,
                         out->corner_x + o, out->corner_y + o, has, out->dx + o, out->dy + o,
                         out->ssd + o, valid);
    else
      lo_search(pyr_ref + poff[l], warped, lw[l], lh[l], p, R, out->corner_x + o,
                out->corner_y + o, has, out->dx + o, out->dy + o, out->ssd + o, valid);
    int32_t bc = -1, bi = -1;
    out->n_valid[l] = lo_weed(nt, out->corner_x + o, out->corner_y + o, out->dx + o,
                              out->dy + o, valid, lw[l], lh[l], l, p, 0, p->weed_iters, inM,
                              &bc, &bi);
    uint8_t* sel = (uint8_t*)calloc((size_t)nt + 1, 1);
    if (bc > lo_weed_delta(out->n_valid[l], p))
      lo_hypothesis_inliers(nt, out->corner_x + o, out->corner_y + o, out->dx + o, out->dy + o,
                            valid, lw[l], lh[l], l, p, bi, sel);
    out->n_inliers[l] = (literal ? lo_fit_level_absolute : lo_fit_level)(
        nt, out->corner_x + o, out->corner_y + o, out->dx + o, out->dy + o, sel, lw[l], lh[l],
        out->H + 9 * (l + 1), out->H + 9 * l);
    out->best_iter[l] = bi;
    for (int t = 0; t < nt; ++t)
      out->flags[o + t] =
          (uint8_t)((has[t] ? 1 : 0) | (valid[t] ? 2 : 0) | (inM[t] ? 4 : 0) | (sel[t] ? 8 : 0));
    if (l == 0 && !literal) memcpy(out->warped0, warped, (size_t)w * h);
    free(sel);
    free(has);
    free(valid);
    free(inM);
  }
  /* level 0 flow and backward warp through H^1 */
  {
    const int nt = out->tile_off[1];
    uint8_t* inM = (uint8_t*)malloc((size_t)nt + 1);
    for (int t = 0; t < nt; ++t) inM[t] = (out->flags[t] & 4) != 0;
    lo_sparse_to_dense(nt, out->corner_x, out->corner_y, out->dx, out->dy, inM, pyr_ref, w, h,
                       p, out->flow_u, out->flow_v, out->ntilde);
    free(inM);
    /* the absolute flow of the paper-literal search is the whole mapping */
    static const double I3p[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double Hp1[9];
    if (literal) memcpy(Hp1, I3p, sizeof(Hp1));
    else lo_pixel_homography(out->H + 9, w, h, Hp1);
    lo_backward_warp(src_y, src_u, src_v, pyr_src, w, h, Hp1, out->flow_u, out->flow_v,
                     out->rgb, out->yeq_warped);
  }
  free(warped);
  free(pyr_src);
  free(pyr_ref);
  return 0;
}
