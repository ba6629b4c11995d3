/*
 * proposal_oracle.c -- plain CPU oracle of the learned displacement proposal
 * (TEST INFRASTRUCTURE ONLY; nothing in the product library links it).
 *
 * The proposal is not part of the paper: it is a small convolutional network
 * that predicts each level-0 tile's displacement, so that the SSD search of
 * Sec. 2.2 only has to scan a small window around the prediction (with the
 * exhaustive search as fallback when the network is not confident). This file
 * defines, as plain loops in double precision, what the network computes, its
 * loss, the gradients of that loss and the AdamW update, plus the windowed
 * search. Rounding to bfloat16 (weights, activations and back-propagated
 * activation gradients) happens at the points listed in the design notes when
 * `rnd` is 1; with `rnd` 0 everything stays in double precision, which is the
 * form the finite-difference pins check.
 *
 * Network (one sample; tensors channel-major [c][y][x]):
 *   x  [4][16][16]  channels 0, 1: the 32 x 32 tile of the reference and of
 *                   the warped source, each value bf16((s - 510) / 512) of the
 *                   sum s of a 2x2 block; channels 2, 3: the 64 x 64 window
 *                   around the tile (16 px on every side, so that the whole
 *                   search range is in view) of the reference and of the
 *                   warped source, each value bf16((s - 2040) / 2048) of the
 *                   sum s of a 4x4 block, coordinates clamped to the image
 *   a1 = relu(conv3x3(x,  W1, b1, stride 1, pad 1))   [32][16][16]
 *   a2 = relu(conv3x3(a1, W2, b2, stride 2, pad 1))   [32][8][8]
 *   a3 = relu(conv3x3(a2, W3, b3, stride 1, pad 1))   [32][8][8]
 *   a4 = relu(conv3x3(a3, W4, b4, stride 2, pad 1))   [32][4][4]
 *   o[j] = bh[j] + sum_f Wh[j][f] a4[f],  f = (y * 4 + x) * 32 + c
 *   prediction dx = 8 o[0], dy = 8 o[1], confidence logit o[2]
 * Parameters, one flat vector: W1[32][4][3][3] b1[32] W2[32][32][3][3] b2[32]
 * W3 b3 W4 b4 Wh[3][512] bh[3] (30,467 values).
 *
 * Loss per sample with label (lx, ly), averaged over the batch:
 *   huber(dx - lx) + huber(dy - ly) + bce(o[2], q),
 *   huber(e) = e^2 / 2 for |e| <= 1, |e| - 1/2 otherwise,
 *   q = 1 / (1 + exp(-4 (2.5 - max(|dx - lx|, |dy - ly|))))  (a soft "the
 *   rounded prediction is within 2 px" target, held constant in the
 *   gradient),
 *   bce(z, q) = max(z, 0) - q z + log(1 + exp(-|z|)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "lnr_oracle.h"

enum { C1 = 4, CH = 32, NF = 512, NX = C1 * 256 };

/* bfloat16 round to nearest even, through float (as a float -> bf16 cast) */
double lo_bf16(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) { /* inf / nan unchanged */
    return (double)f;
  }
  u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double rd(double v, int rnd) { return rnd ? lo_bf16(v) : v; }

/* offsets of each tensor in the flat parameter vector */
typedef struct {
  int W[4], b[4], Wh, bh, total;
} layout;

static layout param_layout(void) {
  layout L;
  int o = 0;
  const int cin[4] = {C1, CH, CH, CH};
  for (int l = 0; l < 4; ++l) {
    L.W[l] = o;
    o += CH * cin[l] * 9;
    L.b[l] = o;
    o += CH;
  }
  L.Wh = o;
  o += 3 * NF;
  L.bh = o;
  o += 3;
  L.total = o;
  return L;
}

int lo_cnn_param_count(void) { return param_layout().total; }

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Network input of one level-0 tile (32 x 32 at origin (x0, y0)) of w x h
 * images: the tile pair at half resolution, then the 64 x 64 windows around
 * it at quarter resolution (pixels outside the image repeat the edge). */
void lo_cnn_tile_input(const uint8_t* ref, const uint8_t* warped, int w, int h, int x0, int y0,
                       double* x /* [4][16][16] */) {
  for (int c = 0; c < 4; ++c) {
    const uint8_t* img = (c & 1) == 0 ? ref : warped;
    const int k = c < 2 ? 2 : 4;           /* block side */
    const int ox = c < 2 ? x0 : x0 - 16, oy = c < 2 ? y0 : y0 - 16;
    for (int i = 0; i < 16; ++i)
      for (int j = 0; j < 16; ++j) {
        int s = 0;
        for (int u = 0; u < k; ++u)
          for (int v = 0; v < k; ++v) {
            const int yy = clampi(oy + k * i + u, 0, h - 1), xx = clampi(ox + k * j + v, 0, w - 1);
            s += img[(size_t)yy * w + xx];
          }
        const double mid = c < 2 ? 510.0 : 2040.0, scale = c < 2 ? 512.0 : 2048.0;
        x[(c * 16 + i) * 16 + j] = lo_bf16(((double)s - mid) / scale);
      }
  }
}

/* z[co][y][x] = b[co] + sum W[co][ci][ky][kx] in[ci][s y + ky - 1][s x + kx - 1] */
static void conv_fwd(const double* in, int cin, int hin, const double* W, const double* b,
                     int stride, int hout, double* z) {
  for (int co = 0; co < CH; ++co)
    for (int y = 0; y < hout; ++y)
      for (int x = 0; x < hout; ++x) {
        double s = b[co];
        for (int ci = 0; ci < cin; ++ci)
          for (int ky = 0; ky < 3; ++ky)
            for (int kx = 0; kx < 3; ++kx) {
              const int iy = stride * y + ky - 1, ix = stride * x + kx - 1;
              if (iy < 0 || iy >= hin || ix < 0 || ix >= hin) continue;
              s += W[((co * cin + ci) * 3 + ky) * 3 + kx] * in[(ci * hin + iy) * hin + ix];
            }
        z[(co * hout + y) * hout + x] = s;
      }
}

typedef struct {
  double a1[CH * 256], a2[CH * 64], a3[CH * 64], a4[CH * 16];
  double o[3];
} acts;

static void forward_one(const double* P, const layout* L, const double* Wr[4], const double* x,
                        int rnd, acts* A) {
  double* z = (double*)malloc(sizeof(double) * CH * 256);
  const double* in[4] = {x, A->a1, A->a2, A->a3};
  double* out[4] = {A->a1, A->a2, A->a3, A->a4};
  const int cin[4] = {C1, CH, CH, CH}, hin[4] = {16, 16, 8, 8}, st[4] = {1, 2, 1, 2},
            hout[4] = {16, 8, 8, 4};
  for (int l = 0; l < 4; ++l) {
    conv_fwd(in[l], cin[l], hin[l], Wr[l], P + L->b[l], st[l], hout[l], z);
    const int n = CH * hout[l] * hout[l];
    for (int i = 0; i < n; ++i) out[l][i] = rd(z[i] > 0.0 ? z[i] : 0.0, rnd);
  }
  free(z);
  for (int j = 0; j < 3; ++j) {
    double s = P[L->bh + j];
    for (int c = 0; c < CH; ++c)
      for (int yx = 0; yx < 16; ++yx)
        s += P[L->Wh + j * NF + yx * CH + c] * A->a4[c * 16 + yx];
    A->o[j] = s;
  }
}

static double* rounded_weights(const double* P, const layout* L, int rnd, const double* Wr[4]) {
  const int cin[4] = {C1, CH, CH, CH};
  int tot = 0;
  for (int l = 0; l < 4; ++l) tot += CH * cin[l] * 9;
  double* buf = (double*)malloc(sizeof(double) * (size_t)tot);
  int o = 0;
  for (int l = 0; l < 4; ++l) {
    const int n = CH * cin[l] * 9;
    for (int i = 0; i < n; ++i) buf[o + i] = rd(P[L->W[l] + i], rnd);
    Wr[l] = buf + o;
    o += n;
  }
  return buf;
}

void lo_cnn_forward(const double* params, const double* x, int n, int rnd, double* out) {
  const layout L = param_layout();
  const double* Wr[4];
  double* wb = rounded_weights(params, &L, rnd, Wr);
  acts* A = (acts*)malloc(sizeof(acts));
  for (int s = 0; s < n; ++s) {
    forward_one(params, &L, Wr, x + (size_t)s * NX, rnd, A);
    for (int j = 0; j < 3; ++j) out[(size_t)s * 3 + j] = A->o[j];
  }
  free(A);
  free(wb);
}

static double huber_grad(double e) { return e > 1.0 ? 1.0 : (e < -1.0 ? -1.0 : e); }
static double huber(double e) { return fabs(e) <= 1.0 ? 0.5 * e * e : fabs(e) - 0.5; }

/* Loss of a batch and its gradient with respect to every parameter
 * (grad has lo_cnn_param_count() entries). Returns the loss. */
double lo_cnn_loss_grad(const double* params, const double* x, const int32_t* label, int n,
                        int rnd, double* grad) {
  const layout L = param_layout();
  const double* Wr[4];
  double* wb = rounded_weights(params, &L, rnd, Wr);
  memset(grad, 0, sizeof(double) * (size_t)L.total);
  acts* A = (acts*)malloc(sizeof(acts));
  double* da = (double*)malloc(sizeof(double) * CH * 256);
  double* dz = (double*)malloc(sizeof(double) * CH * 256);
  double loss = 0.0;
  const int cin[4] = {C1, CH, CH, CH}, hin[4] = {16, 16, 8, 8}, st[4] = {1, 2, 1, 2},
            hout[4] = {16, 8, 8, 4};
  for (int s = 0; s < n; ++s) {
    const double* xs = x + (size_t)s * NX;
    forward_one(params, &L, Wr, xs, rnd, A);
    const double ex = 8.0 * A->o[0] - label[2 * s], ey = 8.0 * A->o[1] - label[2 * s + 1];
    const double em = fabs(ex) > fabs(ey) ? fabs(ex) : fabs(ey);
    const double q = 1.0 / (1.0 + exp(-4.0 * (2.5 - em))), z = A->o[2];
    loss += huber(ex) + huber(ey) + (z > 0 ? z : 0.0) - q * z + log(1.0 + exp(-fabs(z)));
    double dO[3];
    dO[0] = 8.0 * huber_grad(ex) / n;
    dO[1] = 8.0 * huber_grad(ey) / n;
    dO[2] = (1.0 / (1.0 + exp(-z)) - q) / n;
    /* head */
    for (int j = 0; j < 3; ++j) {
      grad[L.bh + j] += dO[j];
      for (int c = 0; c < CH; ++c)
        for (int yx = 0; yx < 16; ++yx)
          grad[L.Wh + j * NF + yx * CH + c] += dO[j] * A->a4[c * 16 + yx];
    }
    for (int c = 0; c < CH; ++c)
      for (int yx = 0; yx < 16; ++yx) {
        double g = 0.0;
        for (int j = 0; j < 3; ++j) g += params[L.Wh + j * NF + yx * CH + c] * dO[j];
        da[c * 16 + yx] = g;
      }
    const double* ain[4] = {xs, A->a1, A->a2, A->a3};
    const double* aout[4] = {A->a1, A->a2, A->a3, A->a4};
    for (int l = 3; l >= 0; --l) {
      const int no = CH * hout[l] * hout[l];
      /* through the ReLU (a > 0), rounded as the kernels consume it */
      for (int i = 0; i < no; ++i) dz[i] = rd(aout[l][i] > 0.0 ? da[i] : 0.0, rnd);
      const int ho = hout[l], hi = hin[l], ci_n = cin[l], S = st[l];
      for (int co = 0; co < CH; ++co)
        for (int y = 0; y < ho; ++y)
          for (int xx = 0; xx < ho; ++xx) {
            const double g = dz[(co * ho + y) * ho + xx];
            grad[L.b[l] + co] += g;
            for (int ci = 0; ci < ci_n; ++ci)
              for (int ky = 0; ky < 3; ++ky)
                for (int kx = 0; kx < 3; ++kx) {
                  const int iy = S * y + ky - 1, ix = S * xx + kx - 1;
                  if (iy < 0 || iy >= hi || ix < 0 || ix >= hi) continue;
                  grad[L.W[l] + ((co * ci_n + ci) * 3 + ky) * 3 + kx] +=
                      g * ain[l][(ci * hi + iy) * hi + ix];
                }
          }
      if (l == 0) break;
      /* gradient of the layer input: transposed convolution */
      for (int i = 0; i < ci_n * hi * hi; ++i) da[i] = 0.0;
      for (int co = 0; co < CH; ++co)
        for (int y = 0; y < ho; ++y)
          for (int xx = 0; xx < ho; ++xx) {
            const double g = dz[(co * ho + y) * ho + xx];
            for (int ci = 0; ci < ci_n; ++ci)
              for (int ky = 0; ky < 3; ++ky)
                for (int kx = 0; kx < 3; ++kx) {
                  const int iy = S * y + ky - 1, ix = S * xx + kx - 1;
                  if (iy < 0 || iy >= hi || ix < 0 || ix >= hi) continue;
                  da[(ci * hi + iy) * hi + ix] += Wr[l][((co * ci_n + ci) * 3 + ky) * 3 + kx] * g;
                }
          }
    }
  }
  free(dz);
  free(da);
  free(A);
  free(wb);
  return loss / n;
}

/* One AdamW step (Loshchilov & Hutter): m, v moments, step t >= 1,
 * decoupled weight decay. */
void lo_adamw(double* w, double* m, double* v, const double* g, int n, int t, double lr,
              double b1, double b2, double eps, double wd) {
  const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (int i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    const double mh = m[i] / c1, vh = v[i] / c2;
    w[i] = w[i] - lr * (mh / (sqrt(vh) + eps) + wd * w[i]);
  }
}

/* Sec. 2.2's search restricted to the window centre[t] + [-R, R]^2 of each
 * tile (same cost, same skipping of patches that leave the image, same tie
 * order on the absolute displacement). */
void lo_search_window(const uint8_t* ref, const uint8_t* wimg, int w, int h, const lo_params* p,
                      int R, const int32_t* ccx, const int32_t* ccy, const int32_t* cx,
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
    int found = 0, bl = 0, bdx = 0, bdy = 0;
    uint32_t bs = 0;
    for (int ddy = ccy[t] - R; ddy <= ccy[t] + R; ++ddy)
      for (int ddx = ccx[t] - R; ddx <= ccx[t] + R; ++ddx) {
        if (px + ddx - P < 0 || px + ddx + P > w - 1) continue;
        if (py + ddy - P < 0 || py + ddy + P > h - 1) continue;
        uint32_t s = 0;
        for (int j = -P; j <= P; ++j)
          for (int i = -P; i <= P; ++i) {
            const int a = ref[(size_t)(py + j) * w + (px + i)];
            const int b = wimg[(size_t)(py + ddy + j) * w + (px + ddx + i)];
            s += (uint32_t)((a - b) * (a - b));
          }
        const int l1 = abs(ddx) + abs(ddy);
        const int better = !found || s < bs ||
                           (s == bs && (l1 < bl || (l1 == bl && (ddy < bdy ||
                                                                 (ddy == bdy && ddx < bdx)))));
        if (better) { found = 1; bs = s; bl = l1; bdx = ddx; bdy = ddy; }
      }
    if (found) { valid[t] = 1; dx[t] = bdx; dy[t] = bdy; ssd[t] = bs; }
  }
}
