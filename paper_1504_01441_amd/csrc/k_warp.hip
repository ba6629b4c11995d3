// k_warp.hip -- backward warp of the source to the reference (paper Sec. 2.1:
// the goal is to warp the source to the reference; Sec. 2.4: the dense flow).
// The sample position m(x) = Hp1(x + F(x)) is computed in double precision (a
// 5 MP frame needs position errors well below 1e-4 px), the samples are FP32
// bilinear with clamp to edge. I420 chroma is upsampled by pixel repetition
// and converted with BT.601 full-range coefficients; outputs are planar FP32
// in [0, 1] plus the warped equalised luma (for the SSIM weight of Sec. 2.5).
#include "lnr_device.h"
#include "lnr_internal.h"

namespace lnr {
namespace {

__device__ inline float bil(float p00, float p10, float p01, float p11, float ax, float ay) {
  return (1.f - ay) * ((1.f - ax) * p00 + ax * p10) + ay * ((1.f - ax) * p01 + ax * p11);
}

__device__ inline void yuv_rgb(float Y, float U, float V, float& r, float& g, float& b) {
  const float up = U - 128.f, vp = V - 128.f;
  r = (Y + 1.402f * vp) / 255.f;
  g = (Y - 0.344136f * up - 0.714136f * vp) / 255.f;
  b = (Y + 1.772f * up) / 255.f;
}

__global__ __launch_bounds__(256) void k_bwarp(const uint8_t* __restrict__ y, int sy,
                                               const uint8_t* __restrict__ u, int su,
                                               const uint8_t* __restrict__ v, int sv, int cs,
                                               const uint8_t* __restrict__ yeq, int W, int H,
                                               const double* __restrict__ Hn,
                                               const float* __restrict__ flow,
                                               float* __restrict__ img, float* __restrict__ yw) {
  int bx, py;
  xcd_block(gridDim.x, gridDim.y, bx, py);  // neighbouring rows gather from shared source rows
  const int px = bx * blockDim.x + threadIdx.x;
  if (px >= W) return;
  double hp[9];  // formed per thread (uniform, no barrier)
  pixel_homography(Hn, W, H, hp);
  const size_t plane = (size_t)W * H, o = (size_t)py * W + px;
  const double X = (double)px + (double)flow[o];
  const double Y = (double)py + (double)flow[plane + o];
  const double den = (hp[6] * X + hp[7] * Y) + hp[8];
  double sx = ((hp[0] * X + hp[1] * Y) + hp[2]) / den;
  double sy2 = ((hp[3] * X + hp[4] * Y) + hp[5]) / den;
  if (!(sx >= -1.0)) sx = -1.0;
  if (sx > (double)W) sx = (double)W;
  if (!(sy2 >= -1.0)) sy2 = -1.0;
  if (sy2 > (double)H) sy2 = (double)H;
  const double fx0 = floor(sx), fy0 = floor(sy2);
  const float ax = (float)(sx - fx0), ay = (float)(sy2 - fy0);
  const int ix = (int)fx0, iy = (int)fy0;
  const int x0 = min(max(ix, 0), W - 1), x1 = min(max(ix + 1, 0), W - 1);
  const int y0 = min(max(iy, 0), H - 1), y1 = min(max(iy + 1, 0), H - 1);
  const float Yv = bil(y[(size_t)y0 * sy + x0], y[(size_t)y0 * sy + x1], y[(size_t)y1 * sy + x0],
                       y[(size_t)y1 * sy + x1], ax, ay);
  const size_t e00 = (size_t)y0 * W + x0, e10 = (size_t)y0 * W + x1;
  const size_t e01 = (size_t)y1 * W + x0, e11 = (size_t)y1 * W + x1;
  yw[o] = bil(yeq[e00], yeq[e10], yeq[e01], yeq[e11], ax, ay) / 255.f;
  if (!u) {
    img[o] = Yv / 255.f;
    return;
  }
  const size_t cx0 = (size_t)(x0 >> 1) * cs, cx1 = (size_t)(x1 >> 1) * cs;
  const size_t c00u = (size_t)(y0 >> 1) * su + cx0, c10u = (size_t)(y0 >> 1) * su + cx1;
  const size_t c01u = (size_t)(y1 >> 1) * su + cx0, c11u = (size_t)(y1 >> 1) * su + cx1;
  const size_t c00v = (size_t)(y0 >> 1) * sv + cx0, c10v = (size_t)(y0 >> 1) * sv + cx1;
  const size_t c01v = (size_t)(y1 >> 1) * sv + cx0, c11v = (size_t)(y1 >> 1) * sv + cx1;
  const float Uv = bil(u[c00u], u[c10u], u[c01u], u[c11u], ax, ay);
  const float Vv = bil(v[c00v], v[c10v], v[c01v], v[c11v], ax, ay);
  float r, g, b;
  yuv_rgb(Yv, Uv, Vv, r, g, b);
  img[o] = r;
  img[plane + o] = g;
  img[2 * plane + o] = b;
}

// Four consecutive pixels per thread: 32-bit luma loads and 128-bit stores
// where the row allows; with yin, the 8-bit plane yin is also mapped to
// [0, 1] into yout (the merge's equalised reference luma).
__global__ __launch_bounds__(256) void k_frame_rgb4(const uint8_t* __restrict__ y, int sy,
                                                    const uint8_t* __restrict__ u, int su,
                                                    const uint8_t* __restrict__ v, int sv, int cs,
                                                    int W,
                                                    int H, float* __restrict__ img,
                                                    const uint8_t* __restrict__ yin,
                                                    float* __restrict__ yout) {
  int bx, py;
  xcd_block(gridDim.x, gridDim.y, bx, py);
  const int px = 4 * (bx * blockDim.x + threadIdx.x);
  if (px >= W) return;
  const size_t plane = (size_t)W * H, o = (size_t)py * W + px;
  const uint8_t* yr = y + (size_t)py * sy + px;
  const bool full = px + 4 <= W;
  const bool vin = full && ((reinterpret_cast<uintptr_t>(yr) & 3u) == 0);
  const bool vout = full && ((reinterpret_cast<uintptr_t>(img + o) & 15u) == 0);
  float Yv[4], r[4], g[4], b[4];
  if (vin) {
    const uint32_t w4 = *reinterpret_cast<const uint32_t*>(yr);
#pragma unroll
    for (int k = 0; k < 4; ++k) Yv[k] = (float)((w4 >> (8 * k)) & 255u);
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) Yv[k] = px + k < W ? (float)yr[k] : 0.f;
  }
  if (u) {
    const uint8_t* ur = u + (size_t)(py >> 1) * su + (size_t)(px >> 1) * cs;
    const uint8_t* vr = v + (size_t)(py >> 1) * sv + (size_t)(px >> 1) * cs;
    const int nc = full ? 2 : (W - px + 1) / 2;  // chroma samples of these pixels
    float U[2] = {128.f, 128.f}, V[2] = {128.f, 128.f};
    for (int c = 0; c < nc; ++c) {
      U[c] = ur[c * cs];
      V[c] = vr[c * cs];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) yuv_rgb(Yv[k], U[k >> 1], V[k >> 1], r[k], g[k], b[k]);
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = Yv[k] / 255.f;
  }
  if (vout) {
    *reinterpret_cast<float4*>(img + o) = make_float4(r[0], r[1], r[2], r[3]);
    if (u) {
      *reinterpret_cast<float4*>(img + plane + o) = make_float4(g[0], g[1], g[2], g[3]);
      *reinterpret_cast<float4*>(img + 2 * plane + o) = make_float4(b[0], b[1], b[2], b[3]);
    }
  } else {
    for (int k = 0; k < 4 && px + k < W; ++k) {
      img[o + k] = r[k];
      if (u) {
        img[plane + o + k] = g[k];
        img[2 * plane + o + k] = b[k];
      }
    }
  }
  if (yin) {
    const uint8_t* q = yin + o;
    if (vout && ((reinterpret_cast<uintptr_t>(q) & 3u) == 0) &&
        ((reinterpret_cast<uintptr_t>(yout + o) & 15u) == 0)) {
      const uint32_t w4 = *reinterpret_cast<const uint32_t*>(q);
      *reinterpret_cast<float4*>(yout + o) =
          make_float4((float)(w4 & 255u) / 255.f, (float)((w4 >> 8) & 255u) / 255.f,
                      (float)((w4 >> 16) & 255u) / 255.f, (float)(w4 >> 24) / 255.f);
    } else {
      for (int k = 0; k < 4 && px + k < W; ++k) yout[o + k] = q[k] / 255.f;
    }
  }
}

}  // namespace

hipError_t launch_backward_warp(const uint8_t* y, int sy, const Chroma& c, const uint8_t* yeq,
                                int W, int H, const double* Hn, const float* flow, float* image,
                                float* yeq_w, hipStream_t st) {
  dim3 grid((W + 255) / 256, H);
  LNR_LAUNCH(k_bwarp, grid, dim3(256), 0, st, y, sy, c.u, c.su, c.v, c.sv, c.cs, yeq, W, H, Hn,
             flow, image, yeq_w);
  return hipGetLastError();
}

hipError_t launch_frame_rgb_unit(const uint8_t* y, int sy, const Chroma& c, int W, int H,
                                 float* image, const uint8_t* yin, float* yout, hipStream_t st) {
  dim3 grid((W + 1023) / 1024, H);
  LNR_LAUNCH(k_frame_rgb4, grid, dim3(256), 0, st, y, sy, c.u, c.su, c.v, c.sv, c.cs, W, H,
             image, yin, yout);
  return hipGetLastError();
}

}  // namespace lnr
