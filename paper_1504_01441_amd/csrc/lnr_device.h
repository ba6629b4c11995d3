// lnr_device.h -- double-precision helpers shared by the GPU kernels. Every
// operation is written in a fixed order (compiled without FMA contraction) so
// results whose rounding decides an integer are reproducible.
#pragma once
#include <hip/hip_runtime.h>

namespace lnr {

// out = a b for row-major 3x3 matrices; each entry sums left to right.
__device__ inline void mat3_mul(const double* a, const double* b, double* out) {
  double t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = a[3 * i + 0] * b[0 + j];
      s = s + a[3 * i + 1] * b[3 + j];
      s = s + a[3 * i + 2] * b[6 + j];
      t[3 * i + j] = s;
    }
  for (int i = 0; i < 9; ++i) out[i] = t[i];
}

// Normalised frame of paper Sec. 2.2 (origin at the image centre, x in [-1, 1],
// y in [-h/w, h/w]): xn ~ C x with C = [[2,0,-(w-1)],[0,2,-(h-1)],[0,0,w]] and
// x ~ B xn with B = [[w,0,w-1],[0,w,h-1],[0,0,2]] (B C = 2w I), so the level
// pixel homography is Hp = B (H C).
__device__ inline void pixel_homography(const double* H, int w, int h, double* Hp) {
  const double B[9] = {(double)w, 0, (double)(w - 1), 0, (double)w, (double)(h - 1), 0, 0, 2};
  const double C[9] = {2, 0, (double)(-(w - 1)), 0, 2, (double)(-(h - 1)), 0, 0, (double)w};
  double T[9];
  mat3_mul(H, C, T);
  mat3_mul(B, T, Hp);
}

}  // namespace lnr
