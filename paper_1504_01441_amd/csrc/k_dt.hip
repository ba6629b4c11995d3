// k_dt.hip -- sparse-to-dense flow (paper Sec. 2.4, Eq. 6-7): the sparse maps
// P_u, P_v (match displacement at each kept corner) and N (1 there) are
// cross-bilateral filtered with the domain transform's recursive filter
// (Gastal & Oliveira 2011), guided by the equalised reference; F = P~ / N~.
//
// Each recursive pass  J[x] = J[x] + c_x (J[x-1] - J[x])  is a chain of affine
// maps z -> c_x z + (1 - c_x) v_x, so it is split into segments whose composed
// maps are combined with a parallel scan, then re-run with the exact carry.
// The step coefficient c = a_i^(1 + sigma_s/sigma_r |dI|) depends only on the
// 8-bit guide difference, so each iteration uses a 256-entry table.
//
//  k_dt_h: one workgroup per row (the row's three maps and guide live in LDS;
//          256 segments, wave shuffles + LDS for the scan). The first pass
//          writes the sparse maps itself from the tile list (no zero-fill pass).
//  k_dt_v: one workgroup per 16-column strip over the full height: 64 row
//          segments x 16 columns, a 6-step scan over segments in LDS; the
//          anti-causal transfer is accumulated during the causal sweep, so a
//          vertical pass reads the maps three times (L2 / MALL resident) and
//          writes them twice. The last pass writes F (and N~) instead.
#include "lnr_internal.h"

namespace lnr {
namespace {

struct DtArgs {
  int iters;
  double sigma_s, ratio;  // ratio = sigma_s / sigma_r
};

// c_i[k] = a_i ^ (1 + ratio * k / 255),  a_i = exp(-sqrt(2) / sigma_i),
// sigma_i = sigma_s sqrt(3) 2^(n - i) / sqrt(4^n - 1)  (i = 1..n)
__global__ void k_dt_coef(DtArgs a, float* __restrict__ coef) {
  const int i = blockIdx.x + 1, k = threadIdx.x;
  const double sig = a.sigma_s * sqrt(3.0) * pow(2.0, (double)(a.iters - i)) /
                     sqrt(pow(4.0, (double)a.iters) - 1.0);
  const double ai = exp(-sqrt(2.0) / sig);
  coef[blockIdx.x * 256 + k] = (float)pow(ai, 1.0 + a.ratio * ((double)k / 255.0));
}

struct Aff {  // z -> A z + B (three channels share A)
  float A, B0, B1, B2;
};

// later o earlier
__device__ inline Aff compose(const Aff& later, const Aff& earlier) {
  Aff r;
  r.A = later.A * earlier.A;
  r.B0 = later.A * earlier.B0 + later.B0;
  r.B1 = later.A * earlier.B1 + later.B1;
  r.B2 = later.A * earlier.B2 + later.B2;
  return r;
}

__device__ inline Aff shfl_up_aff(const Aff& v, int off) {
  Aff r;
  r.A = __shfl_up(v.A, off);
  r.B0 = __shfl_up(v.B0, off);
  r.B1 = __shfl_up(v.B1, off);
  r.B2 = __shfl_up(v.B2, off);
  return r;
}

__device__ inline Aff shfl_down_aff(const Aff& v, int off) {
  Aff r;
  r.A = __shfl_down(v.A, off);
  r.B0 = __shfl_down(v.B0, off);
  r.B1 = __shfl_down(v.B1, off);
  r.B2 = __shfl_down(v.B2, off);
  return r;
}

// Carry into each thread of a 256-thread block: the composition of every
// earlier thread's map (forward: lower tid; backward: higher tid) applied to 0.
template <bool FWD>
__device__ void block_carry(Aff v, Aff* wtot, float& c0, float& c1, float& c2) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  Aff inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const Aff o = FWD ? shfl_up_aff(inc, off) : shfl_down_aff(inc, off);
    const bool ok = FWD ? lane >= off : lane + off < 64;
    if (ok) inc = compose(inc, o);
  }
  if (FWD ? lane == 63 : lane == 0) wtot[wave] = inc;
  __syncthreads();
  float z0 = 0.f, z1 = 0.f, z2 = 0.f;  // carry into this wave
  if (FWD) {
    for (int w = 0; w < wave; ++w) {
      const Aff t = wtot[w];
      z0 = t.A * z0 + t.B0; z1 = t.A * z1 + t.B1; z2 = t.A * z2 + t.B2;
    }
  } else {
    for (int w = 3; w > wave; --w) {
      const Aff t = wtot[w];
      z0 = t.A * z0 + t.B0; z1 = t.A * z1 + t.B1; z2 = t.A * z2 + t.B2;
    }
  }
  const Aff prev = FWD ? shfl_up_aff(inc, 1) : shfl_down_aff(inc, 1);
  const bool edge = FWD ? lane == 0 : lane == 63;
  if (edge) { c0 = z0; c1 = z1; c2 = z2; }
  else {
    c0 = prev.A * z0 + prev.B0;
    c1 = prev.A * z1 + prev.B1;
    c2 = prev.A * z2 + prev.B2;
  }
  __syncthreads();
}

template <bool FIRST>
__global__ __launch_bounds__(256) void k_dt_h(float* __restrict__ maps,
                                              const uint8_t* __restrict__ guide, int W, int H,
                                              const float* __restrict__ coef,
                                              const int32_t* __restrict__ cxy,
                                              const int32_t* __restrict__ disp,
                                              const uint8_t* __restrict__ flags, int ntx,
                                              int nty, int tile) {
  extern __shared__ float sm[];
  __shared__ float cf[256];
  __shared__ Aff wtot[4];
  float* v0 = sm;
  float* v1 = sm + W;
  float* v2 = sm + 2 * W;
  uint8_t* g = reinterpret_cast<uint8_t*>(sm + 3 * W);
  const int y = blockIdx.x, tid = threadIdx.x;
  const size_t plane = (size_t)W * H, ro = (size_t)y * W;
  cf[tid] = coef[tid];
  for (int x = tid; x < W; x += 256) {
    g[x] = guide[ro + x];
    if (FIRST) {
      v0[x] = 0.f; v1[x] = 0.f; v2[x] = 0.f;
    } else {
      v0[x] = maps[ro + x]; v1[x] = maps[plane + ro + x]; v2[x] = maps[2 * plane + ro + x];
    }
  }
  if (FIRST) {
    __syncthreads();
    const int ty = y / tile;
    if (ty < nty)
      for (int tx = tid; tx < ntx; tx += 256) {
        const int t = ty * ntx + tx;
        if ((flags[t] & 4) && cxy[2 * t + 1] == y) {
          const int x = cxy[2 * t];
          v0[x] = (float)disp[2 * t];
          v1[x] = (float)disp[2 * t + 1];
          v2[x] = 1.f;
        }
      }
  }
  __syncthreads();
  const int seg = (W + 255) / 256;
  const int xb = min(W, tid * seg), xe = min(W, xb + seg);
  // causal: J[x] = J[x] + c (J[x-1] - J[x]), c between x-1 and x (0 at x = 0)
  {
    Aff t{1.f, 0.f, 0.f, 0.f};
    for (int x = xb; x < xe; ++x) {
      const float c = x ? cf[abs((int)g[x] - (int)g[x - 1])] : 0.f;
      t.B0 = v0[x] + c * (t.B0 - v0[x]);
      t.B1 = v1[x] + c * (t.B1 - v1[x]);
      t.B2 = v2[x] + c * (t.B2 - v2[x]);
      t.A *= c;
    }
    float p0, p1, p2;
    block_carry<true>(t, wtot, p0, p1, p2);
    for (int x = xb; x < xe; ++x) {
      const float c = x ? cf[abs((int)g[x] - (int)g[x - 1])] : 0.f;
      p0 = v0[x] + c * (p0 - v0[x]); v0[x] = p0;
      p1 = v1[x] + c * (p1 - v1[x]); v1[x] = p1;
      p2 = v2[x] + c * (p2 - v2[x]); v2[x] = p2;
    }
  }
  __syncthreads();
  // anti-causal: J[x] = J[x] + c (J[x+1] - J[x]), c between x and x+1
  {
    Aff t{1.f, 0.f, 0.f, 0.f};
    for (int x = xe - 1; x >= xb; --x) {
      const float c = x + 1 < W ? cf[abs((int)g[x + 1] - (int)g[x])] : 0.f;
      t.B0 = v0[x] + c * (t.B0 - v0[x]);
      t.B1 = v1[x] + c * (t.B1 - v1[x]);
      t.B2 = v2[x] + c * (t.B2 - v2[x]);
      t.A *= c;
    }
    float p0, p1, p2;
    block_carry<false>(t, wtot, p0, p1, p2);
    for (int x = xe - 1; x >= xb; --x) {
      const float c = x + 1 < W ? cf[abs((int)g[x + 1] - (int)g[x])] : 0.f;
      p0 = v0[x] + c * (p0 - v0[x]); v0[x] = p0;
      p1 = v1[x] + c * (p1 - v1[x]); v1[x] = p1;
      p2 = v2[x] + c * (p2 - v2[x]); v2[x] = p2;
    }
  }
  __syncthreads();
  for (int x = tid; x < W; x += 256) {
    maps[ro + x] = v0[x]; maps[plane + ro + x] = v1[x]; maps[2 * plane + ro + x] = v2[x];
  }
}

constexpr int kStrip = 16, kSegs = 64;

template <bool LAST>
__global__ __launch_bounds__(1024) void k_dt_v(float* __restrict__ maps,
                                               const uint8_t* __restrict__ guide, int W, int H,
                                               const float* __restrict__ coef,
                                               float* __restrict__ flow,
                                               float* __restrict__ ntilde, float nmin) {
  __shared__ float cf[256];
  __shared__ Aff T[kSegs][kStrip];
  const int tid = threadIdx.x, cl = tid % kStrip, sg = tid / kStrip;
  const int col = blockIdx.x * kStrip + cl;
  const bool act = col < W;
  const int len = (H + kSegs - 1) / kSegs;
  const int r0 = min(H, sg * len), r1 = min(H, r0 + len);
  const size_t plane = (size_t)W * H;
  if (tid < 256) cf[tid] = coef[tid];
  __syncthreads();
  // phase 1: causal transfer of this segment
  Aff t{1.f, 0.f, 0.f, 0.f};
  if (act) {
    int gp = r0 > 0 ? guide[(size_t)(r0 - 1) * W + col] : 0;
    for (int y = r0; y < r1; ++y) {
      const size_t o = (size_t)y * W + col;
      const int gy = guide[o];
      const float c = y ? cf[abs(gy - gp)] : 0.f;
      const float a0 = maps[o], a1 = maps[plane + o], a2 = maps[2 * plane + o];
      t.B0 = a0 + c * (t.B0 - a0);
      t.B1 = a1 + c * (t.B1 - a1);
      t.B2 = a2 + c * (t.B2 - a2);
      t.A *= c;
      gp = gy;
    }
  }
  T[sg][cl] = t;
  __syncthreads();
  for (int off = 1; off < kSegs; off <<= 1) {  // inclusive scan over segments
    Aff o{1.f, 0.f, 0.f, 0.f};
    if (sg >= off) o = T[sg - off][cl];
    __syncthreads();
    if (sg >= off) t = compose(t, o);
    T[sg][cl] = t;
    __syncthreads();
  }
  float p0 = 0.f, p1 = 0.f, p2 = 0.f;
  if (sg > 0) {  // prefix applied to 0 (segment 0 starts with c = 0)
    const Aff pr = T[sg - 1][cl];
    p0 = pr.B0; p1 = pr.B1; p2 = pr.B2;
  }
  __syncthreads();
  // phase 3: causal sweep with the carry; accumulate the anti-causal transfer
  // K[top] = sum_n (prod_{m=top+1..n} c_m)(1 - c_{n+1}) J[n] + (prod c) e_in
  Aff u{1.f, 0.f, 0.f, 0.f};
  if (act) {
    int gp = r0 > 0 ? guide[(size_t)(r0 - 1) * W + col] : 0;
    for (int y = r0; y < r1; ++y) {
      const size_t o = (size_t)y * W + col;
      const int gy = guide[o];
      const float c = y ? cf[abs(gy - gp)] : 0.f;
      const float a0 = maps[o], a1 = maps[plane + o], a2 = maps[2 * plane + o];
      p0 = a0 + c * (p0 - a0);
      p1 = a1 + c * (p1 - a1);
      p2 = a2 + c * (p2 - a2);
      maps[o] = p0; maps[plane + o] = p1; maps[2 * plane + o] = p2;
      const float cn = y + 1 < H ? cf[abs((int)guide[o + W] - gy)] : 0.f;
      const float wgt = u.A * (1.f - cn);
      u.B0 += wgt * p0; u.B1 += wgt * p1; u.B2 += wgt * p2;
      u.A *= cn;
      gp = gy;
    }
  }
  T[sg][cl] = u;
  __syncthreads();
  for (int off = 1; off < kSegs; off <<= 1) {  // inclusive suffix scan
    Aff o{1.f, 0.f, 0.f, 0.f};
    if (sg + off < kSegs) o = T[sg + off][cl];
    __syncthreads();
    if (sg + off < kSegs) u = compose(u, o);
    T[sg][cl] = u;
    __syncthreads();
  }
  float e0 = 0.f, e1 = 0.f, e2 = 0.f;
  if (sg + 1 < kSegs) {
    const Aff nx = T[sg + 1][cl];
    e0 = nx.B0; e1 = nx.B1; e2 = nx.B2;
  }
  // phase 5: anti-causal sweep upwards
  if (act) {
    int gb = r1 < H ? guide[(size_t)r1 * W + col] : 0;
    for (int y = r1 - 1; y >= r0; --y) {
      const size_t o = (size_t)y * W + col;
      const int gy = guide[o];
      const float cn = y + 1 < H ? cf[abs(gb - gy)] : 0.f;
      const float a0 = maps[o], a1 = maps[plane + o], a2 = maps[2 * plane + o];
      e0 = a0 + cn * (e0 - a0);
      e1 = a1 + cn * (e1 - a1);
      e2 = a2 + cn * (e2 - a2);
      if (LAST) {
        const bool ok = e2 > nmin;
        flow[o] = ok ? e0 / e2 : 0.f;
        flow[plane + o] = ok ? e1 / e2 : 0.f;
        if (ntilde) ntilde[o] = e2;
      } else {
        maps[o] = e0; maps[plane + o] = e1; maps[2 * plane + o] = e2;
      }
      gb = gy;
    }
  }
}

}  // namespace

hipError_t launch_flow(const int32_t* corner_xy, const int32_t* disp, const uint8_t* flags,
                       int ntx, int nty, int tile, const uint8_t* guide, int W, int H,
                       const lnr_params& p, float* maps, float* coef, float* flow,
                       float* ntilde, hipStream_t st) {
  DtArgs a;
  a.iters = p.dt_iters;
  a.sigma_s = p.sigma_s;
  a.ratio = p.sigma_s / p.sigma_r;
  LNR_LAUNCH(k_dt_coef, dim3(a.iters), dim3(256), 0, st, a, coef);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)W * 3 * sizeof(float) + (size_t)W + 16;
  if (lds > 64 * 1024) {  // rows wider than ~5000 px need more than the default LDS
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dt_h<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dt_h<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const float nmin = (float)p.n_min;
  for (int i = 0; i < a.iters; ++i) {
    const float* cf = coef + 256 * i;
    if (i == 0)
      LNR_LAUNCH(k_dt_h<true>, dim3(H), dim3(256), lds, st, maps, guide, W, H, cf,
                         corner_xy, disp, flags, ntx, nty, tile);
    else
      LNR_LAUNCH(k_dt_h<false>, dim3(H), dim3(256), lds, st, maps, guide, W, H, cf,
                         corner_xy, disp, flags, ntx, nty, tile);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((W + kStrip - 1) / kStrip);
    if (i + 1 == a.iters)
      LNR_LAUNCH(k_dt_v<true>, grid, dim3(1024), 0, st, maps, guide, W, H, cf, flow,
                         ntilde, nmin);
    else
      LNR_LAUNCH(k_dt_v<false>, grid, dim3(1024), 0, st, maps, guide, W, H, cf, flow,
                         ntilde, nmin);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lnr
