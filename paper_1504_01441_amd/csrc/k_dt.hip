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
// The recursions run in double precision (the maps are stored as float between
// passes): with c close to 1 (sigma_s = 400) a float recursion amplifies
// rounding by ~1/(1 - c), which would move the flow by ~1e-4 px.
//
// Between passes a pixel is one 12-byte record of the three maps, so that a
// column pass reads whole 24-96 byte runs of neighbouring columns rather than
// 8-32 byte pieces of three planes; the column pass takes the guide from a
// column-major copy (a segment's rows are one aligned load).
//
//  k_dt_row: one workgroup per row; the row is staged in LDS with coalesced
//          loads, each of the 256 or 512 threads keeps a segment in registers, and
//          wave shuffles + LDS combine the segment maps. The first pass writes
//          the sparse maps itself from the tile list (no zero-fill pass); a
//          row that holds no sample stays exactly zero through it, so that
//          pass writes only a row flag for it, and the first column pass
//          reads the records of flagged rows only (the rest are zeros).
//  k_dt_col: one workgroup per strip of 2-8 columns over the full height, as
//          128 or 256 segments per column held in registers; the records are read
//          and written once per pass. The last pass writes F (and N~) instead.
#include "lnr_internal.h"

namespace lnr {
namespace {

struct DtArgs {
  int iters;
  double sigma_s, ratio;  // ratio = sigma_s / sigma_r
};

// c_i[k] = a_i ^ (1 + ratio * k / 255),  a_i = exp(-sqrt(2) / sigma_i),
// sigma_i = sigma_s sqrt(3) 2^(n - i) / sqrt(4^n - 1)  (i = 1..n)
// Block 0 also clears zero[0, nzero), zero64[0, nzero64) and sums[0, 24) and
// sets ident to the identity (the registration's first launch does this
// set-up with the tables: histograms, the top level's weeding bits and sums).
__global__ void k_dt_coef(DtArgs a, double* __restrict__ coef, uint32_t* __restrict__ zero,
                          int nzero, double* __restrict__ ident,
                          unsigned long long* __restrict__ zero64, int nzero64,
                          long long* __restrict__ sums) {
  const int i = blockIdx.x + 1, k = threadIdx.x;
  if (blockIdx.x == 0) {
    for (int j = k; j < nzero; j += 256) zero[j] = 0u;
    for (int j = k; j < nzero64; j += 256) zero64[j] = 0ull;
    if (sums && k < 24) sums[k] = 0;
    if (ident && k < 9) ident[k] = (k % 4 == 0) ? 1.0 : 0.0;
  }
  const double sig = a.sigma_s * sqrt(3.0) * pow(2.0, (double)(a.iters - i)) /
                     sqrt(pow(4.0, (double)a.iters) - 1.0);
  const double ai = exp(-sqrt(2.0) / sig);
  coef[blockIdx.x * 256 + k] = pow(ai, 1.0 + a.ratio * ((double)k / 255.0));
}

struct Rec {  // one pixel of the three maps between passes
  float m0, m1, m2;
};

struct Aff {  // z -> A z + B (three channels share A)
  double A, B0, B1, B2;
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

// Carry into each thread of an NT-thread block: the composition of every
// earlier thread's map (forward: lower tid; backward: higher tid) applied to 0.
template <int NT, bool FWD>
__device__ void block_carry(Aff v, Aff* wtot, double& c0, double& c1, double& c2) {
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
  double z0 = 0.0, z1 = 0.0, z2 = 0.0;  // carry into this wave
  if (FWD) {
    for (int w = 0; w < wave; ++w) {
      const Aff t = wtot[w];
      z0 = t.A * z0 + t.B0; z1 = t.A * z1 + t.B1; z2 = t.A * z2 + t.B2;
    }
  } else {
    for (int w = NT / 64 - 1; w > wave; --w) {
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

// Coefficient between positions i-1 and i of a line: 0 where i - 1 or i is
// outside [0, n) (the recursion starts fresh at both ends).
__device__ inline double coef_at(const double* cf, int gprev, int gcur) {
  return cf[abs(gcur - gprev)];
}

// ---------------------------------------------------------------------------
// Horizontal pass: one block per row; the row is staged in LDS (coalesced),
// each thread keeps a segment of SEG consecutive pixels in registers.
template <int SEG, int NT, bool FIRST>
__global__ __launch_bounds__(NT) void k_dt_row(Rec* __restrict__ maps,
                                                const uint8_t* __restrict__ guide, int W, int H,
                                                const double* __restrict__ coef,
                                                const int32_t* __restrict__ cxy,
                                                const int32_t* __restrict__ disp,
                                                const uint8_t* __restrict__ flags, int ntx,
                                                int nty, int tile,
                                                uint8_t* __restrict__ rowflag) {
  extern __shared__ __align__(16) float sm[];
  __shared__ double cf[256];
  __shared__ Aff wtot[NT / 64];
  float* v0 = sm;
  float* v1 = sm + W;
  float* v2 = sm + 2 * W;
  uint8_t* g = reinterpret_cast<uint8_t*>(sm + 3 * W);
  const int y = blockIdx.x, tid = threadIdx.x;
  const size_t ro = (size_t)y * W;
  if (FIRST) {
    // the row's samples (kept level-0 matches whose corner lies on it)
    int has = 0;
    const int ty = y / tile;
    if (ty < nty)
      for (int tx = tid; tx < ntx; tx += NT) {
        const int t = ty * ntx + tx;
        has |= (flags[t] & 4) && cxy[2 * t + 1] == y;
      }
    has = __syncthreads_or(has);
    if (tid == 0) rowflag[y] = (uint8_t)(has != 0);
    if (!has) return;  // all zeros: the column pass does not read this row
  }
  if (tid < 256) cf[tid] = coef[tid];
  // staging: the whole row's loads in flight at once (NT * SEG covers the
  // row, so SEG per thread), then the stores to workgroup memory
  {
    uint8_t tg[SEG];
    Rec t[SEG];
#pragma unroll
    for (int u = 0; u < SEG; ++u) {
      const int xc = min(u * NT + tid, W - 1);  // in bounds; stored only if x < W
      tg[u] = guide[ro + xc];
      if (FIRST) t[u] = Rec{0.f, 0.f, 0.f};
      else t[u] = maps[ro + xc];
    }
#pragma unroll
    for (int u = 0; u < SEG; ++u) {
      const int x = u * NT + tid;
      if (x >= W) break;
      g[x] = tg[u];
      v0[x] = t[u].m0;
      v1[x] = t[u].m1;
      v2[x] = t[u].m2;
    }
  }
  if (FIRST) {
    __syncthreads();
    const int ty = y / tile;
    if (ty < nty)
      for (int tx = tid; tx < ntx; tx += NT) {
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
  const int xb = tid * SEG;
  // the segment is held as float (as stored between passes); every recursion
  // step and carry is computed in double precision. A whole segment is read
  // with 16-byte accesses where the planes allow (W a multiple of 4): a
  // thread's elements lie SEG apart from its neighbours', which scalar reads
  // would serve four to a bank.
  float a0[SEG], a1[SEG], a2[SEG];
  int gs[SEG + 2];  // guide bytes of pixels xb - 1 .. xb + SEG, 0 outside the row
  const bool vec = SEG % 4 == 0 && (W & 3) == 0 && xb + SEG <= W;
  if (vec) {
#pragma unroll
    for (int q = 0; q < SEG / 4; ++q) {
      const float4 f0 = reinterpret_cast<const float4*>(v0 + xb)[q];
      const float4 f1 = reinterpret_cast<const float4*>(v1 + xb)[q];
      const float4 f2 = reinterpret_cast<const float4*>(v2 + xb)[q];
      a0[4 * q] = f0.x; a0[4 * q + 1] = f0.y; a0[4 * q + 2] = f0.z; a0[4 * q + 3] = f0.w;
      a1[4 * q] = f1.x; a1[4 * q + 1] = f1.y; a1[4 * q + 2] = f1.z; a1[4 * q + 3] = f1.w;
      a2[4 * q] = f2.x; a2[4 * q + 1] = f2.y; a2[4 * q + 2] = f2.z; a2[4 * q + 3] = f2.w;
      const uint32_t w4 = reinterpret_cast<const uint32_t*>(g + xb)[q];
#pragma unroll
      for (int k = 0; k < 4; ++k) gs[1 + 4 * q + k] = (int)((w4 >> (8 * k)) & 255u);
    }
  } else {
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const int x = xb + j;
      a0[j] = x < W ? v0[x] : 0.f;
      a1[j] = x < W ? v1[x] : 0.f;
      a2[j] = x < W ? v2[x] : 0.f;
      gs[1 + j] = x < W ? g[x] : 0;
    }
  }
  gs[0] = xb > 0 && xb - 1 < W ? g[xb - 1] : 0;
  gs[SEG + 1] = xb + SEG < W ? g[xb + SEG] : 0;
  double cc[SEG + 1];  // cc[j]: between xb+j-1 and xb+j
#pragma unroll
  for (int j = 0; j <= SEG; ++j) {
    const int x = xb + j;
    cc[j] = (x > 0 && x < W) ? coef_at(cf, gs[j], gs[j + 1]) : 0.0;
  }
  // causal: J[x] = J[x] + c (J[x-1] - J[x])
  {
    Aff t{1.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      if (xb + j >= W) continue;
      const double c = cc[j];
      const double u0 = a0[j], u1 = a1[j], u2 = a2[j];
      t.B0 = u0 + c * (t.B0 - u0);
      t.B1 = u1 + c * (t.B1 - u1);
      t.B2 = u2 + c * (t.B2 - u2);
      t.A *= c;
    }
    double p0, p1, p2;
    block_carry<NT, true>(t, wtot, p0, p1, p2);
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      if (xb + j >= W) continue;
      const double c = cc[j];
      const double u0 = a0[j], u1 = a1[j], u2 = a2[j];
      p0 = u0 + c * (p0 - u0); a0[j] = (float)p0;
      p1 = u1 + c * (p1 - u1); a1[j] = (float)p1;
      p2 = u2 + c * (p2 - u2); a2[j] = (float)p2;
    }
  }
  // anti-causal: J[x] = J[x] + c (J[x+1] - J[x]), c between x and x+1
  {
    Aff t{1.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = SEG - 1; j >= 0; --j) {
      if (xb + j >= W) continue;
      const double c = cc[j + 1];
      const double u0 = a0[j], u1 = a1[j], u2 = a2[j];
      t.B0 = u0 + c * (t.B0 - u0);
      t.B1 = u1 + c * (t.B1 - u1);
      t.B2 = u2 + c * (t.B2 - u2);
      t.A *= c;
    }
    double p0, p1, p2;
    block_carry<NT, false>(t, wtot, p0, p1, p2);
#pragma unroll
    for (int j = SEG - 1; j >= 0; --j) {
      if (xb + j >= W) continue;
      const double c = cc[j + 1];
      const double u0 = a0[j], u1 = a1[j], u2 = a2[j];
      p0 = u0 + c * (p0 - u0); a0[j] = (float)p0;
      p1 = u1 + c * (p1 - u1); a1[j] = (float)p1;
      p2 = u2 + c * (p2 - u2); a2[j] = (float)p2;
    }
  }
  if (vec) {
#pragma unroll
    for (int q = 0; q < SEG / 4; ++q) {
      reinterpret_cast<float4*>(v0 + xb)[q] =
          make_float4(a0[4 * q], a0[4 * q + 1], a0[4 * q + 2], a0[4 * q + 3]);
      reinterpret_cast<float4*>(v1 + xb)[q] =
          make_float4(a1[4 * q], a1[4 * q + 1], a1[4 * q + 2], a1[4 * q + 3]);
      reinterpret_cast<float4*>(v2 + xb)[q] =
          make_float4(a2[4 * q], a2[4 * q + 1], a2[4 * q + 2], a2[4 * q + 3]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const int x = xb + j;
      if (x < W) { v0[x] = a0[j]; v1[x] = a1[j]; v2[x] = a2[j]; }
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int x = tid; x < W; x += NT) maps[ro + x] = Rec{v0[x], v1[x], v2[x]};
}

// ---------------------------------------------------------------------------
// Vertical pass: a block covers NCOL adjacent columns over the full height as
// NSEG segments of L rows (NCOL * NSEG = 512 threads); each thread keeps its
// segment of one column in registers, so the maps are read and written once.
// Segment carries are combined with wave shuffles (segments of a column sit
// NCOL lanes apart) and per-wave totals in LDS.
template <int NCOL, int NSEG>
__device__ void seg_carry(Aff v, bool fwd, Aff* wt /*[NSEG*NCOL/64][NCOL]*/, double& c0,
                          double& c1, double& c2) {
  constexpr int PER = 64 / NCOL;  // segments of one column per wave
  constexpr int NW = NSEG / PER;  // waves
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, cl = tid % NCOL;
  const int sl = lane / NCOL;  // segment index within the wave
  Aff inc = v;
#pragma unroll
  for (int off = 1; off < PER; off <<= 1) {
    const Aff o = fwd ? shfl_up_aff(inc, off * NCOL) : shfl_down_aff(inc, off * NCOL);
    const bool ok = fwd ? sl >= off : sl + off < PER;
    if (ok) inc = compose(inc, o);
  }
  if (fwd ? sl == PER - 1 : sl == 0) wt[wave * NCOL + cl] = inc;
  __syncthreads();
  double z0 = 0.0, z1 = 0.0, z2 = 0.0;
  if (fwd) {
    for (int w = 0; w < wave; ++w) {
      const Aff t = wt[w * NCOL + cl];
      z0 = t.A * z0 + t.B0; z1 = t.A * z1 + t.B1; z2 = t.A * z2 + t.B2;
    }
  } else {
    for (int w = NW - 1; w > wave; --w) {
      const Aff t = wt[w * NCOL + cl];
      z0 = t.A * z0 + t.B0; z1 = t.A * z1 + t.B1; z2 = t.A * z2 + t.B2;
    }
  }
  const Aff prev = fwd ? shfl_up_aff(inc, NCOL) : shfl_down_aff(inc, NCOL);
  const bool edge = fwd ? sl == 0 : sl == PER - 1;
  if (edge) { c0 = z0; c1 = z1; c2 = z2; }
  else {
    c0 = prev.A * z0 + prev.B0;
    c1 = prev.A * z1 + prev.B1;
    c2 = prev.A * z2 + prev.B2;
  }
  __syncthreads();
}

template <int L, int NCOL, int NSEG, bool LAST>
__global__ __launch_bounds__(NCOL * NSEG) void k_dt_col(Rec* __restrict__ maps,
                                                        const uint8_t* __restrict__ gt, int hp,
                                                        int W, int H,
                                                        const double* __restrict__ coef,
                                                        float* __restrict__ flow,
                                                        float* __restrict__ ntilde, double nmin,
                                                        const uint8_t* __restrict__ rowflag) {
  __shared__ double cf[256];
  __shared__ Aff wt[NSEG * NCOL / 64 * NCOL];
  const int tid = threadIdx.x, cl = tid % NCOL, sg = tid / NCOL;
  // XCD-aware strip order: consecutive blocks run on different XCDs, so
  // neighbouring strips (which share cache lines) are given to one XCD
  const int nb = gridDim.x, b = blockIdx.x, full = nb / 8 * 8;
  const int strip = b < full ? (b % 8) * (nb / 8) + b / 8 : b;
  const int col = strip * NCOL + cl;
  const bool act = col < W;
  const int r0 = sg * L;
  const size_t plane = (size_t)W * H;
  for (int i = tid; i < 256; i += NCOL * NSEG) cf[i] = coef[i];
  __syncthreads();
  // guide bytes of rows r0 .. r0+L-1, four per register, as one aligned load
  // from the column-major copy (r0 is a multiple of L, a multiple of 8, and
  // the copy's rows run past r0 + L), plus the rows r0-1 and r0+L; the
  // coefficient between rows r0+j-1 and r0+j is looked up when needed (0 at
  // the ends)
  static_assert(L % 8 == 0, "segments are whole 8-byte guide words");
  constexpr int NG = L / 4;
  uint32_t gpk[NG];
  uint32_t gup = 0u, gdn = 0u;
  const bool seg_in = act && r0 < H;
  const uint8_t* gcol = gt + (size_t)col * hp;
  if (seg_in) {
    const uint2* gw = reinterpret_cast<const uint2*>(gcol + r0);
#pragma unroll
    for (int q = 0; q < NG / 2; ++q) {
      const uint2 v = gw[q];
      gpk[2 * q] = v.x;
      gpk[2 * q + 1] = v.y;
    }
    if (r0 > 0) gup = gcol[r0 - 1];
    if (r0 + L < H) gdn = gcol[r0 + L];
  } else {
#pragma unroll
    for (int q = 0; q < NG; ++q) gpk[q] = 0u;
  }
  // first pass: the rows the row pass left at zero are not read (their
  // flags, as for the guide, one aligned load per 8 rows; the flag buffer
  // runs past the last row)
  uint32_t rf[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) rf[q] = 0x01010101u;
  if (rowflag) {
    const uint2* rw = reinterpret_cast<const uint2*>(rowflag + r0);
#pragma unroll
    for (int q = 0; q < NG / 2; ++q) {
      const uint2 v = seg_in ? rw[q] : uint2{0u, 0u};
      rf[2 * q] = v.x;
      rf[2 * q + 1] = v.y;
    }
  }
  // the segment is held as float (as stored between passes); every recursion
  // step and carry is computed in double precision
  float a0[L], a1[L], a2[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const int y = r0 + j;
    const bool in = act && y < H && ((rf[j >> 2] >> (8 * (j & 3))) & 255u);
    const Rec r = in ? maps[(size_t)y * W + col] : Rec{0.f, 0.f, 0.f};
    a0[j] = r.m0;
    a1[j] = r.m1;
    a2[j] = r.m2;
  }
#define GB(j)                                                              \
  ((j) < 0 ? (int)gup                                                      \
   : (j) >= L ? (int)gdn                                                   \
              : (int)((gpk[((j) >= 0 && (j) < L ? (j) : 0) >> 2] >> (8 * ((j) & 3))) & 255u))
#define CC(j) ((r0 + (j) > 0 && r0 + (j) < H) ? cf[abs(GB(j) - GB((j) - 1))] : 0.0)
  {
    Aff t{1.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < L; ++j) {
      if (r0 + j >= H) break;
      const double c = CC(j);
      const double v0 = a0[j], v1 = a1[j], v2 = a2[j];
      t.B0 = v0 + c * (t.B0 - v0);
      t.B1 = v1 + c * (t.B1 - v1);
      t.B2 = v2 + c * (t.B2 - v2);
      t.A *= c;
    }
    double p0, p1, p2;
    seg_carry<NCOL, NSEG>(t, true, wt, p0, p1, p2);
#pragma unroll
    for (int j = 0; j < L; ++j) {
      if (r0 + j >= H) break;
      const double c = CC(j);
      const double v0 = a0[j], v1 = a1[j], v2 = a2[j];
      p0 = v0 + c * (p0 - v0); a0[j] = (float)p0;
      p1 = v1 + c * (p1 - v1); a1[j] = (float)p1;
      p2 = v2 + c * (p2 - v2); a2[j] = (float)p2;
    }
  }
  {
    Aff t{1.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = L - 1; j >= 0; --j) {
      if (r0 + j >= H) continue;
      const double c = CC(j + 1);
      const double v0 = a0[j], v1 = a1[j], v2 = a2[j];
      t.B0 = v0 + c * (t.B0 - v0);
      t.B1 = v1 + c * (t.B1 - v1);
      t.B2 = v2 + c * (t.B2 - v2);
      t.A *= c;
    }
    double p0, p1, p2;
    seg_carry<NCOL, NSEG>(t, false, wt, p0, p1, p2);
#pragma unroll
    for (int j = L - 1; j >= 0; --j) {
      if (r0 + j >= H) continue;
      const double c = CC(j + 1);
      const double v0 = a0[j], v1 = a1[j], v2 = a2[j];
      p0 = v0 + c * (p0 - v0); a0[j] = (float)p0;
      p1 = v1 + c * (p1 - v1); a1[j] = (float)p1;
      p2 = v2 + c * (p2 - v2); a2[j] = (float)p2;
    }
  }
#undef CC
#undef GB
  if (!act) return;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const int y = r0 + j;
    if (y >= H) break;
    const size_t o = (size_t)y * W + col;
    if (LAST) {
      const bool ok = (double)a2[j] > nmin;
      flow[o] = ok ? (float)((double)a0[j] / (double)a2[j]) : 0.f;
      flow[plane + o] = ok ? (float)((double)a1[j] / (double)a2[j]) : 0.f;
      if (ntilde) ntilde[o] = a2[j];
    } else {
      maps[o] = Rec{a0[j], a1[j], a2[j]};
    }
  }
}

// The guide's column-major copy for the column pass, one 64 x 64 tile per
// block (used when the equalisation did not write it).
__global__ __launch_bounds__(256) void k_guide_columns(const uint8_t* __restrict__ guide, int W,
                                                       int H, int hp, uint8_t* __restrict__ gt) {
  __shared__ uint8_t tile[64 * 64];
  const int bx = blockIdx.x * 64, by = blockIdx.y * 64;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int i = threadIdx.x + 256 * u, r = i >> 6, c = i & 63;
    tile[i] = (by + r < H && bx + c < W) ? guide[(size_t)(by + r) * W + bx + c] : 0;
  }
  __syncthreads();
  store_tile_columns(tile, bx, by, W, hp, gt);
}

template <int SEG, int NT>
hipError_t launch_row(bool first, Rec* maps, const uint8_t* guide, int W, int H,
                      const double* cf, const int32_t* cxy, const int32_t* disp,
                      const uint8_t* flags, int ntx, int nty, int tile, uint8_t* rowflag,
                      hipStream_t st) {
  const size_t lds = (size_t)W * 3 * sizeof(float) + (size_t)W + 16;
  if (lds > 64 * 1024) {  // rows wider than ~5000 px need more than the default LDS
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(first ? &k_dt_row<SEG, NT, true> : &k_dt_row<SEG, NT, false>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (first)
    LNR_LAUNCH((k_dt_row<SEG, NT, true>), dim3(H), dim3(NT), lds, st, maps, guide, W, H, cf, cxy,
               disp, flags, ntx, nty, tile, rowflag);
  else
    LNR_LAUNCH((k_dt_row<SEG, NT, false>), dim3(H), dim3(NT), lds, st, maps, guide, W, H, cf, cxy,
               disp, flags, ntx, nty, tile, nullptr);
  return hipGetLastError();
}

template <int L, int NCOL, int NSEG>
hipError_t launch_col(bool last, Rec* maps, const uint8_t* gt, int W, int H,
                      const double* cf, float* flow, float* ntilde, double nmin,
                      const uint8_t* rowflag, hipStream_t st) {
  const dim3 grid((W + NCOL - 1) / NCOL);
  const int hp = dt_guide_stride(H);
  if (last)
    LNR_LAUNCH((k_dt_col<L, NCOL, NSEG, true>), grid, dim3(NCOL * NSEG), 0, st, maps, gt, hp, W,
               H, cf, flow, ntilde, nmin, rowflag);
  else
    LNR_LAUNCH((k_dt_col<L, NCOL, NSEG, false>), grid, dim3(NCOL * NSEG), 0, st, maps, gt, hp, W,
               H, cf, flow, ntilde, nmin, rowflag);
  return hipGetLastError();
}

}  // namespace

namespace {
const DtShape kRowShapes[] = {{4, 256, 0, 0, 0}, {8, 256, 0, 0, 0}, {12, 256, 0, 0, 0},
                              {4, 512, 0, 0, 0}, {6, 512, 0, 0, 0}, {8, 512, 0, 0, 0},
                              {12, 512, 0, 0, 0}};
const DtShape kColShapes[] = {{0, 0, 8, 8, 128},  {0, 0, 8, 4, 128},  {0, 0, 16, 4, 128},
                              {0, 0, 8, 2, 256},  {0, 0, 24, 4, 128}, {0, 0, 16, 2, 256},
                              {0, 0, 24, 2, 256}};

hipError_t row_pass(const DtShape& s, bool first, Rec* maps, const uint8_t* guide, int W, int H,
                    const double* cf, const int32_t* cxy, const int32_t* disp,
                    const uint8_t* flags, int ntx, int nty, int tile, uint8_t* rowflag,
                    hipStream_t st) {
#define ROW(SEG, NT)                                                                           \
  if (s.seg == SEG && s.nt == NT)                                                              \
    return launch_row<SEG, NT>(first, maps, guide, W, H, cf, cxy, disp, flags, ntx, nty, tile, \
                               rowflag, st);
  ROW(4, 256) ROW(8, 256) ROW(12, 256) ROW(4, 512) ROW(6, 512) ROW(8, 512) ROW(12, 512)
#undef ROW
  return hipErrorInvalidValue;
}

hipError_t col_pass(const DtShape& s, bool last, Rec* maps, const uint8_t* gt, int W, int H,
                    const double* cf, float* flow, float* ntilde, double nmin,
                    const uint8_t* rowflag, hipStream_t st) {
#define COL(L, NC, NS)                                                                       \
  if (s.l == L && s.ncol == NC && s.nseg == NS)                                               \
    return launch_col<L, NC, NS>(last, maps, gt, W, H, cf, flow, ntilde, nmin, rowflag, st);
  COL(8, 8, 128) COL(8, 4, 128) COL(16, 4, 128) COL(8, 2, 256) COL(24, 4, 128)
  COL(16, 2, 256) COL(24, 2, 256)
#undef COL
  return hipErrorInvalidValue;
}
}  // namespace

bool dt_shape_valid(const DtShape& s, int W, int H) {
  bool row = false, col = false;
  for (const DtShape& r : kRowShapes) row |= r.seg == s.seg && r.nt == s.nt;
  for (const DtShape& c : kColShapes) col |= c.l == s.l && c.ncol == s.ncol && c.nseg == s.nseg;
  return row && col && W <= s.seg * s.nt && H <= s.l * s.nseg;
}

// Every instantiated (row, column) pair that covers W x H.
int dt_shape_candidates(int W, int H, DtShape* out, int max) {
  int n = 0;
  for (const DtShape& r : kRowShapes)
    for (const DtShape& c : kColShapes) {
      const DtShape s{r.seg, r.nt, c.l, c.ncol, c.nseg};
      if (dt_shape_valid(s, W, H) && n < max) out[n++] = s;
    }
  return n;
}

// The default table: the fewest rows / segments per thread that cover the
// image (double-precision segments stay within 256 VGPRs).
DtShape dt_default_shape(int W, int H) {
  DtShape s;
  if (W <= 1024) { s.seg = 4; s.nt = 256; }
  else if (W <= 2048) { s.seg = 8; s.nt = 256; }
  else if (W <= 3072) { s.seg = 12; s.nt = 256; }
  else if (W <= 4096) { s.seg = 8; s.nt = 512; }
  else { s.seg = 12; s.nt = 512; }
  if (H <= 1024) { s.l = 8; s.ncol = 8; s.nseg = 128; }
  else if (H <= 2048) { s.l = 16; s.ncol = 4; s.nseg = 128; }
  else if (H <= 3072) { s.l = 24; s.ncol = 4; s.nseg = 128; }
  else if (H <= 4096) { s.l = 16; s.ncol = 2; s.nseg = 256; }
  else { s.l = 24; s.ncol = 2; s.nseg = 256; }
  return s;
}

hipError_t launch_dt_coef(const lnr_params& p, double* coef, uint32_t* zero, int nzero,
                          double* ident, hipStream_t st, unsigned long long* zero64,
                          int nzero64, long long* sums) {
  DtArgs a;
  a.iters = p.dt_iters;
  a.sigma_s = p.sigma_s;
  a.ratio = p.sigma_s / p.sigma_r;
  LNR_LAUNCH(k_dt_coef, dim3(a.iters), dim3(256), 0, st, a, coef, zero, nzero, ident, zero64,
             zero64 ? nzero64 : 0, sums);
  return hipGetLastError();
}

hipError_t launch_flow(const int32_t* corner_xy, const int32_t* disp, const uint8_t* flags,
                       int ntx, int nty, int tile, const uint8_t* guide, uint8_t* guide_t,
                       int W, int H, const lnr_params& p, void* maps_v, double* coef,
                       float* flow, float* ntilde, hipStream_t st, const DtShape* shape,
                       bool coef_ready, bool guide_t_ready) {
  Rec* maps = static_cast<Rec*>(maps_v);
  uint8_t* rowflag = static_cast<uint8_t*>(maps_v) + dt_rowflag_offset(W, H);
  if (!guide_t_ready) {
    LNR_LAUNCH(k_guide_columns, dim3((W + 63) / 64, (H + 63) / 64), dim3(256), 0, st, guide, W, H,
               dt_guide_stride(H), guide_t);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
  }
  DtArgs a;
  a.iters = p.dt_iters;
  const DtShape sh = shape && dt_shape_valid(*shape, W, H) ? *shape : dt_default_shape(W, H);
  hipError_t e;
  if (!coef_ready && (e = launch_dt_coef(p, coef, nullptr, 0, nullptr, st)) != hipSuccess) return e;
  const double nmin = p.n_min;
  for (int i = 0; i < a.iters; ++i) {
    const double* cf = coef + 256 * i;
    const bool first = i == 0, last = i + 1 == a.iters;
    e = row_pass(sh, first, maps, guide, W, H, cf, corner_xy, disp, flags, ntx, nty, tile,
                 rowflag, st);
    if (e != hipSuccess) return e;
    e = col_pass(sh, last, maps, guide_t, W, H, cf, flow, ntilde, nmin,
                 first ? rowflag : nullptr, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lnr
