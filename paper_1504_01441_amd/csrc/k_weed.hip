// k_weed.hip -- match weeding (paper Sec. 2.3, Eq. 5) and the level
// homography (Sec. 2.2) on the GPU, with no host round trip.
//
// k_compact: one workgroup lists the valid matches of the level in tile order
//   (centred level coordinates: source side p + d - c, reference side p - c).
// k_weedfit: a (256 matches x 8 iterations) block draws four distinct
//   indices per iteration from the counter-based SplitMix64 stream, solves
//   the 8x8 system in double precision (partial pivoting, fixed operation
//   order), and tests its matches; wave ballots form each iteration's inlier
//   bitmask row and the counts are summed with atomics. The last block of an
//   iteration group ORs the accepted rows (count > delta) into M with 64-bit
//   atomics, so M is the same for any execution order (the paper's note that
//   the iterations can be split freely), and keeps the best consensus as a
//   64-bit atomicMax on (count << 32 | ~iteration). The last block overall
//   re-tests the best hypothesis, sums the least-squares normal equations of
//   G: p -> p + d over its inliers exactly in int64 (order-free), and solves
//   and composes H_l = H_{l+1} o G in double precision.
#include "lnr_device.h"
#include "lnr_internal.h"

namespace lnr {
namespace {

__device__ inline unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// 8x8 solve of the augmented system a (row-major 8 x 9): Gaussian elimination
// with partial pivoting (first largest |pivot|); |pivot| < 1e-12 or NaN fails.
__device__ bool solve8(double* a, double* x) {
  for (int c = 0; c < 8; ++c) {
    int piv = c;
    double best = fabs(a[c * 9 + c]);
    for (int r = c + 1; r < 8; ++r) {
      const double v = fabs(a[r * 9 + c]);
      if (v > best) { best = v; piv = r; }
    }
    if (!(best >= 1e-12)) return false;
    if (piv != c)
      for (int j = 0; j < 9; ++j) {
        const double t = a[c * 9 + j];
        a[c * 9 + j] = a[piv * 9 + j];
        a[piv * 9 + j] = t;
      }
    for (int r = c + 1; r < 8; ++r) {
      const double f = a[r * 9 + c] / a[c * 9 + c];
      for (int j = c; j < 9; ++j) a[r * 9 + j] = a[r * 9 + j] - f * a[c * 9 + j];
    }
  }
  for (int c = 7; c >= 0; --c) {
    double s = a[c * 9 + 8];
    for (int j = c + 1; j < 8; ++j) s = s - a[c * 9 + j] * x[j];
    x[c] = s / a[c * 9 + c];
  }
  return true;
}

// inlier test |G(s) - t|^2 < eps^2, fixed operation order
__device__ inline bool is_inlier(const double* g, int4 m, double eps2) {
  const double sx = (double)m.x, sy = (double)m.y;
  const double den = (g[6] * sx + g[7] * sy) + 1.0;
  const double gx = ((g[0] * sx + g[1] * sy) + g[2]) / den;
  const double gy = ((g[3] * sx + g[4] * sy) + g[5]) / den;
  const double ex = gx - (double)m.z, ey = gy - (double)m.w;
  const double e2 = ex * ex + ey * ey;
  return e2 < eps2;
}

__global__ __launch_bounds__(1024) void k_compact(const int32_t* __restrict__ cxy,
                                                  const int32_t* __restrict__ disp,
                                                  const uint8_t* __restrict__ flags, int ntiles,
                                                  int w, int h, int4* __restrict__ matches,
                                                  int32_t* __restrict__ tile_of,
                                                  int32_t* __restrict__ nmatch,
                                                  unsigned long long* __restrict__ mbits,
                                                  unsigned long long* __restrict__ best,
                                                  int32_t* __restrict__ counts, int iters,
                                                  uint32_t* __restrict__ done, int ndone) {
  __shared__ int part[1024];
  const int tid = threadIdx.x;
  const int chunk = (ntiles + 1023) / 1024;
  const int t0 = tid * chunk, t1 = min(ntiles, t0 + chunk);
  int cnt = 0;
  for (int t = t0; t < t1; ++t) cnt += (flags[t] & 2) ? 1 : 0;
  part[tid] = cnt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int add = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  int k = part[tid] - cnt;
  const int ox = w / 2, oy = h / 2;
  for (int t = t0; t < t1; ++t)
    if (flags[t] & 2) {
      const int px = cxy[2 * t], py = cxy[2 * t + 1];
      matches[k] = make_int4(px + disp[2 * t] - ox, py + disp[2 * t + 1] - oy, px - ox, py - oy);
      tile_of[k] = t;
      ++k;
    }
  if (tid == 1023) *nmatch = part[1023];
  for (int i = tid; i < (ntiles + 63) / 64; i += 1024) mbits[i] = 0ull;
  for (int i = tid; i < iters; i += 1024) counts[i] = 0;
  for (int i = tid; i < ndone; i += 1024) done[i] = 0u;
  if (tid == 0) *best = 0ull;
}

struct WeedArgs {
  int iters, level, delta_min, delta_pct;
  double eps2;
  unsigned long long seed;
};

__device__ inline int weed_delta(int N, const WeedArgs& a) {
  const int d = (N * a.delta_pct + 99) / 100;
  return d > a.delta_min ? d : a.delta_min;
}

// Draw and fit hypothesis `it` (identical in every lane). Returns false when
// the draw or the fit is degenerate.
__device__ bool hypothesis(const int4* __restrict__ matches, int N, int it, const WeedArgs& a,
                           double* g) {
  const unsigned long long base = a.seed ^ ((unsigned long long)(uint32_t)a.level << 56);
  int pick[4], np = 0;
  for (int t = 0; t < 16 && np < 4; ++t) {
    const unsigned long long u = splitmix64(base + (unsigned long long)it * 16ull + (unsigned long long)t);
    const int id = (int)(((u >> 32) * (unsigned long long)N) >> 32);
    bool dup = false;
    for (int q = 0; q < np; ++q) dup |= pick[q] == id;
    if (!dup) pick[np++] = id;
  }
  if (np < 4) return false;
  double A[8 * 9];
  for (int q = 0; q < 4; ++q) {
    const int4 m = matches[pick[q]];
    const double sx = (double)m.x, sy = (double)m.y, tx = (double)m.z, ty = (double)m.w;
    double* r0 = A + (2 * q) * 9;
    double* r1 = A + (2 * q + 1) * 9;
    r0[0] = sx; r0[1] = sy; r0[2] = 1; r0[3] = 0; r0[4] = 0; r0[5] = 0;
    r0[6] = -(sx * tx); r0[7] = -(sy * tx); r0[8] = tx;
    r1[0] = 0; r1[1] = 0; r1[2] = 0; r1[3] = sx; r1[4] = sy; r1[5] = 1;
    r1[6] = -(sx * ty); r1[7] = -(sy * ty); r1[8] = ty;
  }
  return solve8(A, g);
}

__device__ inline long long wave_sum_i64(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// index of the upper-triangle entry (i <= j) of the 8x8 normal matrix
__device__ inline int tri(int i, int j) { return i * 8 - (i * (i - 1)) / 2 + (j - i); }

constexpr int kItPerBlock = 8;
constexpr int kWeedThreads = 256;

// Signal that this block is done with its share; returns true in the one
// block that finishes last. Writes before the call are visible to that block.
__device__ inline bool last_to_finish(uint32_t* counter, uint32_t total, int* flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) *flag = atomicAdd(counter, 1u) == total - 1;
  __syncthreads();
  const bool last = *flag != 0;
  if (last) __threadfence();
  return last;
}

// Least-squares level homography over the inliers of the best-consensus
// hypothesis (one block), plus the per-tile flags 4 (in M) and 8 (in the fit).
__device__ void fit_level(const int4* __restrict__ matches, const int32_t* __restrict__ tile_of,
                          int N, const WeedArgs& a, const unsigned long long* mbits,
                          unsigned long long bkey, const double* __restrict__ Gall,
                          uint8_t* __restrict__ flags, int w, int h,
                          const double* __restrict__ Hprev, double* __restrict__ Hout,
                          int32_t* __restrict__ counts) {
  __shared__ long long part[kWeedThreads / 64][45];
  __shared__ long long tot[45];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bc = N >= 4 && bkey ? (int)(bkey >> 32) : -1;
  const int bi = N >= 4 && bkey ? (int)(~(uint32_t)(bkey & 0xffffffffull)) : -1;
  const bool fit = bc > weed_delta(N, a);
  double g[8];
  for (int i = 0; i < 8; ++i) g[i] = fit ? Gall[(size_t)bi * 8 + i] : 0.0;
  long long ata[36], atb[8];
  for (int i = 0; i < 36; ++i) ata[i] = 0;
  for (int i = 0; i < 8; ++i) atb[i] = 0;
  long long m = 0;
  for (int k = tid; k < N; k += kWeedThreads) {
    const int4 mt = matches[k];
    const bool inM = (mbits[k >> 6] >> (k & 63)) & 1ull;
    const bool sel = fit && is_inlier(g, mt, a.eps2);
    const int t = tile_of[k];
    flags[t] = (uint8_t)((flags[t] & 3) | (inM ? 4 : 0) | (sel ? 8 : 0));
    if (!sel) continue;
    ++m;
    const long long x = mt.z, y = mt.w, u = mt.x, v = mt.y;  // G: (x, y) -> (u, v)
    const long long r1[8] = {x, y, 1, 0, 0, 0, -x * u, -y * u};
    const long long r2[8] = {0, 0, 0, x, y, 1, -x * v, -y * v};
    for (int i = 0; i < 8; ++i) {
      for (int j = i; j < 8; ++j) ata[tri(i, j)] += r1[i] * r1[j] + r2[i] * r2[j];
      atb[i] += r1[i] * u + r2[i] * v;
    }
  }
  // exact (order-free) int64 reduction: wave shuffles, then across waves
  for (int i = 0; i < 36; ++i) ata[i] = wave_sum_i64(ata[i]);
  for (int i = 0; i < 8; ++i) atb[i] = wave_sum_i64(atb[i]);
  m = wave_sum_i64(m);
  if (lane == 0) {
    for (int i = 0; i < 36; ++i) part[wave][i] = ata[i];
    for (int i = 0; i < 8; ++i) part[wave][36 + i] = atb[i];
    part[wave][44] = m;
  }
  __syncthreads();
  if (tid < 45) {
    long long s = 0;
    for (int q = 0; q < kWeedThreads / 64; ++q) s += part[q][tid];
    tot[tid] = s;
  }
  __syncthreads();
  if (tid != 0) return;
  const int msel = (int)tot[44];
  counts[0] = N;
  counts[1] = msel;
  counts[2] = bc;
  counts[3] = bi;
  for (int i = 0; i < 9; ++i) Hout[i] = Hprev[i];
  if (msel < 4) return;
  const int ox = w / 2, oy = h / 2;
  int k = 0;
  const int mx = ox > oy ? (ox > 1 ? ox : 1) : (oy > 1 ? oy : 1);
  while ((1 << k) < mx) ++k;
  const int deg[8] = {1, 1, 0, 1, 1, 0, 2, 2};
  double A[8 * 9], hs[8];
  for (int i = 0; i < 8; ++i) {
    for (int j = 0; j < 8; ++j) {
      const long long v = i <= j ? tot[tri(i, j)] : tot[tri(j, i)];
      A[i * 9 + j] = ldexp((double)v, -k * (deg[i] + deg[j]));
    }
    A[i * 9 + 8] = ldexp((double)tot[36 + i], -k * (deg[i] + 1));
  }
  if (!solve8(A, hs)) return;
  double Gc[9];
  for (int i = 0; i < 8; ++i) Gc[i] = ldexp(hs[i], k * (1 - deg[i]));
  Gc[8] = 1.0;
  const double pox = (double)(2 * ox - (w - 1)), poy = (double)(2 * oy - (h - 1));
  const double Pm[9] = {2, 0, pox, 0, 2, poy, 0, 0, (double)w};
  const double Qm[9] = {(double)w, 0, -pox, 0, (double)w, -poy, 0, 0, 2};
  double T1[9], T2[9], T3[9], Hp[9];
  for (int i = 0; i < 9; ++i) Hp[i] = Hprev[i];
  mat3_mul(Pm, Gc, T1);
  mat3_mul(T1, Qm, T2);
  mat3_mul(Hp, T2, T3);
  const double d = T3[8];
  if (d == 0.0) return;
  double Hn[9];
  for (int i = 0; i < 9; ++i) {
    Hn[i] = T3[i] / d;
    if (!isfinite(Hn[i])) return;
  }
  for (int i = 0; i < 9; ++i) Hout[i] = Hn[i];
}

// Block (256 matches, 8 iterations). Every block draws and fits its 8
// hypotheses (8 threads), tests its matches against them (wave ballots form
// the inlier bitmask rows) and adds the counts. The last block of an
// iteration group ORs the accepted rows (count > delta) into M and updates
// the best consensus (count << 32 | ~iteration); the last block overall fits
// the level homography. No block waits for another.
__global__ __launch_bounds__(kWeedThreads) void k_weedfit(
    const int4* __restrict__ matches, const int32_t* __restrict__ tile_of,
    const int32_t* __restrict__ nmatch, WeedArgs a, double* __restrict__ G,
    int32_t* __restrict__ cnt, unsigned long long* __restrict__ bal, int wstride,
    unsigned long long* __restrict__ mbits, unsigned long long* __restrict__ best,
    uint32_t* __restrict__ done, uint8_t* __restrict__ flags, int w, int h,
    const double* __restrict__ Hprev, double* __restrict__ Hout, int32_t* __restrict__ counts) {
  __shared__ double gs[kItPerBlock][8];
  __shared__ int ok[kItPerBlock];
  __shared__ int wc[kItPerBlock][kWeedThreads / 64];
  __shared__ int lastflag;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int it0 = blockIdx.y * kItPerBlock;
  const int N = *nmatch;
  const int k = blockIdx.x * kWeedThreads + tid;
  const bool work = N >= 4 && blockIdx.x * kWeedThreads < N;
  if (work && tid < kItPerBlock) {
    const int it = it0 + tid;
    double g[8];
    const bool good = it < a.iters && hypothesis(matches, N, it, a, g);
    ok[tid] = good;
    for (int i = 0; i < 8; ++i) gs[tid][i] = good ? g[i] : 0.0;
    if (blockIdx.x == 0 && it < a.iters) {  // block 0 of the group publishes G
      if (good)
        for (int i = 0; i < 8; ++i) G[(size_t)it * 8 + i] = g[i];
      else
        cnt[it] = -1;  // degenerate: no block adds to it
    }
  }
  __syncthreads();
  if (work) {
    const int4 m = k < N ? matches[k] : make_int4(0, 0, 0, 0);
    const int word = k >> 6;
    for (int q = 0; q < kItPerBlock; ++q) {
      if (!ok[q]) continue;
      const bool in = k < N && is_inlier(gs[q], m, a.eps2);
      const unsigned long long b = __ballot(in);
      if (lane == 0) {
        if (word * 64 < N) bal[(size_t)(it0 + q) * wstride + word] = b;
        wc[q][wave] = __popcll(b);
      }
    }
    __syncthreads();
    if (tid < kItPerBlock && ok[tid]) {
      int s = 0;
      for (int q = 0; q < kWeedThreads / 64; ++q) s += wc[tid][q];
      if (s) atomicAdd(&cnt[it0 + tid], s);
    }
  }
  // the last block of this iteration group: union of accepted rows into M
  if (last_to_finish(&done[1 + blockIdx.y], gridDim.x, &lastflag) && N >= 4) {
    const int delta = weed_delta(N, a);
    const int nwords = (N + 63) / 64;
    __shared__ int acc[kItPerBlock];
    __shared__ int cval[kItPerBlock];
    if (tid < kItPerBlock) {
      const int it = it0 + tid;
      cval[tid] = it < a.iters ? __atomic_load_n(&cnt[it], __ATOMIC_RELAXED) : -1;
      acc[tid] = cval[tid] > delta;  // -1 marks a degenerate iteration
    }
    __syncthreads();
    for (int wi = tid; wi < nwords; wi += kWeedThreads) {
      unsigned long long v = 0ull;
      for (int q = 0; q < kItPerBlock; ++q)
        if (acc[q]) v |= bal[(size_t)(it0 + q) * wstride + wi];
      if (v) atomicOr(&mbits[wi], v);
    }
    if (tid == 0) {
      unsigned long long bk = 0ull;
      for (int q = 0; q < kItPerBlock; ++q)
        if (cval[q] >= 0) {
          const unsigned long long key = ((unsigned long long)(uint32_t)cval[q] << 32) |
                                         (unsigned long long)(~(uint32_t)(it0 + q));
          bk = key > bk ? key : bk;
        }
      if (bk) atomicMax(best, bk);
    }
  }
  // the last block overall: level homography
  if (last_to_finish(&done[0], gridDim.x * gridDim.y, &lastflag)) {
    const unsigned long long bkey = __atomic_load_n(best, __ATOMIC_RELAXED);
    fit_level(matches, tile_of, N, a, mbits, bkey, G, flags, w, h, Hprev, Hout, counts);
  }
}

}  // namespace

hipError_t launch_weed_fit(const int32_t* corner_xy, const int32_t* disp, uint8_t* flags,
                           int ntiles, int w, int h, int level, const lnr_params& p,
                           const double* H_prev, double* H_out, int32_t* counts,
                           const WeedBufs& b, hipStream_t st) {
  WeedArgs a;
  a.iters = p.weed_iters;
  a.level = level;
  a.delta_min = p.weed_delta_min;
  a.delta_pct = p.weed_delta_pct;
  a.eps2 = p.weed_eps * p.weed_eps;
  a.seed = p.seed;
  const int words = ntiles > 0 ? (ntiles + 63) / 64 : 1;
  const int chunks = ntiles > 0 ? (ntiles + kWeedThreads - 1) / kWeedThreads : 1;
  const int groups = (a.iters + kItPerBlock - 1) / kItPerBlock;
  LNR_LAUNCH(k_compact, dim3(1), dim3(1024), 0, st, corner_xy, disp, flags, ntiles, w, h,
             b.matches, b.tile_of, b.nmatch, b.mbits, b.best, b.cnt, a.iters, b.done, 1 + groups);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  LNR_LAUNCH(k_weedfit, dim3(chunks, groups), dim3(kWeedThreads), 0, st, b.matches, b.tile_of,
             b.nmatch, a, b.G, b.cnt, b.bal, words, b.mbits, b.best, b.done, flags, w, h, H_prev,
             H_out, counts);
  return hipGetLastError();
}

}  // namespace lnr
