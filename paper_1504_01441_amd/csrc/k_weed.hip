// k_weed.hip -- match weeding (paper Sec. 2.3, Eq. 5) and the level
// homography (Sec. 2.2) on the GPU, with no host round trip. Matches are the
// valid tiles of the level, indexed in tile order (centred level coordinates:
// source side p + d - c, reference side p - c).
//
// k_hyp:  one lane per iteration. Each wave counts the valid tiles, draws four
//         distinct match indices from the counter-based SplitMix64 stream,
//         maps them to tiles with a rank-select over ballot masks, and solves
//         the 8x8 system in double precision (partial pivoting, fixed
//         operation order) with the matrix in registers.
// k_test: a (256 tiles x 8 iterations) block tests its tiles against its
//         hypotheses; wave ballots form each iteration's inlier bitmask row,
//         and the block's count per iteration is added atomically.
// k_fit:  one block sums the counts, takes M as the union of the rows whose
//         count exceeds delta (any split of the iterations gives the same M,
//         as the paper notes), finds the best consensus (most inliers, lowest
//         iteration), sums the least-squares normal equations of G: p -> p + d
//         over that hypothesis' inliers exactly in int64 (order-free), and
//         solves and composes H_l = H_{l+1} o G in double precision.
// The three are ordered by the stream; no block waits for another.
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

// 8x8 solve of the augmented system a (row-major 8 x 9), kept in registers
// (every index is a compile-time constant): Gaussian elimination with partial
// pivoting (first largest |pivot|); |pivot| < 1e-12 or NaN fails. Entries left
// of the pivot column are never read again, so row swaps move columns c..8.
__device__ inline bool solve8(double (&a)[72], double (&x)[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    int piv = c;
    double best = fabs(a[c * 9 + c]);
#pragma unroll
    for (int r = c + 1; r < 8; ++r) {
      const double v = fabs(a[r * 9 + c]);
      if (v > best) { best = v; piv = r; }
    }
    if (!(best >= 1e-12)) return false;
#pragma unroll
    for (int r = c + 1; r < 8; ++r)
      if (piv == r) {
#pragma unroll
        for (int j = c; j < 9; ++j) {
          const double t = a[c * 9 + j];
          a[c * 9 + j] = a[r * 9 + j];
          a[r * 9 + j] = t;
        }
      }
#pragma unroll
    for (int r = c + 1; r < 8; ++r) {
      const double f = a[r * 9 + c] / a[c * 9 + c];
#pragma unroll
      for (int j = c; j < 9; ++j) a[r * 9 + j] = a[r * 9 + j] - f * a[c * 9 + j];
    }
  }
#pragma unroll
  for (int c = 7; c >= 0; --c) {
    double s = a[c * 9 + 8];
#pragma unroll
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

__device__ inline int4 tile_match(const int32_t* __restrict__ cxy,
                                  const int32_t* __restrict__ disp, int t, int ox, int oy) {
  const int px = cxy[2 * t], py = cxy[2 * t + 1];
  return make_int4(px + disp[2 * t] - ox, py + disp[2 * t + 1] - oy, px - ox, py - oy);
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

// position of the k-th (0-based) set bit of m (k < popcount(m))
__device__ inline int select_bit(unsigned long long m, int k) {
  int pos = 0;
#pragma unroll
  for (int half = 32; half >= 1; half >>= 1) {
    const unsigned long long lo = m & ((1ull << half) - 1ull);
    const int c = __popcll(lo);
    if (k >= c) {
      k -= c;
      m >>= half;
      pos += half;
    } else {
      m = lo;
    }
  }
  return pos;
}

constexpr int kHypThreads = 256;
constexpr int kItPerBlock = 8;
constexpr int kTestThreads = 256;
constexpr int kFitThreads = 512;  // the final solve needs ~160 VGPRs
constexpr int kMaxIters = 65536;  // the parameter check's bound on weed_iters
constexpr int kMaxWords = 2304;   // tile bitmask words: (6144 / 16)^2 tiles

__global__ __launch_bounds__(kHypThreads) void k_hyp(
    const uint8_t* __restrict__ flags, const int32_t* __restrict__ cxy,
    const int32_t* __restrict__ disp, int ntiles, int w, int h, WeedArgs a,
    double* __restrict__ G, int32_t* __restrict__ cnt, int32_t* __restrict__ nmatch) {
  __shared__ unsigned long long vb[kMaxWords];  // valid-tile bits, tile order
  __shared__ int wpre[kMaxWords + 1];            // valid tiles before each word
  __shared__ int wsum[kHypThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = kHypThreads / 64;
  const int nwords = (ntiles + 63) >> 6;
  // word wi = ballot of tiles 64 wi .. 64 wi + 63 (one coalesced byte load per lane)
  for (int w0 = wave; w0 < nwords; w0 += 8 * NW) {
    uint8_t f[8];  // eight loads in flight, then the ballots
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = (w0 + u * NW) * 64 + lane;
      f[u] = t < ntiles ? flags[t] : 0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const unsigned long long m = __ballot(f[u] & 2);
      if (lane == 0 && w0 + u * NW < nwords) vb[w0 + u * NW] = m;
    }
  }
  __syncthreads();
  // exclusive prefix of the words' popcounts: thread owns a run of K words
  const int K = (nwords + kHypThreads - 1) / kHypThreads;
  int c = 0;
  for (int j = 0; j < K; ++j) {
    const int wi = tid * K + j;
    if (wi < nwords) c += __popcll(vb[wi]);
  }
  int incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int before = 0, N = 0;
  for (int q = 0; q < NW; ++q) {
    before += q < wave ? wsum[q] : 0;
    N += wsum[q];
  }
  int run = before + incl - c;
  for (int j = 0; j < K; ++j) {
    const int wi = tid * K + j;
    if (wi < nwords) {
      wpre[wi] = run;
      run += __popcll(vb[wi]);
    }
  }
  if (tid == 0) wpre[nwords] = N;
  __syncthreads();
  if (blockIdx.x == 0 && tid == 0) *nmatch = N;
  const int it = blockIdx.x * kHypThreads + tid;
  bool ok = N >= 4 && it < a.iters;
  int pk[4] = {-1, -1, -1, -1};
  if (ok) {
    const unsigned long long base = a.seed ^ ((unsigned long long)(uint32_t)a.level << 56);
    int np = 0;
    for (int t = 0; t < 16 && np < 4; ++t) {
      const unsigned long long u =
          splitmix64(base + (unsigned long long)it * 16ull + (unsigned long long)t);
      const int id = (int)(((u >> 32) * (unsigned long long)N) >> 32);
      if (id == pk[0] || id == pk[1] || id == pk[2]) continue;  // a repeat: draw again
      if (np == 0) pk[0] = id;
      else if (np == 1) pk[1] = id;
      else if (np == 2) pk[2] = id;
      else pk[3] = id;
      ++np;
    }
    ok = np == 4;
  }
  if (ok) {
    const int ox = w / 2, oy = h / 2;
    double A[72];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // match index -> tile: last word with wpre <= id, then the bit within it
      const int id = pk[q];
      int lo = 0, hi = nwords - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wpre[mid] <= id) lo = mid;
        else hi = mid - 1;
      }
      const int tq = lo * 64 + select_bit(vb[lo], id - wpre[lo]);
      const int4 m = tile_match(cxy, disp, tq, ox, oy);
      const double sx = (double)m.x, sy = (double)m.y, tx = (double)m.z, ty = (double)m.w;
      double* r0 = A + (2 * q) * 9;
      double* r1 = A + (2 * q + 1) * 9;
      r0[0] = sx; r0[1] = sy; r0[2] = 1; r0[3] = 0; r0[4] = 0; r0[5] = 0;
      r0[6] = -(sx * tx); r0[7] = -(sy * tx); r0[8] = tx;
      r1[0] = 0; r1[1] = 0; r1[2] = 0; r1[3] = sx; r1[4] = sy; r1[5] = 1;
      r1[6] = -(sx * ty); r1[7] = -(sy * ty); r1[8] = ty;
    }
    double g[8];
    ok = solve8(A, g);
    if (ok)
      for (int i = 0; i < 8; ++i) G[(size_t)it * 8 + i] = g[i];
  }
  // k_test adds each tile chunk's inliers; -1: too few matches, degenerate draw or fit
  if (it < a.iters) cnt[it] = ok ? 0 : -1;
}

// Tile chunk blockIdx.x x iteration group blockIdx.y: adds the chunk's inlier
// counts to cnt[iter] and stores the inlier bits in bal[word][iter]
// (word-major, so that the union reads each word's rows contiguously).
__global__ __launch_bounds__(kTestThreads) void k_test(
    const int32_t* __restrict__ cxy, const int32_t* __restrict__ disp,
    const uint8_t* __restrict__ flags, int ntiles, int w, int h, WeedArgs a,
    const double* __restrict__ G, int32_t* __restrict__ cnt,
    unsigned long long* __restrict__ bal, int wstride) {
  __shared__ double gs[kItPerBlock][8];
  __shared__ int ok[kItPerBlock];
  __shared__ int wc[kItPerBlock][kTestThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int it0 = blockIdx.y * kItPerBlock;
  if (tid < kItPerBlock) {
    const int it = it0 + tid;
    // usable hypotheses start at 0 and only grow, so the sign is stable
    const bool good = it < a.iters && __atomic_load_n(&cnt[it], __ATOMIC_RELAXED) >= 0;
    ok[tid] = good;
    for (int i = 0; i < 8; ++i) gs[tid][i] = good ? G[(size_t)it * 8 + i] : 0.0;
  }
  __syncthreads();
  const int t = blockIdx.x * kTestThreads + tid;
  const bool valid = t < ntiles && (flags[t] & 2);
  const int4 m = valid ? tile_match(cxy, disp, t, w / 2, h / 2) : make_int4(0, 0, 0, 0);
  const int word = t >> 6;
  for (int q = 0; q < kItPerBlock; ++q) {
    if (!ok[q]) continue;
    const bool in = valid && is_inlier(gs[q], m, a.eps2);
    const unsigned long long b = __ballot(in);
    if (lane == 0) {
      if (word < wstride) bal[(size_t)word * a.iters + it0 + q] = b;
      wc[q][wave] = __popcll(b);
    }
  }
  __syncthreads();
  if (tid < kItPerBlock && ok[tid]) {
    int s = 0;
    for (int q = 0; q < kTestThreads / 64; ++q) s += wc[tid][q];
    if (s) atomicAdd(&cnt[it0 + tid], s);
  }
}

__device__ inline long long wave_sum_i64(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long u = __shfl_xor(v, o);
    v = u > v ? u : v;
  }
  return v;
}

// distinct sums of the normal equations (see k_fit)
constexpr int kSums = 23;

// polynomial degree of unknown i (h11 h12 h13 h21 h22 h23 h31 h32) in the
// coordinates, for the power-of-two scaling
__device__ inline int deg_of(int i) { return (i == 2 || i == 5) ? 0 : (i >= 6 ? 2 : 1); }

// Entry (i, j) of A^T A from the 23 sums T (order: 1, x, y, xx, xy, yy, u, v,
// xu, yu, xv, yv, xxu, xyu, yyu, xxv, xyv, yyv, xq, yq, xxq, xyq, yyq with
// q = u^2 + v^2).
__device__ inline long long normal_entry(const long long* T, int i, int j) {
  if (i > j) { const int t = i; i = j; j = t; }
  switch (i * 8 + j) {
    case 0: return T[3];   case 1: return T[4];   case 2: return T[1];
    case 6: return -T[12]; case 7: return -T[13];
    case 9: return T[5];   case 10: return T[2];  case 14: return -T[13]; case 15: return -T[14];
    case 18: return T[0];  case 22: return -T[8]; case 23: return -T[9];
    case 27: return T[3];  case 28: return T[4];  case 29: return T[1];
    case 30: return -T[15]; case 31: return -T[16];
    case 36: return T[5];  case 37: return T[2];  case 38: return -T[16]; case 39: return -T[17];
    case 45: return T[0];  case 46: return -T[10]; case 47: return -T[11];
    case 54: return T[20]; case 55: return T[21];
    case 63: return T[22];
    default: return 0;
  }
}

// Entry i of A^T b
__device__ inline long long normal_rhs(const long long* T, int i) {
  switch (i) {
    case 0: return T[8];  case 1: return T[9];  case 2: return T[6];  case 3: return T[10];
    case 4: return T[11]; case 5: return T[7];  case 6: return -T[18];
    default: return -T[19];
  }
}

// The 8x8 solve of solve8 with one row per lane (lanes 0-7 of a wave; the
// other lanes mirror row 7 and are ignored): identical arithmetic per entry,
// the pivot search as a first-largest reduction. Every lane returns the same.
__device__ inline bool solve8_wave(double (&row)[9], double (&x)[8]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    // first largest |a[r][c]| over r >= c; a NaN below the pivot row is never
    // larger, a NaN in the pivot row fails
    const double ac = fabs(row[c]);
    double v = (lane >= c && lane < 8) ? ac : -1.0;
    if (lane != c && !(v >= 0.0)) v = -1.0;
    int idx = lane < 8 ? lane : 8;
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      const double v2 = __shfl_xor(v, o);
      const int i2 = __shfl_xor(idx, o);
      if (v2 > v || (v2 == v && i2 < idx)) { v = v2; idx = i2; }
    }
    const double best = __shfl(v, 0);
    const int piv = __shfl(idx, 0);
    const double diag = __shfl(ac, c);
    if (!(diag == diag) || !(best >= 1e-12)) return false;
    const int src = lane == c ? piv : (lane == piv ? c : lane);
#pragma unroll
    for (int j = c; j < 9; ++j) row[j] = __shfl(row[j], src);
    double pr[9];
#pragma unroll
    for (int j = c; j < 9; ++j) pr[j] = __shfl(row[j], c);
    if (lane > c && lane < 8) {
      const double f = row[c] / pr[c];
#pragma unroll
      for (int j = c; j < 9; ++j) row[j] = row[j] - f * pr[j];
    }
  }
#pragma unroll
  for (int c = 7; c >= 0; --c) {
    double s = row[8];
#pragma unroll
    for (int j = c + 1; j < 8; ++j) s = s - row[j] * x[j];
    x[c] = __shfl(s / row[c], c);
  }
  return true;
}

// One block: union M, best consensus, least-squares level homography, and
// the per-tile flags 4 (in M) and 8 (in the fit).
__global__ __launch_bounds__(kFitThreads) void k_fit(
    const int32_t* __restrict__ cxy, const int32_t* __restrict__ disp,
    uint8_t* __restrict__ flags, int ntiles, int w, int h, WeedArgs a,
    const int32_t* __restrict__ nmatch, const double* __restrict__ G,
    const int32_t* __restrict__ cnt, const unsigned long long* __restrict__ bal, int wstride,
    const double* __restrict__ Hprev, double* __restrict__ Hout, int32_t* __restrict__ counts) {
  extern __shared__ unsigned long long mw[];  // [wstride] union bitmask M
  __shared__ unsigned int accw[kMaxIters / 32];  // accepted iterations
  __shared__ unsigned long long kmax[kFitThreads / 64];
  __shared__ long long part[kFitThreads / 64][kSums];
  __shared__ long long tot[kSums];
  constexpr int NWV = kFitThreads / 64, TPT = 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // The phases below depend on each other (counts -> union and best row ->
  // fit), so each issues all of its loads before using any; the first batch
  // of tile data is loaded up front.
  uint8_t tf[TPT];
  int tpx[TPT], tpy[TPT], tdx[TPT], tdy[TPT];
#pragma unroll
  for (int j = 0; j < TPT; ++j) {
    const int t = tid + j * kFitThreads;
    const bool in = t < ntiles;
    tf[j] = in ? flags[t] : 0;
    tpx[j] = in ? cxy[2 * t] : 0;
    tpy[j] = in ? cxy[2 * t + 1] : 0;
    tdx[j] = in ? disp[2 * t] : 0;
    tdy[j] = in ? disp[2 * t + 1] : 0;
  }
  const int N = *nmatch;
  const int delta = weed_delta(N, a);
  // per-iteration counts, acceptance bits, best key
  unsigned long long kb = 0ull;
  for (int i0 = 0; i0 < a.iters; i0 += 2 * kFitThreads) {
    int c[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int i = i0 + r * kFitThreads + tid;
      c[r] = i < a.iters && N >= 4 ? cnt[i] : -1;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int i = i0 + r * kFitThreads + tid;
      const int ib = i0 + r * kFitThreads + wave * 64;
      const unsigned long long acc = __ballot(c[r] > delta);
      if (lane == 0 && ib < a.iters) {
        accw[ib >> 5] = (unsigned int)acc;
        accw[(ib >> 5) + 1] = (unsigned int)(acc >> 32);
      }
      if (c[r] >= 0) {
        const unsigned long long key =
            ((unsigned long long)(uint32_t)c[r] << 32) | (unsigned long long)(~(uint32_t)i);
        kb = key > kb ? key : kb;
      }
    }
  }
  kb = wave_max_u64(kb);
  if (lane == 0) kmax[wave] = kb;
  __syncthreads();
  unsigned long long bkey = 0ull;
  for (int q = 0; q < NWV; ++q) bkey = kmax[q] > bkey ? kmax[q] : bkey;
  const int bc = N >= 4 && bkey ? (int)(bkey >> 32) : -1;
  const int bi = N >= 4 && bkey ? (int)(~(uint32_t)(bkey & 0xffffffffull)) : -1;
  const bool fit = bc > delta;
  // the best hypothesis' inlier bits for the first tile batch
  unsigned long long brow[TPT];
#pragma unroll
  for (int j = 0; j < TPT; ++j) {
    const int t = tid + j * kFitThreads;
    brow[j] = fit && t < ntiles ? bal[(size_t)(t >> 6) * a.iters + bi] : 0ull;
  }
  // M: OR of the accepted rows; a wave per word (two at a time), its lanes
  // over the iterations
  for (int w0 = wave; w0 < wstride; w0 += 2 * NWV) {
    const int w1 = w0 + NWV;
    unsigned long long v0 = 0ull, v1 = 0ull;
    for (int i0 = 0; i0 < a.iters; i0 += 64 * 16) {
      unsigned long long r0[16], r1[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = i0 + u * 64 + lane;
        r0[u] = i < a.iters ? bal[(size_t)w0 * a.iters + i] : 0ull;
        r1[u] = i < a.iters && w1 < wstride ? bal[(size_t)w1 * a.iters + i] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = i0 + u * 64 + lane;
        if (i < a.iters && ((accw[i >> 5] >> (i & 31)) & 1u)) {
          v0 |= r0[u];
          v1 |= r1[u];
        }
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      v0 |= __shfl_xor(v0, o);
      v1 |= __shfl_xor(v1, o);
    }
    if (lane == 0) {
      mw[w0] = v0;
      if (w1 < wstride) mw[w1] = v1;
    }
  }
  __syncthreads();
  // normal equations of G: (x, y) -> (u, v), reference side to source side,
  // over the best hypothesis' inliers; the 8x8 matrix has 23 distinct sums
  long long s[kSums];
#pragma unroll
  for (int i = 0; i < kSums; ++i) s[i] = 0;
  const int ox = w / 2, oy = h / 2;
  for (int t0 = 0; t0 < ntiles; t0 += TPT * kFitThreads) {
    if (t0 > 0) {  // later batches (levels with more than 8192 tiles)
#pragma unroll
      for (int j = 0; j < TPT; ++j) {
        const int t = t0 + tid + j * kFitThreads;
        const bool in = t < ntiles;
        tf[j] = in ? flags[t] : 0;
        tpx[j] = in ? cxy[2 * t] : 0;
        tpy[j] = in ? cxy[2 * t + 1] : 0;
        tdx[j] = in ? disp[2 * t] : 0;
        tdy[j] = in ? disp[2 * t + 1] : 0;
        brow[j] = fit && in ? bal[(size_t)(t >> 6) * a.iters + bi] : 0ull;
      }
    }
#pragma unroll
    for (int j = 0; j < TPT; ++j) {
      const int t = t0 + tid + j * kFitThreads;
      if (t >= ntiles || !(tf[j] & 2)) continue;
      const bool inM = (mw[t >> 6] >> (t & 63)) & 1ull;
      const bool sel = (brow[j] >> (t & 63)) & 1ull;
      flags[t] = (uint8_t)((tf[j] & 0x13) | (inM ? 4 : 0) | (sel ? 8 : 0));
      if (!sel) continue;
      const long long x = tpx[j] - ox, y = tpy[j] - oy, u = x + tdx[j], v = y + tdy[j];
      const long long xx = x * x, xy = x * y, yy = y * y, q = u * u + v * v;
      s[0] += 1;       s[1] += x;       s[2] += y;
      s[3] += xx;      s[4] += xy;      s[5] += yy;
      s[6] += u;       s[7] += v;
      s[8] += x * u;   s[9] += y * u;   s[10] += x * v;  s[11] += y * v;
      s[12] += xx * u; s[13] += xy * u; s[14] += yy * u;
      s[15] += xx * v; s[16] += xy * v; s[17] += yy * v;
      s[18] += x * q;  s[19] += y * q;
      s[20] += xx * q; s[21] += xy * q; s[22] += yy * q;
    }
  }
  // exact (order-free) int64 reduction
#pragma unroll
  for (int i = 0; i < kSums; ++i) s[i] = wave_sum_i64(s[i]);
  if (lane == 0)
    for (int i = 0; i < kSums; ++i) part[wave][i] = s[i];
  __syncthreads();
  if (tid < kSums) {
    long long z = 0;
    for (int q = 0; q < kFitThreads / 64; ++q) z += part[q][tid];
    tot[tid] = z;
  }
  __syncthreads();
  if (wave != 0) return;
  const int msel = (int)tot[0];
  if (lane == 0) {
    counts[0] = N;
    counts[1] = msel;
    counts[2] = bc;
    counts[3] = bi;
    for (int i = 0; i < 9; ++i) Hout[i] = Hprev[i];
  }
  if (msel < 4) return;
  // A^T A and A^T b of the rows (x, y, 1, 0, 0, 0, -xu, -yu | u) and
  // (0, 0, 0, x, y, 1, -xv, -yv | v), scaled by powers of two; lane r < 8
  // holds row r
  int k = 0;
  const int mx = ox > oy ? (ox > 1 ? ox : 1) : (oy > 1 ? oy : 1);
  while ((1 << k) < mx) ++k;
  const int deg[8] = {1, 1, 0, 1, 1, 0, 2, 2};
  const int r = lane < 8 ? lane : 7;
  double row[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const long long v = j < 8 ? normal_entry(tot, r, j) : normal_rhs(tot, r);
    const int e = j < 8 ? -k * (deg_of(r) + deg[j]) : -k * (deg_of(r) + 1);
    row[j] = ldexp((double)v, e);
  }
  double hs[8];
  if (!solve8_wave(row, hs)) return;
  if (lane != 0) return;
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
  const int chunks = ntiles > 0 ? (ntiles + kTestThreads - 1) / kTestThreads : 1;
  const int groups = (a.iters + kItPerBlock - 1) / kItPerBlock;
  if (words > kMaxWords || a.iters > kMaxIters) return hipErrorInvalidValue;
  LNR_LAUNCH(k_hyp, dim3((a.iters + kHypThreads - 1) / kHypThreads), dim3(kHypThreads), 0, st,
             flags, corner_xy, disp, ntiles, w, h, a, b.G, b.cnt, b.nmatch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ntiles > 0) {
    LNR_LAUNCH(k_test, dim3(chunks, groups), dim3(kTestThreads), 0, st, corner_xy, disp, flags,
               ntiles, w, h, a, b.G, b.cnt, b.bal, words);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  LNR_LAUNCH(k_fit, dim3(1), dim3(kFitThreads), (size_t)words * 8, st, corner_xy, disp, flags,
             ntiles, w, h, a, b.nmatch, b.G, b.cnt, b.bal, words, H_prev, H_out, counts);
  return hipGetLastError();
}

}  // namespace lnr
