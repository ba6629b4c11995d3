// k_weed.hip -- match weeding (paper Sec. 2.3, Eq. 5) and the level
// homography (Sec. 2.2) on the GPU, with no host round trip. Matches are the
// valid tiles of the level, indexed in tile order (centred level coordinates:
// source side p + d - c, reference side p - c).
//
// k_valid: the valid-match bits of the tiles, one 64-bit word per 64 tiles
//         (a wave ballot each); also clears the fit sums. In a registration
//         the level's warp clears them and its search sets the bits instead.
// k_hyp:  one lane per iteration, one wave per block. Each wave prefix-sums
//         the words' popcounts, draws four distinct match indices from the
//         counter-based SplitMix64 stream, maps them to tiles with a
//         rank-select over the words, and solves the 8x8 system in double
//         precision (partial pivoting, fixed operation order) with the matrix
//         in registers.
// k_test: a (256 tiles x 4 or 8 iterations) block tests its tiles against its
//         hypotheses; wave ballots form each iteration's inlier bitmask row,
//         and the block's count per iteration is added atomically.
// k_union: a wave per word of 64 tiles. Every block reads the counts, takes
//         the accepted iterations (count above delta) and the best consensus
//         (most inliers, lowest iteration); a wave ORs the accepted rows of
//         its word (M is the union of those rows; any split of the
//         iterations gives the same M, as the paper notes), writes its tiles'
//         flags and adds their terms of the least-squares normal equations of
//         G: p -> p + d over the best hypothesis' inliers exactly in int64
//         (order-free) to the level's sums.
// k_solve: one lane solves the normal equations in double precision (the
//         solver of k_hyp) and composes H_l = H_{l+1} o G.
// The kernels are ordered by the stream; no block waits for another.
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

constexpr int kValidThreads = 256;
constexpr int kHypThreads = 64;
// hypotheses per k_test block: 4 on levels of up to kTestSmall tiles (more
// blocks for the few tiles), 8 above (fewer re-reads of the tiles)
constexpr int kTestSmall = 2048;
constexpr int kTestThreads = 256;
constexpr int kUnionThreads = 512;
constexpr int kMaxIters = 65536;  // the parameter check's bound on weed_iters
constexpr int kMaxWords = 2304;   // tile bitmask words: (6144 / 16)^2 tiles

// word wi of vb = valid-match bits of tiles 64 wi .. 64 wi + 63; block 0
// also clears the level's least-squares sums
__global__ __launch_bounds__(kValidThreads) void k_valid(const uint8_t* __restrict__ flags,
                                                         int ntiles, int nwords,
                                                         unsigned long long* __restrict__ vb,
                                                         long long* __restrict__ sums) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wi = blockIdx.x * (kValidThreads / 64) + (tid >> 6);
  if (blockIdx.x == 0 && tid < 24) sums[tid] = 0;
  if (wi >= nwords) return;  // whole waves
  const int t = wi * 64 + lane;
  const unsigned long long m = __ballot(t < ntiles && (flags[t] & 2));
  if (lane == 0) vb[wi] = m;
}

// The kernels below take one level of one pair (JOBS false: the job is the
// kernel argument) or a table of jobs, one per blockIdx.z (batches).
template <bool JOBS>
__global__ __launch_bounds__(kHypThreads) void k_hyp(WeedJob one,
                                                     const WeedJob* __restrict__ jobs,
                                                     WeedArgs a) {
  const WeedJob J = JOBS ? jobs[blockIdx.z] : one;
  const unsigned long long* __restrict__ vbg = J.b.vb;
  const int32_t* __restrict__ cxy = J.cxy;
  const int32_t* __restrict__ disp = J.disp;
  const int nwords = J.words, w = J.w, h = J.h;
  double* __restrict__ G = J.b.G;
  int32_t* __restrict__ cnt = J.b.cnt;
  int32_t* __restrict__ nmatch = J.b.nmatch;
  __shared__ unsigned long long vb[kMaxWords];  // valid-tile bits, tile order
  __shared__ int wpre[kMaxWords + 1];            // valid tiles before each word
  const int lane = threadIdx.x;
  for (int q0 = 0; q0 < nwords; q0 += 8 * 64) {
    unsigned long long r[8];  // eight loads in flight per lane
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = vbg[min(q0 + u * 64 + lane, nwords - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int wi = q0 + u * 64 + lane;
      if (wi < nwords) vb[wi] = r[u];
    }
  }
  __syncthreads();
  // exclusive prefix of the words' popcounts: lane owns a run of K words
  const int K = (nwords + 63) / 64;
  int c = 0;
  for (int j = 0; j < K; ++j) {
    const int wi = lane * K + j;
    if (wi < nwords) c += __popcll(vb[wi]);
  }
  int incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  const int N = __shfl(incl, 63);
  int run = incl - c;
  for (int j = 0; j < K; ++j) {
    const int wi = lane * K + j;
    if (wi < nwords) {
      wpre[wi] = run;
      run += __popcll(vb[wi]);
    }
  }
  if (lane == 0) wpre[nwords] = N;
  __syncthreads();
  if (blockIdx.x == 0 && lane == 0) *nmatch = N;
  const int it = blockIdx.x * kHypThreads + lane;
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
template <bool JOBS, int IPB>
__global__ __launch_bounds__(kTestThreads) void k_test(WeedJob one,
                                                       const WeedJob* __restrict__ jobs,
                                                       WeedArgs a) {
  const WeedJob J = JOBS ? jobs[blockIdx.z] : one;
  const int ntiles = J.ntiles, w = J.w, h = J.h, wstride = J.words;
  if (JOBS && (int)blockIdx.x * kTestThreads >= ntiles) return;  // past this job's tiles
  const int32_t* __restrict__ cxy = J.cxy;
  const int32_t* __restrict__ disp = J.disp;
  const uint8_t* __restrict__ flags = J.flags;
  const double* __restrict__ G = J.b.G;
  int32_t* __restrict__ cnt = J.b.cnt;
  unsigned long long* __restrict__ bal = J.b.bal;
  __shared__ double gs[IPB][8];
  __shared__ int ok[IPB];
  __shared__ int wc[IPB][kTestThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int it0 = blockIdx.y * IPB;
  // the tile, the hypotheses and their usability are loaded together
  const int t = blockIdx.x * kTestThreads + tid;
  const int tc = t < ntiles ? t : ntiles - 1;  // ntiles >= 1 here
  const uint8_t tf = flags[tc];
  const int4 mt = tile_match(cxy, disp, tc, w / 2, h / 2);
  if (tid < 8 * IPB) {  // one coefficient per thread
    const int it = min(it0 + (tid >> 3), a.iters - 1);
    gs[tid >> 3][tid & 7] = G[(size_t)it * 8 + (tid & 7)];
  }
  if (tid < IPB) {
    const int it = it0 + tid;
    // usable hypotheses start at 0 and only grow, so the sign is stable
    ok[tid] = it < a.iters && __atomic_load_n(&cnt[min(it, a.iters - 1)], __ATOMIC_RELAXED) >= 0;
  }
  __syncthreads();
  const bool valid = t < ntiles && (tf & 2);
  const int4 m = valid ? mt : make_int4(0, 0, 0, 0);
  const int word = t >> 6;
  for (int q = 0; q < IPB; ++q) {
    if (!ok[q]) continue;
    const bool in = valid && is_inlier(gs[q], m, a.eps2);
    const unsigned long long b = __ballot(in);
    if (lane == 0) {
      if (word < wstride) bal[(size_t)word * a.iters + it0 + q] = b;
      wc[q][wave] = __popcll(b);
    }
  }
  __syncthreads();
  if (tid < IPB && ok[tid]) {
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

// Wave wd of the grid owns tile word wd: union M over the accepted rows,
// flags 4 (in M) and 8 (in the fit) of its tiles, and their least-squares
// terms, added exactly to the level's sums.
template <bool JOBS>
__global__ __launch_bounds__(kUnionThreads) void k_union(WeedJob one,
                                                         const WeedJob* __restrict__ jobs,
                                                         WeedArgs a) {
  const WeedJob J = JOBS ? jobs[blockIdx.z] : one;
  const int ntiles = J.ntiles, w = J.w, h = J.h, wstride = J.words;
  if (JOBS && (int)blockIdx.x * (kUnionThreads / 64) >= wstride) return;  // past its words
  const int32_t* __restrict__ cxy = J.cxy;
  const int32_t* __restrict__ disp = J.disp;
  uint8_t* __restrict__ flags = J.flags;
  const int32_t* __restrict__ nmatch = J.b.nmatch;
  const int32_t* __restrict__ cnt = J.b.cnt;
  const unsigned long long* __restrict__ bal = J.b.bal;
  long long* __restrict__ sums = J.b.sums;
  int32_t* __restrict__ counts = J.counts;
  __shared__ unsigned int accw[kMaxIters / 32];  // accepted iterations
  __shared__ unsigned long long kmax[kUnionThreads / 64];
  __shared__ long long part[kUnionThreads / 64][kSums];
  constexpr int NWV = kUnionThreads / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wd = blockIdx.x * NWV + wave;
  const int t = wd * 64 + lane;
  const bool in = wd < wstride && t < ntiles;
  // this lane's tile, in flight with the counts
  const uint8_t tf = in ? flags[t] : 0;
  const int tpx = in ? cxy[2 * t] : 0, tpy = in ? cxy[2 * t + 1] : 0;
  const int tdx = in ? disp[2 * t] : 0, tdy = in ? disp[2 * t + 1] : 0;
  const int N = *nmatch;
  const int delta = weed_delta(N, a);
  // per-iteration counts -> acceptance bits and the best key
  unsigned long long kb = 0ull;
  for (int i0 = 0; i0 < a.iters; i0 += 2 * kUnionThreads) {
    int c[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {  // loads in flight with the match count
      const int i = i0 + r * kUnionThreads + tid;
      c[r] = cnt[min(i, a.iters - 1)];
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int i = i0 + r * kUnionThreads + tid;
      if (i >= a.iters || N < 4) c[r] = -1;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int i = i0 + r * kUnionThreads + tid;
      const int ib = i0 + r * kUnionThreads + wave * 64;
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
  if (blockIdx.x == 0 && tid == 0) {
    counts[0] = N;
    counts[2] = bc;
    counts[3] = bi;
  }
  long long s[kSums];
#pragma unroll
  for (int i = 0; i < kSums; ++i) s[i] = 0;
  if (wd < wstride) {  // whole waves
    const unsigned long long brow = fit ? bal[(size_t)wd * a.iters + bi] : 0ull;
    unsigned long long v = 0ull;
    for (int i0 = 0; i0 < a.iters; i0 += 64 * 16) {
      unsigned long long r[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = i0 + u * 64 + lane;
        r[u] = bal[(size_t)wd * a.iters + min(i, a.iters - 1)];  // used only if i < iters
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = i0 + u * 64 + lane;
        if (i < a.iters && ((accw[i >> 5] >> (i & 31)) & 1u)) v |= r[u];
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    if (in && (tf & 2)) {
      const bool inM = (v >> lane) & 1ull;
      const bool sel = (brow >> lane) & 1ull;
      flags[t] = (uint8_t)((tf & 0x13) | (inM ? 4 : 0) | (sel ? 8 : 0));
      if (sel) {
        // normal equations of G: (x, y) -> (u, v), reference side to source
        // side; the 8x8 matrix has 23 distinct sums
        const long long x = tpx - w / 2, y = tpy - h / 2, u = x + tdx, vv = y + tdy;
        const long long xx = x * x, xy = x * y, yy = y * y, q = u * u + vv * vv;
        s[0] = 1;        s[1] = x;        s[2] = y;
        s[3] = xx;       s[4] = xy;       s[5] = yy;
        s[6] = u;        s[7] = vv;
        s[8] = x * u;    s[9] = y * u;    s[10] = x * vv;  s[11] = y * vv;
        s[12] = xx * u;  s[13] = xy * u;  s[14] = yy * u;
        s[15] = xx * vv; s[16] = xy * vv; s[17] = yy * vv;
        s[18] = x * q;   s[19] = y * q;
        s[20] = xx * q;  s[21] = xy * q;  s[22] = yy * q;
      }
    }
  }
  // exact (order-free) int64 reduction
  if (__ballot(s[0] != 0)) {
#pragma unroll
    for (int i = 0; i < kSums; ++i) s[i] = wave_sum_i64(s[i]);
  }
  if (lane == 0)
    for (int i = 0; i < kSums; ++i) part[wave][i] = s[i];
  __syncthreads();
  if (tid < kSums) {
    long long z = 0;
    for (int q = 0; q < NWV; ++q) z += part[q][tid];
    if (z != 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(sums + tid), (unsigned long long)z);
  }
}

// The level fit from the sums (A^T A and A^T b of the rows
// (x, y, 1, 0, 0, 0, -xu, -yu | u) and (0, 0, 0, x, y, 1, -xv, -yv | v),
// scaled by powers of two), solved by one lane with the matrix in registers,
// then H_l = Hbase o G with Hbase = H_{l+1} (matches relative to the warped
// source) or the identity (absolute matches); H_l = H_{l+1} when fewer than
// 4 matches were fitted or the solve fails.
template <bool JOBS>
__global__ __launch_bounds__(64) void k_solve(WeedJob one, const WeedJob* __restrict__ jobs) {
  const WeedJob J = JOBS ? jobs[blockIdx.z] : one;
  const int w = J.w, h = J.h;
  const long long* __restrict__ sums = J.b.sums;
  const double* __restrict__ Hprev = J.Hprev;
  const double* __restrict__ Hbase = J.Hbase;
  double* __restrict__ Hout = J.Hout;
  int32_t* __restrict__ counts = J.counts;
  __shared__ long long tot[kSums];
  const int lane = threadIdx.x;
  if (lane < kSums) tot[lane] = sums[lane];
  double Hp[9], Hb[9];  // loaded with the sums
  for (int i = 0; i < 9; ++i) Hp[i] = Hprev[i];
  for (int i = 0; i < 9; ++i) Hb[i] = Hbase[i];
  __syncthreads();
  if (J.clear_vb) {  // the next level's search sets bits and its weeding adds sums
    for (int i = lane; i < J.clear_words; i += 64) J.clear_vb[i] = 0ull;
    if (lane < 24) J.b.sums[lane] = 0;
  }
  if (lane != 0) return;
  const int msel = (int)tot[0];
  counts[1] = msel;
  for (int i = 0; i < 9; ++i) Hout[i] = Hp[i];
  if (msel < 4) return;
  const int ox = w / 2, oy = h / 2;
  int k = 0;
  const int mx = ox > oy ? (ox > 1 ? ox : 1) : (oy > 1 ? oy : 1);
  while ((1 << k) < mx) ++k;
  const int deg[8] = {1, 1, 0, 1, 1, 0, 2, 2};
  double A[72];
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const long long v = j < 8 ? normal_entry(tot, r, j) : normal_rhs(tot, r);
      const int e = j < 8 ? -k * (deg_of(r) + deg[j]) : -k * (deg_of(r) + 1);
      A[r * 9 + j] = ldexp((double)v, e);
    }
  double hs[8];
  if (!solve8(A, hs)) return;
  double Gc[9];
  for (int i = 0; i < 8; ++i) Gc[i] = ldexp(hs[i], k * (1 - deg[i]));
  Gc[8] = 1.0;
  const double pox = (double)(2 * ox - (w - 1)), poy = (double)(2 * oy - (h - 1));
  const double Pm[9] = {2, 0, pox, 0, 2, poy, 0, 0, (double)w};
  const double Qm[9] = {(double)w, 0, -pox, 0, (double)w, -poy, 0, 0, 2};
  double T1[9], T2[9], T3[9];
  mat3_mul(Pm, Gc, T1);
  mat3_mul(T1, Qm, T2);
  mat3_mul(Hb, T2, T3);
  const double d = T3[8];
  if (d == 0.0) return;
  double Hn[9];
  for (int i = 0; i < 9; ++i) {
    Hn[i] = T3[i] / d;
    if (!isfinite(Hn[i])) return;
  }
  for (int i = 0; i < 9; ++i) Hout[i] = Hn[i];
}

WeedArgs weed_args(const lnr_params& p, int level) {
  WeedArgs a;
  a.iters = p.weed_iters;
  a.level = level;
  a.delta_min = p.weed_delta_min;
  a.delta_pct = p.weed_delta_pct;
  a.eps2 = p.weed_eps * p.weed_eps;
  a.seed = p.seed;
  return a;
}

}  // namespace

hipError_t launch_weed_fit(const int32_t* corner_xy, const int32_t* disp, uint8_t* flags,
                           int ntiles, int w, int h, int level, const lnr_params& p,
                           const double* H_prev, double* H_out, int32_t* counts,
                           const WeedBufs& b, hipStream_t st, bool vb_ready,
                           const double* H_base, int clear_words) {
  const WeedArgs a = weed_args(p, level);
  const int words = ntiles > 0 ? (ntiles + 63) / 64 : 1;
  const int chunks = ntiles > 0 ? (ntiles + kTestThreads - 1) / kTestThreads : 1;
  const int ipb = ntiles <= kTestSmall ? 4 : 8;
  const int groups = (a.iters + ipb - 1) / ipb;
  if (words > kMaxWords || a.iters > kMaxIters) return hipErrorInvalidValue;
  WeedJob J;
  J.cxy = corner_xy; J.disp = disp; J.flags = flags;
  J.ntiles = ntiles; J.w = w; J.h = h; J.words = words;
  J.b = b;
  J.Hprev = H_prev; J.Hbase = H_base ? H_base : H_prev; J.Hout = H_out; J.counts = counts;
  J.clear_vb = clear_words > 0 ? b.vb : nullptr;
  J.clear_words = clear_words;
  hipError_t e;
  if (!vb_ready) {  // else the level's search set the bits (and its warp cleared the sums)
    LNR_LAUNCH(k_valid, dim3((words + kValidThreads / 64 - 1) / (kValidThreads / 64)),
               dim3(kValidThreads), 0, st, flags, ntiles, words, b.vb, b.sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  LNR_LAUNCH(k_hyp<false>, dim3((a.iters + kHypThreads - 1) / kHypThreads), dim3(kHypThreads), 0,
             st, J, nullptr, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ntiles > 0) {
    if (ipb == 4)
      LNR_LAUNCH((k_test<false, 4>), dim3(chunks, groups), dim3(kTestThreads), 0, st, J, nullptr,
                 a);
    else
      LNR_LAUNCH((k_test<false, 8>), dim3(chunks, groups), dim3(kTestThreads), 0, st, J, nullptr,
                 a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  LNR_LAUNCH(k_union<false>, dim3((words + kUnionThreads / 64 - 1) / (kUnionThreads / 64)),
             dim3(kUnionThreads), 0, st, J, nullptr, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  LNR_LAUNCH(k_solve<false>, dim3(1), dim3(64), 0, st, J, nullptr);
  return hipGetLastError();
}

hipError_t launch_weed_jobs(const WeedJob* jobs, int njobs, int max_tiles, int level,
                            const lnr_params& p, hipStream_t st) {
  if (njobs < 1) return hipSuccess;
  const WeedArgs a = weed_args(p, level);
  const int words = max_tiles > 0 ? (max_tiles + 63) / 64 : 1;
  const int chunks = max_tiles > 0 ? (max_tiles + kTestThreads - 1) / kTestThreads : 1;
  const int ipb = max_tiles <= kTestSmall ? 4 : 8;
  const int groups = (a.iters + ipb - 1) / ipb;
  if (words > kMaxWords || a.iters > kMaxIters) return hipErrorInvalidValue;
  WeedJob none{};
  hipError_t e;
  LNR_LAUNCH(k_hyp<true>, dim3((a.iters + kHypThreads - 1) / kHypThreads, 1, njobs),
             dim3(kHypThreads), 0, st, none, jobs, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ipb == 4)
    LNR_LAUNCH((k_test<true, 4>), dim3(chunks, groups, njobs), dim3(kTestThreads), 0, st, none,
               jobs, a);
  else
    LNR_LAUNCH((k_test<true, 8>), dim3(chunks, groups, njobs), dim3(kTestThreads), 0, st, none,
               jobs, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  LNR_LAUNCH(k_union<true>,
             dim3((words + kUnionThreads / 64 - 1) / (kUnionThreads / 64), 1, njobs),
             dim3(kUnionThreads), 0, st, none, jobs, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  LNR_LAUNCH(k_solve<true>, dim3(1, 1, njobs), dim3(64), 0, st, none, jobs);
  return hipGetLastError();
}

}  // namespace lnr
