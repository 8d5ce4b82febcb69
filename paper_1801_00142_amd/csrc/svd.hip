// Singular value decomposition by one-sided (Hestenes) block Jacobi, FP64.
//
// The columns of Y (len x p, column-major) are made mutually orthogonal by
// plane rotations from the right, Y V = Z.  The column norms of Z are the
// singular values and the normalised columns the left singular vectors.
// Columns are grouped into blocks of 16 by norm rank; each outer round pairs
// every block with one other block (round-robin tournament, all pairs met
// once per sweep) and one workgroup per block pair orthogonalises its 32
// columns (32 x 32 Gram from the columns on the matrix cores, one sweep of
// small Jacobi on it, one rotation pass).  Sweeps repeat until no pair in a
// sweep needs a rotation.  Several independent problems run in one grouped
// launch per round (blockIdx.y = problem).
//
// Accuracy: the Gram entries are recomputed from the rotated columns at
// every visit and the stopping test is on those fresh cosines, so singular
// values and vectors are resolved to absolute accuracy ~ eps * sigma_1, which
// the thermal-state compression needs: components far below
// sqrt(eps) * sigma_1 carry the high-order terms of the series start and
// must not be lost (a Gram matrix of the whole Y would lose them).
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

namespace xtrg {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxSweeps = 60;
constexpr double kCheckBelow = 1e-6;   // largest cosine of a sweep below which the closing check is a GEMM

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Partner of slot x in round r of a round-robin tournament of n (even) players.
__host__ __device__ inline void rr_pair(int n, int r, int q, int* i, int* j) {
  const int m = n - 1;
  if (q == 0) {
    *i = 0;
    *j = 1 + (r % m);
  } else {
    *i = 1 + ((r + q) % m);
    *j = 1 + ((r - q + m) % m);
  }
}

// One outer round of one-sided block Jacobi.  Block pairing works on
// ranks: rank q is the column with the q-th largest norm at the start of the
// sweep (perm[q]), so each block holds columns of similar norm.  A
// workgroup owns one block pair (kNC = 32 columns):
//  1. the 32 x 32 Gram matrix of the pair is formed from the columns
//     themselves (fresh dot products every visit): 128-row chunks are staged
//     in LDS and every wave accumulates its 16 rows of each chunk on the FP64
//     matrix cores; the wave partials are summed in a fixed order;
//  2. the convergence measure is the largest cosine |z_i . z_j| / (|z_i| |z_j|)
//     of that Gram which exceeds tol; columns with |z|^2 <= zth are
//     numerically zero and take no part.  A pair with nothing to rotate is
//     left untouched;
//  3. one cyclic two-sided Jacobi sweep runs on the small Gram in LDS: 31
//     rounds of 16 disjoint rotations (round r pairs k with k ^ r), each
//     round one step for all threads (thread (q, k) rotates entries k of
//     pair q with its row partner), G ping-ponging between two buffers;
//  4. the accumulated rotation W is applied to the columns in one pass
//     (Z <- Z W).
constexpr int kWT = 576;                  // threads of a round workgroup: 8 update waves + 1 rotation wave
constexpr int kWW = kWT / 64;             // its waves
constexpr int kUW = 8;                    // update waves: Gram, G and W updates, rotation of Z
constexpr int kBlk = 16;                  // columns per block
constexpr int kNC = 2 * kBlk;             // columns per block pair
typedef double d4 __attribute__((ext_vector_type(4)));

// One Jacobi problem of a grouped launch (blockIdx.y selects the problem).
struct JacobiDesc {
  double* Z;
  const int* perm;
  const double* fro2;
  unsigned long long* off;
  double tol, zrel2;
  int len, p, nbk, active;
  int split;        // row slices per block pair (workgroups sharing one pair's round)
  int glen;         // leading rows that define the Gram matrix (<= len; the rest are only rotated)
};

// Rows [a, b) of slice s of `split` (slices start at multiples of 128 rows).
__device__ inline void slice_rows(int len, int split, int s, int* a, int* b) {
  const int per = (((len + split - 1) / split) + 127) / 128 * 128;
  *a = min(len, s * per);
  *b = min(len, *a + per);
}

// Kernel modes: one workgroup per block pair doing the whole round, or the
// round split over `split` workgroups per pair in two launches: partial
// Gram matrices of row slices, then (every slice alike) the sum of the
// partials in slice order, the small Jacobi sweep, and the rotation of the
// slice's rows.  The slices depend only on the column length and the fused
// workgroup sums the same slice partials in the same order, so both modes
// give identical results and a chain gets the same result alone and in a
// batch.
enum { ROUND_FUSED = 0, ROUND_GRAM = 1, ROUND_ROTATE = 2 };
constexpr int kMaxSplit = 4;
constexpr int kMaxPairs = 128;            // p <= 4096 columns in blocks of 16
constexpr int kGramVals = 3 * 256;        // three 16 x 16 tiles

// 1/sqrt(x) from the hardware estimate (relative error ~5e-8) refined by
// one third-order step: with r = 1 - x y^2, x^(-1/2) = y (1 - r)^(-1/2)
// = y (1 + r/2 + 3r^2/8 + O(r^3)); the truncation is ~1e-22, the result is
// within a few ulp (r is formed by one fused multiply-add).
__device__ inline double rsq_refined(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double r = fma(-x * y, y, 1.0);
  return fma(y * r, fma(0.375, r, 0.5), y);
}

// The power of two that brings ||Y||_F^2 into [1/2, 1) (1 if it is zero or
// not finite).  Every Gram entry is at most ||Y||_F^2, so entries times it
// are at most 1 in magnitude and products of two of them cannot overflow;
// the scaling is exact, so every test and ratio formed from scaled entries
// is the one formed from the entries themselves wherever those do not
// overflow or underflow.
__device__ inline double gram_scale(double fro2) {
  int e;
  (void)frexp(fro2, &e);
  return fro2 > 0.0 && isfinite(fro2) ? ldexp(1.0, -e) : 1.0;
}

// Whether the pair with Gram entries [[a, g], [g, b]] needs a rotation:
// both columns above the numerical-zero threshold zth and the cosine
// |g| / sqrt(a b) above tol (tested as g^2 > tol^2 a b on the entries times
// fsc = gram_scale(||Y||_F^2)).  The convergence measure and the rotations
// use this one test.
__device__ inline bool needs_rot(double a, double b, double g, double tol2, double zth, double fsc) {
  const double as = a * fsc, bs = b * fsc, gs = g * fsc;
  return a > zth && b > zth && gs * gs > tol2 * (as * bs);
}

// Squared cosine g^2 / (a b) of a pair, from the scaled entries.
__device__ inline double cos2(double a, double b, double g, double fsc) {
  const double gs = g * fsc;
  return gs * gs / ((a * fsc) * (b * fsc));
}

// Rotation (c, s) that zeroes the off-diagonal of [[a, g], [g, b]] under
// columns x' = c x - s y, y' = s x + c y (the smaller of the two angles,
// tan = sign(d) h / (|d| + r) with d = b - a, h = 2g, r = |(d, h)|), in the
// form c = sqrt(u / 2r), s = sign(d) h / sqrt(2 r u), u = |d| + r, which
// needs one square root and one reciprocal square root in sequence (no
// cancellation: u >= r).  d and h are first multiplied by
// fsc = gram_scale(||Y||_F^2), so |d| < 1 and |h| < 2, and a pair that
// needs a rotation has |h| > 2 tol zth (a fixed fraction ~1e-38 of
// ||Y||_F^2): the squares can neither overflow nor underflow.
// c^2 + s^2 = 1 to a few ulp.  Identity if the pair needs none.
// Branch-free (the value is selected at the end), so that two rotations in
// one thread interleave their chains.
__device__ inline void jacobi_rot(double a, double b, double g, double tol2, double zth, double fsc, double* c,
                                  double* s) {
  const bool need = needs_rot(a, b, g, tol2, zth, fsc);
  // computed whether or not it is needed (a pair that needs none may give
  // NaN here, which the selection drops), so that the test is not on the
  // chain of the square roots
  const double d = b * fsc - a * fsc, h = 2.0 * (g * fsc);
  const double x = fma(d, d, h * h);
  const double r = x * rsq_refined(x);
  const double u = fabs(d) + r;
  const double q = rsq_refined(2.0 * r * u);
  *c = need ? u * q : 1.0;
  *s = need ? copysign(1.0, d) * h * q : 0.0;
}

// Members of pair qq in XOR round rr (rr = 1 .. kNC-1, qq = 0 .. kNC/2-1):
// x = qq with a zero bit inserted at the highest set bit h of rr, y = x ^ rr.
// The kNC - 1 rounds of kNC/2 disjoint pairs each cover every pair once.
__device__ inline int xor_pair_x(int rr, int qq) {
  const int h = 31 - __clz(rr);
  return ((qq >> h) << (h + 1)) | (qq & ((1 << h) - 1));
}

template <int MODE>
__global__ __launch_bounds__(kWT) void jacobi_round(const JacobiDesc* __restrict__ descs, int r, int smax,
                                                    double* __restrict__ parts) {
  const int pair = (int)blockIdx.x / smax, sl = (int)blockIdx.x % smax;
  // A rotate launch's Gram values (this thread's entries of the slices'
  // partials) sit at addresses fixed by the launch alone: their loads go out
  // before the descriptor is read.  Every slot up to kMaxSplit is allocated;
  // those past the problem's split are loaded and not used.
  double* __restrict__ part = parts + ((size_t)blockIdx.y * kMaxPairs + pair) * kMaxSplit * kGramVals;
  double pq[2][kMaxSplit];
  if (MODE == ROUND_ROTATE) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int idx = threadIdx.x + k * kWT;
#pragma unroll
      for (int s2 = 0; s2 < kMaxSplit; ++s2) pq[k][s2] = idx < kGramVals ? part[s2 * kGramVals + idx] : 0.0;
    }
  }
  const JacobiDesc d = descs[blockIdx.y];
  const int split = d.split;
  if (!d.active || r >= d.nbk - 1 || pair >= d.nbk / 2 || sl >= (MODE == ROUND_FUSED ? 1 : split)) return;
  int ra = 0, rb = d.len;                       // rows this workgroup rotates
  if (MODE != ROUND_FUSED) slice_rows(d.len, split, sl, &ra, &rb);
  int ga = 0, gb = d.glen;                      // rows of its Gram partial
  if (MODE == ROUND_GRAM) slice_rows(d.glen, split, sl, &ga, &gb);
  // every pointer of the descriptor is read through its global view, so
  // that the tiles loaded before the small Jacobi sweep stay in flight
  // through its barriers
  const auto Y = gptr(d.Z);
  const int len = d.len, p = d.p, nbk = d.nbk;
  const double tol = d.tol;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // ||Y||_F^2 for the zero threshold (its latency overlaps the column
  // lookup) and, in a rotate launch, the Gram values: the slices' partials
  // summed in slice order
  const double fro2v = MODE == ROUND_GRAM ? 0.0 : gptr(d.fro2)[0];
  double pv[2] = {0.0, 0.0};
  if (MODE == ROUND_ROTATE) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int idx = t + k * kWT;
      if (idx < kGramVals) {
        double v = pq[k][0];
#pragma unroll
        for (int s2 = 1; s2 < kMaxSplit; ++s2)
          if (s2 < split) v += pq[k][s2];
        pv[k] = v;
      }
    }
  }
  __shared__ int colid[kNC];
  __shared__ double buf[kUW * 3 * 4 * 64];   // wave partials of the Gram tiles
  __shared__ double gsum[kGramVals];          // fused round: running sum over the slices
  __shared__ double G[2][kNC][kNC + 1];
  __shared__ double Wt[kNC][kNC + 2];         // W transposed: Wt[c][j] = W[j][c]
  __shared__ double2 rot[2][kNC / 2];          // (c, s) of each pair of a round (double-buffered)
  __shared__ double wmax[kWW];
  __shared__ unsigned wmask[kWW];
  int bi, bj;
  rr_pair(nbk, r, pair, &bi, &bj);
  // Column of member k (0 .. kNC-1) of the pair, -1 past the last column.
  // A Gram launch's lanes look up their own columns (no LDS hop and no
  // barrier before the column loads); a rotate launch first reads colid
  // after the barrier that follows the Gram fill.
  auto col_of = [&](int k) {
    const int rank = (k < kBlk ? bi : bj) * kBlk + (k % kBlk);
    return rank < p ? gptr(d.perm)[rank] : -1;
  };
  if (MODE != ROUND_GRAM && t < kNC) colid[t] = col_of(t);
  if (MODE == ROUND_FUSED) __syncthreads();

  // 1. Gram tiles (0,0), (0,1), (1,1) of the pair on the matrix cores,
  // operands straight from memory: per MFMA step a wave takes 4 rows, lane l
  // row l/16 of column l%16 of each block (4 consecutive rows of a column
  // per 4 lanes, 32-byte sectors fully used).  The update waves interleave
  // 4-row groups (two waves per SIMD, equal shares); a group past the end
  // issues no matrix-core work (an FP64 16x16x4 product occupies a SIMD for
  // 64 cycles).  Partial Gram of rows [a, b): per-wave tiles left in buf.
  auto gram_rows = [&](int a, int b) {
    if (wave >= kUW) return;
    d4 acc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
    const int lr = lane & 15, lk = lane >> 4;
    const int c0 = MODE == ROUND_GRAM ? col_of(lr) : colid[lr];
    const int c1 = MODE == ROUND_GRAM ? col_of(kBlk + lr) : colid[kBlk + lr];
    const auto y0 = Y + (long)(c0 >= 0 ? c0 : 0) * len;
    const auto y1 = Y + (long)(c1 >= 0 ? c1 : 0) * len;
    constexpr int U = 16;                      // row groups in flight per wave
    for (int g0 = a + wave * 4; g0 < b; g0 += kUW * 4 * U) {
      double a0[U], a1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = g0 + u * kUW * 4 + lk;
        a0[u] = (c0 >= 0 && e < b) ? y0[e] : 0.0;
        a1[u] = (c1 >= 0 && e < b) ? y1[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (g0 + u * kUW * 4 >= b) break;      // uniform over the wave
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], a0[u], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], a1[u], acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], a1[u], acc[2], 0, 0, 0);
      }
    }
    // register q of lane l holds tile row l/16 + 4q, column l%16
#pragma unroll
    for (int tt = 0; tt < 3; ++tt)
#pragma unroll
      for (int q = 0; q < 4; ++q) buf[((wave * 3 + tt) * 4 + q) * 64 + lane] = acc[tt][q];
  };
  auto wave_sum = [&](int idx) {
    const int tt = idx >> 8, q = (idx >> 6) & 3, l = idx & 63;
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kUW; ++w) v += buf[((w * 3 + tt) * 4 + q) * 64 + l];
    return v;
  };

  // The Gram matrix is the sum, in slice order, of the slices' partials
  // (each the sum over waves in wave order), whichever way the round runs:
  // the fused workgroup walks the slices itself.
  if (MODE == ROUND_GRAM) {
    gram_rows(ga, gb);
    __syncthreads();
    for (int idx = t; idx < kGramVals; idx += kWT) part[sl * kGramVals + idx] = wave_sum(idx);
    return;
  }
  if (MODE == ROUND_FUSED) {
    for (int s2 = 0; s2 < split; ++s2) {
      int a2, b2;
      slice_rows(d.glen, split, s2, &a2, &b2);
      gram_rows(a2, b2);
      __syncthreads();
      for (int idx = t; idx < kGramVals; idx += kWT) {
        const double v = wave_sum(idx);
        gsum[idx] = s2 == 0 ? v : gsum[idx] + v;
      }
      __syncthreads();
    }
  }
  for (int idx = t; idx < kNC * kNC; idx += kWT) Wt[idx / kNC][idx % kNC] = (idx / kNC == idx % kNC) ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int idx = t + k * kWT;
    if (idx >= kGramVals) break;
    const int tt = idx >> 8, q = (idx >> 6) & 3, l = idx & 63;
    const double v = MODE == ROUND_ROTATE ? pv[k] : gsum[idx];
    const int i = (l >> 4) + 4 * q, j = l & 15;
    const int I = tt == 2 ? kBlk : 0, J = tt == 0 ? 0 : kBlk;
    if (tt == 1) {
      G[0][I + i][J + j] = v;
      G[0][J + j][I + i] = v;
    } else if (i <= j) {            // diagonal tiles: one triangle, mirrored
      G[0][I + i][J + j] = v;
      G[0][J + j][I + i] = v;
    }
  }
  __syncthreads();

  // 2. Convergence measure.
  const double zth = d.zrel2 * fro2v;
  const double tol2 = tol * tol;
  const double fsc = gram_scale(fro2v);
  double off = 0.0;                  // largest squared cosine
  unsigned mask = 0;                 // bit r: some pair (k, k ^ r) needs a rotation
  for (int idx = t; idx < (kNC / 2) * (kNC - 1); idx += kWT) {   // pair qq of XOR round rr
    const int rr = 1 + idx / (kNC / 2), qq = idx % (kNC / 2);
    const int x = xor_pair_x(rr, qq), y = x ^ rr;
    const double a = G[0][x][x], b = G[0][y][y], g = G[0][x][y];
    if (needs_rot(a, b, g, tol2, zth, fsc)) {
      off = fmax(off, cos2(a, b, g, fsc));
      mask |= 1u << rr;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    off = fmax(off, __shfl_xor(off, o, 64));
    mask |= __shfl_xor(mask, o, 64);
  }
  if (lane == 0) {
    wmax[wave] = off;
    wmask[wave] = mask;
  }
  __syncthreads();
  double worst = 0.0;
  mask = 0;
#pragma unroll
  for (int w = 0; w < kWW; ++w) {
    worst = fmax(worst, wmax[w]);
    mask |= wmask[w];
  }
  worst = sqrt(worst);
  // block maximum published as the bit pattern of a non-negative double
  // (monotone under unsigned comparison)
  if (t == 0 && sl == 0 && worst > 0.0)
    __hip_atomic_fetch_max(gptr(d.off), (unsigned long long)__double_as_longlong(worst), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  if (worst == 0.0) return;          // uniform: every thread read the same wmax

  // The first tiles that step 4 rotates are loaded now: their latency
  // passes during the small Jacobi sweep (no other workgroup writes them).
  constexpr int T = 2;                         // 16-row tiles in flight per update wave
  const int lr = lane & 15, lk = lane >> 4;
  int cin[kNC / 4];
#pragma unroll
  for (int kk = 0; kk < kNC / 4; ++kk) cin[kk] = colid[kk * 4 + lk];
  double zb[T][kNC / 4];
  if (wave < kUW) {
    const int e0 = ra + wave * 16;
#pragma unroll
    for (int u = 0; u < T; ++u) {
      const int e = e0 + u * kUW * 16 + lr;
#pragma unroll
      for (int kk = 0; kk < kNC / 4; ++kk) zb[u][kk] = (cin[kk] >= 0 && e < rb) ? Y[(long)cin[kk] * len + e] : 0.0;
    }
  }

  // 3. One sweep of parallel two-sided Jacobi on G; W <- W J per rotation.
  // The 16 rotations of a round are computed once (one thread per pair) and
  // read by all; the threads that compute them work one round ahead: from
  // G before round r and round r's rotations they form the three entries of
  // G after round r that fix their pair's rotation in the next round, so the
  // rotation chains overlap the updates and a round costs one barrier.
  // Waves 0-3 update G (thread (qc, lo): the 2 x 2 block of G on the rows
  // of pair lo and the columns of pair qc), waves 4-7 update W (thread
  // (qc, lo): rows lo and lo + 16 of W, columns of pair qc), lanes 0-15 of
  // wave 8 compute the rotations.
  {
    const bool gupd = t < 256, wupd = t >= 256 && t < 512;
    const int qc = (t >> 4) & 15, lo = t & 15;
    const int qr = t - 512;                   // rotation lane: pair index
    auto next_round = [&](int r0) {            // next round after r0 with a rotation, 0 if none
      const unsigned later = mask & ~((2u << r0) - 1u);
      return later ? __builtin_ctz(later) : 0;
    };
    auto pair_x = [](int rr, int qq) { return xor_pair_x(rr, qq); };
    // pair index of member a in round rr
    auto pair_of = [](int rr, int a) {
      const int h = 31 - __clz(rr);
      const int am = min(a, a ^ rr);
      return ((am >> (h + 1)) << h) | (am & ((1 << h) - 1));
    };
    int rc = next_round(0);
    if (qr >= 0 && qr < kNC / 2 && rc) {
      const int x = pair_x(rc, qr), y = x ^ rc;
      double c, sn;
      jacobi_rot(G[0][x][x], G[0][y][y], G[0][x][y], tol2, zth, fsc, &c, &sn);
      rot[0][qr] = make_double2(c, sn);
    }
    __syncthreads();
    int src = 0, rb = 0;
    while (rc) {
      const int rn = next_round(rc);
      if (gupd) {
        const int x = pair_x(rc, qc), y = x ^ rc;     // columns
        const int k = pair_x(rc, lo), kb = k ^ rc;    // rows, k < kb
        const double2 cs = rot[rb][qc], cs2 = rot[rb][lo];
        const double c = cs.x, sn = cs.y, c2 = cs2.x, s2 = cs2.y;
        const double gkx = G[src][k][x], gky = G[src][k][y];
        const double gbx = G[src][kb][x], gby = G[src][kb][y];
        const double hkx = c * gkx - sn * gky, hky = sn * gkx + c * gky;   // columns rotated
        const double hbx = c * gbx - sn * gby, hby = sn * gbx + c * gby;
        G[src ^ 1][k][x] = c2 * hkx - s2 * hbx;                              // then rows
        G[src ^ 1][k][y] = c2 * hky - s2 * hby;
        G[src ^ 1][kb][x] = s2 * hkx + c2 * hbx;
        G[src ^ 1][kb][y] = s2 * hky + c2 * hby;
      } else if (wupd) {
        const int x = pair_x(rc, qc), y = x ^ rc;
        const double2 cs = rot[rb][qc];
        const double c = cs.x, sn = cs.y;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = lo + 16 * h;
          const double wx = Wt[x][k], wy = Wt[y][k];
          Wt[x][k] = c * wx - sn * wy;
          Wt[y][k] = sn * wx + c * wy;
        }
      } else if (qr < kNC / 2 && rn) {
        // entry (a, b) of G after round rc: sum over i in {a, a^rc}, j in
        // {b, b^rc} of J[i][a] G[i][j] J[j][b]; column a of J holds
        // (u, v) = (c, -s) on rows (a, a^rc) if a is the smaller member of
        // its pair, (c, s) if it is the larger.  Every LDS value is read
        // first, in one batch (one LDS latency on the rotation chain).
        const int xn = pair_x(rn, qr), yn = xn ^ rn;
        const int xr = xn ^ rc, yr = yn ^ rc;
        const int qx = pair_of(rc, xn), qy = pair_of(rc, yn);
        const double2 csx = rot[rb][qx], csy = rot[rb][qy];
        const double cx = csx.x, sx = csx.y, cy = csy.x, sy = csy.y;
        const double gxx = G[src][xn][xn], gxX = G[src][xn][xr], gXx = G[src][xr][xn], gXX = G[src][xr][xr];
        const double gyy = G[src][yn][yn], gyY = G[src][yn][yr], gYy = G[src][yr][yn], gYY = G[src][yr][yr];
        const double gxy = G[src][xn][yn], gxY = G[src][xn][yr], gXy = G[src][xr][yn], gXY = G[src][xr][yr];
        const double ux = cx, vx = xn < xr ? -sx : sx;
        const double uy = cy, vy = yn < yr ? -sy : sy;
        const double na = ux * (ux * gxx + vx * gxX) + vx * (ux * gXx + vx * gXX);
        const double nb = uy * (uy * gyy + vy * gyY) + vy * (uy * gYy + vy * gYY);
        const double ng = ux * (uy * gxy + vy * gxY) + vx * (uy * gXy + vy * gXY);
        double c, sn;
        jacobi_rot(na, nb, ng, tol2, zth, fsc, &c, &sn);
        rot[rb ^ 1][qr] = make_double2(c, sn);
      }
      src ^= 1;
      rb ^= 1;
      rc = rn;
      __syncthreads();
    }
  }

  // 4. Z <- Z W on this pair's columns, as (Z W)^T = W^T Z^T on the matrix
  // cores: W^T (the A operand) stays in registers, each update wave takes
  // 16-row tiles of Z (the B operand, 16 consecutive rows of a column per 16
  // lanes; tile k to wave k mod 8, no products for tiles past the end) and
  // writes the rotated rows back in place (no other wave touches them).
  if (wave < kUW) {
    double wa[2][kNC / 4];
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int kk = 0; kk < kNC / 4; ++kk) wa[I][kk] = Wt[I * 16 + lr][kk * 4 + lk];
    int cout[2][4];
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int q = 0; q < 4; ++q) cout[I][q] = colid[I * 16 + lk + 4 * q];
    for (int e0 = ra + wave * 16; e0 < rb; e0 += kUW * 16 * T) {
      if (e0 != ra + wave * 16) {              // later tiles (the first are loaded)
#pragma unroll
        for (int u = 0; u < T; ++u) {
          const int e = e0 + u * kUW * 16 + lr;
#pragma unroll
          for (int kk = 0; kk < kNC / 4; ++kk)
            zb[u][kk] = (cin[kk] >= 0 && e < rb) ? Y[(long)cin[kk] * len + e] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < T; ++u) {
        if (e0 + u * kUW * 16 >= rb) break;    // uniform over the wave
        const int e = e0 + u * kUW * 16 + lr;
        d4 o[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
        for (int kk = 0; kk < kNC / 4; ++kk) {
          o[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[0][kk], zb[u][kk], o[0], 0, 0, 0);
          o[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[1][kk], zb[u][kk], o[1], 0, 0, 0);
        }
        // register q of lane l: column I*16 + l/16 + 4q of Z W, row e
        if (e < rb) {
#pragma unroll
          for (int I = 0; I < 2; ++I)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (cout[I][q] >= 0) Y[(long)cout[I][q] * len + e] = o[I][q];
        }
      }
    }
  }
}

// Largest cosine over all column pairs x < y of Z from G = Z^T Z (p x p,
// row-major), with the rotation test of the rounds, into *off (bit
// pattern of a non-negative double; 0 if no pair needs a rotation).
__global__ __launch_bounds__(256) void gram_check(const double* __restrict__ G, int p, double tol2, double zrel2,
                                                  const double* __restrict__ fro2, unsigned long long* off) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  double worst = 0.0;
  if (idx < (long)p * p) {
    const int x = (int)(idx / p), y = (int)(idx % p);
    if (y > x) {
      const double a = G[(long)x * p + x], b = G[(long)y * p + y], g = G[(long)x * p + y];
      const double f2 = fro2[0], fsc = gram_scale(f2);
      if (needs_rot(a, b, g, tol2, zrel2 * f2, fsc)) worst = cos2(a, b, g, fsc);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) worst = fmax(worst, __shfl_xor(worst, o, 64));
  if ((threadIdx.x & 63) == 0 && worst > 0.0) atomicMax(off, (unsigned long long)__double_as_longlong(sqrt(worst)));
}

// Norms of the columns of Y (stride len) over their first glen rows.
__global__ void column_norms(const double* __restrict__ Y, int len, int glen, int p, double* __restrict__ out) {
  const int col = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col >= p) return;
  const double* c = Y + (long)col * len;
  double s = 0.0;
  for (int e = lane; e < glen; e += 64) s = fma(c[e], c[e], s);
  s = wave_sum(s);
  if (lane == 0) out[col] = sqrt(s);
}

// *out = sum of x[i]^2 for i < n, one workgroup, a fixed summation order.
__global__ __launch_bounds__(256) void sum_squares_ordered(const double* __restrict__ x, int n,
                                                           double* __restrict__ out) {
  __shared__ double part[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v = fma(x[i], x[i], v);
  part[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

// Descending bitonic sort of (value, index) in one workgroup, n <= 4096:
// larger value first, ties by smaller index (deterministic).  sm holds
// pow2(p) doubles and as many ints.
__device__ inline void sort_desc_body(const double* __restrict__ val, int p, double* __restrict__ sorted,
                                      int* __restrict__ perm, unsigned char* sm) {
  int n = 1;
  while (n < p) n <<= 1;
  double* v = reinterpret_cast<double*>(sm);
  int* ix = reinterpret_cast<int*>(v + n);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    v[i] = i < p ? val[i] : -1.0;
    ix[i] = i < p ? i : 0x7fffffff;
  }
  __syncthreads();
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool desc = (i & k) == 0;
          const bool i_first = (v[i] > v[l]) || (v[i] == v[l] && ix[i] < ix[l]);
          if (desc != i_first) {
            const double tv = v[i]; v[i] = v[l]; v[l] = tv;
            const int ti = ix[i]; ix[i] = ix[l]; ix[l] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    sorted[i] = v[i];
    perm[i] = ix[i];
  }
}

__global__ __launch_bounds__(1024) void sort_desc(const double* __restrict__ val, int p,
                                                   double* __restrict__ sorted, int* __restrict__ perm) {
  extern __shared__ unsigned char sm[];
  sort_desc_body(val, p, sorted, perm, sm);
}

// The ranking of every active problem of a grouped SVD at once
// (blockIdx.y, or blockIdx.x for the one-workgroup kernels, selects the
// problem; per problem the arithmetic of column_norms and sort_desc above,
// so the same bits): column norms over the Gram rows, their descending
// order, and how many of them have norm^2 > zth / 2 (the margin keeps every
// column that a Gram diagonal could find above zth; the others are never
// rotated again).
// Problem workspace: Z (len x p), then raw norms, sorted norms, order.
__global__ void column_norms_group(const JacobiDesc* __restrict__ descs) {
  const JacobiDesc& D = descs[blockIdx.y];
  if (!D.active) return;
  const int col = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col >= D.p) return;
  const double* c = D.Z + (long)col * D.len;
  double s = 0.0;
  for (int e = lane; e < D.glen; e += 64) s = fma(c[e], c[e], s);
  s = wave_sum(s);
  if (lane == 0) D.Z[(long)D.len * D.p + col] = sqrt(s);
}

__global__ __launch_bounds__(1024) void sort_desc_group(const JacobiDesc* __restrict__ descs) {
  const JacobiDesc& D = descs[blockIdx.x];
  if (!D.active) return;
  extern __shared__ unsigned char sm[];
  const int p = D.p;
  double* raw = D.Z + (long)D.len * p;
  sort_desc_body(raw, p, raw + p, reinterpret_cast<int*>(raw + 2 * (long)p), sm);
}

__global__ __launch_bounds__(256) void count_alive_group(const JacobiDesc* __restrict__ descs,
                                                         int* __restrict__ out, double* __restrict__ f2out) {
  const JacobiDesc& D = descs[blockIdx.x];
  if (!D.active) return;
  __shared__ int part[256];
  const double* sorted = D.Z + (long)D.len * D.p + D.p;
  const double th = 0.5 * D.zrel2 * D.fro2[0];
  int c = 0;
  for (int i = threadIdx.x; i < D.p; i += 256) c += sorted[i] * sorted[i] > th;
  part[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[blockIdx.x] = part[0];
    f2out[blockIdx.x] = D.fro2[0];   // ||Y||_F^2 of the problem, for the host's finiteness check
  }
}

// U column j = Z column perm[j] / sigma[j] (zero if sigma[j] == 0).
__global__ void gather_columns(const double* __restrict__ Z, int len, const double* __restrict__ sigma,
                               const int* __restrict__ perm, int k, double* __restrict__ U, long ldu,
                               int rowmajor) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)len * k) return;
  const int j = (int)(idx / len), e = (int)(idx % len);
  const double s = sigma[j];
  const double v = s > 0.0 ? Z[(long)perm[j] * len + e] / s : 0.0;
  if (rowmajor) U[(long)e * ldu + j] = v;
  else U[(long)j * ldu + e] = v;
}


}  // namespace

// work layout: [Z: len*p][sigma_raw: p][sigma: p][perm: p ints][offmax: 1][fro2: 1][part: 1024]
size_t svd_work(int len, int p) { return (size_t)len * p + 3 * (size_t)p + 1040; }

static double* sv_sorted(double* work, int len, int p) { return work + (size_t)len * p + p; }
static int* sv_perm(double* work, int len, int p) {
  return reinterpret_cast<int*>(work + (size_t)len * p + 2 * (size_t)p);
}

// [descs: n][off: n][||Y||_F^2: n doubles][alive: n ints][pad to 256 B]
// [Gram partials: n x kMaxPairs x kMaxSplit x kGramVals doubles]
static size_t parts_offset(int n) {
  return (sizeof(JacobiDesc) * (size_t)n + sizeof(unsigned long long) * (size_t)n + sizeof(double) * (size_t)n +
          sizeof(int) * (size_t)n + 255) /
         256 * 256;
}
size_t svd_desc_bytes(int n) {
  return parts_offset(n) + sizeof(double) * (size_t)n * kMaxPairs * kMaxSplit * kGramVals;
}

static int pow2_at_least(int p) {
  int n = 1;
  while (n < p) n <<= 1;
  return n;
}

// Row slices per block pair: long columns are split so that one round of a
// single chain spreads over more compute units.
static int split_for(int len) { return len >= 1024 ? 4 : len >= 512 ? 2 : 1; }

void svd_batched(std::vector<SvdJob>& jobs, void* desc_dev, hipStream_t s, RoundTimer* timer) {
  const int n = (int)jobs.size();
  if (n == 0) return;
  JacobiDesc* d_desc = reinterpret_cast<JacobiDesc*>(desc_dev);
  unsigned long long* d_off = reinterpret_cast<unsigned long long*>(d_desc + n);
  double* d_f2 = reinterpret_cast<double*>(d_off + n);
  int* d_alive = reinterpret_cast<int*>(d_f2 + n);
  double* d_parts = reinterpret_cast<double*>(static_cast<char*>(desc_dev) + parts_offset(n));
  std::vector<JacobiDesc> h(n);
  std::vector<int> n2(n);
  int max_nbk = 0, max_half = 0;
  for (int j = 0; j < n; ++j) {
    SvdJob& J = jobs[j];
    J.sweeps = 0;
    J.status = 0;
    JacobiDesc& D = h[j];
    D = JacobiDesc{};
    D.len = J.len;
    D.p = J.p;
    const int glen = J.glen > 0 ? J.glen : J.len;
    if (glen > J.len) throw Error(-1, "svd: Gram rows beyond the column length");
    D.glen = glen;
    if (J.len <= 0 || J.p <= 0) continue;
    if (J.len > 4096) throw Error(-1, "svd: column length above 4096");
    if (J.p > 4096) throw Error(-1, "svd: more than 4096 columns");
    double* w = J.work;
    D.Z = w;
    D.perm = sv_perm(w, J.len, J.p);
    D.fro2 = w + (size_t)J.len * J.p + 3 * (size_t)J.p + 1;
    D.off = d_off + j;
    D.tol = 8.0 * std::sqrt((double)glen) * 2.220446049250313e-16;
    // Columns below a quarter of the keep floor are numerically zero: they
    // are neither rotated nor counted for convergence.  Columns of pure
    // rounding noise (the null space of a rank-deficient Y) otherwise never
    // settle, since every rotation leaves them a fresh O(1) relative error.
    // The margin to the keep floor lets content near the floor that is still
    // spread over several columns be gathered before the count is taken.
    const double zrel = 0.25 * svd_keep_rel(glen, J.p);
    D.zrel2 = zrel * zrel;
    D.nbk = (J.p + kBlk - 1) / kBlk;
    if (D.nbk % 2) ++D.nbk;
    D.active = J.p > 1;
    D.split = split_for(glen);
    XTRG_HIP(hipMemcpyAsync(w, J.Y, sizeof(double) * J.len * J.p, hipMemcpyDeviceToDevice, s));
    if (glen == J.len) {
      sumsq(w, (size_t)J.len * J.p, w + (size_t)J.len * J.p + 3 * (size_t)J.p + 1,
            w + (size_t)J.len * J.p + 3 * (size_t)J.p + 2, s);
    } else {   // ||Y||_F^2 of the leading rows, from the column norms in fixed order
      double* raw = w + (size_t)J.len * J.p;
      hipLaunchKernelGGL(column_norms, dim3((J.p + 3) / 4), dim3(256), 0, s, w, J.len, glen, J.p, raw);
      hipLaunchKernelGGL(sum_squares_ordered, dim3(1), dim3(256), 0, s, raw, J.p,
                         w + (size_t)J.len * J.p + 3 * (size_t)J.p + 1);
    }
    n2[j] = 1;
    while (n2[j] < J.p) n2[j] <<= 1;
  }
  std::vector<int> full_nbk(n), hal(n, 0);
  for (int j = 0; j < n; ++j) full_nbk[j] = h[j].nbk;
  // Ranks for the next sweep and the count of columns still above the
  // numerical zero: the rest sort last, are never rotated again (a pair is
  // rotated only if both columns are above it, and rotations alone change
  // a column), and are left out of the block schedule.
  // The same for every active problem at once (three grouped launches; the
  // device descriptors must be current).
  auto prepare_all = [&](bool count) {
    int maxp = 0, maxn2 = 1;
    for (int j = 0; j < n; ++j)
      if (h[j].active) {
        maxp = std::max(maxp, h[j].p);
        maxn2 = std::max(maxn2, n2[j]);
      }
    if (maxp == 0) return;
    hipLaunchKernelGGL(column_norms_group, dim3((maxp + 3) / 4, n), dim3(256), 0, s, d_desc);
    hipLaunchKernelGGL(sort_desc_group, dim3(n), dim3(1024), (sizeof(double) + sizeof(int)) * maxn2, s, d_desc);
    if (count) hipLaunchKernelGGL(count_alive_group, dim3(n), dim3(256), 0, s, d_desc, d_alive, d_f2);
    XTRG_HIP(hipGetLastError());
  };
  bool dirty = true;
  auto set_nbk = [&](int j) {
    int nb = (std::max(hal[j], 2) + kBlk - 1) / kBlk;
    if (nb % 2) ++nb;
    nb = std::min(nb, full_nbk[j]);
    if (nb != h[j].nbk) {
      h[j].nbk = nb;
      dirty = true;
    }
  };
  XTRG_HIP(hipMemcpyAsync(d_desc, h.data(), sizeof(JacobiDesc) * n, hipMemcpyHostToDevice, s));
  prepare_all(true);
  XTRG_HIP(hipMemcpyAsync(hal.data(), d_alive, sizeof(int) * n, hipMemcpyDeviceToHost, s));
  // ||Y||_F^2 must be finite: a NaN or Inf entry, or a norm beyond the
  // double range, would leave every rotation test false
  std::vector<double> f2(n, 0.0);   // written for the active problems by the count
  XTRG_HIP(hipMemcpyAsync(f2.data(), d_f2, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  XTRG_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < n; ++j)
    if (h[j].active && !std::isfinite(f2[j])) {   // non-finite entry or ||Y||_F^2 beyond the double range
      jobs[j].status = -4;
      h[j].active = 0;
    }
  for (int j = 0; j < n; ++j)
    if (h[j].active) set_nbk(j);
  // Sliced launches pay off while the fused rounds would leave most compute
  // units idle; the results are the same either way.
  int smax = 1;
  auto plan = [&]() {
    max_nbk = 0;
    max_half = 0;
    smax = 1;
    long wgs = 0;
    for (const auto& D : h)
      if (D.active) {
        smax = std::max(smax, D.split);
        wgs += (long)(D.nbk / 2) * D.split;
        max_nbk = std::max(max_nbk, D.nbk);
        max_half = std::max(max_half, D.nbk / 2);
      }
    if (wgs > 256) smax = 1;
  };
  auto round = [&](int r) {
    if (smax == 1) {
      hipLaunchKernelGGL(jacobi_round<ROUND_FUSED>, dim3(max_half, n), dim3(kWT), 0, s, d_desc, r, 1, d_parts);
    } else {
      hipLaunchKernelGGL(jacobi_round<ROUND_GRAM>, dim3(max_half * smax, n), dim3(kWT), 0, s, d_desc, r, smax,
                         d_parts);
      hipLaunchKernelGGL(jacobi_round<ROUND_ROTATE>, dim3(max_half * smax, n), dim3(kWT), 0, s, d_desc, r, smax,
                         d_parts);
    }
  };
  std::vector<unsigned long long> hoff(n);
  std::vector<double> last(n, 0.0);
  int n_active = 0;
  for (auto& D : h) n_active += D.active;
  for (int sweep = 0; n_active > 0; ++sweep) {
    if (sweep >= kMaxSweeps) {   // not converged: the problems still active fail
      for (int j = 0; j < n; ++j)
        if (h[j].active) {
          jobs[j].status = -4;
          h[j].active = 0;
        }
      break;
    }
    plan();
    if (dirty) {   // the active set or a block count changed: refresh the device descriptors
      XTRG_HIP(hipMemcpyAsync(d_desc, h.data(), sizeof(JacobiDesc) * n, hipMemcpyHostToDevice, s));
      dirty = false;
    }
    XTRG_HIP(hipMemsetAsync(d_off, 0, sizeof(unsigned long long) * n, s));
    if (timer) timer->begin(s);
    for (int r = 0; r < max_nbk - 1; ++r) round(r);
    XTRG_HIP(hipGetLastError());
    if (timer) {
      double fl = 0.0, by = 0.0;
      for (const auto& D : h)
        if (D.active) {
          const double pairs = 0.5 * D.nbk * (D.nbk - 1);          // over the whole sweep
          fl += pairs * (kNC * (kNC + 1) / 2 * 2.0 + 2.0 * kNC * kNC) * D.len;
          by += (D.nbk - 1) * 16.0 * D.len * std::min(D.p, D.nbk * kBlk);
        }
      timer->end(s, (long)(max_nbk - 1) * (smax > 1 ? 2 : 1), fl, by, smax > 1);
    }
    prepare_all(true);   // the descriptors on the device are those of this sweep
    XTRG_HIP(hipMemcpyAsync(hoff.data(), d_off, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, s));
    XTRG_HIP(hipMemcpyAsync(hal.data(), d_alive, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    XTRG_HIP(hipStreamSynchronize(s));
    std::vector<int> chk;
    for (int j = 0; j < n; ++j) {
      if (!h[j].active) continue;
      double m;
      std::memcpy(&m, &hoff[j], sizeof(m));
      if (!(m == m)) {           // NaN in the input
        jobs[j].status = -4;
        h[j].active = 0;
        --n_active;
        dirty = true;
        continue;
      }
      last[j] = m;
      jobs[j].sweeps = sweep + 1;
      if (m == 0.0) {            // no pair needed a rotation
        h[j].active = 0;
        --n_active;
        dirty = true;
      } else if (m < kCheckBelow && jobs[j].gram) {
        chk.push_back(j);
      }
    }
    // Nearly converged: the closing sweep would only confirm it.  One GEMM
    // gives every pair's fresh Gram entries at once; the job stops here if
    // none needs a rotation (what that sweep would find, with no rotation
    // in it the columns do not change while it runs).
    if (!chk.empty()) {
      XTRG_HIP(hipMemsetAsync(d_off, 0, sizeof(unsigned long long) * n, s));
      for (int j : chk) {
        const SvdJob& J = jobs[j];
        Gemm g;
        g.M = J.p;
        g.N = J.p;
        g.K = h[j].glen;
        g.A = J.work;
        g.lda = J.len;
        g.B = J.work;
        g.ldb = J.len;
        g.transB = 1;
        g.C = J.gram;
        g.ldc = J.p;
        g.tiles64 = 1;
        gemm(g, s);
        const long np = (long)J.p * J.p;
        hipLaunchKernelGGL(gram_check, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, J.gram, J.p,
                           h[j].tol * h[j].tol, h[j].zrel2, h[j].fro2, d_off + j);
      }
      XTRG_HIP(hipGetLastError());
      XTRG_HIP(hipMemcpyAsync(hoff.data(), d_off, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, s));
      XTRG_HIP(hipStreamSynchronize(s));
      for (int j : chk)
        if (hoff[j] == 0ull) {
          h[j].active = 0;
          --n_active;
          dirty = true;
        }
    }
    for (int j = 0; j < n; ++j)
      if (h[j].active) set_nbk(j);
  }
  // final ranking of every problem that succeeded (also those with one column)
  for (int j = 0; j < n; ++j) h[j].active = jobs[j].len > 0 && jobs[j].p > 0 && jobs[j].status == 0;
  XTRG_HIP(hipMemcpyAsync(d_desc, h.data(), sizeof(JacobiDesc) * n, hipMemcpyHostToDevice, s));
  prepare_all(false);
}

void svd_left(int len, int p, const double* Y, double* sigma, int k, double* U, long ldu, int u_rowmajor,
              double* work, void* desc_dev, hipStream_t s, int* sweeps_out, RoundTimer* timer) {
  std::vector<SvdJob> jobs(1);
  jobs[0] = SvdJob{len, p, Y, work, 0};
  svd_batched(jobs, desc_dev, s, timer);
  if (jobs[0].status != 0)
    throw Error(-4, "svd: non-finite entry, ||Y||_F^2 beyond the double range, or no convergence (len " +
                        std::to_string(len) + ", p " + std::to_string(p) + ")");
  if (len > 0 && p > 0) {
    if (sigma) XTRG_HIP(hipMemcpyAsync(sigma, sv_sorted(work, len, p), sizeof(double) * p, hipMemcpyDeviceToDevice, s));
    if (k > 0 && U) svd_gather(len, p, work, k, U, ldu, u_rowmajor, s);
  }
  if (sweeps_out) *sweeps_out = jobs[0].sweeps;
}

// Second stage after the caller has chosen k from the sorted values.
void svd_gather(int len, int p, double* work, int k, double* U, long ldu, int u_rowmajor, hipStream_t s) {
  if (k <= 0) return;
  const long n = (long)len * k;
  hipLaunchKernelGGL(gather_columns, dim3((n + 255) / 256), dim3(256), 0, s, work, len, sv_sorted(work, len, p),
                     sv_perm(work, len, p), k, U, ldu, u_rowmajor);
  XTRG_HIP(hipGetLastError());
}

void svd_adopt(int len, int p, const double* Z, double* work, hipStream_t s) {
  if (len <= 0 || p <= 0) return;
  if (p > 4096) throw Error(-1, "svd: more than 4096 columns");
  XTRG_HIP(hipMemcpyAsync(work, Z, sizeof(double) * len * p, hipMemcpyDeviceToDevice, s));
  sumsq(work, (size_t)len * p, work + (size_t)len * p + 3 * (size_t)p + 1, work + (size_t)len * p + 3 * (size_t)p + 2,
        s);
  double* raw = work + (size_t)len * p;
  hipLaunchKernelGGL(column_norms, dim3((p + 3) / 4), dim3(256), 0, s, work, len, len, p, raw);
  hipLaunchKernelGGL(sort_desc, dim3(1), dim3(1024), (sizeof(double) + sizeof(int)) * (size_t)pow2_at_least(p), s,
                     raw, p, sv_sorted(work, len, p), sv_perm(work, len, p));
  XTRG_HIP(hipGetLastError());
}

const double* svd_column_norms(const double* work, int len, int p) { return work + (size_t)len * p; }

const double* svd_sorted_values(const double* work, int len, int p) {
  return work + (size_t)len * p + p;
}

const double* svd_fro2(const double* work, int len, int p) {
  return work + (size_t)len * p + 3 * (size_t)p + 1;
}

double svd_noise_rel(int len, int p) {
  return 8.0 * 2.220446049250313e-16 * std::sqrt((double)std::max(len, p));
}

double svd_keep_rel(int len, int p) {
  return 40.0 * 2.220446049250313e-16 * std::sqrt((double)std::max(len, p));
}

}  // namespace xtrg
