// Singular value decomposition by one-sided (Hestenes) block Jacobi, FP64.
//
// The columns of Y (len x p, column-major) are made mutually orthogonal by
// plane rotations from the right, Y V = Z.  The column norms of Z are the
// singular values and the normalised columns the left singular vectors.
// Columns are grouped into blocks of 4 by norm rank; each outer round pairs
// every block with one other block (round-robin tournament, all pairs met
// once per sweep) and one workgroup per block pair orthogonalises its 8
// columns (8 x 8 Gram from the columns, one sweep of small Jacobi on it,
// one rotation pass).  Sweeps repeat until no pair in a sweep needs a
// rotation.
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
// workgroup owns one block pair (kNC = 8 columns): every thread keeps its R
// rows of the 8 columns in registers, the 8 x 8 Gram matrix of the pair is
// formed from the columns themselves (fresh dot products every visit),
// one cyclic two-sided Jacobi sweep is run on that small matrix, and the
// accumulated 8 x 8 rotation W is applied to the columns in one pass
// (Z <- Z W).  The convergence measure is the largest cosine
// |z_i . z_j| / (|z_i| |z_j|) of the fresh Gram that exceeds tol; columns
// with |z|^2 <= zth are numerically zero and take no part.
constexpr int kNC = 8;
constexpr int kPairs = kNC * (kNC + 1) / 2;   // 36 Gram entries

template <int R>
__global__ __launch_bounds__(kThreads) void jacobi_round(double* __restrict__ Y, int len, int p, int nbk, int r,
                                                          double tol, const int* __restrict__ perm,
                                                          const double* __restrict__ fro2, double zrel2,
                                                          unsigned long long* __restrict__ offmax) {
  constexpr int b = kNC / 2;
  __shared__ int colid[kNC];
  __shared__ double red[kWaves][64];
  __shared__ double Gsh[kNC][kNC + 1];
  __shared__ double Wsh[kNC][kNC + 1];
  __shared__ double rot_c[kNC / 2], rot_s[kNC / 2];
  __shared__ int rot_x[kNC / 2], rot_y[kNC / 2];
  __shared__ double worst_sh;
  int bi, bj;
  rr_pair(nbk, r, blockIdx.x, &bi, &bj);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t < kNC) {
    const int rank = (t < b ? bi : bj) * b + (t < b ? t : t - b);
    colid[t] = rank < p ? perm[rank] : -1;
  }
  __syncthreads();

  double z[kNC][R];
#pragma unroll
  for (int c = 0; c < kNC; ++c) {
    const int col = colid[c];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int e = t + kThreads * i;
      z[c][i] = (col >= 0 && e < len) ? Y[(long)col * len + e] : 0.0;
    }
  }
  // partial Gram entries of this thread's rows, padded to 64 for the
  // recursive-halving reduction (after it, lane l holds the sum of entry l)
  double g[64];
#pragma unroll
  for (int q = 0; q < 64; ++q) g[q] = 0.0;
  {
    int q = 0;
#pragma unroll
    for (int x = 0; x < kNC; ++x)
#pragma unroll
      for (int y = x; y < kNC; ++y, ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) g[q] = fma(z[x][i], z[y][i], g[q]);
  }
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) {
    const bool up = (lane & h) != 0;
#pragma unroll
    for (int k = 0; k < h; ++k) {
      const double send = up ? g[k] : g[k + h];
      const double keep = up ? g[k + h] : g[k];
      g[k] = keep + __shfl_xor(send, h, 64);
    }
  }
  red[wave][lane] = g[0];
  __syncthreads();

  // Small Gram G (8 x 8) and accumulated rotation W in LDS.
  if (t < kPairs) {
    int x = 0, q = t;
    while (q >= kNC - x) { q -= kNC - x; ++x; }      // entry t <-> (x, x + q), row-major upper triangle
    const int y = x + q;
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) v += red[w][t];
    Gsh[x][y] = v;
    Gsh[y][x] = v;
  }
  if (t < kNC * kNC) Wsh[t / kNC][t % kNC] = (t / kNC == t % kNC) ? 1.0 : 0.0;
  __syncthreads();
  const double zth = zrel2 * fro2[0];
  // Convergence measure from the fresh Gram: largest cosine above tol.
  if (wave == 0) {
    double off = 0.0;
    if (lane < kNC * (kNC - 1) / 2) {
      int x = 0, q = lane;
      while (q >= kNC - 1 - x) { q -= kNC - 1 - x; ++x; }
      const int y = x + 1 + q;
      const double a = Gsh[x][x], be = Gsh[y][y];
      if (a > zth && be > zth) {
        const double c = fabs(Gsh[x][y]) / sqrt(a) / sqrt(be);
        if (c > tol) off = c;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o, 64));
    if (lane == 0) {
      worst_sh = off;
      // block maximum published as the bit pattern of a non-negative double
      // (monotone under unsigned comparison)
      atomicMax(offmax, (unsigned long long)__double_as_longlong(off));
    }
  }
  __syncthreads();
  // One cyclic sweep of two-sided Jacobi on G, parallel over the 4 disjoint
  // pairs of each round-robin round (the outer iteration recomputes G from
  // the columns at the next visit).  Columns x' = c x - s y, y' = s x + c y:
  // G <- J^T G J, W <- W J.
  if (worst_sh > 0.0) {
    for (int ir = 0; ir < kNC - 1; ++ir) {
      if (t < kNC / 2) {
        int x, y;
        rr_pair(kNC, ir, t, &x, &y);
        const double a = Gsh[x][x], be = Gsh[y][y], gg = Gsh[x][y];
        double c = 1.0, sn = 0.0;
        if (a > zth && be > zth && fabs(gg) > tol * sqrt(a) * sqrt(be)) {
          const double zeta = (be - a) / (2.0 * gg);
          const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
          c = 1.0 / sqrt(fma(tt, tt, 1.0));
          sn = c * tt;
        }
        rot_c[t] = c;
        rot_s[t] = sn;
        rot_x[t] = x;
        rot_y[t] = y;
      }
      __syncthreads();
      if (t < 2 * kNC * (kNC / 2)) {             // columns x, y of G and of W
        const int q = (t / kNC) % (kNC / 2), k = t % kNC;
        const int x = rot_x[q], y = rot_y[q];
        const double c = rot_c[q], sn = rot_s[q];
        if (t < kNC * (kNC / 2)) {
          const double gx = Gsh[k][x], gy = Gsh[k][y];
          Gsh[k][x] = c * gx - sn * gy;
          Gsh[k][y] = sn * gx + c * gy;
        } else {
          const double wx = Wsh[k][x], wy = Wsh[k][y];
          Wsh[k][x] = c * wx - sn * wy;
          Wsh[k][y] = sn * wx + c * wy;
        }
      }
      __syncthreads();
      if (t < kNC * (kNC / 2)) {                 // rows x, y of G
        const int q = t / kNC, k = t % kNC;
        const int x = rot_x[q], y = rot_y[q];
        const double c = rot_c[q], sn = rot_s[q];
        const double gx = Gsh[x][k], gy = Gsh[y][k];
        Gsh[x][k] = c * gx - sn * gy;
        Gsh[y][k] = sn * gx + c * gy;
      }
      __syncthreads();
    }
  }

#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int e = t + kThreads * i;
    if (e >= len) continue;
#pragma unroll
    for (int c = 0; c < kNC; ++c) {
      const int col = colid[c];
      if (col < 0) continue;
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < kNC; ++j) v = fma(z[j][i], Wsh[j][c], v);
      Y[(long)col * len + e] = v;
    }
  }
}

__global__ void column_norms(const double* __restrict__ Y, int len, int p, double* __restrict__ out) {
  const int col = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col >= p) return;
  const double* c = Y + (long)col * len;
  double s = 0.0;
  for (int e = lane; e < len; e += 64) s = fma(c[e], c[e], s);
  s = wave_sum(s);
  if (lane == 0) out[col] = sqrt(s);
}

// Descending bitonic sort of (value, index) in one workgroup, n <= 4096.
__global__ __launch_bounds__(1024) void sort_desc(const double* __restrict__ val, int p,
                                                   double* __restrict__ sorted, int* __restrict__ perm) {
  extern __shared__ unsigned char sm[];
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
          // order: larger value first; ties by smaller index (deterministic)
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

void svd_left(int len, int p, const double* Y, double* sigma, int k, double* U, long ldu, int u_rowmajor,
              double* work, hipStream_t s, int* sweeps_out) {
  if (len <= 0 || p <= 0) {
    if (sweeps_out) *sweeps_out = 0;
    return;
  }
  if (len > 4096) throw Error(-1, "svd_left: column length above 4096");
  if (p > 4096) throw Error(-1, "svd_left: more than 4096 columns");
  double* Z = work;
  double* raw = work + (size_t)len * p;
  double* srt = sv_sorted(work, len, p);
  int* perm = sv_perm(work, len, p);
  double* tail = work + (size_t)len * p + 3 * (size_t)p;
  unsigned long long* off = reinterpret_cast<unsigned long long*>(tail);
  double* fro2 = tail + 1;
  double* part = tail + 2;
  XTRG_HIP(hipMemcpyAsync(Z, Y, sizeof(double) * len * p, hipMemcpyDeviceToDevice, s));
  sumsq(Z, (size_t)len * p, fro2, part, s);

  int n2 = 1;
  while (n2 < p) n2 <<= 1;
  const size_t sort_lds = (sizeof(double) + sizeof(int)) * n2;
  auto rank_columns = [&]() {
    hipLaunchKernelGGL(column_norms, dim3((p + 3) / 4), dim3(256), 0, s, Z, len, p, raw);
    hipLaunchKernelGGL(sort_desc, dim3(1), dim3(1024), sort_lds, s, raw, p, srt, perm);
    XTRG_HIP(hipGetLastError());
  };

  const int b = kNC / 2;
  int nbk = (p + b - 1) / b;
  if (nbk % 2) ++nbk;
  const double tol = 8.0 * std::sqrt((double)len) * 2.220446049250313e-16;
  // Columns below a quarter of the keep floor are numerically zero: they
  // are neither rotated nor counted for convergence.  Columns of pure
  // rounding noise (the null space of a rank-deficient Y) otherwise never
  // settle, since every rotation leaves them a fresh O(1) relative error.
  // The margin to the keep floor lets content near the floor that is still
  // spread over several columns be gathered before the count is taken.
  const double zrel = 0.25 * svd_keep_rel(len, p);
  const double zrel2 = zrel * zrel;
  const int R = (len + kThreads - 1) / kThreads;
  int sweeps = 0;
  double last = 0.0;
  auto round = [&](int r) {
    const dim3 g(nbk / 2), blk(kThreads);
    if (R <= 1) hipLaunchKernelGGL(jacobi_round<1>, g, blk, 0, s, Z, len, p, nbk, r, tol, perm, fro2, zrel2, off);
    else if (R <= 2) hipLaunchKernelGGL(jacobi_round<2>, g, blk, 0, s, Z, len, p, nbk, r, tol, perm, fro2, zrel2, off);
    else if (R <= 4) hipLaunchKernelGGL(jacobi_round<4>, g, blk, 0, s, Z, len, p, nbk, r, tol, perm, fro2, zrel2, off);
    else if (R <= 8) hipLaunchKernelGGL(jacobi_round<8>, g, blk, 0, s, Z, len, p, nbk, r, tol, perm, fro2, zrel2, off);
    else hipLaunchKernelGGL(jacobi_round<16>, g, blk, 0, s, Z, len, p, nbk, r, tol, perm, fro2, zrel2, off);
  };
  if (p > 1) {
    for (; sweeps < kMaxSweeps; ++sweeps) {
      rank_columns();
      XTRG_HIP(hipMemsetAsync(off, 0, sizeof(unsigned long long), s));
      for (int r = 0; r < nbk - 1; ++r) round(r);
      XTRG_HIP(hipGetLastError());
      unsigned long long h = 0;
      XTRG_HIP(hipMemcpyAsync(&h, off, sizeof(h), hipMemcpyDeviceToHost, s));
      XTRG_HIP(hipStreamSynchronize(s));
      double m;
      std::memcpy(&m, &h, sizeof(m));
      if (!(m == m)) throw Error(-4, "svd_left: NaN in input");
      last = m;
      if (m == 0.0) { ++sweeps; break; }   // no pair needed a rotation
    }
    if (sweeps >= kMaxSweeps)
      throw Error(-4, "svd_left: Jacobi did not converge (len " + std::to_string(len) + ", p " +
                          std::to_string(p) + ", largest cosine " + std::to_string(last) + ")");
  }
  rank_columns();
  if (sigma) XTRG_HIP(hipMemcpyAsync(sigma, srt, sizeof(double) * p, hipMemcpyDeviceToDevice, s));
  if (k > 0 && U) {
    const long n = (long)len * k;
    hipLaunchKernelGGL(gather_columns, dim3((n + 255) / 256), dim3(256), 0, s, Z, len, srt, perm, k, U, ldu,
                       u_rowmajor);
    XTRG_HIP(hipGetLastError());
  }
  if (sweeps_out) *sweeps_out = sweeps;
}

// Second stage after the caller has chosen k from the sorted values.
void svd_gather(int len, int p, double* work, int k, double* U, long ldu, int u_rowmajor, hipStream_t s) {
  if (k <= 0) return;
  const long n = (long)len * k;
  hipLaunchKernelGGL(gather_columns, dim3((n + 255) / 256), dim3(256), 0, s, work, len, sv_sorted(work, len, p),
                     sv_perm(work, len, p), k, U, ldu, u_rowmajor);
  XTRG_HIP(hipGetLastError());
}

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
