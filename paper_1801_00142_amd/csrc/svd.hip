// Singular value decomposition by one-sided (Hestenes) block Jacobi, FP64.
//
// The columns of Y (len x p, column-major) are made mutually orthogonal by
// plane rotations from the right, Y V = Z.  The column norms of Z are the
// singular values and the normalised columns the left singular vectors.
// Columns are grouped into blocks of b; each outer round pairs every block
// with one other block (round-robin tournament, all pairs met once per
// sweep), one workgroup per block pair holds its 2b columns in LDS and runs
// one inner sweep of rotations over them.  Sweeps repeat until the largest
// cosine |z_i . z_j| / (|z_i| |z_j|) seen in a sweep is below tol.
//
// Accuracy: the rotations act on the columns themselves (no Gram matrix is
// formed), so singular values and vectors are resolved to absolute
// accuracy ~ eps * sigma_1, which the thermal-state compression needs:
// components far below sqrt(eps) * sigma_1 carry the high-order terms of
// the series start and must not be lost.
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

// Block pairing works on ranks: rank q is the column with the q-th largest
// norm at the start of the sweep (perm[q]), so each block holds columns of
// similar norm (sorted one-sided Jacobi converges in fewer sweeps on graded
// spectra).  Pairs are skipped when a column is numerically zero
// (|z|^2 <= zth) or when both columns rank at or beyond kneed (both will be
// discarded by the truncation that follows).
__global__ __launch_bounds__(kThreads) void jacobi_round(double* __restrict__ Y, int len, int p, int b,
                                                          int nbk, int r, double tol,
                                                          const int* __restrict__ perm,
                                                          const double* __restrict__ fro2, double zrel2,
                                                          double noise_coef, int kneed,
                                                          unsigned long long* __restrict__ offmax) {
  extern __shared__ double cols[];     // [2b][len]
  __shared__ int colid[32];
  int bi, bj;
  rr_pair(nbk, r, blockIdx.x, &bi, &bj);
  const int nc = 2 * b;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const double zth = zrel2 * fro2[0];
  const double nscale = noise_coef * sqrt(fro2[0]);
  if (t < nc) {
    const int rank = (t < b ? bi : bj) * b + (t < b ? t : t - b);
    colid[t] = rank < p ? perm[rank] : -1;
  }
  __syncthreads();

  // load the 2b columns (absent columns read as zero)
  for (int s = 0; s < nc; ++s) {
    const int col = colid[s];
    double* dst = cols + (long)s * len;
    if (col >= 0) {
      const double* src = Y + (long)col * len;
      for (int e = t; e < len; e += kThreads) dst[e] = src[e];
    } else {
      for (int e = t; e < len; e += kThreads) dst[e] = 0.0;
    }
  }
  __syncthreads();

  double worst = 0.0;
  // one inner sweep: round-robin over the nc slots
  for (int ir = 0; ir < nc - 1; ++ir) {
    for (int q = wave; q < b; q += kWaves) {
      int x, y;
      rr_pair(nc, ir, q, &x, &y);
      if (colid[x] < 0 || colid[y] < 0) continue;
      const int rx = (x < b ? bi : bj) * b + (x < b ? x : x - b);
      const int ry = (y < b ? bi : bj) * b + (y < b ? y : y - b);
      if (rx >= kneed && ry >= kneed) continue;
      double* cx = cols + (long)x * len;
      double* cy = cols + (long)y * len;
      double a = 0.0, be = 0.0, g = 0.0;
      for (int e = lane; e < len; e += 64) {
        const double u = cx[e], v = cy[e];
        a = fma(u, u, a);
        be = fma(v, v, be);
        g = fma(u, v, g);
      }
      a = wave_sum(a);
      be = wave_sum(be);
      g = wave_sum(g);
      if (a > zth && be > zth && g != 0.0) {
        // converged when the overlap is below the relative tolerance or below
        // the rounding noise that columns of size sqrt(fro2) leave in it
        const double sa = sqrt(a), sb = sqrt(be);
        const double off = fabs(g) / sa / sb;
        if (fabs(g) > fmax(tol * sa * sb, nscale * (sa + sb))) {
          worst = fmax(worst, off);
          const double zeta = (be - a) / (2.0 * g);
          const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
          const double c = 1.0 / sqrt(fma(tt, tt, 1.0));
          const double s = c * tt;
          for (int e = lane; e < len; e += 64) {
            const double u = cx[e], v = cy[e];
            cx[e] = c * u - s * v;
            cy[e] = s * u + c * v;
          }
        }
      }
    }
    __syncthreads();
  }

  for (int s = 0; s < nc; ++s) {
    const int col = colid[s];
    if (col >= 0) {
      const double* src = cols + (long)s * len;
      double* dst = Y + (long)col * len;
      for (int e = t; e < len; e += kThreads) dst[e] = src[e];
    }
  }
  // block-wide max of the cosines seen, published as the bit pattern of a
  // non-negative double (monotone under unsigned comparison)
  __shared__ double wmax[kWaves];
  if (lane == 0) wmax[wave] = worst;
  __syncthreads();
  if (t == 0) {
    double m = 0.0;
    for (int w = 0; w < kWaves; ++w) m = fmax(m, wmax[w]);
    atomicMax(offmax, (unsigned long long)__double_as_longlong(m));
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

int block_cols(int len) { return std::max(1, std::min(16, 4096 / std::max(len, 1))); }

}  // namespace

// work layout: [Z: len*p][sigma_raw: p][sigma: p][perm: p ints][offmax: 1][fro2: 1][part: 1024]
size_t svd_work(int len, int p) { return (size_t)len * p + 3 * (size_t)p + 1040; }

static double* sv_sorted(double* work, int len, int p) { return work + (size_t)len * p + p; }
static int* sv_perm(double* work, int len, int p) {
  return reinterpret_cast<int*>(work + (size_t)len * p + 2 * (size_t)p);
}

void svd_left(int len, int p, const double* Y, double* sigma, int k, double* U, long ldu, int u_rowmajor,
              double* work, hipStream_t s, int* sweeps_out, int kneed) {
  if (len <= 0 || p <= 0) {
    if (sweeps_out) *sweeps_out = 0;
    return;
  }
  if (len > 4096) throw Error(-1, "svd_left: column length above 4096");
  if (p > 4096) throw Error(-1, "svd_left: more than 4096 columns");
  if (kneed <= 0 || kneed > p) kneed = p;
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

  const int b = block_cols(len);
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
  const double noise_coef = 0.0;
  const size_t lds = sizeof(double) * 2 * b * len;
  int sweeps = 0;
  double last = 0.0;
  if (p > 1) {
    for (; sweeps < kMaxSweeps; ++sweeps) {
      rank_columns();
      XTRG_HIP(hipMemsetAsync(off, 0, sizeof(unsigned long long), s));
      for (int r = 0; r < nbk - 1; ++r) {
        hipLaunchKernelGGL(jacobi_round, dim3(nbk / 2), dim3(kThreads), lds, s, Z, len, p, b, nbk, r, tol,
                           perm, fro2, zrel2, noise_coef, kneed, off);
      }
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
