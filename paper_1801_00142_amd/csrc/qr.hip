// Householder QR with column pivoting (triangular factor only), FP64.
//
// Used for the SVD of a two-site overlap that has no singular basis from an
// earlier visit: with Y P = Q R, the one-sided Jacobi on R^T converges in a
// fraction of the sweeps it needs on Y itself (the pivoted factor is graded:
// its rows fall off in norm, and the column scaling that remains after the
// grading is well conditioned).  Run on [R^T; I], it accumulates its
// rotations W below: R^T W = U_R Sigma, R = W Sigma U_R^T, and Y's left
// singular vectors are Q W, formed by applying the reflectors (qr_apply_q).
//
// Layout: the columns are never moved.  Step i takes the remaining column
// of largest norm below row i (its index is the pivot piv[i]), forms the
// reflector H_i = I - tau v v^T that maps that column to beta e_i, and
// applies it to rows i.. of every column not yet pivoted.  Row i of a
// column not pivoted before step i is then final: it is R's entry at row i.
// The factorisation stops once every remaining column is below a threshold
// (the numerical zero of the Jacobi), so R has keff <= min(len, p) rows.
//
// One launch per step, one wave per column.  Every workgroup forms the
// reflector itself from the pivot column (the same arithmetic in every
// workgroup, so all agree).  The next pivot is the largest packed
// (norm^2, column) key: each workgroup writes the largest of its waves'
// keys to its own slot, and every workgroup of the next step reduces the
// slots itself (no atomics on one address, which would serialise).
#include "internal.h"

#include <algorithm>
#include <climits>
#include <cmath>

namespace xtrg {

namespace {

constexpr int kQT = 256;                      // threads of a step workgroup (4 waves, one column each)
constexpr int kIdxBits = 12;                  // column index in the low bits of a pivot key
constexpr unsigned long long kIdxMask = (1ull << kIdxBits) - 1;
constexpr int kChunk = 64;                    // steps launched between checks for the stop

// The kernels reach these pointers through their global views (gptr): no
// flat access, so no store in flight holds up a barrier.
struct QrDesc {
  double* A;                                  // len x p column-major, overwritten
  unsigned long long* keys;                   // 2 x nslot: workgroup keys, by step parity
  int* piv;                                   // kmax: pivot column of each step
  int* stepof;                                // p: step at which a column was pivoted (INT_MAX: never)
  double* rdiag;                              // kmax: diagonal of R (beta of each step)
  int* keff;                                  // rows of R (starts at kmax, lowered at the stop)
  const double* fro2;                         // ||Y||_F^2
  double stop_rel2;
  int len, p, kmax;
  int nslot;                                  // workgroups with columns: ceil(p / 4)
};

// Pivot key: the bit pattern of a non-negative double is monotone under
// unsigned comparison; its low 12 mantissa bits carry the column index
// (a relative change of 2^-40 in the compared norm, which only decides
// between columns of equal norm to that precision).
__device__ inline unsigned long long qr_key(double n2, int c) {
  return ((unsigned long long)__double_as_longlong(n2) & ~kIdxMask) | (unsigned long long)c;
}
__device__ inline double qr_key_norm2(unsigned long long k) {
  return __longlong_as_double((long long)(k & ~kIdxMask));
}

__device__ inline double qr_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline unsigned long long qr_wave_max(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// Largest of the waves' keys (lane 0 of each holds its wave's key) into
// the workgroup's slot of the given step parity.  All threads call it.
__device__ inline void qr_post(const QrDesc& d, int parity, unsigned long long key, unsigned long long* red) {
  const int t = threadIdx.x;
  if ((t & 63) == 0) red[t >> 6] = key;
  __syncthreads();
  if (t == 0 && (int)blockIdx.x < d.nslot) {
    unsigned long long m = red[0];
    for (int w = 1; w < kQT / 64; ++w) m = red[w] > m ? red[w] : m;
    gptr(d.keys)[(size_t)parity * d.nslot + blockIdx.x] = m;
  }
}

// Largest key of all workgroups of the previous step (every thread gets it).
__device__ inline unsigned long long qr_pivot_key(const QrDesc& d, int parity, unsigned long long* red) {
  const int t = threadIdx.x;
  unsigned long long m = 0;
  for (int q = t; q < d.nslot; q += kQT) {
    const unsigned long long k = gptr(d.keys)[(size_t)parity * d.nslot + q];
    m = k > m ? k : m;
  }
  m = qr_wave_max(m);
  if ((t & 63) == 0) red[t >> 6] = m;
  __syncthreads();
  m = red[0];
  for (int w = 1; w < kQT / 64; ++w) m = red[w] > m ? red[w] : m;
  return m;
}

// Column norms of Y: the keys of the first pivot; marks every column not
// pivoted.
__global__ __launch_bounds__(kQT) void qr_init(const QrDesc* __restrict__ descs) {
  const QrDesc d = descs[blockIdx.y];
  if (d.kmax <= 0 || (int)blockIdx.x >= d.nslot) return;   // (a workgroup past nslot has no column)
  __shared__ unsigned long long red[kQT / 64];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int gt = blockIdx.x * kQT + t;
  if (gt < d.p) gptr(d.stepof)[gt] = INT_MAX;
  const int c = blockIdx.x * (kQT / 64) + wave;
  double ss = 0.0;
  if (c < d.p) {
    const auto y = gptr(d.A) + (size_t)c * d.len;
    for (int r = lane; r < d.len; r += 64) ss = fma(y[r], y[r], ss);
  }
  ss = qr_wave_sum(ss);
  qr_post(d, 0, c < d.p ? qr_key(ss, c) : 0ull, red);
}

// Step i.  R: rows per lane (len - i <= 64 R).
template <int R>
__global__ __launch_bounds__(kQT) void qr_step(const QrDesc* __restrict__ descs, int i) {
  const QrDesc d = descs[blockIdx.y];
  if (i >= d.kmax || (int)blockIdx.x >= d.nslot) return;
  const int m = d.len - i;                    // rows i .. len-1
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int c = blockIdx.x * (kQT / 64) + wave;
  // this wave's column if not pivoted before: its loads are issued first,
  // the pivot (which it may turn out to be) is known after the reduction
  bool mine = c < d.p && gptr(d.stepof)[c] > i;
  const auto yc = gptr(d.A) + (size_t)(mine ? c : 0) * d.len + i;
  double y[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    y[u] = (mine && r < m) ? yc[r] : 0.0;
  }
  __shared__ unsigned long long red[kQT / 64];
  const unsigned long long key = qr_pivot_key(d, i & 1, red);
  if (!(qr_key_norm2(key) > d.stop_rel2 * gptr(d.fro2)[0])) {     // every remaining column is numerically zero
    if (t == 0) {
      gptr(d.keys)[(size_t)((i + 1) & 1) * d.nslot + blockIdx.x] = 0;   // so that every later step stops too
      if (blockIdx.x == 0) __hip_atomic_fetch_min(gptr(d.keff), i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  const int ci = (int)(key & kIdxMask);
  mine = mine && c != ci;
  // the reflector, from the pivot column (read only in this step)
  __shared__ double v[64 * R];
  __shared__ double rsum[kQT / 64];
  const auto xc = gptr(static_cast<const double*>(d.A)) + (size_t)ci * d.len + i;
  double ss = 0.0;
  for (int r = t; r < m; r += kQT) {
    const double x = xc[r];
    v[r] = x;
    ss = fma(x, x, ss);
  }
  ss = qr_wave_sum(ss);
  if (lane == 0) rsum[wave] = ss;
  __syncthreads();
  const double sig2 = (rsum[0] + rsum[1]) + (rsum[2] + rsum[3]);
  const double alpha = v[0];
  const double beta = -copysign(sqrt(sig2), alpha);   // |alpha - beta| = |alpha| + sigma > 0
  const double tau = (beta - alpha) / beta;
  const double sc = 1.0 / (alpha - beta);
  __syncthreads();                            // v[0] read by all before it is overwritten
  for (int r = t; r < m; r += kQT) v[r] = r == 0 ? 1.0 : v[r] * sc;
  __syncthreads();
  // y <- (I - tau v v^T) y; norm^2 of rows i+1.. for the next pivot.  Every
  // wave runs it on all its registers (rows past m hold zeros and stay
  // zero; a wave with no column of its own, or with the pivot column,
  // computes values that it neither stores nor posts): no register keeps a
  // predicated-off load, so the stores below need no wait on memory.
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    s = fma(r < m ? v[r] : 0.0, y[u], s);
  }
  s = qr_wave_sum(s) * tau;
  double n2 = 0.0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    y[u] = fma(-s, r < m ? v[r] : 0.0, y[u]);
    const double w = r > 0 ? y[u] : 0.0;
    n2 = fma(w, w, n2);
  }
  n2 = qr_wave_sum(n2);
  qr_post(d, (i + 1) & 1, mine ? qr_key(n2, c) : 0ull, red);
  // Stores after the key: nothing in this launch waits for them, so their
  // latency overlaps that of the key's store (the next step reads both).
  if (blockIdx.x == 0 && t == 0) {
    gptr(d.piv)[i] = ci;
    gptr(d.rdiag)[i] = beta;
    gptr(d.stepof)[ci] = i;
  }
  if (mine) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int r = lane + 64 * u;
      if (r < m) yc[r] = y[u];
    }
  }
}

// R^T (p x keff, column-major, leading dimension ld): entry (c, r) is R's
// entry at row r for column c: beta_r for the pivot of step r, row r of the
// updated column if c was pivoted after step r (or never), else zero; rows
// p .. p + rows_id - 1 hold the first rows_id rows of an identity.
// 32 x 32 tiles through LDS (reads along A's columns, writes along R^T's).
__global__ __launch_bounds__(256) void qr_rt(const double* __restrict__ A, int len, int p, int keff, int rows_id,
                                             const int* __restrict__ piv, const int* __restrict__ stepof,
                                             const double* __restrict__ rdiag, double* __restrict__ RT, long ld) {
  __shared__ double tile[32][33];
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;    // 32 x 8
  const int rows = p + rows_id;
  for (int q = ty; q < 32; q += 8) {
    const int c = c0 + q, r = r0 + tx;
    double v = 0.0;
    if (c < p && r < keff) {
      if (piv[r] == c) v = rdiag[r];
      else if (stepof[c] > r) v = A[(size_t)c * len + r];
    } else if (c >= p && c < rows && r < keff) {
      v = c - p == r ? 1.0 : 0.0;
    }
    tile[q][tx] = v;
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {
    const int r = r0 + q, c = c0 + tx;
    if (r < keff && c < rows) RT[(size_t)r * ld + c] = tile[tx][q];
  }
}

// M <- Q M = H_0 (H_1 (... (H_{keff-1} M))).  Every column of M is
// transformed on its own, so one launch does it all: a wave keeps its column
// in registers and applies the reflectors from the last to the first; the
// workgroup stages them through LDS, kQC at a time, each rebuilt from its
// pivot column (which no later step of the factorisation changed) with the
// arithmetic of the factorisation step.
struct QrApply {
  const double* A;
  const int* piv;
  const double* rdiag;
  double* M;
  int len, keff, ncols;
};
constexpr int kQC = 4;                        // reflectors per LDS stage

template <int R>
__global__ __launch_bounds__(kQT) void qr_apply_kernel(const QrApply* __restrict__ descs) {
  const QrApply d = descs[blockIdx.y];
  if (d.keff <= 0 || (int)blockIdx.x * (kQT / 64) >= d.ncols) return;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int c = blockIdx.x * (kQT / 64) + wave;
  const bool mine = c < d.ncols;
  const auto mc = gptr(d.M) + (size_t)(mine ? c : 0) * d.len;
  double y[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    y[u] = (mine && r < d.len) ? mc[r] : 0.0;
  }
  __shared__ double v[kQC][64 * R];
  __shared__ double tau[kQC];
  for (int i1 = d.keff; i1 > 0; i1 -= kQC) {
    const int i0 = max(0, i1 - kQC);           // reflectors i0 .. i1-1 of this stage
    __syncthreads();                          // the previous stage's reflectors are used up
    for (int q = 0; q < i1 - i0; ++q) {
      const int i = i0 + q;
      const auto xc = gptr(d.A) + (size_t)gptr(d.piv)[i] * d.len;
      const double alpha = xc[i], beta = gptr(d.rdiag)[i];
      const double sc = 1.0 / (alpha - beta);
      for (int r = t; r < 64 * R; r += kQT) v[q][r] = (r < i || r >= d.len) ? 0.0 : r == i ? 1.0 : xc[r] * sc;
      if (t == 0) tau[q] = (beta - alpha) / beta;
    }
    __syncthreads();
    if (!mine) continue;
    for (int q = i1 - i0 - 1; q >= 0; --q) {
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < R; ++u) s = fma(v[q][lane + 64 * u], y[u], s);
      s = qr_wave_sum(s) * tau[q];
#pragma unroll
      for (int u = 0; u < R; ++u) y[u] = fma(-s, v[q][lane + 64 * u], y[u]);
    }
  }
  if (!mine) return;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    if (r < d.len) mc[r] = y[u];
  }
}

// M (len x keff, column-major) = [W Sigma; 0]: W = rows p .. p + keff - 1 of
// the Jacobi columns Z (leading dimension ldz), Sigma = their norms over the
// first p rows.
__global__ void qr_lift_kernel(const double* __restrict__ Z, long ldz, int p, int keff,
                               const double* __restrict__ norms, double* __restrict__ M, int len) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)len * keff) return;
  const int c = (int)(idx / len), r = (int)(idx % len);
  M[idx] = r < keff ? Z[(long)c * ldz + p + r] * norms[c] : 0.0;
}

// Workspace layout (doubles): A (len p), fro2 (1), sumsq scratch (1024),
// rdiag (kmax), keys (2 nslot), piv (kmax ints), stepof (p ints).
int qr_nslot(int p) { return (p + kQT / 64 - 1) / (kQT / 64); }
struct QrLayout {
  double* A;
  double* fro2;
  double* part;
  double* rdiag;
  unsigned long long* keys;
  int* piv;
  int* stepof;
};
QrLayout qr_layout(double* w, int len, int p) {
  const size_t kmax = (size_t)std::min(len, p);
  QrLayout L;
  L.A = w;
  L.fro2 = w + (size_t)len * p;
  L.part = L.fro2 + 1;
  L.rdiag = L.part + 1024;
  L.keys = reinterpret_cast<unsigned long long*>(L.rdiag + kmax);
  L.piv = reinterpret_cast<int*>(L.keys + 2 * (size_t)qr_nslot(p));
  L.stepof = L.piv + kmax;
  return L;
}

}  // namespace

size_t qr_work(int len, int p) {
  const size_t kmax = (size_t)std::min(len, p);
  return (size_t)len * p + 1 + 1024 + kmax + 2 * (size_t)qr_nslot(p) + (kmax + 1) / 2 + ((size_t)p + 1) / 2 + 2;
}

size_t qr_desc_bytes(int n) { return (sizeof(QrDesc) + sizeof(int)) * (size_t)n + 256; }

void qrcp_batched(std::vector<QrJob>& jobs, void* desc_dev, hipStream_t s) {
  const int n = (int)jobs.size();
  if (n == 0) return;
  QrDesc* d_desc = reinterpret_cast<QrDesc*>(desc_dev);
  int* d_keff = reinterpret_cast<int*>(d_desc + n);
  std::vector<QrDesc> h(n);
  std::vector<int> kmax(n);
  int kmax_all = 0, pmax = 0, lenmax = 0;
  for (int j = 0; j < n; ++j) {
    QrJob& J = jobs[j];
    if (J.len < 0 || J.p < 0) throw Error(-1, "qrcp: negative size");
    if (J.len > kQrMaxLen) throw Error(-1, "qrcp: column length above 2048");
    if (J.p > (int)kIdxMask + 1) throw Error(-1, "qrcp: more than 4096 columns");
    kmax[j] = std::min(J.len, J.p);
    J.keff = 0;
    QrLayout L = qr_layout(J.work, J.len, J.p);
    h[j] = QrDesc{L.A,   L.keys,  L.piv,  L.stepof,  L.rdiag, d_keff + j, L.fro2, J.stop_rel * J.stop_rel,
                  J.len, J.p, kmax[j], qr_nslot(J.p)};
    if (kmax[j] == 0) continue;
    XTRG_HIP(hipMemcpyAsync(L.A, J.Y, sizeof(double) * J.len * J.p, hipMemcpyDeviceToDevice, s));
    sumsq(L.A, (size_t)J.len * J.p, L.fro2, L.part, s);
    kmax_all = std::max(kmax_all, kmax[j]);
    pmax = std::max(pmax, J.p);
    lenmax = std::max(lenmax, J.len);
  }
  XTRG_HIP(hipMemcpyAsync(d_desc, h.data(), sizeof(QrDesc) * n, hipMemcpyHostToDevice, s));
  XTRG_HIP(hipMemcpyAsync(d_keff, kmax.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  std::vector<int> keff(kmax);
  if (kmax_all > 0) {
    const dim3 grid((pmax + kQT / 64 - 1) / (kQT / 64), n);
    hipLaunchKernelGGL(qr_init, grid, dim3(kQT), 0, s, d_desc);
    for (int i0 = 0; i0 < kmax_all; i0 += kChunk) {
      const int i1 = std::min(kmax_all, i0 + kChunk);
      for (int i = i0; i < i1; ++i) {
        if (lenmax <= 256) hipLaunchKernelGGL(qr_step<4>, grid, dim3(kQT), 0, s, d_desc, i);
        else if (lenmax <= 512) hipLaunchKernelGGL(qr_step<8>, grid, dim3(kQT), 0, s, d_desc, i);
        else if (lenmax <= 1024) hipLaunchKernelGGL(qr_step<16>, grid, dim3(kQT), 0, s, d_desc, i);
        else hipLaunchKernelGGL(qr_step<32>, grid, dim3(kQT), 0, s, d_desc, i);
      }
      XTRG_HIP(hipGetLastError());
      XTRG_HIP(hipMemcpyAsync(keff.data(), d_keff, sizeof(int) * n, hipMemcpyDeviceToHost, s));
      XTRG_HIP(hipStreamSynchronize(s));
      bool more = false;
      for (int j = 0; j < n; ++j) more = more || (keff[j] == kmax[j] && kmax[j] > i1);
      if (!more) break;
    }
  }
  for (int j = 0; j < n; ++j) jobs[j].keff = keff[j];
}

void qr_rt(const QrJob& J, double* RT, long ld, bool identity, hipStream_t s) {
  if (J.keff <= 0 || J.p <= 0) return;
  const int rows_id = identity ? J.keff : 0;
  if (ld < (long)J.p + rows_id) throw Error(-1, "qr_rt: leading dimension too small");
  QrLayout L = qr_layout(J.work, J.len, J.p);
  hipLaunchKernelGGL(qr_rt, dim3((J.keff + 31) / 32, (J.p + rows_id + 31) / 32), dim3(256), 0, s, L.A, J.len, J.p,
                     J.keff, rows_id, L.piv, L.stepof, L.rdiag, RT, ld);
  XTRG_HIP(hipGetLastError());
}

void qr_apply_q(std::vector<QrJob>& jobs, const std::vector<double*>& M, const std::vector<int>& ncols,
                void* desc_dev, hipStream_t s) {
  const int n = (int)jobs.size();
  if (n == 0) return;
  static_assert(sizeof(QrApply) <= sizeof(QrDesc), "descriptor space");
  QrApply* d_desc = reinterpret_cast<QrApply*>(desc_dev);
  std::vector<QrApply> h(n);
  int kmax = 0, cmax = 0, lenmax = 0;
  for (int j = 0; j < n; ++j) {
    const QrJob& J = jobs[j];
    QrLayout L = qr_layout(J.work, J.len, J.p);
    h[j] = QrApply{L.A, L.piv, L.rdiag, M[j], J.len, J.keff, ncols[j]};
    if (J.keff <= 0 || ncols[j] <= 0) continue;
    if (J.len > kQrMaxLen) throw Error(-1, "qr_apply_q: column length above 2048");
    kmax = std::max(kmax, J.keff);
    cmax = std::max(cmax, ncols[j]);
    lenmax = std::max(lenmax, J.len);
  }
  if (kmax == 0) return;
  XTRG_HIP(hipMemcpyAsync(d_desc, h.data(), sizeof(QrApply) * n, hipMemcpyHostToDevice, s));
  const dim3 grid((cmax + kQT / 64 - 1) / (kQT / 64), n);
  if (lenmax <= 256) hipLaunchKernelGGL(qr_apply_kernel<4>, grid, dim3(kQT), 0, s, d_desc);
  else if (lenmax <= 512) hipLaunchKernelGGL(qr_apply_kernel<8>, grid, dim3(kQT), 0, s, d_desc);
  else if (lenmax <= 1024) hipLaunchKernelGGL(qr_apply_kernel<16>, grid, dim3(kQT), 0, s, d_desc);
  else hipLaunchKernelGGL(qr_apply_kernel<32>, grid, dim3(kQT), 0, s, d_desc);
  XTRG_HIP(hipGetLastError());
}

void qr_lift(const double* Z, long ldz, int p, int keff, const double* norms, double* M, int len, hipStream_t s) {
  if (keff <= 0 || len <= 0) return;
  if (keff > len) throw Error(-1, "qr_lift: more columns than rows");
  const long n = (long)len * keff;
  hipLaunchKernelGGL(qr_lift_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Z, ldz, p, keff, norms, M, len);
  XTRG_HIP(hipGetLastError());
}

const int* qr_pivots(const QrJob& J) { return qr_layout(J.work, J.len, J.p).piv; }

}  // namespace xtrg
