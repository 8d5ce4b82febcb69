// Small elementwise, permutation and reduction kernels (memory-bound; one
// thread per element, grid-stride loops).
#include "internal.h"

#include <algorithm>

namespace xtrg {

namespace {

constexpr int kT = 256;

inline dim3 grid_for(size_t n) {
  size_t b = (n + kT - 1) / kT;
  if (b > 65535u * 8u) b = 65535u * 8u;
  return dim3((unsigned)(b ? b : 1));
}

__global__ void k_fill(double* __restrict__ d, double v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    d[i] = v;
}

__global__ void k_scale(double* __restrict__ d, double a, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    d[i] *= a;
}

__global__ void k_axpby(double* __restrict__ y, double a, const double* __restrict__ x, double b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * y[i] + b * x[i];
}

__global__ void k_transpose(double* __restrict__ dst, long ldd, const double* __restrict__ src, long lds,
                            int rows, int cols) {
  __shared__ double tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  for (int y = threadIdx.y; y < 32; y += 8) {
    const int c = c0 + y, r = r0 + threadIdx.x;       // read src column-major: src[c*lds + r]
    tile[y][threadIdx.x] = (c < cols && r < rows) ? src[(long)c * lds + r] : 0.0;
  }
  __syncthreads();
  for (int y = threadIdx.y; y < 32; y += 8) {
    const int r = r0 + y, c = c0 + threadIdx.x;       // write dst row-major: dst[r*ldd + c]
    if (r < rows && c < cols) dst[(long)r * ldd + c] = tile[threadIdx.x][y];
  }
}

__global__ void k_swap_phys(double* __restrict__ dst, const double* __restrict__ src, int Dl, int Dr) {
  const long n = (long)Dl * 4 * Dr;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long ar = i % Dr;
    const long q = i / Dr;
    const int t = (int)(q % 2), s = (int)((q / 2) % 2);
    const long al = q / 4;
    dst[((al * 2 + t) * 2 + s) * Dr + ar] = src[i];
  }
}

// Fixed-order block sums, then one block adds the partials: deterministic.
__global__ void k_sumsq_partial(const double* __restrict__ x, size_t n, double* __restrict__ part) {
  __shared__ double sm[kT];
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    s = fma(x[i], x[i], s);
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_sum_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sm[kT];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kT) s += part[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

__global__ void k_site_product(double* __restrict__ C, const double* __restrict__ A, int Dla, int Dra,
                               const double* __restrict__ B, int Dlb, int Drb) {
  // C[(a,b), s, u, (a',b')] = sum_t A[a,s,t,a'] B[b,t,u,b']
  const long n = (long)Dla * Dlb * 4 * Dra * Drb;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    long q = i;
    const int bp = (int)(q % Drb); q /= Drb;
    const int ap = (int)(q % Dra); q /= Dra;
    const int u = (int)(q % 2); q /= 2;
    const int s = (int)(q % 2); q /= 2;
    const int b = (int)(q % Dlb); q /= Dlb;
    const int a = (int)q;
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t)
      v += A[(((long)a * 2 + s) * 2 + t) * Dra + ap] * B[(((long)b * 2 + t) * 2 + u) * Drb + bp];
    C[i] = v;
  }
}

__global__ void k_phys_trace(double* __restrict__ out, const double* __restrict__ W, int Dl, int Dr) {
  const long n = (long)Dl * Dr;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long a = i / Dr, ap = i % Dr;
    out[i] = W[((a * 2 + 0) * 2 + 0) * Dr + ap] + W[((a * 2 + 1) * 2 + 1) * Dr + ap];
  }
}

__global__ void k_contract(Contract c, long n_out_total) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n_out_total; i += (long)gridDim.x * blockDim.x) {
    long q = i, bt = 0, bw = 0;
    for (int d = c.n_out - 1; d >= 0; --d) {
      const long v = q % c.oe[d];
      q /= c.oe[d];
      bt += v * c.ots[d];
      bw += v * c.ows[d];
    }
    double acc = 0.0;
    for (int i0 = 0; i0 < c.ce[0]; ++i0)
      for (int i1 = 0; i1 < c.ce[1]; ++i1)
        for (int i2 = 0; i2 < c.ce[2]; ++i2) {
          const long ot = bt + i0 * c.cts[0] + i1 * c.cts[1] + i2 * c.cts[2];
          const long ow = bw + i0 * c.cws[0] + i1 * c.cws[1] + i2 * c.cws[2];
          acc = fma(c.T[ot], c.W[ow], acc);
        }
    c.out[i] = acc;
  }
}

__global__ void k_to_f32(float* __restrict__ dst, const double* __restrict__ src, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

__global__ void k_fill_f32(float* __restrict__ dst, float v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

// Uniform values in (-1, 1) from a counter-based hash (splitmix64 of the
// element index plus seed): reproducible, independent of the launch shape.
__global__ void k_fill_hash(double* __restrict__ d, size_t n, unsigned long long seed) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    d[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

// Partial maxima of |G[i][j] - delta_ij| over a k x k row-major matrix.
__global__ void k_eye_dev_partial(const double* __restrict__ G, int k, double* __restrict__ part) {
  __shared__ double sm[kT];
  double m = 0.0;
  const size_t n = (size_t)k * k;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double v = G[i] - ((i / k == i % k) ? 1.0 : 0.0);
    m = fmax(m, fabs(v));
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_max_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sm[kT];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += kT) m = fmax(m, part[i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

}  // namespace

void fill_hash(double* dst, size_t n, unsigned long long seed, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill_hash, grid_for(n), dim3(kT), 0, s, dst, n, seed);
  XTRG_HIP(hipGetLastError());
}

void eye_dev(const double* G, int k, double* out, double* part, hipStream_t s) {
  const size_t n = (size_t)k * k;
  unsigned nb = (unsigned)std::min<size_t>(1024, (n + kT - 1) / kT);
  if (nb == 0) nb = 1;
  hipLaunchKernelGGL(k_eye_dev_partial, dim3(nb), dim3(kT), 0, s, G, k, part);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kT), 0, s, part, (int)nb, out);
  XTRG_HIP(hipGetLastError());
}

void to_f32(float* dst, const double* src, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_to_f32, grid_for(n), dim3(kT), 0, s, dst, src, n);
  XTRG_HIP(hipGetLastError());
}

void fill_f32(float* dst, float v, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill_f32, grid_for(n), dim3(kT), 0, s, dst, v, n);
  XTRG_HIP(hipGetLastError());
}

void copy(double* dst, const double* src, size_t n, hipStream_t s) {
  if (n) XTRG_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
}

void fill(double* dst, double v, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill, grid_for(n), dim3(kT), 0, s, dst, v, n);
  XTRG_HIP(hipGetLastError());
}

void scale(double* x, double a, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_scale, grid_for(n), dim3(kT), 0, s, x, a, n);
  XTRG_HIP(hipGetLastError());
}

void axpby(double* y, double a, const double* x, double b, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_axpby, grid_for(n), dim3(kT), 0, s, y, a, x, b, n);
  XTRG_HIP(hipGetLastError());
}

void transpose(double* dst, long ldd, const double* src, long lds, int rows, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  dim3 g((cols + 31) / 32, (rows + 31) / 32);
  hipLaunchKernelGGL(k_transpose, g, dim3(32, 8), 0, s, dst, ldd, src, lds, rows, cols);
  XTRG_HIP(hipGetLastError());
}

void swap_phys(double* dst, const double* src, int Dl, int Dr, hipStream_t s) {
  const size_t n = (size_t)Dl * 4 * Dr;
  if (!n) return;
  hipLaunchKernelGGL(k_swap_phys, grid_for(n), dim3(kT), 0, s, dst, src, Dl, Dr);
  XTRG_HIP(hipGetLastError());
}

void sumsq(const double* x, size_t n, double* out, double* part, hipStream_t s) {
  unsigned nb = (unsigned)std::min<size_t>(1024, (n + kT - 1) / kT);
  if (nb == 0) nb = 1;
  hipLaunchKernelGGL(k_sumsq_partial, dim3(nb), dim3(kT), 0, s, x, n, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kT), 0, s, part, (int)nb, out);
  XTRG_HIP(hipGetLastError());
}

void site_product(double* C, const double* A, int Dla, int Dra, const double* B, int Dlb, int Drb,
                  hipStream_t s) {
  const size_t n = (size_t)Dla * Dlb * 4 * Dra * Drb;
  if (!n) return;
  hipLaunchKernelGGL(k_site_product, grid_for(n), dim3(kT), 0, s, C, A, Dla, Dra, B, Dlb, Drb);
  XTRG_HIP(hipGetLastError());
}

void phys_trace(double* out, const double* W, int Dl, int Dr, hipStream_t s) {
  const size_t n = (size_t)Dl * Dr;
  if (!n) return;
  hipLaunchKernelGGL(k_phys_trace, grid_for(n), dim3(kT), 0, s, out, W, Dl, Dr);
  XTRG_HIP(hipGetLastError());
}

// dst[i + j*rows] = src[ri[i] + ci[j]*ld]: one charge block of a matrix.
__global__ void k_gather_block(double* __restrict__ dst, const double* __restrict__ src, long ld,
                               const int* __restrict__ ri, int rows, const int* __restrict__ ci, int cols) {
  const long n = (long)rows * cols;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), j = (int)(e / rows);
    dst[e] = src[ri[i] + (long)ci[j] * ld];
  }
}

__global__ void k_gather_values(ValGather g) {
  const int e = blockIdx.x;
  if (e == 0 && threadIdx.x == 0) g.out[0] = g.head[0];
  if (threadIdx.x == 0) g.out[g.off[e]] = g.f2[e][0];
  for (int i = threadIdx.x; i < g.r[e]; i += blockDim.x) g.out[g.off[e] + 1 + i] = g.v[e][i];
}

// Column t of src (rows x cols, column-major) goes to column pos[t] of a
// dense len x k matrix, row i to row ri[i]: dst[r*k + j] (rowmajor) or
// dst[j*len + r].
__global__ void k_scatter_cols(double* __restrict__ dst, int len, int k, int rowmajor, const double* __restrict__ src,
                               int rows, int cols, const int* __restrict__ ri, const int* __restrict__ pos) {
  const long n = (long)rows * cols;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), t = (int)(e / rows);
    const long r = ri[i], j = pos[t];
    dst[rowmajor ? r * k + j : j * len + r] = src[e];
  }
}

// out (row-major over the n dims, extents e) = src at offset sum_d i_d st_d.
__global__ void k_permute(Permute p, long n_total) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += (long)gridDim.x * blockDim.x) {
    long q = i, off = 0;
    for (int d = p.n - 1; d >= 0; --d) {
      const long v = q % p.e[d];
      q /= p.e[d];
      off += v * p.st[d];
    }
    p.out[i] = p.src[off];
  }
}

void gather_block(double* dst, const double* src, long ld, const int* ri, int rows, const int* ci, int cols,
                  hipStream_t s) {
  const size_t n = (size_t)rows * cols;
  if (!n) return;
  hipLaunchKernelGGL(k_gather_block, grid_for(n), dim3(kT), 0, s, dst, src, ld, ri, rows, ci, cols);
  XTRG_HIP(hipGetLastError());
}

void gather_values(const ValGather& g, hipStream_t s) {
  if (g.n <= 0) return;
  hipLaunchKernelGGL(k_gather_values, dim3(g.n), dim3(kT), 0, s, g);
  XTRG_HIP(hipGetLastError());
}

void scatter_cols(double* dst, int len, int k, int rowmajor, const double* src, int rows, int cols, const int* ri,
                  const int* pos, hipStream_t s) {
  const size_t n = (size_t)rows * cols;
  if (!n) return;
  hipLaunchKernelGGL(k_scatter_cols, grid_for(n), dim3(kT), 0, s, dst, len, k, rowmajor, src, rows, cols, ri, pos);
  XTRG_HIP(hipGetLastError());
}

void permute(const Permute& p, hipStream_t s) {
  long n = 1;
  for (int d = 0; d < p.n; ++d) n *= p.e[d];
  if (n <= 0) return;
  hipLaunchKernelGGL(k_permute, grid_for((size_t)n), dim3(kT), 0, s, p, n);
  XTRG_HIP(hipGetLastError());
}

void contract(const Contract& c, hipStream_t s) {
  long n = 1;
  for (int d = 0; d < c.n_out; ++d) n *= c.oe[d];
  if (n <= 0) return;
  hipLaunchKernelGGL(k_contract, grid_for((size_t)n), dim3(kT), 0, s, c, n);
  XTRG_HIP(hipGetLastError());
}

}  // namespace xtrg
