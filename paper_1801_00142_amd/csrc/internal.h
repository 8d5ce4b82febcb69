// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace xtrg {

// Error carried to the C ABI boundary and turned into a status code there.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Global-memory view of a pointer that a kernel reads from a descriptor in
// memory (the compiler cannot tell its address space and would emit flat
// accesses).  Flat loads and stores also count against the LDS wait that
// precedes every barrier, so a load in flight or a store not yet
// acknowledged holds up the next barrier; through this view they do not.
template <class T>
__device__ inline __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

#define XTRG_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::xtrg::Error(-3, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

// Batched, strided GEMM on the matrix cores:  C[b] = A[b] * B[b]
//   A element (m, k): transA ? A[k*lda + m] : A[m*lda + k]
//   B element (k, n): transB ? B[n*ldb + k] : B[k*ldb + n]
//   C element (m, n): C[m*ldc + n]
// The batch index is split into up to three levels b = (b0*nb1 + b1)*nb2 + b2,
// each with its own offset stride (in elements) for A, B and C.
// Precision: GEMM_F64 (double in, double out, FP64 MFMA), GEMM_F32 (float
// in, FP32 MFMA with FP32 accumulation) or GEMM_BF16X3 (float in, each
// operand split into two bf16 terms, three bf16 MFMA products with FP32
// accumulation); for the float modes out64 selects a double or a float C.
enum { GEMM_F64 = 0, GEMM_F32 = 1, GEMM_BF16X3 = 2 };   // BF16X3: float operands split hi + lo
struct Gemm {
  int M = 0, N = 0, K = 0;
  int transA = 0, transB = 0;
  long lda = 0, ldb = 0, ldc = 0;
  int nb[3] = {1, 1, 1};
  long sA[3] = {0, 0, 0}, sB[3] = {0, 0, 0}, sC[3] = {0, 0, 0};
  const void* A = nullptr;
  const void* B = nullptr;
  void* C = nullptr;
  int tag = 0;    // 1: the two-site overlap C_E (its own kernel symbol for profiling)
  int prec = GEMM_F64;
  int out64 = 1;  // GEMM_F32 only: C is double (1) or float (0)
  int tiles64 = 0;  // 64 x 64 output tiles even for large M and N (more workgroups without split-K)
};

// Launch; split-K (for small M*N and large K, unbatched only) uses `work`
// (device, >= splitk*M*N doubles) and a deterministic reduction.
void gemm(const Gemm& g, hipStream_t s, double* work = nullptr, size_t work_cap = 0);
size_t gemm_splitk_work(const Gemm& g);
// Independent problems in as few launches as their kernels allow (one per
// kernel and 8 problems; each problem's tiles, split-K and summation order
// as in gemm(), so it gets the same bits as alone).  `work` holds
// gemm_grouped_work(gs) doubles (the problems' split-K partials side by side).
void gemm_grouped(const std::vector<Gemm>& gs, hipStream_t s, double* work, size_t work_cap);
size_t gemm_grouped_work(const std::vector<Gemm>& gs);

// One-sided block Jacobi SVD of Y (len x p, column-major, device).
// On return sigma (device, p) holds the singular values descending and,
// if k > 0, U (device, column-major len x k, leading dim ldu) the leading
// left singular vectors.  `work` must hold svd_work(len, p) doubles.
size_t svd_work(int len, int p);
// desc_dev: device scratch of svd_desc_bytes(n) bytes (n problems).
size_t svd_desc_bytes(int n);
struct RoundTimer;
void svd_left(int len, int p, const double* Y, double* sigma, int k, double* U, long ldu,
              int u_rowmajor, double* work, void* desc_dev, hipStream_t s, int* sweeps_out,
              RoundTimer* timer = nullptr);
// Several independent SVDs at once: every Jacobi round of all problems is one
// grouped launch, so latency-bound rounds of independent chains overlap.
struct SvdJob {
  int len, p;
  const double* Y;   // len x p column-major (device)
  double* work;      // svd_work(len, p) doubles
  int sweeps;        // out
  // optional p x p doubles: once a sweep's largest cosine is below 1e-6,
  // the closing sweep is replaced by one check of all pairs on Z^T Z (a
  // GEMM); the Jacobi stops if no pair needs a rotation, as that sweep would
  double* gram = nullptr;
  // rows that define the Gram matrix (0: all len): the columns are
  // orthogonalised on their first glen rows and the remaining rows are only
  // rotated with them (rows of an identity appended below accumulate V)
  int glen = 0;
  // out: 0, or -4 (XTRG_ENUMERIC) if this problem failed (a non-finite
  // entry, ||Y||_F^2 beyond the double range, no convergence); a failed
  // problem leaves the others of the grouped launch untouched
  int status = 0;
};
// Optional timing of the Jacobi rounds (event pair around each sweep's
// back-to-back round launches on the stream).
struct RoundTimer {
  virtual ~RoundTimer() = default;
  virtual void begin(hipStream_t s) = 0;
  // launches: round kernels in the bracket; flops: Gram (symmetric) plus
  // rotation of every visited pair; bytes: each column read and written once
  // sliced: the rounds were split over row slices (two launches per round)
  virtual void end(hipStream_t s, long launches, double flops, double bytes, bool sliced) = 0;
};
// Problems that fail are marked in their status and dropped from the
// remaining rounds; the call itself throws only on runtime errors.
void svd_batched(std::vector<SvdJob>& jobs, void* desc_dev, hipStream_t s, RoundTimer* timer = nullptr);

// Householder QR with column pivoting of Y (len x p, column-major), the
// triangular factor only, stopped once every remaining column has norm^2
// <= stop_rel^2 ||Y||_F^2 (keff rows; each job its own stop_rel).  Columns stay in place: R's entry
// at row r for column c is read with qr_rt.  Several problems per launch.
constexpr int kQrMaxLen = 2048;
struct QrJob {
  int len, p;
  const double* Y;   // len x p column-major (device), not modified
  double* work;      // qr_work(len, p) doubles
  double stop_rel;
  int keff;          // out: rows of R
};
size_t qr_work(int len, int p);
size_t qr_desc_bytes(int n);
void qrcp_batched(std::vector<QrJob>& jobs, void* desc_dev, hipStream_t s);
// R^T into RT (p x keff, column-major, leading dimension ld >= p); with
// identity, rows p .. p + keff - 1 of RT hold the keff x keff identity
// (ld >= p + keff).
void qr_rt(const QrJob& J, double* RT, long ld, bool identity, hipStream_t s);
// M <- Q M for the orthogonal factor Q = H_0 H_1 ... H_{keff-1} of each job
// (M: len x ncols, column-major, leading dimension len; jobs with keff = 0
// are left alone).  One launch per reflector.
void qr_apply_q(std::vector<QrJob>& jobs, const std::vector<double*>& M, const std::vector<int>& ncols,
                void* desc_dev, hipStream_t s);
// M = [W Sigma; 0] (len x keff) from the Jacobi columns Z of [R^T; I]
// (leading dimension ldz): W = their rows p .., Sigma = norms (device, keff).
void qr_lift(const double* Z, long ldz, int p, int keff, const double* norms, double* M, int len, hipStream_t s);
// Pivot column of each step (device, keff ints).
const int* qr_pivots(const QrJob& J);

// Put Z (len x p, column-major, device) into an SVD workspace as if the
// Jacobi had produced it: ||Z||_F^2, column norms, their descending order.
void svd_adopt(int len, int p, const double* Z, double* work, hipStream_t s);
// Column norms over the first glen rows, as the Jacobi left them (device, p).
const double* svd_column_norms(const double* work, int len, int p);

// Two-stage use: svd_left with k = 0, read the sorted values, then gather.
void svd_gather(int len, int p, double* work, int k, double* U, long ldu, int u_rowmajor, hipStream_t s);
const double* svd_sorted_values(const double* work, int len, int p);
// ||Y||_F^2 (device scalar in work) and the relative rounding-noise level:
// singular values below svd_noise_rel(len, p) * ||Y||_F are numerically zero
// (not resolvable by any FP64 factorisation of Y) and are never kept.
const double* svd_fro2(const double* work, int len, int p);
double svd_noise_rel(int len, int p);
// Smallest singular value (relative to ||Y||_F) whose vector the Jacobi
// keeps orthogonal to the larger ones to better than ~10% (the rotation of a
// pair stops once its overlap is below the rounding noise 4 sqrt(n) eps
// ||Y||_F |z|); values below svd_keep_rel(len, p) * ||Y||_F are not kept.
double svd_keep_rel(int len, int p);

// Small elementwise / reduction kernels (misc.hip).
void copy(double* dst, const double* src, size_t n, hipStream_t s);
void fill(double* dst, double v, size_t n, hipStream_t s);
void to_f32(float* dst, const double* src, size_t n, hipStream_t s);   // round to nearest
// n values uniform in (-1, 1) from a counter-based hash of (seed, index).
void fill_hash(double* dst, size_t n, unsigned long long seed, hipStream_t s);
// *out = max |G - I| of the k x k matrix G (device); part: >= 1024 doubles.
void eye_dev(const double* G, int k, double* out, double* part, hipStream_t s);
void fill_f32(float* dst, float v, size_t n, hipStream_t s);
void scale(double* x, double a, size_t n, hipStream_t s);
// y = a*y + b*x
void axpby(double* y, double a, const double* x, double b, size_t n, hipStream_t s);
// dst[r*ldd + c] = src[c*lds + r] for r < rows, c < cols
void transpose(double* dst, long ldd, const double* src, long lds, int rows, int cols, hipStream_t s);
// swap the two physical indices of a site tensor [Dl][2][2][Dr]
void swap_phys(double* dst, const double* src, int Dl, int Dr, hipStream_t s);
// sum of squares into *out (device double), deterministic; part: 1024 doubles scratch
void sumsq(const double* x, size_t n, double* out, double* part, hipStream_t s);
// C[(a,b), s, u, (a',b')] = sum_t A[a,s,t,a'] B[b,t,u,b'] (exact MPO product site)
void site_product(double* C, const double* A, int Dla, int Dra, const double* B, int Dlb, int Drb,
                  hipStream_t s);
// dst (rows x cols, column-major) = src[ri[i] + ci[j]*ld]: the rows ri and
// columns ci of a column-major matrix (index arrays on the device).
void gather_block(double* dst, const double* src, long ld, const int* ri, int rows, const int* ci, int cols,
                  hipStream_t s);
// out[0] = head[0]; then for every entry e: out[off[e]] = f2[e][0] and
// out[off[e] + 1 + i] = v[e][i] for i < r[e] (one launch for many small
// device-to-device copies; the table is passed by value).
struct ValGather {
  static constexpr int kMax = 64;
  int n = 0;
  const double* f2[kMax] = {};
  const double* v[kMax] = {};
  int r[kMax] = {};
  int off[kMax] = {};
  const double* head = nullptr;
  double* out = nullptr;
};
void gather_values(const ValGather& g, hipStream_t s);
// Column t of src (rows x cols, column-major) into column pos[t] of a dense
// len x k matrix at rows ri: dst[ri[i]*k + pos[t]] (rowmajor) or
// dst[pos[t]*len + ri[i]]; other entries of dst are left as they are.
void scatter_cols(double* dst, int len, int k, int rowmajor, const double* src, int rows, int cols, const int* ri,
                  const int* pos, hipStream_t s);
// out[a][a'] = sum_s W[a][s][s][a']
void phys_trace(double* out, const double* W, int Dl, int Dr, hipStream_t s);

// Generic pairwise contraction (observables): see misc.hip.
struct Contract {
  int n_out = 0;            // <= 6 output dims (row-major, in this order)
  int oe[6] = {1, 1, 1, 1, 1, 1};
  long ots[6] = {0}, ows[6] = {0};  // stride of each output dim in T and in W
  int n_c = 0;              // <= 3 contracted dims
  int ce[3] = {1, 1, 1};
  long cts[3] = {0}, cws[3] = {0};
  const double* T = nullptr;
  const double* W = nullptr;
  double* out = nullptr;
};
void contract(const Contract& c, hipStream_t s);
// Strided gather into a row-major block: out[i_0..i_{n-1}] = src[sum_d i_d st[d]]
// (a stride may cover a repeated index: a diagonal).
struct Permute {
  int n = 0;                // <= 8 dims
  long e[8] = {1, 1, 1, 1, 1, 1, 1, 1};
  long st[8] = {0};
  const double* src = nullptr;
  double* out = nullptr;
};
void permute(const Permute& p, hipStream_t s);

}  // namespace xtrg
