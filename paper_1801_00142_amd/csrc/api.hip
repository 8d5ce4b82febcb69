// C ABI of the library: contexts, MPO handles, the automaton Hamiltonian,
// the series start, one XTRG doubling (variational product compression)
// and the thermodynamic observables.  Host code here only orchestrates:
// every tensor operation is a kernel on the context stream.
#include "xtrg.h"

#include <algorithm>
#include <limits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <tuple>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "context.h"
#include "host_rules.h"

using xtrg::Error;
using xtrg::Gemm;
using xtrg_host::col_charges;
using xtrg_host::keep_count;
using xtrg_host::row_charges;

// Device scratch of xtrg_dgemm_noalloc (the split-K partial products):
// one fixed array per GPU, in the library's code object, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (in
// host code the name is a stand-in, not a device address): the address is
// looked up once per device when a context is created there.
constexpr size_t kNoAllocDoubles = size_t(1) << 23;   // 8 Mi doubles = 64 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// With `device` current: the device address of this device's scratch.
double* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error(XTRG_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    XTRG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error(XTRG_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[device];
}
}  // namespace

namespace {

// Phases of the doubling step timed by the profiler.
// svd_rounds is the part of svd spent in the Jacobi round kernels; its
// "calls" count kernel launches.
// warm is the building of the warm-start bases and the rotation of the SVD input.
// svd_rounds: the sweeps of rounds split over row slices (a Gram and a
// rotate launch per round); svd_rounds_fused: those of one-launch rounds.
enum { P_THETA = 0, P_BLOCK, P_ENV, P_SVD, P_SPLIT, P_ROUNDS, P_WARM, P_QR, P_ROUNDS0, P_NCAT };
const char* const kPhase[P_NCAT] = {"theta_gemm", "block_gemm", "env_gemm", "svd",
                                    "split", "svd_rounds", "warm", "qr_start", "svd_rounds_fused"};

// RAII event pair around the work enqueued in its scope.
struct Timed {
  xtrg_ctx c;
  xtrg_ctx_s::Prof r{};
  Timed(xtrg_ctx ctx, int cat, double flops, double bytes) : c(ctx) {
    if (!c->prof) return;
    r.cat = cat;
    r.flops = flops;
    r.bytes = bytes;
    r.launches = 1;
    XTRG_HIP(hipEventCreate(&r.a));
    XTRG_HIP(hipEventCreate(&r.b));
    XTRG_HIP(hipEventRecord(r.a, c->stream));
  }
  ~Timed() {
    if (!c->prof) return;
    (void)hipEventRecord(r.b, c->stream);
    c->prof_recs.push_back(r);
  }
};

template <class F>
int guarded(xtrg_ctx ctx, F&& f) {
  if (ctx && ctx->serving.load()) return XTRG_EBUSY;   // the serving loop owns the stream
  try {
    f();
    if (ctx) ctx->err.clear();
    return XTRG_OK;
  } catch (const Error& e) {
    if (ctx) ctx->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return XTRG_EINVAL;
  } catch (...) {
    if (ctx) ctx->err = "unknown error";
    return XTRG_EINVAL;
  }
}

void set_device(xtrg_ctx c) { XTRG_HIP(hipSetDevice(c->device)); }

std::unique_ptr<xtrg_mpo_s> new_mpo(xtrg_ctx c, const std::vector<int>& dims) {
  auto m = std::make_unique<xtrg_mpo_s>();
  m->ctx = c;
  m->L = (int)dims.size() - 1;
  m->dims = dims;
  m->site.resize(m->L);
  for (int i = 0; i < m->L; ++i) {
    m->site[i].n = m->elems(i);
    m->site[i].p = c->alloc(m->site[i].n);
  }
  return m;
}

void upload(xtrg_ctx c, double* dst, const double* src, size_t n) {
  XTRG_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
}

double read_scalar(xtrg_ctx c, const double* d) {
  double h = 0.0;
  XTRG_HIP(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  XTRG_HIP(hipStreamSynchronize(c->stream));
  return h;
}

// Event pairs around the Jacobi round launches of each sweep (back to back
// on the stream, so the bracket over a sweep's launches divided by their
// number is the mean launch duration).
struct RoundProf : xtrg::RoundTimer {
  xtrg_ctx c;
  xtrg_ctx_s::Prof r{};
  explicit RoundProf(xtrg_ctx ctx) : c(ctx) {}
  void begin(hipStream_t s) override {
    if (!c->prof) return;
    XTRG_HIP(hipEventCreate(&r.a));
    XTRG_HIP(hipEventCreate(&r.b));
    XTRG_HIP(hipEventRecord(r.a, s));
  }
  void end(hipStream_t s, long launches, double flops, double bytes, bool sliced) override {
    if (!c->prof) return;
    XTRG_HIP(hipEventRecord(r.b, s));
    r.cat = sliced ? P_ROUNDS : P_ROUNDS0;
    r.flops = flops;
    r.bytes = bytes;
    r.launches = launches;
    c->prof_recs.push_back(r);
  }
};

// Device descriptors of a grouped SVD launch over n problems.
void* svd_desc(xtrg_ctx c, int n) { return c->need("svd_desc", xtrg::svd_desc_bytes(n) / sizeof(double) + 1); }
// Workspace of the Jacobi's closing check (Z^T Z), for SVDs of up to 2048 columns.
double* svd_gram(xtrg_ctx c, const std::string& tag, int p) {
  return p <= 2048 ? c->need("svd_gram" + tag, (size_t)p * p) : nullptr;
}
void* qr_desc(xtrg_ctx c, int n) { return c->need("qr_desc", xtrg::qr_desc_bytes(n) / sizeof(double) + 1); }

void gemm(xtrg_ctx c, const Gemm& g) {
  const size_t w = xtrg::gemm_splitk_work(g);
  double* work = w ? c->need("splitk", w) : nullptr;
  xtrg::gemm(g, c->stream, work, w);
}

// Independent GEMMs (one per chain of a batch step) in grouped launches.
void gemm_group(xtrg_ctx c, const std::vector<Gemm>& gs) {
  if (gs.empty()) return;
  const size_t w = xtrg::gemm_grouped_work(gs);
  double* work = w ? c->need("splitk_group", w) : nullptr;
  xtrg::gemm_grouped(gs, c->stream, work, w);
}

// Plain row-major C[MxN] = op(A) op(B).
Gemm plain(int M, int N, int K, const void* A, long lda, bool tA, const void* B, long ldb, bool tB,
           void* C, long ldc, int prec = xtrg::GEMM_F64, int out64 = 1) {
  Gemm g;
  g.M = M; g.N = N; g.K = K;
  g.prec = prec; g.out64 = out64;
  g.A = A; g.lda = lda; g.transA = tA;
  g.B = B; g.ldb = ldb; g.transB = tB;
  g.C = C; g.ldc = ldc;
  return g;
}

// ---------------------------------------------------------------------------
// Automaton Hamiltonian MPO (App. B.1)
// ---------------------------------------------------------------------------

struct Automaton {
  int n = 0;
  std::vector<int> dims;                 // n+1 open dims (2 at both ends)
  std::vector<std::vector<double>> T;    // [Dl][2][2][Dr]
};

Automaton build_automaton(int n, int nb, const int* bonds, const double* jxy, const double* jz) {
  std::map<std::pair<int, int>, std::pair<double, double>> coup;
  for (int b = 0; b < nb; ++b) {
    int i = bonds[2 * b], j = bonds[2 * b + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) throw Error(XTRG_EINVAL, "bad bond index");
    if (i > j) std::swap(i, j);
    auto& v = coup[{i, j}];
    v.first += jxy[b];
    v.second += jz[b];
  }
  // pending[p]: sites i <= p with a partner j > p (interaction terms open across cut p)
  std::vector<std::vector<int>> pend(std::max(n - 1, 0));
  for (int p = 0; p + 1 < n; ++p) {
    std::vector<int> s;
    for (auto& kv : coup)
      if (kv.first.first <= p && p < kv.first.second) s.push_back(kv.first.first);
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    pend[p] = s;
  }
  auto chan = [&](int cut, int site, int a) {
    const auto& P = pend[cut];
    const int k = (int)(std::lower_bound(P.begin(), P.end(), site) - P.begin());
    return 2 + 3 * k + a;
  };
  // local operators: basis (up, down); S+ = |up><down|
  const double Sp[2][2] = {{0, 1}, {0, 0}}, Sm[2][2] = {{0, 0}, {1, 0}}, Sz[2][2] = {{0.5, 0}, {0, -0.5}};
  const double Id[2][2] = {{1, 0}, {0, 1}};
  const double (*open_op[3])[2] = {Sp, Sm, Sz};
  const double (*close_op[3])[2] = {Sm, Sp, Sz};

  Automaton A;
  A.n = n;
  A.dims.resize(n + 1);
  A.dims[0] = 2;
  A.dims[n] = 2;
  for (int p = 0; p + 1 < n; ++p) A.dims[p + 1] = 2 + 3 * (int)pend[p].size();
  A.T.resize(n);
  for (int p = 0; p < n; ++p) {
    const int Dl = A.dims[p], Dr = A.dims[p + 1];
    std::vector<double> T((size_t)Dl * 4 * Dr, 0.0);
    auto put = [&](int a, int b, const double (*op)[2], double cf) {
      for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t) T[(((size_t)a * 2 + s) * 2 + t) * Dr + b] += cf * op[s][t];
    };
    put(0, 0, Id, 1.0);  // start -> start
    put(1, 1, Id, 1.0);  // stop -> stop
    if (p + 1 < n && std::binary_search(pend[p].begin(), pend[p].end(), p))
      for (int a = 0; a < 3; ++a) put(0, chan(p, p, a), open_op[a], 1.0);   // open at site p
    if (p > 0) {
      for (int i : pend[p - 1]) {
        if (p + 1 < n && std::binary_search(pend[p].begin(), pend[p].end(), i))
          for (int a = 0; a < 3; ++a) put(chan(p - 1, i, a), chan(p, i, a), Id, 1.0);  // carry
        auto it = coup.find({i, p});
        if (it != coup.end()) {                                                   // close at p
          const double cf[3] = {0.5 * it->second.first, 0.5 * it->second.first, it->second.second};
          for (int a = 0; a < 3; ++a) put(chan(p - 1, i, a), 1, close_op[a], cf[a]);
        }
      }
    }
    A.T[p] = std::move(T);
  }
  return A;
}

// Cap the outer bonds: left with e_start, right with the vector `r` (length 2).
std::vector<std::vector<double>> cap(const Automaton& A, const double r[2], std::vector<int>* dims) {
  const int n = A.n;
  std::vector<std::vector<double>> S(n);
  dims->assign(n + 1, 0);
  for (int p = 0; p < n; ++p) (*dims)[p] = A.dims[p];
  (*dims)[n] = 1;
  (*dims)[0] = 1;
  for (int p = 0; p < n; ++p) {
    const int Dl = A.dims[p], Dr = A.dims[p + 1];
    const int dl = (p == 0) ? 1 : Dl, dr = (p == n - 1) ? 1 : Dr;
    std::vector<double> T((size_t)dl * 4 * dr, 0.0);
    for (int a = 0; a < dl; ++a)
      for (int st = 0; st < 4; ++st)
        for (int b = 0; b < dr; ++b) {
          double v;
          if (p == n - 1) {
            v = 0.0;
            for (int q = 0; q < 2; ++q) v += A.T[p][((size_t)a * 4 + st) * Dr + q] * r[q];
          } else {
            v = A.T[p][((size_t)a * 4 + st) * Dr + b];
          }
          T[((size_t)a * 4 + st) * dr + b] = v;   // p == 0: a = 0 is the start row
        }
    S[p] = std::move(T);
  }
  return S;
}

// ---------------------------------------------------------------------------
// Canonical forms by SVD sweeps (all on device)
// ---------------------------------------------------------------------------

std::vector<double> read_vec(xtrg_ctx c, const double* d, size_t n) {
  std::vector<double> h(n);
  if (n) {
    XTRG_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    XTRG_HIP(hipStreamSynchronize(c->stream));
  }
  return h;
}

// Absolute rounding-noise floor of the matrix last decomposed in `work`.
// work holds an SVD of len x p_work columns; p is the column count of the
// matrix whose rounding noise is meant (C_E itself when the SVD ran on C_E
// rotated into extra columns).
double noise_floor(xtrg_ctx c, const double* work, int len, int p_work, int p) {
  const double f2 = read_vec(c, xtrg::svd_fro2(work, len, p_work), 1)[0];
  return xtrg::svd_keep_rel(len, p) * std::sqrt(std::max(f2, 0.0));
}
double noise_floor(xtrg_ctx c, const double* work, int len, int p) { return noise_floor(c, work, len, p, p); }

// Enforce orthonormal columns on the len x k isometry U by Newton-Schulz
// polar iterations U <- U (3I - U^T U)/2: the column space is kept and the
// deviation from orthonormality e goes to (3/4) e^2 per iteration.  U is
// stored row-major [len][k] (rowmajor) or as U^T row-major [k][len].  The
// Jacobi columns of tiny singular values are orthogonal only to the
// rounding noise of the large ones; this restores the canonical form.
void orthonormalize(xtrg_ctx c, double* U, int len, int k, bool rowmajor) {
  if (k <= 0 || len <= 0) return;
  double* X = c->need("ns_X", (size_t)k * k);
  double* T = c->need("ns_T", (size_t)len * k);
  for (int it = 0; it < 4; ++it) {
    if (rowmajor) {
      gemm(c, plain(k, k, len, U, k, true, U, k, false, X, k));        // U^T U
      gemm(c, plain(len, k, k, U, k, false, X, k, false, T, k));       // U (U^T U)
    } else {
      gemm(c, plain(k, k, len, U, len, false, U, len, true, X, k));    // U^T U from U^T
      gemm(c, plain(k, len, k, X, k, false, U, len, false, T, len));   // (U^T U) U^T
    }
    xtrg::axpby(U, 1.5, T, -0.5, (size_t)len * k, c->stream);
  }
}

// ---------------------------------------------------------------------------
// U(1) charge sectors (Sec. II.A: the XXZ models conserve S^z_tot, and the
// paper's tensors are blocked by it; App. B.2).  The tensors stay dense; the
// S^z charges label the bond indices, and a matrix that conserves the charge
// is factorised block by block.
// ---------------------------------------------------------------------------

// Charges of every bond index from the non-zero entries of host copies of
// the sites (xtrg_host::infer_charges), with the library's error code.
std::vector<std::vector<int>> infer_charges(const std::vector<std::vector<double>>& W, const std::vector<int>& dims) {
  try {
    return xtrg_host::infer_charges(W, dims);
  } catch (const std::invalid_argument& e) {
    throw Error(XTRG_EINVAL, e.what());
  }
}

// Factorisation of a len x p column-major matrix Y whose entries vanish
// unless the charge of the row (ql) equals that of the column (qp): sorted by
// charge it is block diagonal, and its singular triples are those of its
// blocks.  Every block is one problem of a grouped Jacobi SVD.
struct BlockSvd {
  struct Blk {
    int q = 0, len = 0, p = 0;
    size_t off = 0;         // its index lists in idx: rows, then columns, then the merged positions of the kept triples
    int* d_idx = nullptr;   // the same on the device
    double* Y = nullptr;
    double* work = nullptr;
    int psvd = 0;           // columns of the SVD input (p, or more with a warm basis)
    std::vector<double> S;  // after merge(): the block's values, descending
    int kept = 0;
  };
  std::vector<Blk> b;
  std::vector<int> idx;           // the index lists of all blocks (one upload each way)
  int* d_idx = nullptr;
  const double* Y = nullptr;
  int len = 0, p = 0;
  double* chk = nullptr;          // device: ||Y||_F^2, then 1024 partials
  // after merge(): the values of all blocks, descending (equal values in
  // increasing charge), with their charge, block and rank in the block
  std::vector<double> S;
  std::vector<int> qs, from, rank;
  double fro2 = 0.0;              // sum of the blocks' ||Y_q||_F^2
};

// warm(q, len_q, p_q, Y_q): the SVD input of block q (Y_q itself, or Y_q
// rotated into a warm basis) and its column count.
using WarmHook = std::function<std::pair<const double*, int>(int, int, int, const double*)>;

// Split Y into its charge blocks and append one SVD problem per block to
// jobs.  `tag` names the workspaces (one set per concurrent factorisation).
void bsvd_prepare(xtrg_ctx c, const std::string& tag, const double* Y, int len, int p, const std::vector<int>& ql,
                  const std::vector<int>& qp, BlockSvd& B, std::vector<xtrg::SvdJob>& jobs,
                  const WarmHook& warm = nullptr) {
  if ((int)ql.size() != len || (int)qp.size() != p) throw Error(XTRG_EINVAL, "charge lists do not match the tensor");
  hipStream_t s = c->stream;
  B = BlockSvd{};
  B.Y = Y;
  B.len = len;
  B.p = p;
  for (const auto& cb : xtrg_host::charge_blocks(ql, qp)) {
    BlockSvd::Blk k;
    k.q = cb.q;
    k.len = (int)cb.rows.size();
    k.p = (int)cb.cols.size();
    k.off = B.idx.size();
    B.idx.insert(B.idx.end(), cb.rows.begin(), cb.rows.end());
    B.idx.insert(B.idx.end(), cb.cols.begin(), cb.cols.end());
    B.idx.resize(B.idx.size() + std::min(k.len, k.p), 0);
    B.b.push_back(std::move(k));
  }
  if (B.b.empty()) throw Error(XTRG_EINVAL, "no S^z charge is shared by the rows and the columns");
  // one upload for all blocks (an upload from pageable memory waits for the stream)
  B.d_idx = reinterpret_cast<int*>(c->need("u1_idx" + tag, B.idx.size() / 2 + 1));
  XTRG_HIP(hipMemcpyAsync(B.d_idx, B.idx.data(), sizeof(int) * B.idx.size(), hipMemcpyHostToDevice, s));
  B.chk = c->need("u1_chk" + tag, 1026);
  xtrg::sumsq(Y, (size_t)len * p, B.chk, B.chk + 2, s);
  for (size_t t = 0; t < B.b.size(); ++t) {
    auto& k = B.b[t];
    const std::string nm = tag + "/" + std::to_string(t);
    k.d_idx = B.d_idx + k.off;
    k.Y = c->need("u1_Y" + nm, (size_t)k.len * k.p);
    xtrg::gather_block(k.Y, Y, len, k.d_idx, k.len, k.d_idx + k.len, k.p, s);
    const double* in = k.Y;
    k.psvd = k.p;
    if (warm) std::tie(in, k.psvd) = warm(k.q, k.len, k.p, k.Y);
    k.work = c->need("u1_svd" + nm, xtrg::svd_work(k.len, k.psvd));
    jobs.push_back(xtrg::SvdJob{k.len, k.psvd, in, k.work, 0, svd_gram(c, "u1" + nm, k.psvd)});
  }
}

// After the grouped SVD: the values of all blocks, merged and sorted; throws
// if Y has weight between different charges (beyond rounding).
void bsvd_merge(xtrg_ctx c, const std::string& tag, BlockSvd& B) {
  hipStream_t s = c->stream;
  size_t n = 1;
  for (auto& k : B.b) n += 1 + std::min(k.len, k.p);
  double* st = c->need("u1_vals" + tag, n);
  if (B.b.size() <= (size_t)xtrg::ValGather::kMax) {   // one launch for all blocks
    xtrg::ValGather g;
    g.n = (int)B.b.size();
    g.head = B.chk;
    g.out = st;
    size_t o = 1;
    for (int t = 0; t < g.n; ++t) {
      const auto& k = B.b[t];
      g.f2[t] = xtrg::svd_fro2(k.work, k.len, k.psvd);
      g.v[t] = xtrg::svd_sorted_values(k.work, k.len, k.psvd);
      g.r[t] = std::min(k.len, k.p);
      g.off[t] = (int)o;
      o += 1 + g.r[t];
    }
    xtrg::gather_values(g, s);
  } else {
    XTRG_HIP(hipMemcpyAsync(st, B.chk, sizeof(double), hipMemcpyDeviceToDevice, s));
    size_t o = 1;
    for (auto& k : B.b) {
      const int r = std::min(k.len, k.p);
      XTRG_HIP(hipMemcpyAsync(st + o, xtrg::svd_fro2(k.work, k.len, k.psvd), sizeof(double),
                              hipMemcpyDeviceToDevice, s));
      XTRG_HIP(hipMemcpyAsync(st + o + 1, xtrg::svd_sorted_values(k.work, k.len, k.psvd), sizeof(double) * r,
                              hipMemcpyDeviceToDevice, s));
      o += 1 + r;
    }
  }
  size_t o = 1;
  const std::vector<double> h = read_vec(c, st, n);
  B.fro2 = 0.0;
  o = 1;
  std::vector<int> qb(B.b.size());
  std::vector<std::vector<double>> Sb(B.b.size());
  for (size_t t = 0; t < B.b.size(); ++t) {
    auto& k = B.b[t];
    const int r = std::min(k.len, k.p);
    k.S.assign(h.begin() + o + 1, h.begin() + o + 1 + r);
    for (double v : k.S)
      if (!std::isfinite(v)) throw Error(XTRG_ENUMERIC, "non-finite singular value");
    B.fro2 += h[o];
    qb[t] = k.q;
    Sb[t] = k.S;
    o += 1 + r;
  }
  const double full = h[0];
  if (!std::isfinite(full)) throw Error(XTRG_ENUMERIC, "non-finite entries in the two-site tensor");
  if (std::fabs(full - B.fro2) > 1e-10 * full)
    throw Error(XTRG_EINVAL, "the tensor has weight between different S^z charges: the inputs do not conserve "
                             "S^z in their bond bases");
  xtrg_host::Merged m = xtrg_host::merge_block_values(qb, Sb);
  B.S = std::move(m.S);
  B.qs = std::move(m.qs);
  B.from = std::move(m.from);
  B.rank = std::move(m.rank);
}

// The first k merged singular vectors as a dense len x k matrix: dst[r*k + j]
// (rowmajor) or dst[j*len + r]; zero outside each vector's block.
void bsvd_scatter(xtrg_ctx c, const std::string& tag, BlockSvd& B, int k, double* dst, int rowmajor) {
  hipStream_t s = c->stream;
  xtrg::fill(dst, 0.0, (size_t)B.len * k, s);
  for (auto& blk : B.b) blk.kept = 0;
  for (int j = 0; j < k; ++j) {
    auto& blk = B.b[B.from[j]];
    if (B.rank[j] != blk.kept) throw Error(XTRG_EINVAL, "block SVD: kept values out of order");
    B.idx[blk.off + blk.len + blk.p + blk.kept] = j;
    blk.kept += 1;
  }
  XTRG_HIP(hipMemcpyAsync(B.d_idx, B.idx.data(), sizeof(int) * B.idx.size(), hipMemcpyHostToDevice, s));
  for (auto& blk : B.b) {
    if (blk.kept == 0) continue;
    int* pos = blk.d_idx + blk.len + blk.p;
    double* tmp = c->need("u1_vec" + tag, (size_t)blk.len * blk.kept);
    xtrg::svd_gather(blk.len, blk.psvd, blk.work, blk.kept, tmp, blk.len, 0, s);
    xtrg::scatter_cols(dst, B.len, k, rowmajor, tmp, blk.len, blk.kept, blk.d_idx, pos, s);
  }
}

// One block factorisation on its own (the canonical sweeps of the start).
void bsvd_run(xtrg_ctx c, const std::string& tag, const double* Y, int len, int p, const std::vector<int>& ql,
              const std::vector<int>& qp, BlockSvd& B) {
  std::vector<xtrg::SvdJob> jobs;
  bsvd_prepare(c, tag, Y, len, p, ql, qp, B, jobs);
  xtrg::svd_batched(jobs, svd_desc(c, (int)jobs.size()), c->stream);
  for (const auto& j : jobs)
    if (j.status != 0) throw Error(XTRG_ENUMERIC, "block SVD: non-finite entries or no convergence");
  bsvd_merge(c, tag, B);
}

// Replace site i's buffer by a new one of n doubles.
double* reshape_site(xtrg_mpo m, int i, size_t n) {
  xtrg_ctx c = m->ctx;
  if (m->site[i].n < n) {
    c->release(m->site[i].p, m->site[i].n);
    m->site[i].p = c->alloc(n);
    m->site[i].n = n;
  }
  return m->site[i].p;
}

// Left-to-right: site i = U (left-isometric), R = S V^T pushed into site i+1.
// Singular values <= floor * s_1 are dropped (floor = 0 keeps all nonzero).
void left_sweep(xtrg_mpo m, double floor, std::vector<std::vector<double>>* sv) {
  xtrg_ctx c = m->ctx;
  hipStream_t s = c->stream;
  for (int i = 0; i + 1 < m->L; ++i) {
    const int Dl = m->dims[i], Dr = m->dims[i + 1], Dn = m->dims[i + 2];
    const int rows = Dl * 4;
    double* Y = c->need("cs_Y", (size_t)rows * Dr);
    xtrg::transpose(Y, rows, m->site[i].p, Dr, Dr, rows, s);          // Y col-major (rows x Dr)
    // note: transpose(dst, ldd, src, lds, R, C) reads src column-major (C cols of R);
    // the site matrix [rows][Dr] row-major is (Dr x rows) column-major.
    double* work = c->need("cs_work", xtrg::svd_work(rows, Dr));
    xtrg::svd_left(rows, Dr, Y, nullptr, 0, nullptr, 0, 0, work, svd_desc(c, 1), s, nullptr);
    std::vector<double> S = read_vec(c, xtrg::svd_sorted_values(work, rows, Dr), Dr);
    const int lim = std::min(rows, Dr);
    S.resize(lim);
    const double nf = noise_floor(c, work, rows, Dr);
    int k = 0;
    for (double v : S)
      if (v > floor * S[0] && v > nf && v > 0) ++k;
    k = std::max(k, 1);
    if (sv) sv->push_back(S);
    double* U = c->need("cs_U", (size_t)rows * k);
    xtrg::svd_gather(rows, Dr, work, k, U, k, 1, s);                   // U row-major [rows][k]
    orthonormalize(c, U, rows, k, true);
    double* R = c->need("cs_R", (size_t)k * Dr);
    gemm(c, plain(k, Dr, rows, U, k, true, m->site[i].p, Dr, false, R, Dr));   // R = U^T M
    double* Nn = c->need("cs_N", (size_t)k * 4 * Dn);
    gemm(c, plain(k, 4 * Dn, Dr, R, Dr, false, m->site[i + 1].p, 4 * Dn, false, Nn, 4 * Dn));
    xtrg::copy(reshape_site(m, i, (size_t)rows * k), U, (size_t)rows * k, s);
    xtrg::copy(reshape_site(m, i + 1, (size_t)k * 4 * Dn), Nn, (size_t)k * 4 * Dn, s);
    m->dims[i + 1] = k;
  }
}

// Right-to-left: site i = V^T (right-isometric), U S pushed into site i-1.
// Keeps at most Dmax (if > 0; with degen > 0 backing off as the keep rule
// of the doubling does, so that a multiplet is not split) and drops values
// <= floor * s_1.  Records the singular values of every bond (bond i-1 | i)
// in sv (indexed by bond).
void right_sweep(xtrg_mpo m, double floor, int Dmax, std::vector<std::vector<double>>* sv, double degen = 0.0) {
  xtrg_ctx c = m->ctx;
  hipStream_t s = c->stream;
  if (sv) sv->assign(std::max(m->L - 1, 0), {});
  for (int i = m->L - 1; i >= 1; --i) {
    const int Dl = m->dims[i], Dr = m->dims[i + 1], Dp = m->dims[i - 1];
    const int len = 4 * Dr;
    double* work = c->need("cs_work", xtrg::svd_work(len, Dl));
    xtrg::svd_left(len, Dl, m->site[i].p, nullptr, 0, nullptr, 0, 0, work, svd_desc(c, 1), s, nullptr);
    std::vector<double> S = read_vec(c, xtrg::svd_sorted_values(work, len, Dl), Dl);
    S.resize(std::min(len, Dl));
    const double nf = noise_floor(c, work, len, Dl);
    const int k = keep_count(S, Dmax > 0 ? Dmax : std::numeric_limits<int>::max(), degen, floor, nf);
    if (sv) (*sv)[i - 1] = S;
    double* V = c->need("cs_V", (size_t)len * k);
    xtrg::svd_gather(len, Dl, work, k, V, len, 0, s);                 // V col-major = V^T row-major [k][len]
    orthonormalize(c, V, len, k, false);
    double* US = c->need("cs_R", (size_t)Dl * k);
    gemm(c, plain(Dl, k, len, m->site[i].p, len, false, V, len, true, US, k));   // U S = M V
    double* Pn = c->need("cs_N", (size_t)Dp * 4 * k);
    gemm(c, plain(Dp * 4, k, Dl, m->site[i - 1].p, Dl, false, US, k, false, Pn, k));
    xtrg::copy(reshape_site(m, i, (size_t)k * len), V, (size_t)k * len, s);
    xtrg::copy(reshape_site(m, i - 1, (size_t)Dp * 4 * k), Pn, (size_t)Dp * 4 * k, s);
    m->dims[i] = k;
  }
}

// left_sweep and right_sweep with charge-definite bonds: every site matrix
// is factorised by charge blocks (m->charges labels its bonds and is kept up
// to date), so the new bond indices carry their block's charge.
void left_sweep_u1(xtrg_mpo m, double floor) {
  xtrg_ctx c = m->ctx;
  hipStream_t s = c->stream;
  auto& q = m->charges;
  BlockSvd B;
  for (int i = 0; i + 1 < m->L; ++i) {
    const int Dl = m->dims[i], Dr = m->dims[i + 1], Dn = m->dims[i + 2];
    const int rows = Dl * 4;
    double* Y = c->need("cs_Y", (size_t)rows * Dr);
    xtrg::transpose(Y, rows, m->site[i].p, Dr, Dr, rows, s);          // Y col-major (rows x Dr)
    bsvd_run(c, "cs", Y, rows, Dr, row_charges(q[i]), q[i + 1], B);
    const double nf = xtrg::svd_keep_rel(rows, Dr) * std::sqrt(B.fro2);
    int k = 0;
    for (double v : B.S)
      if (v > floor * B.S[0] && v > nf && v > 0) ++k;
    k = std::max(k, 1);
    double* U = c->need("cs_U", (size_t)rows * k);
    bsvd_scatter(c, "cs", B, k, U, 1);                                 // U row-major [rows][k]
    orthonormalize(c, U, rows, k, true);
    double* R = c->need("cs_R", (size_t)k * Dr);
    gemm(c, plain(k, Dr, rows, U, k, true, m->site[i].p, Dr, false, R, Dr));   // R = U^T M
    double* Nn = c->need("cs_N", (size_t)k * 4 * Dn);
    gemm(c, plain(k, 4 * Dn, Dr, R, Dr, false, m->site[i + 1].p, 4 * Dn, false, Nn, 4 * Dn));
    xtrg::copy(reshape_site(m, i, (size_t)rows * k), U, (size_t)rows * k, s);
    xtrg::copy(reshape_site(m, i + 1, (size_t)k * 4 * Dn), Nn, (size_t)k * 4 * Dn, s);
    m->dims[i + 1] = k;
    q[i + 1].assign(B.qs.begin(), B.qs.begin() + k);
  }
}

void right_sweep_u1(xtrg_mpo m, double floor, int Dmax) {
  xtrg_ctx c = m->ctx;
  hipStream_t s = c->stream;
  auto& q = m->charges;
  BlockSvd B;
  for (int i = m->L - 1; i >= 1; --i) {
    const int Dl = m->dims[i], Dr = m->dims[i + 1], Dp = m->dims[i - 1];
    const int len = 4 * Dr;
    bsvd_run(c, "cs", m->site[i].p, len, Dl, col_charges(q[i + 1]), q[i], B);
    const double nf = xtrg::svd_keep_rel(len, Dl) * std::sqrt(B.fro2);
    const int k = keep_count(B.S, Dmax > 0 ? Dmax : std::numeric_limits<int>::max(), 0.0, floor, nf);
    double* V = c->need("cs_V", (size_t)len * k);
    bsvd_scatter(c, "cs", B, k, V, 0);                                 // V^T row-major [k][len]
    orthonormalize(c, V, len, k, false);
    double* US = c->need("cs_R", (size_t)Dl * k);
    gemm(c, plain(Dl, k, len, m->site[i].p, len, false, V, len, true, US, k));   // U S = M V
    double* Pn = c->need("cs_N", (size_t)Dp * 4 * k);
    gemm(c, plain(Dp * 4, k, Dl, m->site[i - 1].p, Dl, false, US, k, false, Pn, k));
    xtrg::copy(reshape_site(m, i, (size_t)k * len), V, (size_t)k * len, s);
    xtrg::copy(reshape_site(m, i - 1, (size_t)Dp * 4 * k), Pn, (size_t)Dp * 4 * k, s);
    m->dims[i] = k;
    q[i].assign(B.qs.begin(), B.qs.begin() + k);
  }
}

// Host copies of the sites.
std::vector<std::vector<double>> download_sites(xtrg_mpo m) {
  std::vector<std::vector<double>> W(m->L);
  for (int i = 0; i < m->L; ++i) W[i] = read_vec(m->ctx, m->site[i].p, m->elems(i));
  return W;
}

double site_norm(xtrg_mpo m, int i) {
  xtrg_ctx c = m->ctx;
  xtrg::sumsq(m->site[i].p, m->elems(i), c->scratch, c->scratch + 1024, c->stream);
  return std::sqrt(read_scalar(c, c->scratch));
}

std::unique_ptr<xtrg_mpo_s> clone(xtrg_mpo src) {
  auto m = new_mpo(src->ctx, src->dims);
  for (int i = 0; i < src->L; ++i) xtrg::copy(m->site[i].p, src->site[i].p, src->elems(i), src->ctx->stream);
  m->charges = src->charges;
  return m;
}

// ---------------------------------------------------------------------------
// The doubling step (App. D.1, Fig. VMPO)
// ---------------------------------------------------------------------------

using xtrg_host::Step;
using xtrg_host::schedule;

struct Doubler {
  xtrg_ctx c;
  int L;
  std::vector<int> Da;                  // bonds of A (the left factor; rho in a doubling)
  std::vector<int> Db;                  // bonds of B (the right factor; rho in a doubling)
  std::vector<int> Dc;                  // bonds of C
  std::vector<int> cap;                 // largest possible bond of C
  // Working precision of the contractions: GEMM_F64, or GEMM_F32 with FP32
  // copies of rho, the environments, the blocks and C (the SVD, the split
  // and the output sites stay FP64).
  int prec = xtrg::GEMM_F64;
  std::vector<const void*> A;           // sites of A (working precision)
  std::vector<const void*> B;           // sites of B (working precision)
  std::vector<void*> Bp;                // sites of B with the physical indices swapped
  std::string tag;                      // suffix of the chain's workspace names
  std::vector<Site> C;                  // output sites, FP64 (capacity at cap)
  std::vector<void*> Cw;                // working-precision copies of C (C itself in FP64)
  std::map<int, void*> slot;            // Lb_i or Rb_i: one named workspace per site

  // Named workspace of n elements of the working precision.
  void* needw(const std::string& name, size_t n) {
    if (prec == xtrg::GEMM_F64) return c->need(name, n);
    return c->need(name + "/f32", (n + 1) / 2);
  }
  // Refresh the working copy of C_i (n leading elements) after C_i changed.
  void sync_cw(int i, size_t n) {
    if (prec != xtrg::GEMM_F64) xtrg::to_f32(static_cast<float*>(Cw[i]), C[i].p, n, c->stream);
  }
  Gemm wplain(int M, int N, int K, const void* A_, long lda, bool tA, const void* B_, long ldb, bool tB,
              void* C_, long ldc) const {
    return plain(M, N, K, A_, lda, tA, B_, ldb, tB, C_, ldc, prec, 0);
  }

  // Slot i holds Lb_i (4 cap_i Da_{i+1} Db_{i+1}) or Rb_i (Da_i Db_i 4 cap_{i+1}).
  void* slot_need(int i) {
    const size_t n = std::max((size_t)4 * cap[i] * Da[i + 1] * Db[i + 1], (size_t)Da[i] * Db[i] * 4 * cap[i + 1]);
    return slot[i] = needw("slot" + std::to_string(i) + tag, n);
  }

  // Lb[(c,s,s'')][(a',b')] = sum_{a,b,s'} E[c][a][b] A_i[a][s][s'][a'] B_i[b][s'][s''][b']:
  // two batched GEMMs, the second reading the first's output X (the chain's own)
  std::pair<Gemm, Gemm> left_block_gemms(int i, const void* E, void* out) {
    const int dc = Dc[i], da = Da[i], db = Db[i], da2 = Da[i + 1], db2 = Db[i + 1];
    void* X = needw("X" + tag, (size_t)dc * 4 * db * da2);
    Gemm g1;
    g1.prec = prec; g1.out64 = 0;   // X[c][s][b][(s',a')] = sum_a E[c][a][b] A[a][s][(s',a')]   batch (c, s)
    g1.M = db; g1.N = 2 * da2; g1.K = da;
    g1.transA = 1; g1.A = E; g1.lda = db;
    g1.B = A[i]; g1.ldb = 4 * da2;
    g1.C = X; g1.ldc = 2 * da2;
    g1.nb[0] = dc; g1.nb[1] = 2;
    g1.sA[0] = (long)da * db;
    g1.sB[1] = 2L * da2;
    g1.sC[0] = 4L * db * da2; g1.sC[1] = 2L * db * da2;
    Gemm g2;
    g2.prec = prec; g2.out64 = 0;
    //         Lb[c][s][s''][a'][b'] = sum_{(b,s')} X[c][s][(b,s')][a'] B[(b,s')][s''][b']  batch (c,s,s'')
    g2.M = da2; g2.N = db2; g2.K = 2 * db;
    g2.transA = 1; g2.A = X; g2.lda = da2;
    g2.B = B[i]; g2.ldb = 2 * db2;
    g2.C = out; g2.ldc = db2;
    g2.nb[0] = dc; g2.nb[1] = 2; g2.nb[2] = 2;
    g2.sA[0] = 4L * db * da2; g2.sA[1] = 2L * db * da2;
    g2.sB[2] = db2;
    g2.sC[0] = 4L * da2 * db2; g2.sC[1] = 2L * da2 * db2; g2.sC[2] = (long)da2 * db2;
    return {g1, g2};
  }

  // Rb[(a,b)][(t,t'',c'')] = sum_{a'',b'',t'} A_j[a][t][t'][a''] B_j[b][t'][t''][b''] F[a''][b''][c'']
  std::pair<Gemm, Gemm> right_block_gemms(int j, const void* F, void* out) {
    const int da = Da[j], db = Db[j], da2 = Da[j + 1], db2 = Db[j + 1], dc2 = Dc[j + 1];
    void* Z = needw("X" + tag, (size_t)4 * da * db2 * dc2);
    const Gemm g1 = wplain(4 * da, db2 * dc2, da2, A[j], da2, false, F, (long)db2 * dc2, false, Z, (long)db2 * dc2);
    Gemm g;
    g.prec = prec; g.out64 = 0;
    //         batch (a, t, t''): Rb[a][b][t][t''][c''] = sum_{(t',b'')} Bp[b][t''][(t',b'')] Z[a][t][(t',b'')][c'']
    g.M = db; g.N = dc2; g.K = 2 * db2;
    g.A = Bp[j]; g.lda = 4 * db2;
    g.B = Z; g.ldb = dc2;
    g.C = out; g.ldc = 4 * dc2;
    g.nb[0] = da; g.nb[1] = 2; g.nb[2] = 2;
    g.sA[2] = 2L * db2;
    g.sB[0] = 4L * db2 * dc2; g.sB[1] = 2L * db2 * dc2;
    g.sC[0] = 4L * db * dc2; g.sC[1] = 2L * dc2; g.sC[2] = dc2;
    return {g1, g};
  }

  void left_block(int i, const void* E, void* out) {
    const auto g = left_block_gemms(i, E, out);
    gemm(c, g.first);
    gemm(c, g.second);
  }
  void right_block(int j, const void* F, void* out) {
    const auto g = right_block_gemms(j, F, out);
    gemm(c, g.first);
    gemm(c, g.second);
  }

  static double step_flops(int dc, int da, int db, int da2, int db2, int dc2) {
    const double k1 = 2.0 * dc * db * da * 4 * da2;
    const double k2 = 2.0 * dc * 2 * da2 * db * 4 * db2;
    const double th = 2.0 * (4.0 * dc) * ((double)da2 * db2) * (4.0 * dc2);
    const double k3 = 2.0 * da2 * db2 * (4.0 * dc) * dc;
    return k1 + k2 + th + k3;
  }
};

// State of one chain of a (possibly batched) doubling.
struct Chain {
  Doubler d;
  xtrg_compress_opts o;
  std::vector<Step> sched;
  std::string tag;                        // suffix of this chain's workspace names
  void* E = nullptr;                      // left environment of the current bond (working precision)
  void* F = nullptr;                      // right environment
  double* th = nullptr;                   // two-site overlap C_E
  double* work = nullptr;                 // SVD workspace
  std::vector<std::vector<double>> sv;
  std::vector<int> kept;
  std::vector<double> disc;
  double flops = 0.0, last_norm = 0.0;
  // Warm start of the SVD at each bond: an orthogonal basis from the
  // previous visit of the bond (side 0: left index of C_E, 1: right index).
  struct WarmQ {
    int side = -1;
    int dim = 0;      // rows of the basis block Q (the index dimension)
    int cols = 0;     // its columns: dim, plus the extra columns of the completion
  };
  std::vector<WarmQ> warm;
  std::vector<char> revisit;              // step st: its bond is visited again later
  size_t st = 0;                          // current step
  // current step
  int i = 0;
  bool gauge_right = false;
  const double* Y = nullptr;              // SVD input: C_E, or C_E rotated by the warm basis
  void* Lb = nullptr;
  void* Rb = nullptr;
  int mL = 0, mR = 0, Kt = 0, len = 0, p = 0;
  int psvd = 0;                           // columns of the SVD input (p, or p + extra with a warm start)
  bool svd_done = false;                  // the QR start produced this step's factorisation
  bool warm_now = false;                  // this step's SVD input was rotated by a warm basis
  int status = 0;                         // XTRG_OK, or the code that stopped this chain
  std::string err;                        // and its message
  // U(1) charge sectors: charges of C's bonds, and the block factorisation
  // of the current step
  bool u1 = false;
  std::vector<std::vector<int>> qc;
  BlockSvd bs;
  std::map<std::pair<int, int>, WarmQ> wq1;   // warm bases per (bond, charge block)
  std::string wq1_name(int i, int q) const { return "wq1_" + std::to_string(i) + "_" + std::to_string(q) + tag; }

};

void check_opts(const xtrg_compress_opts& o) {
  if (o.D_max < 1 || o.n_sweeps < 1) throw Error(XTRG_EINVAL, "D_max and n_sweeps must be >= 1");
  if (o.precision != XTRG_FP64 && o.precision != XTRG_FP32 && o.precision != XTRG_BF16X3)
    throw Error(XTRG_EINVAL, "precision must be XTRG_FP64, XTRG_FP32 or XTRG_BF16X3");
}

// Set up chain q of C ~ A B: initial guess C = B (right-canonical), working
// copies of A's and B's sites (B also with its physical indices swapped),
// and the static right blocks Rb_j, j = L-1 .. 1 (the first left-to-right
// half-sweep reads Rb_{i+1} for every bond i).  A doubling is A = B = rho.
void chain_setup(xtrg_ctx c, Chain& C, xtrg_mpo ina, xtrg_mpo inb, int q) {
  hipStream_t s = c->stream;
  const int L = inb->L;
  Doubler& d = C.d;
  C.tag = q == 0 ? "" : "#" + std::to_string(q);
  C.sched = schedule(L, C.o.n_sweeps);
  C.revisit.assign(C.sched.size(), 0);
  {
    std::vector<char> seen(L, 0);
    for (size_t q = C.sched.size(); q-- > 0;) {
      C.revisit[q] = seen[C.sched[q].bond];
      seen[C.sched[q].bond] = 1;
    }
  }
  d.c = c;
  d.L = L;
  d.tag = C.tag;
  d.prec = C.o.precision == XTRG_FP32     ? xtrg::GEMM_F32
           : C.o.precision == XTRG_BF16X3 ? xtrg::GEMM_BF16X3
                                          : xtrg::GEMM_F64;
  const bool same = ina == inb;
  C.u1 = C.o.u1 != 0;
  if (C.u1) {
    if (ina->charges.empty() || inb->charges.empty())
      throw Error(XTRG_EINVAL, "u1: the input MPOs carry no S^z charges (xtrg_init_rho_u1, xtrg_mpo_label_charges)");
    C.qc = inb->charges;                   // C = B
  }
  d.Da = ina->dims;
  d.Db = inb->dims;
  d.Dc = inb->dims;                        // initial guess C = B (right-canonical)
  d.cap.resize(L + 1);
  for (int i = 0; i <= L; ++i) {
    double cp = 1.0;
    for (int k = 0; k < std::min(i, L - i) && cp < 1e9; ++k) cp *= 4.0;
    d.cap[i] = (int)std::min<double>(cp, (double)std::max(C.o.D_max, inb->dims[i]));
  }
  d.A.resize(L);
  d.B.resize(L);
  d.Bp.resize(L);
  d.C.resize(L);
  d.Cw.resize(L);
  const bool f32 = d.prec != xtrg::GEMM_F64;
  for (int i = 0; i < L; ++i) {
    const std::string si = std::to_string(i) + C.tag;
    const size_t na = ina->elems(i), nb = inb->elems(i);
    d.C[i].n = (size_t)d.cap[i] * 4 * d.cap[i + 1];
    d.C[i].p = c->need("C" + si, d.C[i].n);
    xtrg::copy(d.C[i].p, inb->site[i].p, nb, s);
    if (!f32) {
      d.A[i] = ina->site[i].p;
      d.B[i] = inb->site[i].p;
      double* bp = c->need("Bp" + si, nb);
      xtrg::swap_phys(bp, inb->site[i].p, inb->dims[i], inb->dims[i + 1], s);
      d.Bp[i] = bp;
      d.Cw[i] = d.C[i].p;
    } else {
      float* a32 = static_cast<float*>(d.needw("A" + si, na));
      xtrg::to_f32(a32, ina->site[i].p, na, s);
      d.A[i] = a32;
      if (same) {
        d.B[i] = a32;
      } else {
        float* b32 = static_cast<float*>(d.needw("B" + si, nb));
        xtrg::to_f32(b32, inb->site[i].p, nb, s);
        d.B[i] = b32;
      }
      double* tmp = c->need("Bp_swap", nb);
      xtrg::swap_phys(tmp, inb->site[i].p, inb->dims[i], inb->dims[i + 1], s);
      float* bp32 = static_cast<float*>(d.needw("Bp" + si, nb));
      xtrg::to_f32(bp32, tmp, nb, s);
      d.Bp[i] = bp32;
      d.Cw[i] = d.needw("Cw" + si, d.C[i].n);
      d.sync_cw(i, nb);
    }
  }
  size_t env_max = 1;
  for (int i = 0; i <= L; ++i) env_max = std::max(env_max, (size_t)d.cap[i] * d.Da[i] * d.Db[i]);
  C.E = d.needw("E" + C.tag, env_max);
  C.F = d.needw("F" + C.tag, env_max);
  if (!f32) {
    xtrg::fill(static_cast<double*>(C.E), 1.0, 1, s);
    xtrg::fill(static_cast<double*>(C.F), 1.0, 1, s);
  } else {
    xtrg::fill_f32(static_cast<float*>(C.E), 1.0f, 1, s);
    xtrg::fill_f32(static_cast<float*>(C.F), 1.0f, 1, s);
  }
  C.sv.resize(L - 1);
  C.warm.assign(L - 1, Chain::WarmQ{});
  C.kept.assign(L - 1, 1);
  C.disc.assign(L - 1, 0.0);
  for (int j = L - 1; j >= 1; --j) {
    void* Rb = d.slot_need(j);
    d.right_block(j, C.F, Rb);
    if (j == 1) break;
    const int mR = 4 * d.Dc[j + 1];
    const int k = d.Dc[j];
    gemm(c, d.wplain(d.Da[j] * d.Db[j], k, mR, Rb, mR, false, d.Cw[j], mR, true, C.F, k));
  }
}

// ---------------------------------------------------------------------------
// Warm start of the SVD.  Consecutive visits of bond i share one index basis
// of C_E: a left-to-right step and the right-to-left step that follows it
// at the same bond share the left index (C_{i-1} is unchanged in between),
// that step and the next left-to-right one share the right index (C_{i+2}
// is unchanged).  The singular vectors of the previous visit on the shared
// side, completed to an orthogonal basis Q, rotate the next SVD input:
// Y Q has the same left singular vectors and values as Y for any orthogonal
// Q, and nearly orthogonal columns when Q is close to the new right
// singular vectors, so the one-sided Jacobi needs far fewer sweeps.  Q only
// steers the convergence; its orthogonality (to 1e-13) is what the result
// relies on, and it is checked.
// ---------------------------------------------------------------------------
constexpr int kWarmMin = 128;   // smallest SVD column count worth a warm start
// The same for a charge block: the blocks of one two-site tensor share the
// grouped Jacobi launches until the last of them converges, so a cold small
// block would add sweeps of its own after the warm large ones are done.
constexpr int kWarmMinBlock = 32;

// it Newton-Schulz steps X <- X (3I - X^T X)/2 on the columns of X
// (column-major len x k, sigma_max(X) < sqrt(3)): singular values below 1
// grow by up to 1.5 per step, then converge quadratically.
void ns_steps(xtrg_ctx c, double* X, int len, int k, int it) {
  double* G = c->need("wq_G", (size_t)k * k);
  double* T = c->need("wq_T", (size_t)len * k);
  for (int q = 0; q < it; ++q) {
    gemm(c, plain(k, k, len, X, len, false, X, len, true, G, k));       // X^T X
    gemm(c, plain(k, len, k, G, k, false, X, len, false, T, len));       // X (X^T X)
    xtrg::axpby(X, 1.5, T, -0.5, (size_t)len * k, c->stream);
  }
}

// Polar factor of X (column-major len x k, singular values in [s0, 1]):
// quintic steps X <- X (a I + b X^T X + c (X^T X)^2), which multiply small
// singular values by a = 3.4445 and map [s, 1] with s >= 0.3 into
// [0.70, 1.19], until the lower bound passes 0.3 (tracked on the host with
// the same polynomial), then 7 cubic Newton-Schulz steps, which converge
// quadratically from there (deviation 0.51 -> ~1e-26).
void polar_ns(xtrg_ctx c, double* X, int len, int k, double s0) {
  constexpr double a = 3.4445, b = -4.7750, cq = 2.0315;
  double* G = c->need("wq_G", (size_t)k * k);
  double* G2 = c->need("wq_G2", (size_t)k * k);
  double* T = c->need("wq_T", (size_t)len * k);
  double s = s0;
  for (int q = 0; s < 0.3 && q < 8; ++q) {
    gemm(c, plain(k, k, len, X, len, false, X, len, true, G, k));        // X^T X
    gemm(c, plain(k, k, k, G, k, false, G, k, false, G2, k));            // (X^T X)^2
    xtrg::axpby(G2, cq, G, b, (size_t)k * k, c->stream);                 // b G + c G^2
    gemm(c, plain(k, len, k, G2, k, false, X, len, false, T, len));      // X (b G + c G^2)
    xtrg::axpby(X, a, T, 1.0, (size_t)len * k, c->stream);
    s = s * (a + s * s * (b + cq * s * s));
  }
  ns_steps(c, X, len, k, 7);
}

// max |X^T X - I| for X column-major len x k.
double orth_dev(xtrg_ctx c, const double* X, int len, int k) {
  double* G = c->need("wq_G", (size_t)k * k);
  gemm(c, plain(k, k, len, X, len, false, X, len, true, G, k));
  xtrg::eye_dev(G, k, c->scratch, c->scratch + 1024, c->stream);
  return read_scalar(c, c->scratch);
}

// After the SVD of this visit: a basis block Q for the next visit of the
// bond, with Q Q^T = I on the row space of Y.  The normalised Jacobi columns
// above the noise level (r of them) are orthonormal to the Jacobi tolerance.
// The complement (dimension m = len - r) is represented by m + o hashed
// noise vectors projected off them (twice) and driven by Newton-Schulz to
// their polar factor X, for which X X^T is the projector onto the complement
// (the o surplus directions have singular values that stay at rounding
// level and add ~1e-25 to X X^T).  The surplus keeps the noise block
// rectangular and so well conditioned: a square random block has a smallest
// singular value with a tail towards zero.  The next SVD runs on Y [Q0 X]
// (len + o columns), whose left singular vectors and values are those of Y.
constexpr int kWarmExtra = 32;

// The block from the Jacobi workspace `work` of a dim x pw problem (sorted
// values S) into Q (dim x (dim + kWarmExtra) doubles, column-major).
// Returns its column count, 0 if none is built (small, or mostly noise), or
// -1 if it fails the orthogonality check; *m_out: the completion size.
// *dev (device) = max |Q Q^T - I| of the len x cols basis Q.
void basis_check(xtrg_ctx c, const double* Q, int len, int cols, double* dev) {
  double* G = c->need("wq_G", (size_t)len * len);
  gemm(c, plain(len, len, cols, Q, len, true, Q, len, false, G, len));  // Q Q^T
  xtrg::eye_dev(G, len, dev, c->scratch + 1024, c->stream);
}

// The Jacobi leaves cosines <= 8 sqrt(len) eps between kept columns; a
// basis passes when Q Q^T is the identity to 4x that.
double basis_lim(int len) { return 32.0 * std::sqrt((double)len) * 2.220446049250313e-16; }

// A basis that failed its first check: up to two rounds of further
// Newton-Schulz steps on its completion (m + o columns after the first
// len - m), each followed by the check.  Returns cols, or -1.
int basis_retry(xtrg_ctx c, double* Q, int len, int cols, int m) {
  if (m == 0) return -1;
  const int o = cols - len, r = len - m;
  for (int attempt = 1; attempt <= 2; ++attempt) {
    ns_steps(c, Q + (size_t)len * r, len, m + o, 3);
    basis_check(c, Q, len, cols, c->scratch);
    if (read_scalar(c, c->scratch) <= basis_lim(len)) return cols;
  }
  return -1;
}

// dev_out (device, optional): leave the first orthogonality check there for
// the caller to read (together with other bases) and return the columns
// the basis has if it passes; basis_retry then handles one that does not.
int build_basis(xtrg_ctx c, double* work, int dim, int pw, const std::vector<double>& S, double keep_floor,
                unsigned long long seed, double* Q, int* m_out, int min_len = kWarmMin, double* dev_out = nullptr) {
  hipStream_t s = c->stream;
  const int len = dim;
  *m_out = 0;
  if (len < min_len || pw < 1) return 0;
  int r = 0;
  const int rmax = std::min(len, pw);
  while (r < rmax && S[r] > 0.5 * keep_floor) ++r;
  const int m = len - r;
  if (4 * r < len) return 0;                // mostly noise: the completion would dominate
  const int o = m > 0 ? kWarmExtra : 0;
  const int cols = len + o;
  xtrg::svd_gather(len, pw, work, r, Q, len, 0, s);
  if (m > 0) {
    const int mo = m + o;
    double* R = Q + (size_t)len * r;
    xtrg::fill_hash(R, (size_t)len * mo, seed, s);
    double* T1 = c->need("wq_T1", (size_t)r * mo);
    double* P = c->need("wq_P", (size_t)len * mo);
    for (int pass = 0; pass < 2; ++pass) {
      gemm(c, plain(r, mo, len, Q, len, false, R, len, true, T1, mo));   // Q0^T R
      gemm(c, plain(mo, len, r, T1, mo, true, Q, len, false, P, len));   // Q0 (Q0^T R)
      xtrg::axpby(R, 1.0, P, -1.0, (size_t)len * mo, s);
    }
    // coordinates of R in the complement: an m x (m + o) block of variance
    // 1/3, singular values within sqrt(1/3) (sqrt(m + o) -+ sqrt(m))
    const double hi = 1.1 * std::sqrt(1.0 / 3.0) * (std::sqrt((double)mo) + std::sqrt((double)m));
    const double lo = std::sqrt(1.0 / 3.0) * (std::sqrt((double)mo) - std::sqrt((double)m));
    xtrg::scale(R, 1.0 / hi, (size_t)len * mo, s);
    polar_ns(c, R, len, mo, 0.5 * lo / hi);
  }
  // Q Q^T = I on R^len?  A completion whose smallest singular value
  // started below the estimate gets up to two rounds of further steps.
  *m_out = m;
  if (dev_out) {
    basis_check(c, Q, len, cols, dev_out);
    return cols;
  }
  basis_check(c, Q, len, cols, c->scratch);
  if (read_scalar(c, c->scratch) <= basis_lim(len)) return cols;
  return basis_retry(c, Q, len, cols, m);
}

void build_warm(xtrg_ctx c, Chain& C, const std::vector<double>& S, double keep_floor, unsigned long long seed) {
  auto& w = C.warm[C.i];
  w.side = -1;
  const int len = C.len;
  if (len < kWarmMin || C.psvd < 1) return;
  double* Q = c->need("wq" + std::to_string(C.i) + C.tag, (size_t)len * (len + kWarmExtra));
  int m = 0;
  const int cols = build_basis(c, C.work, len, C.psvd, S, keep_floor, seed, Q, &m);
  c->warm_m += m;
  if (cols < 0) c->warm_rejected += 1;
  if (cols <= 0) return;
  c->warm_built += 1;
  w.side = C.gauge_right ? 0 : 1;   // Z lives in the row space of Y
  w.dim = len;
  w.cols = cols;
}

// First visits of a bond (no basis from an earlier visit): the SVD of Y
// through a column-pivoted QR.  With Y P = Q R, the one-sided Jacobi runs
// on [R^T; I] (the Gram matrices from the first p rows): it converges in a
// fraction of the sweeps that it needs on Y (the pivoted factor is graded)
// and accumulates its rotations W in the identity rows, R^T W = U_R Sigma.
// Then R = W Sigma U_R^T, and Q [W Sigma; 0] (Y's left singular vectors
// times their values) becomes Y's SVD workspace: no Jacobi runs on Y.  The
// QR stops at the Jacobi's numerical zero (a quarter of the keep floor),
// since directions below it are never rotated; a factorisation with fewer
// than a quarter as many rows as Y has columns is mostly noise, and that
// chain runs the Jacobi on Y itself.  All chains at once: one grouped QR
// and one grouped Jacobi.
constexpr int kQrMin = 256;   // smallest SVD (rows and columns) that gets the QR start

// One SVD routed through the QR: Y (len x p, column-major) in, on success
// an SVD workspace of len x psvd columns (Q [W Sigma; 0]) that the Jacobi
// would have left, with done = true.  `tag` names the workspaces.
struct QrTask {
  int len = 0, p = 0;
  const double* Y = nullptr;
  std::string tag;
  double* work = nullptr;   // out: SVD workspace
  int psvd = 0;             // out: its columns (the rows of R kept)
  bool done = false;        // out: false if the factorisation was rejected (mostly noise)
  bool failed = false;      // out: the Jacobi on [R^T; I] failed (non-finite input, no convergence)
};

void qr_factorise(xtrg_ctx c, std::vector<QrTask*>& tasks, xtrg::RoundTimer* rt) {
  hipStream_t s = c->stream;
  const int n = (int)tasks.size();
  std::vector<xtrg::QrJob> qj;
  for (QrTask* T : tasks)
    qj.push_back(xtrg::QrJob{T->len, T->p, T->Y, c->need("qr" + T->tag, xtrg::qr_work(T->len, T->p)),
                             0.25 * xtrg::svd_keep_rel(T->len, T->p), 0});
  xtrg::qrcp_batched(qj, qr_desc(c, n), s);
  // Jacobi on [R^T; I]: orthogonal columns on the first p rows, the
  // accumulated rotation W below
  std::vector<xtrg::SvdJob> sj;
  std::vector<int> at;
  for (int q = 0; q < n; ++q) {
    QrTask* T = tasks[q];
    const auto& J = qj[q];
    c->qr_calls += 1;
    c->qr_rows += J.keff;
    if (4 * J.keff < T->p) {                 // mostly noise: the Jacobi on Y itself
      c->qr_rejected += 1;
      continue;
    }
    const long ld = (long)T->p + J.keff;
    double* RT = c->need("qr_rt" + T->tag, (size_t)ld * J.keff);
    xtrg::qr_rt(J, RT, ld, true, s);
    sj.push_back(xtrg::SvdJob{(int)ld, J.keff, RT, c->need("qr_svd" + T->tag, xtrg::svd_work((int)ld, J.keff)), 0,
                              svd_gram(c, T->tag, J.keff), T->p});
    at.push_back(q);
  }
  if (sj.empty()) return;
  xtrg::svd_batched(sj, svd_desc(c, (int)sj.size()), s, rt);
  // Y P = Q R and R^T W = U_R Sigma give R = W Sigma U_R^T, so Y's left
  // singular vectors are Q W: the SVD workspace of Y takes Q [W Sigma; 0]
  std::vector<xtrg::QrJob> aj;
  std::vector<double*> Ms;
  std::vector<int> nc;
  for (size_t t = 0; t < sj.size(); ++t) {
    QrTask* T = tasks[at[t]];
    if (sj[t].status != 0) {
      T->failed = true;
      continue;
    }
    const int keff = sj[t].p;
    c->qr_sweeps += sj[t].sweeps;
    double* Mm = c->need("qr_M" + T->tag, (size_t)T->len * keff);
    xtrg::qr_lift(sj[t].work, sj[t].len, T->p, keff, xtrg::svd_column_norms(sj[t].work, sj[t].len, keff), Mm,
                  T->len, s);
    aj.push_back(qj[at[t]]);
    Ms.push_back(Mm);
    nc.push_back(keff);
  }
  if (!aj.empty()) xtrg::qr_apply_q(aj, Ms, nc, qr_desc(c, n), s);
  for (size_t t = 0; t < sj.size(); ++t) {
    QrTask* T = tasks[at[t]];
    if (T->failed) continue;
    const int keff = sj[t].p;
    T->work = c->need("svd" + T->tag, xtrg::svd_work(T->len, keff));
    xtrg::svd_adopt(T->len, keff, Ms[t], T->work, s);
    T->psvd = keff;
    T->done = true;
    c->qr_used += 1;
  }
}

void qr_start(xtrg_ctx c, const std::vector<Chain*>& pre, xtrg::RoundTimer* rt) {
  std::vector<QrTask> tk(pre.size());
  std::vector<QrTask*> tp;
  for (size_t q = 0; q < pre.size(); ++q) {
    tk[q].len = pre[q]->len;
    tk[q].p = pre[q]->p;
    tk[q].Y = pre[q]->th;
    tk[q].tag = pre[q]->tag;
    tp.push_back(&tk[q]);
  }
  qr_factorise(c, tp, rt);
  for (size_t q = 0; q < pre.size(); ++q)
    if (tk[q].failed) {
      pre[q]->status = XTRG_ENUMERIC;
      pre[q]->err = "two-site tensor: non-finite entries or no convergence of the SVD (QR route)";
    } else if (tk[q].done) {
      pre[q]->work = tk[q].work;
      pre[q]->psvd = tk[q].psvd;
      pre[q]->svd_done = true;
    }
}

// After the SVD of the chain's two-site overlap: choose k, split into C_i and
// C_{i+1} (the side the sweep moves away from takes the isometry), and
// advance the environment on that side.
void chain_truncate_split(xtrg_ctx c, Chain& C) {
  hipStream_t s = c->stream;
  auto& d = C.d;
  const int i = C.i;
  const int mL = C.mL, mR = C.mR, Kt = C.Kt, len = C.len, p = C.p, pw = C.psvd;
  std::vector<double> S, S_all;
  double kf = 0.0;
  if (C.u1) {
    bsvd_merge(c, C.tag, C.bs);
    S = C.bs.S;
    kf = xtrg::svd_keep_rel(len, p) * std::sqrt(C.bs.fro2);
  } else {
    S = read_vec(c, xtrg::svd_sorted_values(C.work, len, pw), pw);
    for (double v : S)
      if (!std::isfinite(v)) throw Error(XTRG_ENUMERIC, "non-finite singular value");
    S_all = S;
    S.resize(std::min(mL, mR));
    kf = noise_floor(c, C.work, len, pw, p);
  }
  const int k = keep_count(S, C.o.D_max, C.o.degen_rtol, C.o.sv_floor, kf);
  double tot = 0.0, kw = 0.0;
  for (size_t q = 0; q < S.size(); ++q) {
    tot += S[q] * S[q];
    if ((int)q < k) kw += S[q] * S[q];
  }
  if (!(tot > 0)) throw Error(XTRG_ENUMERIC, "zero two-site tensor");
  C.sv[i] = S;
  C.kept[i] = k;
  C.disc[i] = (tot - kw) / tot;
  C.last_norm = std::sqrt(kw);
  double* Ci = d.C[i].p;
  double* Cn = d.C[i + 1].p;
  if (C.gauge_right) {
    {
      Timed tm(c, P_SPLIT, 2.0 * k * (double)mL * mR, 0.0);
      if (C.u1)
        bsvd_scatter(c, C.tag, C.bs, k, Ci, 1);
      else
        xtrg::svd_gather(len, pw, C.work, k, Ci, k, 1, s);                            // C_i = U [mL][k]
      orthonormalize(c, Ci, mL, k, true);
      gemm(c, plain(k, mR, mL, Ci, k, true, C.th, mL, true, Cn, mR));                 // C_{i+1} = U^T theta
    }
    Timed tm(c, P_ENV, 2.0 * k * (double)Kt * mL, 8.0 * ((double)mL * Kt + (double)k * Kt));
    d.sync_cw(i, (size_t)mL * k);
    gemm(c, d.wplain(k, Kt, mL, d.Cw[i], k, true, C.Lb, Kt, false, C.E, Kt));          // E_{i+1} = C_i^T Lb
  } else {
    {
      Timed tm(c, P_SPLIT, 2.0 * k * (double)mL * mR, 0.0);
      if (C.u1)
        bsvd_scatter(c, C.tag, C.bs, k, Cn, 0);
      else
        xtrg::svd_gather(len, pw, C.work, k, Cn, len, 0, s);                          // C_{i+1} = V^T [k][mR]
      orthonormalize(c, Cn, mR, k, false);
      gemm(c, plain(mL, k, mR, C.th, mR, false, Cn, mR, true, Ci, k));                // C_i = theta V
    }
    Timed tm(c, P_ENV, 2.0 * k * (double)Kt * mR, 8.0 * ((double)mR * Kt + (double)k * Kt));
    d.sync_cw(i + 1, (size_t)k * mR);
    gemm(c, d.wplain(d.Da[i + 1] * d.Db[i + 1], k, mR, C.Rb, mR, false, d.Cw[i + 1], mR, true, C.F, k));  // F_{i+1}
  }
  d.Dc[i + 1] = k;
  if (C.u1) C.qc[i + 1].assign(C.bs.qs.begin(), C.bs.qs.begin() + k);
  if (C.u1 && !C.o.no_warm_start && C.revisit[C.st]) {
    // a basis per charge block for the next visit of the bond (as
    // build_warm does for the whole tensor)
    Timed tm(c, P_WARM, 0.0, 0.0);
    const size_t nb = C.bs.b.size();
    std::vector<int> colsv(nb, 0), mv(nb, 0);
    double* devs = c->need("u1_dev" + C.tag, nb + 1);
    bool any = false;
    for (size_t t = 0; t < nb; ++t) {
      const auto& blk = C.bs.b[t];
      C.wq1.erase(std::make_pair(i, blk.q));
      if (blk.len < kWarmMinBlock) continue;
      double* Q = c->need(C.wq1_name(i, blk.q), (size_t)blk.len * (blk.len + kWarmExtra));
      std::vector<double> Sb = blk.S;
      Sb.resize(std::max<size_t>(Sb.size(), blk.psvd), 0.0);
      const unsigned long long seed = 0x5EEDull + 7919ull * (unsigned long long)i + 104729ull * (unsigned)(blk.q + 4096);
      colsv[t] = build_basis(c, blk.work, blk.len, blk.psvd, Sb, kf, seed, Q, &mv[t], kWarmMinBlock, devs + t);
      any |= colsv[t] > 0;
    }
    // the orthogonality checks of all blocks in one read
    const std::vector<double> hd = any ? read_vec(c, devs, nb) : std::vector<double>(nb, 0.0);
    for (size_t t = 0; t < nb; ++t) {
      const auto& blk = C.bs.b[t];
      const auto key = std::make_pair(i, blk.q);
      int cols = colsv[t];
      if (cols > 0 && !(hd[t] <= basis_lim(blk.len)))
        cols = basis_retry(c, c->need(C.wq1_name(i, blk.q), (size_t)blk.len * (blk.len + kWarmExtra)), blk.len, cols,
                           mv[t]);
      c->warm_m += mv[t];
      if (cols < 0) c->warm_rejected += 1;
      if (cols <= 0) continue;
      c->warm_built += 1;
      Chain::WarmQ w;
      w.side = C.gauge_right ? 0 : 1;
      w.dim = blk.len;
      w.cols = cols;
      C.wq1[key] = w;
    }
  }
  if (!C.u1 && !C.o.no_warm_start && C.revisit[C.st]) {
    Timed tm(c, P_WARM, 0.0, 0.0);
    build_warm(c, C, S_all, kf, 0x5EEDull + 7919ull * (unsigned long long)i);
  }
}

// Runs f for one chain; an error that belongs to that chain alone (bad
// numbers in its tensors, its memory refused by the budget) stops only
// that chain, runtime errors stop the call.
template <class F>
void per_chain(Chain& C, F&& f) {
  if (C.status != XTRG_OK) return;
  try {
    f();
  } catch (const Error& e) {
    if (e.code != XTRG_ENUMERIC && e.code != XTRG_ENOMEM) throw;
    C.status = e.code;
    C.err = e.what();
  }
}

// One XTRG doubling of n independent chains at once.  Every chain follows
// its own bond schedule (lengths and sweep counts may differ); step st of
// all chains that still have one is issued together: the GEMMs per chain on
// the one stream, and the Jacobi rounds of all their SVDs as one grouped
// launch per round.  n = 1 is the plain single-chain doubling.  A chain
// whose numbers turn non-finite or whose memory the budget refuses stops
// with its own status (outs[q] = NULL, infos[q].status); the others finish.
// Returns the number of chains that failed.
// insb: the right factors and initial guesses (NULL: insb = ins, a doubling).
int square_compress_impl(xtrg_ctx c, int n, const xtrg_mpo* ins, const xtrg_compress_opts* opts,
                         xtrg_mpo* outs, xtrg_compress_info* infos, std::string* first_err,
                         const xtrg_mpo* insb = nullptr) {
  if (n < 1) throw Error(XTRG_EINVAL, "need at least one chain");
  if (!insb) insb = ins;
  for (int q = 0; q < n; ++q) {
    if (!ins[q] || !insb[q]) throw Error(XTRG_EINVAL, "null input MPO");
    if (ins[q]->ctx != c || insb[q]->ctx != c) throw Error(XTRG_EINVAL, "input MPO belongs to another context");
    if (ins[q]->L < 2) throw Error(XTRG_EINVAL, "the compression needs at least two sites");
    if (insb[q]->L != ins[q]->L) throw Error(XTRG_EINVAL, "the two factors differ in length");
    check_opts(opts[q]);
  }
  hipStream_t s = c->stream;
  std::vector<Chain> ch(n);
  size_t n_steps = 0;
  for (int q = 0; q < n; ++q) {
    ch[q].o = opts[q];
    per_chain(ch[q], [&] { chain_setup(c, ch[q], ins[q], insb[q], q); });
    n_steps = std::max(n_steps, ch[q].sched.size());
  }

  std::vector<Chain*> act;
  std::vector<xtrg::SvdJob> jobs;
  std::vector<Chain*> job_chain;
  for (size_t st = 0; st < n_steps; ++st) {
    act.clear();
    for (auto& C : ch) {
      if (C.status != XTRG_OK || st >= C.sched.size()) continue;
      const Step& sp = C.sched[st];
      const bool final_step = st + 1 == C.sched.size();
      C.i = sp.bond;
      C.st = st;
      C.gauge_right = xtrg_host::gauge_right(sp, final_step);
      act.push_back(&C);
    }
    if (act.empty()) break;
    {
      // left block: 8 Dc Da Db Da' + 16 Dc Da' Db Db' (two substeps of Fig. VMPO(c));
      // the right block mirrors it with the right bond of C
      double fb = 0.0;
      for (Chain* C : act) {
        const auto& d = C->d;
        const int i = C->i;
        if (C->sched[st].dir > 0)
          fb += 8.0 * d.Dc[i] * d.Da[i] * (double)d.Db[i] * d.Da[i + 1] +
                16.0 * d.Dc[i] * d.Da[i + 1] * (double)d.Db[i] * d.Db[i + 1];
        else
          fb += 8.0 * d.Dc[i + 2] * d.Da[i + 2] * (double)d.Db[i + 2] * d.Da[i + 1] +
                16.0 * d.Dc[i + 2] * d.Da[i + 1] * (double)d.Db[i + 2] * d.Db[i + 1];
      }
      Timed tm(c, P_BLOCK, fb, 0.0);
      std::vector<Gemm> g1, g2;   // the two substeps of every chain, each stage one grouped launch
      for (Chain* C : act)
        per_chain(*C, [&] {
          auto& d = C->d;
          const int i = C->i;
          std::pair<Gemm, Gemm> gg;
          if (C->sched[st].dir > 0) {
            C->Lb = d.slot_need(i);
            gg = d.left_block_gemms(i, C->E, C->Lb);
            C->Rb = d.slot.at(i + 1);
          } else {
            C->Rb = d.slot_need(i + 1);
            gg = d.right_block_gemms(i + 1, C->F, C->Rb);
            C->Lb = d.slot.at(i);
          }
          g1.push_back(gg.first);
          g2.push_back(gg.second);
        });
      gemm_group(c, g1);
      gemm_group(c, g2);
    }
    {
      double fth = 0.0, bth = 0.0;
      for (Chain* C : act) {
        if (C->status != XTRG_OK) continue;
        const auto& d = C->d;
        const int i = C->i;
        C->mL = 4 * d.Dc[i];
        C->mR = 4 * d.Dc[i + 2];
        C->Kt = d.Da[i + 1] * d.Db[i + 1];
        C->len = C->gauge_right ? C->mL : C->mR;
        C->p = C->gauge_right ? C->mR : C->mL;
        fth += 2.0 * C->mL * (double)C->mR * C->Kt;
        bth += 8.0 * ((double)C->mL * C->Kt + (double)C->Kt * C->mR + (double)C->mL * C->mR);
      }
      Timed tm(c, P_THETA, fth, bth);
      std::vector<Gemm> gt;
      for (Chain* C : act)
        per_chain(*C, [&] {
          const auto& d = C->d;
          const int i = C->i;
          C->flops += Doubler::step_flops(d.Dc[i], d.Da[i], d.Db[i], d.Da[i + 1], d.Db[i + 1], d.Dc[i + 2]);
          C->th = c->need("theta" + C->tag, (size_t)C->mL * C->mR);
          const int pr = C->d.prec;   // FP64 output in every precision: the SVD is FP64
          Gemm g = C->gauge_right
                       ? plain(C->mR, C->mL, C->Kt, C->Rb, C->mR, true, C->Lb, C->Kt, true, C->th, C->mL, pr, 1)  // column-major
                       : plain(C->mL, C->mR, C->Kt, C->Lb, C->Kt, false, C->Rb, C->mR, false, C->th, C->mR, pr, 1);
          g.tag = 1;
          gt.push_back(g);
        });
      gemm_group(c, gt);
    }
    {
      double fw = 0.0;
      for (Chain* C : act) {
        const auto& w = C->warm[C->i];
        if (C->status == XTRG_OK && !C->u1 && !C->o.no_warm_start && C->p >= kWarmMin &&
            w.side == (C->gauge_right ? 1 : 0) &&
            w.dim == C->p)
          fw += 2.0 * C->len * (double)C->p * w.cols;
      }
      Timed tm(c, P_WARM, fw, 0.0);
      std::vector<Gemm> gw;
      for (Chain* C : act)
        per_chain(*C, [&] {
          C->Y = C->th;
          C->psvd = C->p;
          C->svd_done = false;
          C->warm_now = false;
          const auto& w = C->warm[C->i];
          const int need_side = C->gauge_right ? 1 : 0;   // the column index of Y
          if (!C->u1 && !C->o.no_warm_start && C->p >= kWarmMin && w.side == need_side && w.dim == C->p) {
            const double* Q = c->need("wq" + std::to_string(C->i) + C->tag, (size_t)C->p * w.cols);
            double* Yw = c->need("svd_in" + C->tag, (size_t)C->len * w.cols);
            gw.push_back(plain(w.cols, C->len, C->p, Q, C->p, false, C->th, C->len, false, Yw, C->len));   // Y [Q0 X]
            C->Y = Yw;
            C->psvd = w.cols;
            C->warm_now = true;
            c->warm_used += 1;
          }
          if (!C->u1) C->work = c->need("svd" + C->tag, xtrg::svd_work(C->len, C->psvd));
        });
      gemm_group(c, gw);
    }
    {
      std::vector<Chain*> pre;
      for (Chain* C : act)
        // first visits only: a warm basis (square when the previous visit's
        // spectrum was all above the noise) already gives a cheap Jacobi
        if (C->status == XTRG_OK && !C->u1 && !C->warm_now && !C->o.no_warm_start && !C->o.no_qr_start &&
            C->p >= kQrMin && C->len >= kQrMin && C->len <= xtrg::kQrMaxLen && C->p <= 2048)
          pre.push_back(C);
      if (!pre.empty()) {
        Timed tm(c, P_QR, 0.0, 0.0);
        RoundProf rp(c);
        // workspace allocations that the budget refuses stop the chains of this QR group
        try {
          qr_start(c, pre, &rp);
        } catch (const Error& e) {
          if (e.code != XTRG_ENOMEM) throw;
          for (Chain* C : pre) {
            C->status = e.code;
            C->err = e.what();
          }
        }
      }
    }
    {
      double bs = 0.0;
      jobs.clear();
      job_chain.clear();
      for (Chain* C : act) {
        if (C->status != XTRG_OK || C->svd_done) continue;
        if (C->u1) {
          // one problem per charge block of C_E (len side: the index that
          // takes the isometry)
          const int i = C->i;
          const auto qr = row_charges(C->qc[i]), qcol = col_charges(C->qc[i + 2]);
          const size_t j0 = jobs.size();
          // warm start of a block: the basis of the previous visit of the
          // bond for the same charge block, on the side this visit shares
          const int need_side = C->gauge_right ? 1 : 0;
          const WarmHook hook = [&, C, i, need_side](int q, int len_q, int p_q,
                                                     const double* Yq) -> std::pair<const double*, int> {
            if (C->o.no_warm_start || p_q < kWarmMinBlock) return {Yq, p_q};
            const auto it = C->wq1.find({i, q});
            if (it == C->wq1.end() || it->second.side != need_side || it->second.dim != p_q) return {Yq, p_q};
            const auto& w = it->second;
            const double* Q = c->need(C->wq1_name(i, q), (size_t)p_q * w.cols);
            double* Yw = c->need("u1_in" + C->tag + "/" + std::to_string(q), (size_t)len_q * w.cols);
            gemm(c, plain(w.cols, len_q, p_q, Q, p_q, false, Yq, len_q, false, Yw, len_q));   // Y_q [Q0 X]
            c->warm_used += 1;
            return {Yw, w.cols};
          };
          per_chain(*C, [&] {
            bsvd_prepare(c, C->tag, C->th, C->len, C->p, C->gauge_right ? qr : qcol, C->gauge_right ? qcol : qr,
                         C->bs, jobs, hook);
          });
          if (C->status != XTRG_OK) {   // its workspaces refused by the budget
            jobs.resize(j0);
            continue;
          }
          for (size_t j = j0; j < jobs.size(); ++j) {
            job_chain.push_back(C);
            bs += 8.0 * jobs[j].len * (double)jobs[j].p;
          }
          continue;
        }
        jobs.push_back(xtrg::SvdJob{C->len, C->psvd, C->Y, C->work, 0, svd_gram(c, C->tag, C->psvd)});
        job_chain.push_back(C);
        bs += 8.0 * C->len * (double)C->psvd;
      }
      Timed tm(c, P_SVD, 0.0, bs);
      RoundProf rp(c);
      xtrg::svd_batched(jobs, svd_desc(c, (int)jobs.size()), s, &rp);
      for (size_t j = 0; j < jobs.size(); ++j) {
        if (jobs[j].status != 0) {
          job_chain[j]->status = XTRG_ENUMERIC;
          job_chain[j]->err = "two-site tensor: non-finite entries or no convergence of the SVD";
          continue;
        }
        c->svd_calls += 1;
        c->svd_sweeps += jobs[j].sweeps;
      }
    }
    for (Chain* C : act) per_chain(*C, [&] { chain_truncate_split(c, *C); });
  }
  // normalise: the centre is site 0 after the final right-to-left step
  std::vector<std::unique_ptr<xtrg_mpo_s>> res(n);
  for (int q = 0; q < n; ++q)
    per_chain(ch[q], [&] {
      auto& d = ch[q].d;
      if (!(ch[q].last_norm > 0) || !std::isfinite(ch[q].last_norm))
        throw Error(XTRG_ENUMERIC, "non-finite or zero norm of the compressed product");
      xtrg::scale(d.C[0].p, 1.0 / ch[q].last_norm, (size_t)4 * d.Dc[1], s);
      res[q] = new_mpo(c, d.Dc);
      for (int i = 0; i < d.L; ++i) xtrg::copy(res[q]->site[i].p, d.C[i].p, res[q]->elems(i), s);
      if (ch[q].u1) res[q]->charges = ch[q].qc;
    });
  XTRG_HIP(hipStreamSynchronize(s));
  int failed = 0;
  for (int q = 0; q < n; ++q) {
    const Chain& C = ch[q];
    xtrg_compress_info* info = infos ? infos + q : nullptr;
    if (C.status != XTRG_OK) {
      ++failed;
      if (first_err && first_err->empty()) *first_err = "chain " + std::to_string(q) + ": " + C.err;
      if (info) info->status = C.status;
      outs[q] = nullptr;
      continue;
    }
    if (info) {
      info->status = XTRG_OK;
      info->dlog_norm = std::log(C.last_norm);
      info->trunc_err_max = *std::max_element(C.disc.begin(), C.disc.end());
      info->sweeps_done = C.o.n_sweeps;
      info->D_kept_max = *std::max_element(C.d.Dc.begin(), C.d.Dc.end());
      info->steps = (int)C.sched.size();
      info->flops = C.flops;
      if (info->sv && info->sv_stride > 0)
        for (int b = 0; b < C.d.L - 1; ++b)
          for (int k = 0; k < info->sv_stride; ++k)
            info->sv[(size_t)b * info->sv_stride + k] = k < (int)C.sv[b].size() ? C.sv[b][k] : 0.0;
    }
    outs[q] = res[q].release();
  }
  return failed;
}

// ---------------------------------------------------------------------------
// Observables: traces of MPO products by environment contractions
// ---------------------------------------------------------------------------

struct Named {
  std::vector<std::string> name;
  std::vector<int> ext;
  long size() const {
    long n = 1;
    for (int e : ext) n *= e;
    return n;
  }
  long stride(const std::string& nm) const {   // sum over repeated names (diagonal)
    long st = 1, out = 0;
    for (int d = (int)name.size() - 1; d >= 0; --d) {
      if (name[d] == nm) out += st;
      st *= ext[d];
    }
    return out;
  }
  int extent(const std::string& nm) const {
    for (size_t d = 0; d < name.size(); ++d)
      if (name[d] == nm) return ext[d];
    throw Error(XTRG_EINVAL, "internal: no dim " + nm);
  }
};

// out (row-major in `outd` order) = sum over `sum` of T * W, as a batched
// GEMM on the matrix cores: T is gathered into [batch][M][K] and W into
// [batch][K][N] (batch: output indices of both, M / N: of one only, K: the
// summed ones; an index missing from one tensor has stride 0 there, and a
// repeated index is a diagonal), then C[batch][M][N] = T' W', scattered
// into the order of `outd`.
void contract_named(xtrg_ctx c, const Named& T, const double* Tp, const Named& W, const double* Wp,
                    const Named& outd, double* outp, const std::vector<std::string>& sum, hipStream_t s) {
  auto has = [](const Named& X, const std::string& nm) {
    return std::find(X.name.begin(), X.name.end(), nm) != X.name.end();
  };
  struct Dim {
    long e, st_t, st_w;
    int out_pos;
  };
  std::vector<Dim> bat, mm, nn, kk;
  for (size_t d = 0; d < outd.name.size(); ++d) {
    const std::string& nm = outd.name[d];
    const bool it = has(T, nm), iw = has(W, nm);
    if (!it && !iw) throw Error(XTRG_EINVAL, "internal: output index in neither factor");
    Dim x{outd.ext[d], it ? T.stride(nm) : 0, iw ? W.stride(nm) : 0, (int)d};
    (it && iw ? bat : it ? mm : nn).push_back(x);
  }
  for (const std::string& nm : sum) {
    const long e = has(T, nm) ? T.extent(nm) : W.extent(nm);
    kk.push_back(Dim{e, has(T, nm) ? T.stride(nm) : 0, has(W, nm) ? W.stride(nm) : 0, -1});
  }
  auto prod = [](const std::vector<Dim>& v) {
    long n = 1;
    for (const Dim& x : v) n *= x.e;
    return n;
  };
  const long nb = prod(bat), nm_ = prod(mm), nn_ = prod(nn), nk = prod(kk);
  if (bat.size() + mm.size() + kk.size() > 8 || bat.size() + kk.size() + nn.size() > 8)
    throw Error(XTRG_EINVAL, "internal: contraction too wide");
  auto gather = [&](const double* src, const std::vector<const std::vector<Dim>*>& groups, bool t_side,
                    double* dst) {
    xtrg::Permute p;
    for (const auto* g : groups)
      for (const Dim& x : *g) {
        p.e[p.n] = x.e;
        p.st[p.n] = t_side ? x.st_t : x.st_w;
        ++p.n;
      }
    p.src = src;
    p.out = dst;
    xtrg::permute(p, s);
  };
  double* Tg = c->need("ct_T", (size_t)std::max(nb * nm_ * nk, 1L));
  double* Wg = c->need("ct_W", (size_t)std::max(nb * nk * nn_, 1L));
  gather(Tp, {&bat, &mm, &kk}, true, Tg);
  gather(Wp, {&bat, &kk, &nn}, false, Wg);
  // the GEMM's row-major [batch][M][N] is the requested order when the
  // output indices come batch first, then T's, then W's
  bool direct = true;
  {
    int pos = 0;
    for (const auto* g : {&bat, &mm, &nn})
      for (const Dim& x : *g) direct &= x.out_pos == pos++;
  }
  double* Cg = direct ? outp : c->need("ct_C", (size_t)std::max(nb * nm_ * nn_, 1L));
  Gemm g;
  g.M = (int)nm_;
  g.N = (int)nn_;
  g.K = (int)nk;
  g.A = Tg;
  g.lda = nk;
  g.B = Wg;
  g.ldb = nn_;
  g.C = Cg;
  g.ldc = nn_;
  g.nb[0] = (int)nb;
  g.sA[0] = nm_ * nk;
  g.sB[0] = nk * nn_;
  g.sC[0] = nm_ * nn_;
  gemm(c, g);
  if (direct) return;
  // scatter: output position d reads C' at the row-major stride of its index there
  xtrg::Permute p;
  std::vector<long> cst(outd.name.size(), 0);
  {
    long st = 1;
    std::vector<const Dim*> order;
    for (const auto* grp : {&bat, &mm, &nn})
      for (const Dim& x : *grp) order.push_back(&x);
    for (int q = (int)order.size() - 1; q >= 0; --q) {
      cst[order[q]->out_pos] = st;
      st *= order[q]->e;
    }
  }
  for (size_t d = 0; d < outd.name.size(); ++d) {
    p.e[p.n] = outd.ext[d];
    p.st[p.n] = cst[d];
    ++p.n;
  }
  p.src = Cg;
  p.out = outp;
  xtrg::permute(p, s);
}

// Tr(M_1 M_2 ... M_k) for k <= 4; trans[j]: use M_j^T.
double trace_chain(xtrg_ctx c, const std::vector<xtrg_mpo>& M, const std::vector<bool>& trans) {
  const int k = (int)M.size();
  const int L = M[0]->L;
  hipStream_t s = c->stream;
  auto bname = [](const char* p, int j) { return std::string(p) + std::to_string(j); };
  size_t cap = 1;   // largest intermediate: open a's of site i, b's of site i+1, two physical indices
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < k; ++j) {
      size_t e = 4;
      for (int q = 0; q < k; ++q) e *= (size_t)(q > j ? M[q]->dims[i] : M[q]->dims[i + 1]);
      cap = std::max(cap, e);
    }
  double* bufA = c->need("tr_a", cap);
  double* bufB = c->need("tr_b", cap);
  Named E;
  for (int j = 0; j < k; ++j) {
    E.name.push_back(bname("a", j));
    E.ext.push_back(1);
  }
  xtrg::fill(bufA, 1.0, 1, s);
  double* cur = bufA;
  double* nxt = bufB;
  for (int i = 0; i < L; ++i) {
    // T_0 = E with dims a_0..a_{k-1}
    Named T = E;
    for (int j = 0; j < k; ++j) {
      Named W;
      const int Dl = M[j]->dims[i], Dr = M[j]->dims[i + 1];
      // physical: output index s_j, input index s_{j+1}; transposed swaps them
      const std::string so = "s" + std::to_string(j);
      const std::string si = (j + 1 < k) ? "s" + std::to_string(j + 1) : "s0";
      W.name = {bname("a", j), trans[j] ? si : so, trans[j] ? so : si, bname("b", j)};
      W.ext = {Dl, 2, 2, Dr};
      Named O;
      std::vector<std::string> sum = {bname("a", j)};
      if (j > 0) sum.push_back(so);
      if (j + 1 == k && k > 1) sum.push_back("s0");
      if (k == 1) sum.push_back("s0");           // W has s0 twice: the diagonal
      // output dims: remaining a's, s0 (if still open), b_0..b_j, s_{j+1} (if open)
      for (int q = j + 1; q < k; ++q) {
        O.name.push_back(bname("a", q));
        O.ext.push_back(M[q]->dims[i]);
      }
      if (j + 1 < k) {
        O.name.push_back("s0");
        O.ext.push_back(2);
      }
      for (int q = 0; q <= j; ++q) {
        O.name.push_back(bname("b", q));
        O.ext.push_back(M[q]->dims[i + 1]);
      }
      if (j + 1 < k) {
        O.name.push_back(si);
        O.ext.push_back(2);
      }
      contract_named(c, T, cur, W, M[j]->site[i].p, O, nxt, sum, s);
      std::swap(cur, nxt);
      T = O;
    }
    // rename b -> a for the next site
    E = T;
    for (auto& nm : E.name) nm[0] = 'a';
  }
  return read_scalar(c, cur);
}

// MPO of sum_i O_i for a single-site operator O (2 x 2, row = output
// index): bond 2 (states "before" and "after" the site that carries O).
std::unique_ptr<xtrg_mpo_s> local_sum_mpo(xtrg_ctx c, int L, const double O[2][2]) {
  std::vector<int> dims(L + 1, 2);
  dims[0] = dims[L] = 1;
  auto m = new_mpo(c, dims);
  for (int i = 0; i < L; ++i) {
    const int Dl = dims[i], Dr = dims[i + 1];
    std::vector<double> T((size_t)Dl * 4 * Dr, 0.0);
    for (int a = 0; a < Dl; ++a)
      for (int b = 0; b < Dr; ++b) {
        // virtual state 0: O not placed yet, 1: placed; the left edge is in
        // state 0, the right edge in state 1
        const int ga = L == 1 ? 0 : (i == 0 ? 0 : a), gb = L == 1 ? 1 : (i == L - 1 ? 1 : b);
        for (int s1 = 0; s1 < 2; ++s1)
          for (int s2 = 0; s2 < 2; ++s2) {
            double v = 0.0;
            if (ga == gb) v = s1 == s2 ? 1.0 : 0.0;     // identity while the state is kept
            else if (ga == 0 && gb == 1) v = O[s1][s2];  // the site that carries O
            T[(((size_t)a * 2 + s1) * 2 + s2) * Dr + b] = v;
          }
      }
    upload(c, m->site[i].p, T.data(), T.size());
  }
  return m;
}

// MPO of (sum_i S^z_i)^power for power 1 (bond 2) or 2 (bond 3): virtual
// states 0 (no S^z placed yet), 1 (one placed), 2 (done); for the square,
// 0 -> 1 carries 2 S^z (each unordered pair i < j once, times 2), 1 -> 2
// S^z, 0 -> 2 (S^z)^2 = I/4 (the diagonal terms i = j).
std::unique_ptr<xtrg_mpo_s> spin_sum_mpo(xtrg_ctx c, int L, int power) {
  const double Sz[2][2] = {{0.5, 0.0}, {0.0, -0.5}};
  if (power == 1) return local_sum_mpo(c, L, Sz);
  const int nv = 3;
  std::vector<int> dims(L + 1, nv);
  dims[0] = dims[L] = 1;
  auto m = new_mpo(c, dims);
  for (int i = 0; i < L; ++i) {
    const int Dl = dims[i], Dr = dims[i + 1];
    std::vector<double> T((size_t)Dl * 4 * Dr, 0.0);
    auto put = [&](int a, int b, const double (*op)[2], double cf) {
      for (int s1 = 0; s1 < 2; ++s1)
        for (int s2 = 0; s2 < 2; ++s2) T[(((size_t)a * 2 + s1) * 2 + s2) * Dr + b] += cf * op[s1][s2];
    };
    const double Id[2][2] = {{1.0, 0.0}, {0.0, 1.0}};
    for (int a = 0; a < Dl; ++a)
      for (int b = 0; b < Dr; ++b) {
        const int ga = i == 0 ? 0 : a, gb = i == L - 1 ? 2 : b;   // left edge in 0, right edge in 2
        if (ga == gb) put(a, b, Id, 1.0);
        else if (ga == 0 && gb == 1) put(a, b, Sz, 2.0);
        else if (ga == 1 && gb == 2) put(a, b, Sz, 1.0);
        else if (ga == 0 && gb == 2) put(a, b, Id, 0.25);
      }
    upload(c, m->site[i].p, T.data(), T.size());
  }
  return m;
}

// MPO of sum_j w_j S_c . S_j (real form S+S-/2 + S-S+/2 + SzSz; j = c gives
// w_c S_c . S_c = 3/4 w_c): bond 5 with states start, done and one per
// spin component of the one spin already placed.  A spin placed before c
// carries its weight; at c the partner closes it, or c's own spin opens a
// channel that a later site j closes with weight w_j.
std::unique_ptr<xtrg_mpo_s> correlation_mpo(xtrg_ctx c, int L, int center, const double* w) {
  const double Sp[2][2] = {{0, 1}, {0, 0}}, Sm[2][2] = {{0, 0}, {1, 0}}, Sz[2][2] = {{0.5, 0}, {0, -0.5}};
  const double Id[2][2] = {{1, 0}, {0, 1}};
  const double (*open_op[3])[2] = {Sp, Sm, Sz};
  const double (*close_op[3])[2] = {Sm, Sp, Sz};
  const double half[3] = {0.5, 0.5, 1.0};
  std::vector<int> dims(L + 1, 5);
  dims[0] = dims[L] = 1;
  auto m = new_mpo(c, dims);
  for (int i = 0; i < L; ++i) {
    const int Dl = dims[i], Dr = dims[i + 1];
    std::vector<double> T((size_t)Dl * 4 * Dr, 0.0);
    // state index: 0 start, 1 done, 2 + a open channel of component a
    auto idx_l = [&](int st) { return i == 0 ? (st == 0 ? 0 : -1) : st; };
    auto idx_r = [&](int st) { return i == L - 1 ? (st == 1 ? 0 : -1) : st; };
    auto put = [&](int sa, int sb, const double (*op)[2], double cf) {
      const int a = idx_l(sa), b = idx_r(sb);
      if (a < 0 || b < 0 || cf == 0.0) return;
      for (int s1 = 0; s1 < 2; ++s1)
        for (int s2 = 0; s2 < 2; ++s2) T[(((size_t)a * 2 + s1) * 2 + s2) * Dr + b] += cf * op[s1][s2];
    };
    put(0, 0, Id, 1.0);
    put(1, 1, Id, 1.0);
    // an open channel passes every site but the centre, where it must close
    // (else a pair j < c < j' would be picked up)
    if (i != center)
      for (int a = 0; a < 3; ++a) put(2 + a, 2 + a, Id, 1.0);
    if (i < center) {
      for (int a = 0; a < 3; ++a) put(0, 2 + a, open_op[a], w[i]);           // S_i^a, weight w_i
    } else if (i == center) {
      for (int a = 0; a < 3; ++a) put(2 + a, 1, close_op[a], half[a]);       // closes j < c
      for (int a = 0; a < 3; ++a) put(0, 2 + a, open_op[a], 1.0);            // opens for j > c
      put(0, 1, Id, 0.75 * w[i]);                                            // S_c . S_c = 3/4
    } else {
      for (int a = 0; a < 3; ++a) put(2 + a, 1, close_op[a], half[a] * w[i]); // closes c with weight w_j
    }
    upload(c, m->site[i].p, T.data(), T.size());
  }
  return m;
}

void observables_impl(xtrg_ctx c, xtrg_mpo rho, double lam, double tau, xtrg_mpo H, int n_sites,
                      xtrg_obs* at_tau, xtrg_obs* at_2tau, double* SE) {
  if (H->L != rho->L) throw Error(XTRG_EINVAL, "H and rho differ in length");
  if (n_sites <= 0) n_sites = rho->L;
  const double N = n_sites;
  const int L = rho->L;
  // total-spin MPOs for the invariants (real form: S^x = (S^+ + S^-)/2)
  const double Sz[2][2] = {{0.5, 0.0}, {0.0, -0.5}}, Sx[2][2] = {{0.0, 0.5}, {0.5, 0.0}};
  auto SZ = local_sum_mpo(c, L, Sz);
  auto SX = local_sum_mpo(c, L, Sx);
  // ||rho - rho^T||_F^2 / ||rho||_F^2 = 2 (1 - Tr(rho rho) / Tr(rho^T rho))
  double nrm = 0.0, herm = 0.0;
  if (at_tau || at_2tau) {
    nrm = trace_chain(c, {rho, rho}, {true, false});
    if (!(nrm > 0)) throw Error(XTRG_ENUMERIC, "||rho|| = 0");
    herm = 2.0 * (1.0 - trace_chain(c, {rho, rho}, {false, false}) / nrm);
  }
  if (at_tau) {
    const double tr = trace_chain(c, {rho}, {false});
    if (!(tr > 0)) throw Error(XTRG_ENUMERIC, "Tr rho <= 0");
    const double e1 = trace_chain(c, {H, rho}, {false, false}) / tr;
    const double e2 = trace_chain(c, {H, H, rho}, {false, false, false}) / tr;
    const double sz = trace_chain(c, {SZ.get(), rho}, {false, false}) / tr;
    const double z2 = trace_chain(c, {SZ.get(), SZ.get(), rho}, {false, false, false}) / tr;
    const double x2 = trace_chain(c, {SX.get(), SX.get(), rho}, {false, false, false}) / tr;
    const double b = tau, lnZ = lam + std::log(tr);
    *at_tau = xtrg_obs{b, lnZ, -lnZ / (N * b), e1 / N, b * b * (e2 - e1 * e1) / N, tr, 0.0, 0.0,
                       herm, sz, (x2 - z2) / std::max(z2, 1.0)};
  }
  double Sc = 0.0, Smax = 0.0;
  if (SE) {
    auto m = clone(rho);
    left_sweep(m.get(), 0.0, nullptr);
    std::vector<std::vector<double>> sv;
    right_sweep(m.get(), 0.0, 0, &sv);
    for (int bnd = 0; bnd + 1 < rho->L; ++bnd) {
      double tot = 0.0;
      for (double v : sv[bnd]) tot += v * v;
      double e = 0.0;
      for (double v : sv[bnd]) {
        const double q = v * v / tot;
        if (q > 0) e -= q * std::log(q);
      }
      if (SE) SE[bnd] = e;
      Smax = std::max(Smax, e);
      if (bnd == (rho->L - 1) / 2) Sc = e;
    }
  }
  if (at_2tau) {
    const double g1 = trace_chain(c, {H, rho, rho}, {false, true, false}) / nrm;
    const double g2 = trace_chain(c, {H, H, rho, rho}, {false, false, true, false}) / nrm;
    const double sz = trace_chain(c, {SZ.get(), rho, rho}, {false, true, false}) / nrm;
    const double z2 = trace_chain(c, {SZ.get(), SZ.get(), rho, rho}, {false, false, true, false}) / nrm;
    const double x2 = trace_chain(c, {SX.get(), SX.get(), rho, rho}, {false, false, true, false}) / nrm;
    const double b = 2 * tau, lnZ = 2 * lam + std::log(nrm);
    *at_2tau = xtrg_obs{b, lnZ, -lnZ / (N * b), g1 / N, b * b * (g2 - g1 * g1) / N, nrm, Sc, Smax,
                        herm, sz, (x2 - z2) / std::max(z2, 1.0)};
  }
}

}  // namespace

namespace xtrg_impl {

std::unique_ptr<xtrg_mpo_s> hamiltonian(xtrg_ctx c, int n_sites, int n_bonds, const int* bonds, const double* jxy,
                                        const double* jz) {
  Automaton A = build_automaton(n_sites, n_bonds, bonds, jxy, jz);
  const double r[2] = {0.0, 1.0};   // stop state: H
  std::vector<int> dims;
  auto S = cap(A, r, &dims);
  auto m = new_mpo(c, dims);
  for (int i = 0; i < n_sites; ++i) upload(c, m->site[i].p, S[i].data(), S[i].size());
  m->has_open = true;
  m->open_last = A.T[n_sites - 1];
  XTRG_HIP(hipStreamSynchronize(c->stream));
  return m;
}

std::unique_ptr<xtrg_mpo_s> init_rho(xtrg_ctx c, xtrg_mpo H, double tau0, int order, int D0_max,
                                   double* log_norm, bool u1) {
  if (!H->has_open || order < 1 || order > 2 || !(tau0 > 0))
  throw Error(XTRG_EINVAL, "init_rho: H from xtrg_hamiltonian_xxz, order 1 or 2, tau0 > 0");
  hipStream_t s = c->stream;
  const int L = H->L;
  // The right end of the automaton is left open over {start, stop}; a
  // right boundary r selects r_start * I + r_stop * H (App. B.1, App. C.2).
  std::unique_ptr<xtrg_mpo_s> m;
  if (order == 1) {
    std::vector<int> dims = H->dims;
    m = new_mpo(c, dims);
    for (int i = 0; i + 1 < L; ++i) xtrg::copy(m->site[i].p, H->site[i].p, H->elems(i), s);
    const int Dl = H->dims[L - 1];
    std::vector<double> last((size_t)Dl * 4);
    for (size_t q = 0; q < last.size(); ++q)
      last[q] = H->open_last[2 * q + 0] * 1.0 + H->open_last[2 * q + 1] * (-tau0);
    upload(c, m->site[L - 1].p, last.data(), last.size());
  } else {
    // exact product of two automata; each factor ends in start (I) or stop (H):
    // weights r[(x,y)] with x,y in {start, stop} give I - tau H + tau^2/2 H^2
    std::vector<int> dims(L + 1);
    for (int i = 0; i <= L; ++i) dims[i] = H->dims[i] * H->dims[i];
    dims[L] = 1;
    m = new_mpo(c, dims);
    for (int i = 0; i + 1 < L; ++i)
      xtrg::site_product(m->site[i].p, H->site[i].p, H->dims[i], H->dims[i + 1], H->site[i].p, H->dims[i],
                         H->dims[i + 1], s);
    const int Dl = H->dims[L - 1];
    double* openp = c->need("init_open", (size_t)Dl * 4 * 2);
    upload(c, openp, H->open_last.data(), H->open_last.size());
    double* prod = c->need("init_prod", (size_t)Dl * Dl * 4 * 4);
    xtrg::site_product(prod, openp, Dl, 2, openp, Dl, 2, s);     // [(a,b)][s][u][(x,y)]
    const double r[4] = {1.0, -0.5 * tau0, -0.5 * tau0, 0.5 * tau0 * tau0};
    double* rv = c->need("init_r", 4);
    upload(c, rv, r, 4);
    gemm(c, plain(Dl * Dl * 4, 1, 4, prod, 4, false, rv, 1, false, m->site[L - 1].p, 1));
  }
  // lossless compression to canonical form: exact zeros dropped
  if (u1) {
    // charges of the automaton states from H's entries; the product of two
    // automata carries q_a + q_b on its state (a, b)
    const std::vector<std::vector<int>> qH =
        H->charges.empty() ? infer_charges(download_sites(H), H->dims) : H->charges;
    auto& q = m->charges;
    q.assign(L + 1, {});
    for (int i = 0; i <= L; ++i) {
      const auto& h = qH[i];
      if (i == L) {
        q[i].assign(m->dims[L], 0);
      } else if (order == 1) {
        q[i] = h;
      } else {
        for (int a = 0; a < (int)h.size(); ++a)
          for (int b = 0; b < (int)h.size(); ++b) q[i].push_back(h[a] + h[b]);
      }
    }
    left_sweep_u1(m.get(), 1e-14);
    right_sweep_u1(m.get(), 1e-14, D0_max);
  } else {
    left_sweep(m.get(), 1e-14, nullptr);
    right_sweep(m.get(), 1e-14, D0_max, nullptr);
  }
  const double nrm = site_norm(m.get(), 0);
  if (!(nrm > 0) || !std::isfinite(nrm)) throw Error(XTRG_ENUMERIC, "rho(tau0) has zero norm");
  xtrg::scale(m->site[0].p, 1.0 / nrm, m->elems(0), s);
  XTRG_HIP(hipStreamSynchronize(s));
  *log_norm = std::log(nrm);
  // shrink the buffers to the final shapes
  auto fin = clone(m.get());
  XTRG_HIP(hipStreamSynchronize(s));
  return fin;
}

// The exact sum of MPOs of one length (App. D.2, Eq. MPO:plus): site 0
// concatenates the terms' columns, the last site their rows, the sites
// between are block diagonal.  The bonds add up; the site matrices the SVD
// sweeps factorise afterwards must stay within 4096 columns.
std::unique_ptr<xtrg_mpo_s> block_sum(xtrg_ctx c, const std::vector<xtrg_mpo>& terms) {
  hipStream_t s = c->stream;
  const int L = terms[0]->L;
  std::vector<int> dims(L + 1, 0);
  dims[0] = dims[L] = 1;
  std::vector<std::vector<int>> off(terms.size(), std::vector<int>(L + 1, 0));
  for (size_t t = 0; t < terms.size(); ++t)
    for (int b = 1; b < L; ++b) {
      off[t][b] = dims[b];
      dims[b] += terms[t]->dims[b];
    }
  for (int b = 1; b < L; ++b)
    if (dims[b] > 4096)
      throw Error(XTRG_EINVAL, "MPO sum: bond " + std::to_string(dims[b]) + " > 4096 (lower the bond budget)");
  auto S = new_mpo(c, dims);
  for (int i = 0; i < L; ++i) xtrg::fill(S->site[i].p, 0.0, S->elems(i), s);
  for (size_t t = 0; t < terms.size(); ++t) {
    xtrg_mpo T = terms[t];
    for (int i = 0; i < L; ++i) {
      const int Dl = T->dims[i], Dr = T->dims[i + 1], Drs = dims[i + 1];
      double* dst = S->site[i].p + (size_t)off[t][i] * 4 * Drs + off[t][i + 1];
      XTRG_HIP(hipMemcpy2DAsync(dst, (size_t)Drs * sizeof(double), T->site[i].p, (size_t)Dr * sizeof(double),
                                (size_t)Dr * sizeof(double), (size_t)Dl * 4, hipMemcpyDeviceToDevice, s));
    }
  }
  return S;
}

// sum_{k=0}^{N_c} x^k / k! H^k X for a normalised, right-canonical X, the
// series of Sec. II.C (Eq. RhoTau for X = I, Eq. Tay for X = rho_n with
// x = tau_n - tau_{n+1}).  H^k X = H (H^(k-1) X) by the compressed product
// of App. D.1 (the doubling's sweeps with A = H and the previous term as B
// and initial guess); HX, if given, is the first term already (normalised,
// log-norm l_hx relative to X).  Every term is kept normalised with its
// log-norm l_k; the expansion stops at the first order whose term,
// |x^k / k!| e^(l_k), is at most tol relative to X.  The terms are added one
// at a time, each exact sum of two MPOs (App. D.2 Eq. MPO:plus) compressed
// by the direct route of App. D.1: a left-to-right SVD sweep that drops the
// numerical zeros, then a right-to-left sweep with the keep rule of the
// doublings (exact when nothing is cut; the sums stay at bond <= 2 D).
// Returns the normalised sum and, in *dlog, the log of its norm.
std::unique_ptr<xtrg_mpo_s> expand_series(xtrg_ctx c, xtrg_mpo H, std::unique_ptr<xtrg_mpo_s> X,
                                          std::unique_ptr<xtrg_mpo_s> HX, double l_hx, double x, int D,
                                          int n_sweeps, double tol, double* dlog, int* n_terms) {
  constexpr int kMaxOrder = 80;
  hipStream_t s = c->stream;
  std::vector<std::unique_ptr<xtrg_mpo_s>> terms;
  std::vector<double> coef;
  terms.push_back(std::move(X));
  coef.push_back(1.0);
  xtrg_compress_opts o{};
  o.D_max = D;
  o.n_sweeps = n_sweeps;
  o.precision = XTRG_FP64;
  o.degen_rtol = 1e-6;
  o.sv_floor = 1e-14;
  double l = 0.0, omega = 1.0;
  int nc = 0;
  for (int k = 1; k <= kMaxOrder; ++k) {
    std::unique_ptr<xtrg_mpo_s> P;
    if (k == 1 && HX) {
      P = std::move(HX);
      l = l_hx;
    } else {
      xtrg_mpo A = H, B = terms.back().get();
      xtrg_mpo out = nullptr;
      xtrg_compress_info info{};
      std::string err;
      if (square_compress_impl(c, 1, &A, &o, &out, &info, &err, &B) > 0) throw Error(info.status, err);
      P.reset(out);
      l += info.dlog_norm;
    }
    omega *= x / k;
    const double a = omega * std::exp(l);
    terms.push_back(std::move(P));
    coef.push_back(a);
    nc = k;
    if (std::fabs(a) <= tol) break;
  }
  // the sum, one term at a time: S <- compress(S + a_k T_k)
  for (size_t t = 1; t < terms.size(); ++t) xtrg::scale(terms[t]->site[0].p, coef[t], terms[t]->elems(0), s);
  std::unique_ptr<xtrg_mpo_s> S = std::move(terms[0]);
  for (size_t t = 1; t < terms.size(); ++t) {
    S = block_sum(c, {S.get(), terms[t].get()});
    terms[t].reset();
    left_sweep(S.get(), 1e-14, nullptr);
    right_sweep(S.get(), 1e-14, D, nullptr, 1e-6);
  }
  terms.clear();
  const double nrm = site_norm(S.get(), 0);
  if (!(nrm > 0) || !std::isfinite(nrm)) throw Error(XTRG_ENUMERIC, "series: the sum has zero norm");
  xtrg::scale(S->site[0].p, 1.0 / nrm, S->elems(0), s);
  *dlog = std::log(nrm);
  *n_terms = nc;
  auto fin = clone(S.get());
  XTRG_HIP(hipStreamSynchronize(s));
  return fin;
}

// The series start of Sec. II.C, Eq. (RhoTau): rho(tau0) = sum_k (-tau0)^k / k! H^k
// with the cutoff order chosen by the expansion error (expand_series with
// X = I / 2^(L/2)).  The first term is H itself, compressed without loss:
// from the bond-1 identity as the initial guess the product's sweeps would
// see only the parts of H that project onto the identity elsewhere, and
// the traceless couplings project to zero.
std::unique_ptr<xtrg_mpo_s> settn_init(xtrg_ctx c, xtrg_mpo H, double tau0, int D, int n_sweeps, double tol,
                                       double* log_norm, int* n_terms) {
  if (!(tau0 > 0) || !std::isfinite(tau0) || D < 1 || n_sweeps < 1 || !(tol > 0))
    throw Error(XTRG_EINVAL, "settn_init: tau0 > 0, D >= 1, n_sweeps >= 1, tol > 0");
  hipStream_t s = c->stream;
  const int L = H->L;
  const double l0 = 0.5 * L * std::log(2.0);            // ln ||I||_F
  auto I = new_mpo(c, std::vector<int>(L + 1, 1));     // I / sqrt(2) on every site: norm 1, right-canonical
  const double v[4] = {std::sqrt(0.5), 0.0, 0.0, std::sqrt(0.5)};
  for (int i = 0; i < L; ++i) upload(c, I->site[i].p, v, 4);
  auto P = clone(H);
  left_sweep(P.get(), 1e-14, nullptr);
  right_sweep(P.get(), 1e-14, 0, nullptr);
  const double h = site_norm(P.get(), 0);
  if (!(h > 0) || !std::isfinite(h)) throw Error(XTRG_ENUMERIC, "settn_init: ||H|| is zero or not finite");
  xtrg::scale(P->site[0].p, 1.0 / h, P->elems(0), s);
  double dl = 0.0;
  auto out = expand_series(c, H, std::move(I), std::move(P), std::log(h) - l0, -tau0, D, n_sweeps, tol, &dl,
                           n_terms);
  *log_norm = l0 + dl;
  return out;
}

// One step of Eq. (Tay): rho(tau + dtau) from the normalised, right-canonical
// rho(tau) (expand_series with X = rho, x = -dtau).
std::unique_ptr<xtrg_mpo_s> taylor_step(xtrg_ctx c, xtrg_mpo H, xtrg_mpo rho, double dtau, int D, int n_sweeps,
                                        double tol, double* dlog, int* n_terms) {
  if (!std::isfinite(dtau) || D < 1 || n_sweeps < 1 || !(tol > 0))
    throw Error(XTRG_EINVAL, "taylor_step: finite dtau, D >= 1, n_sweeps >= 1, tol > 0");
  if (H->L != rho->L) throw Error(XTRG_EINVAL, "taylor_step: H and rho differ in length");
  return expand_series(c, H, clone(rho), nullptr, 0.0, -dtau, D, n_sweeps, tol, dlog, n_terms);
}

int square_compress(xtrg_ctx c, int n, const xtrg_mpo* ins, const xtrg_compress_opts* opts, xtrg_mpo* outs,
                    xtrg_compress_info* infos, std::string* first_err) {
  return square_compress_impl(c, n, ins, opts, outs, infos, first_err);
}

void observables(xtrg_ctx c, xtrg_mpo rho, double lam, double tau, xtrg_mpo H, int n_sites, xtrg_obs* at_tau,
                 xtrg_obs* at_2tau, double* S_E) {
  observables_impl(c, rho, lam, tau, H, n_sites, at_tau, at_2tau, S_E);
}

void trim(xtrg_ctx c) {
  XTRG_HIP(hipStreamSynchronize(c->stream));
  for (auto& kv : c->ws) c->release(kv.second.p, kv.second.cap);
  c->ws.clear();
}

}  // namespace xtrg_impl

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

int xtrg_ctx_create(int device, void* hip_stream, size_t hbm_budget, xtrg_ctx* out) {
  if (!out) return XTRG_EINVAL;
  *out = nullptr;
  auto c = new xtrg_ctx_s();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->budget = hbm_budget;
  const int rc = guarded(c, [&] {
    int n = 0;
    XTRG_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) throw Error(XTRG_EINVAL, "no such device");
    set_device(c);
    c->scratch = c->alloc(2048);
    (void)scratch_address(device);   // the no-allocation entry point's scratch on this device
  });
  if (rc != XTRG_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return XTRG_OK;
}

int xtrg_ctx_destroy(xtrg_ctx c) {
  if (!c) return XTRG_EINVAL;
  xtrg::server_shutdown(c);
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (auto& kv : c->ws) c->release(kv.second.p, kv.second.cap);
  c->release(c->scratch, 2048);
  delete c;
  return XTRG_OK;
}

const char* xtrg_last_error(xtrg_ctx c) { return c ? c->err.c_str() : "null context"; }

size_t xtrg_ctx_bytes(xtrg_ctx c) { return c ? c->bytes : 0; }

int xtrg_ctx_trim(xtrg_ctx c) {
  if (!c) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    XTRG_HIP(hipStreamSynchronize(c->stream));
    for (auto& kv : c->ws) c->release(kv.second.p, kv.second.cap);
    c->ws.clear();
  });
}

int xtrg_hamiltonian_xxz(xtrg_ctx c, int n_sites, int n_bonds, const int* bonds, const double* jxy,
                         const double* jz, xtrg_mpo* H_out) {
  if (!c || !H_out || n_sites < 2 || n_bonds < 0 || (n_bonds > 0 && (!bonds || !jxy || !jz)))
    return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    *H_out = xtrg_impl::hamiltonian(c, n_sites, n_bonds, bonds, jxy, jz).release();
  });
}

int xtrg_mpo_from_host(xtrg_ctx c, int L, int d, const int* bond_dims, const double* const* site_tensors,
                       xtrg_mpo* out) {
  if (!c || !out || L < 1 || d != 2 || !bond_dims || !site_tensors) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    std::vector<int> dims(bond_dims, bond_dims + L + 1);
    if (dims[0] != 1 || dims[L] != 1) throw Error(XTRG_EINVAL, "outer bonds must be 1");
    for (int v : dims)
      if (v < 1) throw Error(XTRG_EINVAL, "bond dimension < 1");
    auto m = new_mpo(c, dims);
    for (int i = 0; i < L; ++i) {
      if (!site_tensors[i]) throw Error(XTRG_EINVAL, "null site tensor");
      upload(c, m->site[i].p, site_tensors[i], m->elems(i));
    }
    XTRG_HIP(hipStreamSynchronize(c->stream));
    *out = m.release();
  });
}

int xtrg_mpo_shape(xtrg_mpo m, int* L, int* bond_dims) {
  if (!m) return XTRG_EINVAL;
  if (L) *L = m->L;
  if (bond_dims) std::copy(m->dims.begin(), m->dims.end(), bond_dims);
  return XTRG_OK;
}

int xtrg_mpo_to_host(xtrg_mpo m, double* const* site_tensors) {
  if (!m || !site_tensors) return XTRG_EINVAL;
  xtrg_ctx c = m->ctx;
  return guarded(c, [&] {
    set_device(c);
    for (int i = 0; i < m->L; ++i) {
      if (!site_tensors[i]) throw Error(XTRG_EINVAL, "null site tensor");
      XTRG_HIP(hipMemcpyAsync(site_tensors[i], m->site[i].p, m->elems(i) * sizeof(double),
                              hipMemcpyDeviceToHost, c->stream));
    }
    XTRG_HIP(hipStreamSynchronize(c->stream));
  });
}

int xtrg_mpo_destroy(xtrg_mpo m) {
  if (!m) return XTRG_EINVAL;
  (void)hipSetDevice(m->ctx->device);
  (void)hipStreamSynchronize(m->ctx->stream);
  delete m;
  return XTRG_OK;
}

int xtrg_init_rho(xtrg_ctx c, xtrg_mpo H, double tau0, int order, int D0_max, xtrg_mpo* rho_out,
                  double* log_norm) {
  if (!c || !H || !rho_out || !log_norm || !(tau0 > 0) || order < 1 || order > 2) return XTRG_EINVAL;
  if (!H->has_open) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    *rho_out = xtrg_impl::init_rho(c, H, tau0, order, D0_max, log_norm).release();
  });
}

int xtrg_init_rho_u1(xtrg_ctx c, xtrg_mpo H, double tau0, int order, int D0_max, xtrg_mpo* rho_out,
                     double* log_norm) {
  if (!c || !H || !rho_out || !log_norm || !(tau0 > 0) || order < 1 || order > 2) return XTRG_EINVAL;
  if (!H->has_open) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    *rho_out = xtrg_impl::init_rho(c, H, tau0, order, D0_max, log_norm, true).release();
  });
}

int xtrg_mpo_label_charges(xtrg_mpo m) {
  if (!m) return XTRG_EINVAL;
  return guarded(m->ctx, [&] {
    set_device(m->ctx);
    m->charges = infer_charges(download_sites(m), m->dims);
  });
}

int xtrg_mpo_charges(xtrg_mpo m, int* charges) {
  if (!m || !charges || m->charges.empty()) return XTRG_EINVAL;
  size_t o = 0;
  for (const auto& q : m->charges)
    for (int v : q) charges[o++] = v;
  return XTRG_OK;
}

int xtrg_settn_init(xtrg_ctx c, xtrg_mpo H, double tau0, int D_max, int n_sweeps, double tol, xtrg_mpo* rho_out,
                    double* log_norm, int* n_terms) {
  if (!c || !H || !rho_out || !log_norm) return XTRG_EINVAL;
  *rho_out = nullptr;
  return guarded(c, [&] {
    set_device(c);
    int nt = 0;
    *rho_out = xtrg_impl::settn_init(c, H, tau0, D_max, n_sweeps, tol, log_norm, &nt).release();
    if (n_terms) *n_terms = nt;
  });
}

int xtrg_taylor_step(xtrg_ctx c, xtrg_mpo H, xtrg_mpo rho, double dtau, int D_max, int n_sweeps, double tol,
                     xtrg_mpo* rho_out, double* dlog_norm, int* n_terms) {
  if (!c || !H || !rho || !rho_out || !dlog_norm) return XTRG_EINVAL;
  *rho_out = nullptr;
  return guarded(c, [&] {
    set_device(c);
    int nt = 0;
    *rho_out = xtrg_impl::taylor_step(c, H, rho, dtau, D_max, n_sweeps, tol, dlog_norm, &nt).release();
    if (n_terms) *n_terms = nt;
  });
}

int xtrg_square_compress(xtrg_ctx c, xtrg_mpo rho_in, const xtrg_compress_opts* opts, xtrg_mpo* rho_out,
                         xtrg_compress_info* info) {
  if (!c || !rho_in || !opts || !rho_out) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    std::string err;
    xtrg_compress_info tmp{};
    xtrg_compress_info* inf = info ? info : &tmp;
    if (square_compress_impl(c, 1, &rho_in, opts, rho_out, inf, &err) > 0) throw Error(inf->status, err);
  });
}

int xtrg_product_compress(xtrg_ctx c, xtrg_mpo A, xtrg_mpo B, const xtrg_compress_opts* opts, xtrg_mpo* out,
                          xtrg_compress_info* info) {
  if (!c || !A || !B || !opts || !out) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    std::string err;
    xtrg_compress_info tmp{};
    xtrg_compress_info* inf = info ? info : &tmp;
    if (square_compress_impl(c, 1, &A, opts, out, inf, &err, &B) > 0) throw Error(inf->status, err);
  });
}

int xtrg_square_compress_batched(xtrg_ctx c, int n, const xtrg_mpo* rho_in, const xtrg_compress_opts* opts,
                                 xtrg_mpo* rho_out, xtrg_compress_info* info) {
  if (!c || n < 1 || !rho_in || !opts || !rho_out) return XTRG_EINVAL;
  for (int q = 0; q < n; ++q) rho_out[q] = nullptr;
  int first_code = XTRG_OK;
  std::string err;
  const int rc = guarded(c, [&] {
    set_device(c);
    std::vector<xtrg_compress_info> tmp;
    xtrg_compress_info* inf = info;
    if (!inf) {
      tmp.assign(n, xtrg_compress_info{});
      inf = tmp.data();
    }
    if (square_compress_impl(c, n, rho_in, opts, rho_out, inf, &err) > 0)
      for (int q = 0; q < n && first_code == XTRG_OK; ++q)
        if (!rho_out[q]) first_code = inf[q].status;
  });
  if (rc != XTRG_OK) {            // nothing left to release
    for (int q = 0; q < n; ++q)
      if (rho_out[q]) {
        delete rho_out[q];
        rho_out[q] = nullptr;
      }
    return rc;
  }
  if (first_code != XTRG_OK) c->err = err;
  return first_code;
}

int xtrg_observables(xtrg_ctx c, xtrg_mpo rho, double log_norm, double tau_n, xtrg_mpo H, int n_sites,
                     xtrg_obs* at_tau, xtrg_obs* at_2tau, double* S_E_per_bond) {
  if (!c || !rho || !H || !(tau_n > 0)) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    observables_impl(c, rho, log_norm, tau_n, H, n_sites, at_tau, at_2tau, S_E_per_bond);
  });
}

int xtrg_spin_sum_mpo(xtrg_ctx c, int L, int power, xtrg_mpo* out) {
  if (!c || !out || L < 1 || (power != 1 && power != 2)) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    auto m = spin_sum_mpo(c, L, power);
    XTRG_HIP(hipStreamSynchronize(c->stream));
    *out = m.release();
  });
}

int xtrg_correlation_mpo(xtrg_ctx c, int L, int center, const double* weights, xtrg_mpo* out) {
  if (!c || !out || !weights || L < 1 || center < 0 || center >= L) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    auto m = correlation_mpo(c, L, center, weights);
    XTRG_HIP(hipStreamSynchronize(c->stream));
    *out = m.release();
  });
}

int xtrg_expectation(xtrg_ctx c, xtrg_mpo rho, int n_ops, const xtrg_mpo* ops, double* at_tau, double* at_2tau) {
  if (!c || !rho || n_ops < 1 || n_ops > 2 || !ops) return XTRG_EINVAL;
  for (int k = 0; k < n_ops; ++k)
    if (!ops[k] || ops[k]->L != rho->L) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    std::vector<xtrg_mpo> m(ops, ops + n_ops);
    std::vector<bool> tr(n_ops, false);
    if (at_tau) {
      const double z = trace_chain(c, {rho}, {false});
      if (!(z > 0)) throw Error(XTRG_ENUMERIC, "Tr rho <= 0");
      auto mm = m;
      auto tt = tr;
      mm.push_back(rho);
      tt.push_back(false);
      *at_tau = trace_chain(c, mm, tt) / z;
    }
    if (at_2tau) {
      const double z = trace_chain(c, {rho, rho}, {true, false});
      if (!(z > 0)) throw Error(XTRG_ENUMERIC, "||rho|| = 0");
      auto mm = m;
      auto tt = tr;
      mm.push_back(rho);
      tt.push_back(true);
      mm.push_back(rho);
      tt.push_back(false);
      *at_2tau = trace_chain(c, mm, tt) / z;
    }
  });
}

int xtrg_profile_enable(xtrg_ctx c, int on) {
  if (!c) return XTRG_EINVAL;
  c->prof = on != 0;
  return XTRG_OK;
}

int xtrg_profile_report(xtrg_ctx c, char* buf, size_t cap) {
  if (!c || !buf || cap == 0) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    XTRG_HIP(hipStreamSynchronize(c->stream));
    double ms[P_NCAT] = {0}, fl[P_NCAT] = {0}, by[P_NCAT] = {0};
    long n[P_NCAT] = {0};
    for (auto& r : c->prof_recs) {
      float t = 0.f;
      XTRG_HIP(hipEventElapsedTime(&t, r.a, r.b));
      ms[r.cat] += t;
      fl[r.cat] += r.flops;
      by[r.cat] += r.bytes;
      n[r.cat] += r.launches;
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    c->prof_recs.clear();
    std::string out = "{";
    for (int q = 0; q < P_NCAT; ++q) {
      char tmp[256];
      std::snprintf(tmp, sizeof tmp, "%s\"%s\": {\"ms\": %.6f, \"calls\": %ld, \"flops\": %.6e, \"bytes\": %.6e}",
                    q ? ", " : "", kPhase[q], ms[q], n[q], fl[q], by[q]);
      out += tmp;
    }
    char tail[512];
    std::snprintf(tail, sizeof tail,
                  ", \"svd_calls\": %ld, \"svd_sweeps\": %ld, \"warm_built\": %ld, \"warm_rejected\": %ld, "
                  "\"warm_used\": %ld, \"warm_m\": %ld, \"qr_calls\": %ld, \"qr_rows\": %ld, "
                  "\"qr_sweeps\": %ld, \"qr_used\": %ld, \"qr_rejected\": %ld}",
                  c->svd_calls, c->svd_sweeps, c->warm_built, c->warm_rejected, c->warm_used, c->warm_m,
                  c->qr_calls, c->qr_rows, c->qr_sweeps, c->qr_used, c->qr_rejected);
    out += tail;
    c->svd_calls = c->svd_sweeps = 0;
    c->warm_built = c->warm_rejected = c->warm_used = c->warm_m = 0;
    c->qr_calls = c->qr_rows = c->qr_sweeps = c->qr_used = c->qr_rejected = 0;
    if (out.size() + 1 > cap) throw Error(XTRG_EINVAL, "profile report buffer too small");
    std::memcpy(buf, out.c_str(), out.size() + 1);
  });
}

int xtrg_dgemm(xtrg_ctx c, int M, int N, int K, int transA, int transB, const double* A, long lda,
               const double* B, long ldb, double* C, long ldc) {
  if (!c || M < 0 || N < 0 || K < 0 || (M * (long)N > 0 && (!A || !B || !C))) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    gemm(c, plain(M, N, K, A, lda, transA != 0, B, ldb, transB != 0, C, ldc));
    XTRG_HIP(hipStreamSynchronize(c->stream));
  });
}

int xtrg_dgemm_noalloc(xtrg_ctx c, int M, int N, int K, int transA, int transB, const double* A, long lda,
                       const double* B, long ldb, double* C, long ldc) {
  if (!c || M < 0 || N < 0 || K < 0 || (M * (long)N > 0 && (!A || !B || !C))) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    const Gemm g = plain(M, N, K, A, lda, transA != 0, B, ldb, transB != 0, C, ldc);
    const size_t need = xtrg::gemm_splitk_work(g);
    if (need > kNoAllocDoubles)
      throw Error(XTRG_EINVAL, "xtrg_dgemm_noalloc: the split-K partials of this shape need " + std::to_string(need) +
                                   " doubles, the fixed scratch holds " + std::to_string(kNoAllocDoubles));
    // every partial is written before it is read: nothing to clear
    xtrg::gemm(g, c->stream, need ? scratch_address(c->device) : nullptr, kNoAllocDoubles);
    XTRG_HIP(hipGetLastError());
  });
}

int xtrg_sgemm(xtrg_ctx c, int M, int N, int K, int transA, int transB, const float* A, long lda,
               const float* B, long ldb, void* C, long ldc, int c_double) {
  if (!c || M < 0 || N < 0 || K < 0 || (M * (long)N > 0 && (!A || !B || !C))) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    gemm(c, plain(M, N, K, A, lda, transA != 0, B, ldb, transB != 0, C, ldc, xtrg::GEMM_F32, c_double != 0));
    XTRG_HIP(hipStreamSynchronize(c->stream));
  });
}

int xtrg_gemm_bf16x3(xtrg_ctx c, int M, int N, int K, int transA, int transB, const float* A, long lda,
                     const float* B, long ldb, void* C, long ldc, int c_double) {
  if (!c || M < 0 || N < 0 || K < 0 || (M * (long)N > 0 && (!A || !B || !C))) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    gemm(c, plain(M, N, K, A, lda, transA != 0, B, ldb, transB != 0, C, ldc, xtrg::GEMM_BF16X3, c_double != 0));
    XTRG_HIP(hipStreamSynchronize(c->stream));
  });
}

int xtrg_dsvd_left(xtrg_ctx c, int len, int p, const double* Y, double* sigma, int k, double* U) {
  if (!c || len < 0 || p < 0 || k < 0 || k > p || (len * (long)p > 0 && !Y)) return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    double* work = c->need("svd", xtrg::svd_work(len, p));
    int sw = 0;
    RoundProf rp(c);
    xtrg::svd_left(len, p, Y, sigma, k, U, len, 0, work, svd_desc(c, 1), c->stream, &sw, &rp);
    c->svd_calls += 1;
    c->svd_sweeps += sw;
    if (k > 0 && U) orthonormalize(c, U, len, k, false);
    XTRG_HIP(hipStreamSynchronize(c->stream));
  });
}

int xtrg_dsvd_left_qr(xtrg_ctx c, int len, int p, const double* Y, double* sigma, int k, double* U, int* keff) {
  if (!c || len < 1 || p < 1 || k < 0 || k > p || !Y || !sigma || (k > 0 && !U) || len > xtrg::kQrMaxLen ||
      p > 2048)
    return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    QrTask T;
    T.len = len;
    T.p = p;
    T.Y = Y;
    T.tag = "#kernel";
    std::vector<QrTask*> tp{&T};
    qr_factorise(c, tp, nullptr);
    if (T.failed) throw Error(XTRG_ENUMERIC, "QR route: non-finite entries or no convergence of the Jacobi");
    if (!T.done) throw Error(XTRG_ENUMERIC, "QR route rejected: fewer than p/4 rows of R above the stop");
    if (k > T.psvd) throw Error(XTRG_EINVAL, "k exceeds the number of values the QR route resolves");
    XTRG_HIP(hipMemsetAsync(sigma, 0, sizeof(double) * p, c->stream));
    XTRG_HIP(hipMemcpyAsync(sigma, xtrg::svd_sorted_values(T.work, len, T.psvd), sizeof(double) * T.psvd,
                            hipMemcpyDeviceToDevice, c->stream));
    if (k > 0) {
      xtrg::svd_gather(len, T.psvd, T.work, k, U, len, 0, c->stream);
      orthonormalize(c, U, len, k, false);
    }
    XTRG_HIP(hipStreamSynchronize(c->stream));
    if (keff) *keff = T.psvd;
  });
}

int xtrg_dqrcp(xtrg_ctx c, int len, int p, const double* Y, double stop_rel, int* piv, double* RT, int* keff) {
  if (!c || len < 0 || p < 0 || !keff || !(stop_rel >= 0.0) || len > xtrg::kQrMaxLen || p > 4096 ||
      (len * (long)p > 0 && (!Y || !piv || !RT)))
    return XTRG_EINVAL;
  return guarded(c, [&] {
    set_device(c);
    std::vector<xtrg::QrJob> jobs{xtrg::QrJob{len, p, Y, c->need("qr", xtrg::qr_work(len, p)), stop_rel, 0}};
    xtrg::qrcp_batched(jobs, qr_desc(c, 1), c->stream);
    const int k = jobs[0].keff;
    if (k > 0) {
      xtrg::qr_rt(jobs[0], RT, p, false, c->stream);
      XTRG_HIP(hipMemcpyAsync(piv, xtrg::qr_pivots(jobs[0]), sizeof(int) * k, hipMemcpyDeviceToDevice, c->stream));
    }
    XTRG_HIP(hipStreamSynchronize(c->stream));
    *keff = k;
  });
}

}  // extern "C"
