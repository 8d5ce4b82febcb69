// Context and MPO handles of the C ABI, shared by the translation units that
// implement it (api.hip: the paper's calls; serve.hip: the serving loop).
#pragma once

#include <algorithm>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "xtrg.h"

namespace xtrg {
struct Server;   // serve.hip
}

// ---------------------------------------------------------------------------
// Context and device memory
// ---------------------------------------------------------------------------

struct DevBuf {
  double* p = nullptr;
  size_t cap = 0;  // doubles
};

struct xtrg_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  size_t bytes = 0;
  std::string err;
  std::map<std::string, DevBuf> ws;   // named, grow-only workspaces
  double* scratch = nullptr;          // 2048 doubles: reductions, small vectors

  // Optional timing of the doubling's phases with HIP events on `stream`.
  struct Prof {
    int cat;
    hipEvent_t a, b;
    double flops, bytes;
    long launches;
  };
  bool prof = false;
  std::vector<Prof> prof_recs;
  long svd_calls = 0, svd_sweeps = 0;
  // warm-start statistics: bases built, rejected, used; sum of completion sizes m
  long warm_built = 0, warm_rejected = 0, warm_used = 0, warm_m = 0;
  // QR-preconditioned first visits: factorisations, their rows, Jacobi
  // sweeps on R^T, starts used, bases rejected by the orthogonality check
  long qr_calls = 0, qr_rows = 0, qr_sweeps = 0, qr_used = 0, qr_rejected = 0;

  // Allocation bookkeeping is shared with the serving thread (user calls may
  // release MPO handles while it runs).
  std::mutex mem_mu;
  // The serving loop (xtrg_serve_submit) owns the stream and workspaces while
  // it runs; the compute calls of the ABI then return XTRG_EBUSY.
  xtrg::Server* server = nullptr;
  std::atomic<bool> serving{false};
  int serve_lanes = 2;      // lanes of the serving loop (xtrg_serve_set_lanes)

  double* alloc(size_t n) {
    std::lock_guard<std::mutex> lk(mem_mu);
    const size_t b = std::max<size_t>(n, 1) * sizeof(double);
    if (budget && bytes + b > budget)
      throw xtrg::Error(XTRG_ENOMEM, "HBM budget exceeded (" + std::to_string(bytes + b) + " > " +
                                   std::to_string(budget) + " bytes)");
    double* p = nullptr;
    if (hipMalloc(&p, b) != hipSuccess) {
      (void)hipGetLastError();
      throw xtrg::Error(XTRG_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
    }
    bytes += b;
    return p;
  }
  void release(double* p, size_t n) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mem_mu);
    // work queued on the stream may still read p
    if (stream) (void)hipStreamSynchronize(stream);
    else (void)hipDeviceSynchronize();
    (void)hipFree(p);
    bytes -= std::max<size_t>(n, 1) * sizeof(double);
  }
  double* need(const std::string& name, size_t n) {
    DevBuf& d = ws[name];
    if (d.cap < n) {
      release(d.p, d.cap);
      d.p = nullptr;
      d.cap = 0;
      d.p = alloc(n);
      d.cap = n;
    }
    return d.p;
  }
};

struct Site {
  double* p = nullptr;
  size_t n = 0;
};

struct xtrg_mpo_s {
  xtrg_ctx ctx = nullptr;
  int L = 0;
  std::vector<int> dims;      // L+1
  std::vector<Site> site;     // device [Dl][2][2][Dr]
  // Hamiltonians built here keep the un-capped right end ([Dl][2][2][2],
  // last index: start, stop) on the host for the series start.
  bool has_open = false;
  std::vector<double> open_last;
  // S^z charge of every bond index (L+1 lists, bond i has dims[i] entries),
  // or empty: the MPO's bond bases are not known to be charge-definite.
  // Index s = 0 of a site is up; the entry W[a][s][s'][b] is non-zero only
  // if q_b = q_a + (s' - s).
  std::vector<std::vector<int>> charges;

  ~xtrg_mpo_s() {
    for (auto& s : site) ctx->release(s.p, s.n);
  }
  size_t elems(int i) const { return (size_t)dims[i] * 4 * dims[i + 1]; }
};


// The paper's calls as the C ABI runs them, for the serving loop (no status
// codes: errors are thrown as xtrg::Error).
namespace xtrg_impl {
std::unique_ptr<xtrg_mpo_s> hamiltonian(xtrg_ctx c, int n_sites, int n_bonds, const int* bonds, const double* jxy,
                                        const double* jz);
std::unique_ptr<xtrg_mpo_s> init_rho(xtrg_ctx c, xtrg_mpo H, double tau0, int order, int D0_max,
                                     double* log_norm, bool u1 = false);
std::unique_ptr<xtrg_mpo_s> settn_init(xtrg_ctx c, xtrg_mpo H, double tau0, int D, int n_sweeps, double tol,
                                       double* log_norm, int* n_terms);
std::unique_ptr<xtrg_mpo_s> taylor_step(xtrg_ctx c, xtrg_mpo H, xtrg_mpo rho, double dtau, int D, int n_sweeps,
                                        double tol, double* dlog, int* n_terms);
// Returns the number of chains that stopped (their outs[q] = NULL, infos[q].status).
int square_compress(xtrg_ctx c, int n, const xtrg_mpo* ins, const xtrg_compress_opts* opts, xtrg_mpo* outs,
                    xtrg_compress_info* infos, std::string* first_err);
void observables(xtrg_ctx c, xtrg_mpo rho, double lam, double tau, xtrg_mpo H, int n_sites, xtrg_obs* at_tau,
                 xtrg_obs* at_2tau, double* S_E);
// Release the named workspaces (waits for the stream).
void trim(xtrg_ctx c);
}  // namespace xtrg_impl

// Serving loop (serve.hip): stop and join the worker, release its requests.
namespace xtrg {
void server_shutdown(xtrg_ctx c);
}
