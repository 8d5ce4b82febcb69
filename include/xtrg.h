/*
 * xtrg.h -- C ABI of the MI355X XTRG library (libxtrg.so).
 *
 * XTRG (exponential thermal tensor renormalization group) cools a thermal
 * state by repeated squaring, rho(2 tau) = rho(tau) * rho(tau), with the
 * product of two matrix product operators (MPOs) compressed back to a bond
 * dimension D by variational two-site sweeps (paper: Sec. II.B, Eqs.
 * (rhoinit), (rho:scale2); App. D.1, Eqs. (MPO:prod), (LSEProd), Fig. VMPO).
 *
 * Conventions for every call:
 *  - Return value: XTRG_OK (0) on success, a negative XTRG_E* code on
 *    failure.  No C++ exception and no abort crosses this interface; the
 *    message of the last failure on a context is xtrg_last_error(ctx).
 *  - Ownership: the library owns all device memory behind xtrg_ctx and
 *    xtrg_mpo handles.  Every *_out handle is newly created and must be
 *    released by the caller with xtrg_mpo_destroy / xtrg_ctx_destroy.
 *    Input handles are never modified (xtrg_mpo_label_charges, which
 *    attaches charge labels to its argument, is the one exception; the
 *    tensors stay unchanged).  Host arrays are caller-owned and
 *    are only read or written during the call.
 *  - Threading: a context serialises its work on one HIP stream; use one
 *    context per host thread.
 *  - Numbers: FP64 at the interface.  MPO site tensors are real, row-major
 *    [D_left][d][d][D_right] with W[a][s][s'][a'] = <s| W_{a a'} |s'>
 *    (row = output index, column = input index), d = 2 (spin 1/2), and the
 *    outermost bonds have dimension 1.
 */
#ifndef XTRG_H
#define XTRG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xtrg_ctx_s* xtrg_ctx;
typedef struct xtrg_mpo_s* xtrg_mpo;

enum {
  XTRG_OK = 0,
  XTRG_EINVAL = -1,   /* bad argument (null pointer, size, shape) */
  XTRG_ENOMEM = -2,   /* device allocation failed or HBM budget exceeded */
  XTRG_EDEVICE = -3,  /* HIP runtime error */
  XTRG_ENUMERIC = -4, /* NaN/Inf, non-positive norm or trace, SVD not converged */
  XTRG_EBUSY = -5
};

/* Precision of the contractions of a doubling (xtrg_compress_opts.precision).
 * XTRG_FP64: everything FP64.
 * XTRG_FP32: the contractions (environment blocks, two-site overlap C_E,
 *   environment advance) take FP32 copies of rho, C and the environments and
 *   run on the FP32 matrix cores with FP32 accumulation (split-K partials are
 *   summed in FP64); C_E is handed to the SVD in FP64, and the SVD, the
 *   truncation, the split, the output sites and the normalisation stay FP64.
 *   Free energies agree with the FP64 path to about 1e-6 relative (tested).
 * XTRG_BF16X3: as XTRG_FP32, but the contractions split every FP32 operand
 *   into two bf16 terms (hi = bf16(x), lo = bf16(x - hi)) and accumulate
 *   hi*hi + hi*lo + lo*hi in FP32 on the bf16 matrix cores (about 16
 *   significant bits per product). */
enum { XTRG_FP64 = 0, XTRG_FP32 = 1, XTRG_BF16X3 = 2 };

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (e.g. torch.cuda.current_stream().cuda_stream) or NULL for the null
 * stream.  `hbm_budget` bounds the bytes the context may hold (0 = no
 * bound); an allocation beyond it fails with XTRG_ENOMEM. */
int xtrg_ctx_create(int device, void* hip_stream, size_t hbm_budget, xtrg_ctx* out);
int xtrg_ctx_destroy(xtrg_ctx ctx);
/* Message of the last failure on ctx ("" if none).  Owned by ctx. */
const char* xtrg_last_error(xtrg_ctx ctx);
/* Device bytes currently held by ctx (MPOs + workspaces). */
size_t xtrg_ctx_bytes(xtrg_ctx ctx);
/* Release the context's workspaces (environment blocks, SVD and GEMM
 * scratch), which otherwise stay allocated at their largest size for reuse;
 * MPO handles are untouched.  Waits for the context stream. */
int xtrg_ctx_trim(xtrg_ctx ctx);

/* Hamiltonian MPO of the spin-1/2 XXZ model on an arbitrary bond list,
 * H = sum_b jxy_b (Sx Sx + Sy Sy) + jz_b Sz Sz
 *   = sum_b jxy_b/2 (S+ S- + S- S+) + jz_b Sz Sz   (real form, App. F),
 * built by the automaton construction of App. B.1: virtual states start,
 * stop and one state per operator still pending across a cut, so
 * D_H = 2 + 3 * (max number of sites with an open bond across a cut).
 * bonds: 2*n_bonds site indices (0-based, in the 1D MPO ordering), i != j.
 * The handle also keeps the un-capped right end (start/stop open) for
 * xtrg_init_rho. */
int xtrg_hamiltonian_xxz(xtrg_ctx ctx, int n_sites, int n_bonds, const int* bonds,
                         const double* jxy, const double* jz, xtrg_mpo* H_out);

/* Upload an MPO.  bond_dims: L+1 entries (first and last must be 1);
 * site_tensors[i]: host array of bond_dims[i]*d*d*bond_dims[i+1] doubles. */
int xtrg_mpo_from_host(xtrg_ctx ctx, int L, int d, const int* bond_dims,
                       const double* const* site_tensors, xtrg_mpo* out);
/* Number of sites and bond dimensions (bond_dims: L+1 entries, caller-sized). */
int xtrg_mpo_shape(xtrg_mpo mpo, int* L, int* bond_dims);
/* Download an MPO into caller-allocated host arrays sized from xtrg_mpo_shape. */
int xtrg_mpo_to_host(xtrg_mpo mpo, double* const* site_tensors);
int xtrg_mpo_destroy(xtrg_mpo mpo);

/* Initial state rho(tau0) = sum_{k<=order} (-tau0)^k/k! H^k (Eq. RhoTau;
 * order 1 is the linear start I - tau0 H of App. C.2, exact at bond D_H).
 * H must come from xtrg_hamiltonian_xxz.  order is 1 or 2.  The result is
 * compressed without loss (numerically zero singular values dropped, never
 * more than D0_max kept if D0_max > 0), right-canonical and normalised:
 * rho(tau0) = exp(*log_norm) * rho_out with ||rho_out||_F = 1. */
int xtrg_init_rho(xtrg_ctx ctx, xtrg_mpo H, double tau0, int order, int D0_max,
                  xtrg_mpo* rho_out, double* log_norm);
/* xtrg_init_rho with S^z charges on every bond (Sec. II.A; App. B.2): the
 * same operator, normalised and right-canonical, compressed by block SVD
 * sweeps, so that every bond index has a definite charge (a dense SVD mixes
 * degenerate values of different charges); the handle carries the charges
 * for doublings with opts.u1 = 1.  The charges of H's automaton states are
 * read from its non-zero entries. */
int xtrg_init_rho_u1(xtrg_ctx ctx, xtrg_mpo H, double tau0, int order, int D0_max,
                     xtrg_mpo* rho_out, double* log_norm);
/* Attach S^z charges to an MPO whose bond bases are charge-definite (e.g. one
 * uploaded with xtrg_mpo_from_host), read from its non-zero entries: site
 * index 0 is up, W[a][s][s'][b] != 0 requires q_b = q_a + (s' - s), q = 0 at
 * the left end; an index that no non-zero entry reaches from the left gets
 * charge 0.  Downloads the sites (host work O(sum_i D_i D_{i+1})).
 * XTRG_EINVAL if some index would need two charges. */
int xtrg_mpo_label_charges(xtrg_mpo mpo);
/* The charges of every bond, bond 0 first (sum of the L+1 bond dimensions
 * ints, caller-sized).  XTRG_EINVAL if the MPO carries none. */
int xtrg_mpo_charges(xtrg_mpo mpo, int* charges);


/* The series start of Sec. II.C, Eq. (RhoTau), for larger tau0: the series
 * sum_k (-tau0)^k/k! H^k up to the first order whose term is at most tol
 * (e.g. 1e-15) relative to the identity term, i.e. an expansion error
 * below tol.  The powers H^k = H (H^(k-1)) are compressed products (the
 * sweeps of xtrg_product_compress at bond <= D_max with n_sweeps sweeps,
 * starting from H itself), each kept normalised with its log-norm; the
 * terms are then added one at a time, each exact sum of two MPOs
 * compressed by SVD sweeps to bond <= D_max with the keep rule of the
 * doublings (App. D.1 direct route, App. D.2 Eq. MPO:plus).  H is any MPO
 * (from xtrg_hamiltonian_xxz or xtrg_mpo_from_host); at most 80 orders.
 * Result: right-canonical and normalised, rho(tau0) = exp(*log_norm) *
 * rho_out; n_terms (may be NULL) receives the cutoff order.
 * Errors: XTRG_EINVAL for tau0 <= 0, D_max < 1, n_sweeps < 1 or tol <= 0,
 * or a two-term sum beyond bond 4096 (D_max above 2048). */
int xtrg_settn_init(xtrg_ctx ctx, xtrg_mpo H, double tau0, int D_max, int n_sweeps, double tol,
                    xtrg_mpo* rho_out, double* log_norm, int* n_terms);

/* One pointwise expansion step of Sec. II.C, Eq. (Tay):
 * rho(tau + dtau) = sum_k (-dtau)^k/k! H^k rho(tau), with the terms
 * H^k rho = H (H^(k-1) rho) built and summed as in xtrg_settn_init, up to
 * the first order whose term is at most tol relative to rho (the series
 * start is this step from rho = I, tau = 0).  rho must be normalised and
 * right-canonical (every output of this library is); the result is too:
 * rho(tau + dtau) = exp(lambda + *dlog_norm) * rho_out for
 * rho(tau) = exp(lambda) * rho.  Steps on the exponential grid
 * (dtau = tau) reach the same temperatures as the doublings.
 * Errors: XTRG_EINVAL for a non-finite dtau, D_max < 1, n_sweeps < 1,
 * tol <= 0, or H and rho of different lengths. */
int xtrg_taylor_step(xtrg_ctx ctx, xtrg_mpo H, xtrg_mpo rho, double dtau, int D_max, int n_sweeps, double tol,
                     xtrg_mpo* rho_out, double* dlog_norm, int* n_terms);

/* Options of one doubling. */
typedef struct {
  int D_max;         /* bond dimension budget D (> 0) */
  int n_sweeps;      /* full sweeps (left-to-right then right-to-left), >= 1 */
  int precision;     /* XTRG_FP64, XTRG_FP32 or XTRG_BF16X3 */
  double degen_rtol; /* multiplet-safe cut: back off to a gap > degen_rtol*sigma_k (1e-6) */
  double sv_floor;   /* singular values <= sv_floor*sigma_1 count as zero (1e-14) */
  int no_warm_start; /* 0: each SVD after the first visit of a bond starts from the
                        previous visit's singular basis (same result, fewer Jacobi
                        sweeps); 1: every SVD starts cold (and no_qr_start is implied) */
  int no_qr_start;   /* 0: a first visit (no basis from an earlier visit) with at least
                        256 rows and columns (at most 2048 of each) is factorised through
                        a column-pivoted QR of its two-site tensor, Y P = Q R, and the
                        one-sided Jacobi on R^T with its rotations W accumulated: the
                        singular values are those of R, the left singular vectors Q W
                        (same result to rounding, fewer Jacobi sweeps);
                        1: such SVDs run the Jacobi on the two-site tensor itself */
  int u1;            /* 0: C_E is factorised as one dense matrix.  1: U(1) charge sectors
                        (Sec. II.A: the XXZ models conserve S^z_tot; App. B.2): the
                        input MPOs must carry S^z charges on their bonds (xtrg_init_rho_u1,
                        xtrg_mpo_label_charges, or an earlier u1 doubling); C_E, block
                        diagonal in the charge of the bond being cut, is factorised block by
                        block (one grouped Jacobi launch per round over all blocks; a block of
                        at least 32 columns starts from the previous visit's basis of the same
                        block unless no_warm_start; no QR start), the keep rule runs on the
                        merged values of all blocks, and every kept singular vector carries its
                        block's charge into the output's bond, which is charge-definite
                        too.  The tensors stay dense.  XTRG_EINVAL if an input has no
                        charges or C_E has weight between different charges. */
} xtrg_compress_opts;

/* Diagnostics of one doubling. */
typedef struct {
  double dlog_norm;     /* ln c, c = ||C||_F before normalisation */
  double trunc_err_max; /* max over bonds of discarded weight sum_{k>kept} s_k^2 / sum s_k^2 */
  int sweeps_done;
  int D_kept_max;
  int steps;            /* two-site steps performed */
  double flops;         /* algorithmic flops of the contractions (64 D^4 per uniform step) */
  double* sv;           /* optional, caller-sized (L-1)*sv_stride: per-bond sigma of the last visit */
  int sv_stride;        /* entries per bond in sv (values beyond the bond's count are zero) */
  int status;           /* out: XTRG_OK, or the code that stopped this chain (batched call) */
} xtrg_compress_info;

/* One XTRG doubling (Eqs. rhoinit, rho:scale2): rho_out ~ rho_in * rho_in
 * compressed to bond <= D_max by n_sweeps variational two-site sweeps
 * (App. D.1, Eq. LSEProd, Fig. VMPO).  rho_in must be normalised and
 * right-canonical (as returned by xtrg_init_rho or this call).  The result
 * is normalised and right-canonical; lambda_{n+1} = 2 lambda_n + info->dlog_norm.
 * Initial guess: rho_in.  Truncation: at most D_max states per bond, backed
 * off to the largest k >= D_max/2 with sigma_k - sigma_{k+1} > degen_rtol*sigma_k
 * (never split a degenerate multiplet; a gap must also exceed the rounding
 * noise of the values, and degen_rtol = 0 cuts at exactly D_max);
 * sigma <= sv_floor*sigma_1 dropped. */
int xtrg_square_compress(xtrg_ctx ctx, xtrg_mpo rho_in, const xtrg_compress_opts* opts,
                         xtrg_mpo* rho_out, xtrg_compress_info* info);

/* Product of two different MPOs, out ~ A B / c compressed to bond <= D_max by
 * the same variational sweeps (App. D.1, Eq. MPO:prod): the cross products
 * rho_{n,n'} = rho_{n-1} rho_{n'-1} of the interleaved temperature grids
 * (Sec. II.B) and the steps H (H^{k-1} rho) of the pointwise expansion
 * (Sec. II.C, Eq. Tay).  B is the initial guess and must be right-canonical
 * (sites 1..L-1 isometric, as every output of xtrg_init_rho and of the
 * compressions is); A is any MPO of the same length (an H from
 * xtrg_hamiltonian_xxz included).  The result is normalised and
 * right-canonical, info->dlog_norm = ln c with c = ||C||_F before
 * normalisation.  With A == B it is xtrg_square_compress. */
int xtrg_product_compress(xtrg_ctx ctx, xtrg_mpo A, xtrg_mpo B, const xtrg_compress_opts* opts,
                          xtrg_mpo* out, xtrg_compress_info* info);

/* The same doubling for n independent chains at once, e.g. the interleaved
 * temperature grids tau0 = 2^(z-1) tau0' of the z-shift average (Sec. II.B, Eq. zshift),
 * other couplings, lengths or bond budgets.  Chain q runs with opts[q]; the
 * chains advance one two-site step each per batch step (each on its own bond
 * schedule, so lengths and sweep counts may differ), and the latency-bound
 * SVD rounds of all chains run as one grouped launch.  Each result equals
 * what xtrg_square_compress returns for that chain alone: the same kernels
 * on the same data in the same order.
 * rho_in, opts, rho_out: n entries each.  rho_out entries are set to NULL on
 * entry.  The chains are independent (Sec. II.B: each z-shift is its own
 * run), and so are their failures: a chain whose tensors turn non-finite
 * (XTRG_ENUMERIC) or whose memory the HBM budget refuses (XTRG_ENOMEM) stops
 * with rho_out[q] = NULL and info[q].status set, while every other chain
 * finishes with the result it would have had alone.  Return value: XTRG_OK
 * if every chain finished; otherwise the status of the first chain that
 * stopped (the finished chains' handles are still returned and must be
 * released; xtrg_last_error names the chain).  Argument and runtime errors
 * (XTRG_EINVAL, XTRG_EDEVICE) stop the whole call with no handle to release.
 * info: NULL or n entries (each with its own optional sv buffer).
 * Device memory grows with n: one set of per-site environment blocks per
 * chain (about 4 D^3 (L-1) doubles at bond D). */
int xtrg_square_compress_batched(xtrg_ctx ctx, int n, const xtrg_mpo* rho_in,
                                 const xtrg_compress_opts* opts, xtrg_mpo* rho_out,
                                 xtrg_compress_info* info);

/* Thermodynamics of a normalised MPO rho (rho_true = exp(log_norm) rho),
 * Eq. (ThermalQuan): f = -ln Z/(N beta), u = <H>/N, c = beta^2 (<H^2> - <H>^2)/N.
 * at_tau : beta = tau_n, Z = Tr rho.
 * at_2tau: beta = 2 tau_n, Z = Tr rho^T rho = ||rho||_F^2 (Sec. II.B).
 * S_E_per_bond (optional, L-1 entries): von Neumann entropy of the
 * normalised vectorised MPO across every bond (Eq. purif), at beta = 2 tau_n;
 * at_2tau->S_E_center / S_E_max are filled only when it is given (the
 * canonical pass it needs costs a sweep of SVDs), else 0. */
typedef struct {
  double beta, lnZ, f, u, c;
  double tr_rho;      /* Tr rho (at_tau) or ||rho||_F^2 (at_2tau) of the normalised MPO */
  double S_E_center, S_E_max;
  /* Invariants of the exact thermal state, as checks of the compression:
   * herm_resid = ||rho - rho^T||_F^2 / ||rho||_F^2 (0: rho is symmetric),
   * sz_tot     = <S^z_tot> (0 for any XXZ Hamiltonian: U(1) symmetry),
   * su2_resid  = (<(S^x_tot)^2> - <(S^z_tot)^2>) / max(<(S^z_tot)^2>, 1)
   *              (0 for the SU(2)-symmetric Heisenberg case jxy = jz, and
   *              only while no multiplet is split), with the expectation
   *              values of the row's estimator. */
  double herm_resid, sz_tot, su2_resid;
} xtrg_obs;

int xtrg_observables(xtrg_ctx ctx, xtrg_mpo rho, double log_norm, double tau_n, xtrg_mpo H,
                     int n_sites, xtrg_obs* at_tau, xtrg_obs* at_2tau, double* S_E_per_bond);

/* Small operator MPOs and their thermal expectation values, for the
 * observables the paper evaluates by MPO sandwiches (Sec. IV.D, Eq. Binder:
 * the Binder ratio U_4 = <M^2>^2 / <M^4> of M = S^z_tot from the exact MPOs
 * of M and M^2; Sec. III.D: the static structure factor
 * S(q) = sum_j e^{-i q r_0j} <S_0 . S_j> from one MPO).
 * xtrg_spin_sum_mpo: (sum_i S^z_i)^power, power 1 (bond 2) or 2 (bond 3).
 * xtrg_correlation_mpo: sum_j weights[j] S_center . S_j (L weights, the
 *   j = center term 3/4 weights[center]; bond 5).  With weights
 *   cos(q r_0j) its expectation value is the real part of S(q).
 * xtrg_expectation: <O_1 ... O_n> for n = 1 or 2 operators of rho's length:
 *   at_tau = Tr(O_1..O_n rho)/Tr rho (beta = tau_n), at_2tau =
 *   Tr(O_1..O_n rho^T rho)/Tr(rho^T rho) (beta = 2 tau_n); either may be NULL.
 *   <M^4> = <M^2 M^2> takes the M^2 MPO twice. */
int xtrg_spin_sum_mpo(xtrg_ctx ctx, int L, int power, xtrg_mpo* out);
int xtrg_correlation_mpo(xtrg_ctx ctx, int L, int center, const double* weights, xtrg_mpo* out);
int xtrg_expectation(xtrg_ctx ctx, xtrg_mpo rho, int n_ops, const xtrg_mpo* ops, double* at_tau, double* at_2tau);

/* Serving (continuous batching of thermal solves, Sec. II.B: independent
 * runs such as the z-shifted grids of Eq. (zshift) advance together).
 *
 * xtrg_serve_submit queues one XTRG run given as a JSON object:
 *   {"n_sites": L, "bonds": [[i, j], ...], "jxy": x or [x per bond],
 *    "jz": x or [...], "tau0": t, "n_doublings": n, "D": D,
 *    "n_sweeps": 2, "order": 1, "precision": "fp64"|"fp32"|"bf16x3",
 *    "beta_mix": 1.0, "series_tol": 0, "u1": false}
 * (the last seven optional, with these defaults; precision applies to the
 * doublings that reach beta >= beta_mix, earlier ones run in FP64;
 * series_tol > 0 starts from xtrg_settn_init at bond <= D with that
 * expansion error instead of the order-1/2 start; u1 = true runs the solve
 * with S^z charges on its bonds, xtrg_init_rho_u1 and opts.u1, and needs
 * series_tol = 0) and
 * returns its id.  The runs are served in lanes (xtrg_serve_set_lanes,
 * default 2): a run goes to lane k if its work per doubling (sites x D^4)
 * is 8^k times below the largest seen so far (the last lane takes the rest),
 * so runs of very different size do not wait on each other's doublings.
 * Each lane is a worker thread with its own stream (lane 0 on the
 * context's, the others on contexts of their own on the same device), and
 * the lanes run concurrently on the device.  A lane admits its queued runs
 * in arrival order whenever their device-memory estimates fit the budget
 * (the context's hbm_budget, or 85% of the free device memory when the
 * first worker starts if that is 0; shared by all lanes), after the lane's
 * shared workspaces (64 MiB plus 128 (4D)^2 bytes for the largest D it
 * admitted) and what the other lanes hold; per run
 * 8 [4 D^3 (L-1) + (4D)(4D+32)(L+9) + 16 D^2 L + 6 D^3 + (4D+32)^2] bytes
 * plus 4 MiB.  A run that could not fit even alone fails with XTRG_ENOMEM.
 * The allocator enforces the same budget, so an estimate that falls short
 * fails that run with XTRG_ENOMEM, not the others.  A lane advances all its admitted runs by one doubling per batch
 * step with xtrg_square_compress_batched, accumulates lambda and the
 * observables after every doubling, and retires finished runs at once;
 * runs submitted meanwhile join at the next step.  A run whose numbers turn
 * non-finite or whose memory the budget refuses fails alone.  Each run's
 * records equal those of the same run served alone.
 * While a lane has work, the context's other compute calls return
 * XTRG_EBUSY; submit and poll may be called from any thread.
 * Errors: XTRG_EINVAL for malformed requests (nothing queued).
 *
 * xtrg_serve_poll: XTRG_EBUSY while the run is queued or running (result_json
 * then holds {"id", "state": "queued"|"running", "doublings"}: its progress
 * at the last batch step), XTRG_EINVAL
 * for an unknown id or a buffer (cap bytes) too small; otherwise XTRG_OK
 * and the result JSON:
 *   {"id", "status" (XTRG_OK or the code that stopped the run), "error",
 *    "submitted_s", "admitted_s", "finished_s", "latency_s" (seconds on the
 *    server's clock), "doublings", "flops" (algorithmic flops of its
 *    doublings), "records": [{"n", "tau", "lam", "bond_dims", "f_tau",
 *    "u_tau", "c_tau", "f_2tau", "u_2tau", "c_2tau", "herm_resid", "sz_tot",
 *    "su2_resid", "trunc_err", "flops"}, ...]}
 * with one record for rho(tau0) and one per completed doubling.
 *
 * xtrg_serve_set_lanes: the number of lanes (1 to 4; 1 serves every run in
 * one lockstep batch).  XTRG_EBUSY while a lane has work; the results of
 * earlier runs stay available to xtrg_serve_poll. */
int xtrg_serve_submit(xtrg_ctx ctx, const char* request_json, unsigned long long* id);
int xtrg_serve_poll(xtrg_ctx ctx, unsigned long long id, char* result_json, size_t cap);
int xtrg_serve_set_lanes(xtrg_ctx ctx, int n_lanes);

/* Timing of the doubling's phases (two-site overlap GEMM, left/right block
 * GEMMs, environment GEMMs, SVD, split/projection) with HIP events on the
 * context stream.  xtrg_profile_report writes a JSON object
 * {"theta_gemm": {"ms", "calls", "flops", "bytes"}, ...} accumulated since
 * the last report into buf (cap bytes) and resets the counters. */
int xtrg_profile_enable(xtrg_ctx ctx, int on);
int xtrg_profile_report(xtrg_ctx ctx, char* buf, size_t cap);

/* Kernel-level entry points (device pointers, FP64, on the context stream).
 * Used by the parity tests of the individual kernels.
 *
 * xtrg_dgemm: C = A * B with A (M x K) stored row-major (lda) or, if transA,
 * as K x M row-major; B (K x N) row-major (ldb) or, if transB, as N x K;
 * C (M x N) row-major (ldc).  Inputs and output must not alias. */
int xtrg_dgemm(xtrg_ctx ctx, int M, int N, int K, int transA, int transB,
               const double* A, long lda, const double* B, long ldb, double* C, long ldc);
/* xtrg_dgemm_noalloc: the product of xtrg_dgemm (same kernels, same
 * result bit for bit) for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It allocates nothing: the split-K partial products live in a
 * fixed device array of 8 Mi doubles (64 MiB) per GPU, part of the library
 * and held until the process ends.  Shapes whose partials need more
 * (xtrg_dgemm splits K for small M*N and large K) are rejected with
 * XTRG_EINVAL and a message naming the size.  The call is enqueued on the
 * context stream and returns without waiting.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (other
 * streams or contexts) race; calls ordered on one stream do not.  Nothing
 * in the array needs to start at zero (every partial is written before it
 * is read). */
int xtrg_dgemm_noalloc(xtrg_ctx ctx, int M, int N, int K, int transA, int transB, const double* A, long lda,
                       const double* B, long ldb, double* C, long ldc);
/* xtrg_sgemm: the same product in the XTRG_FP32 contraction precision:
 * A, B float (device), FP32 matrix cores with FP32 accumulation (split-K
 * partials summed in FP64); C is double if c_double, else float. */
int xtrg_sgemm(xtrg_ctx ctx, int M, int N, int K, int transA, int transB,
               const float* A, long lda, const float* B, long ldb, void* C, long ldc, int c_double);
/* xtrg_gemm_bf16x3: the same product in the XTRG_BF16X3 contraction
 * precision (float operands split into bf16 hi + lo, three bf16 products,
 * FP32 accumulation, split-K partials summed in FP64). */
int xtrg_gemm_bf16x3(xtrg_ctx ctx, int M, int N, int K, int transA, int transB,
                     const float* A, long lda, const float* B, long ldb, void* C, long ldc, int c_double);
/* xtrg_dsvd_left: singular values of the len x p matrix Y stored
 * column-major (column j at Y + j*len, device), descending, into sigma
 * (device, p entries), and the left singular vectors of the first k of them
 * into U (device, column-major len x k; a zero column for a zero singular
 * value).  Y is not modified.  One-sided
 * (Hestenes) Jacobi with column blocks.  Range: ||Y||_F^2 must be a finite
 * double (||Y||_F below ~1.3e154); the results scale exactly with a
 * power-of-two scaling of Y as long as no squared column norm leaves the
 * normal double range.  Len or p above 4096, or a NaN in Y, gives an
 * error status. */
int xtrg_dsvd_left(xtrg_ctx ctx, int len, int p, const double* Y, double* sigma, int k, double* U);
/* xtrg_dsvd_left_qr: the same truncated SVD routed as a first visit of a
 * bond is in xtrg_square_compress (App. D.1, SVD of C_E): column-pivoted
 * QR Y P = Q R stopped at a quarter of the numerical-zero level, one-sided
 * Jacobi on [R^T; I] with its rotations W accumulated, left singular
 * vectors Q W.  sigma (device, p entries): the *keff (host) resolved values
 * descending, zeros after them; U (device, column-major len x k, k <= *keff):
 * the leading left singular vectors.  Y is not modified.  Requires
 * 1 <= len <= 2048, 1 <= p <= 2048; XTRG_EINVAL otherwise, XTRG_ENUMERIC if
 * fewer than p/4 rows of R lie above the stop (a matrix that is mostly
 * rounding noise, which the doubling factorises by the Jacobi on Y). */
int xtrg_dsvd_left_qr(xtrg_ctx ctx, int len, int p, const double* Y, double* sigma, int k, double* U, int* keff);
/* xtrg_dqrcp: Householder QR with column pivoting of Y (len x p stored
 * column-major, device, not modified), triangular factor only: the first
 * stage of the truncated SVD of App. D.1 on a first visit of a bond (the
 * one-sided Jacobi then runs on R^T; the singular values and vectors agree
 * with the Jacobi on Y to rounding).  Step r pivots the remaining
 * column of largest norm below row r, so that Y[:, piv] = Q R with R upper
 * triangular and |R_rr| non-increasing.  The factorisation stops when every
 * remaining column has norm^2 <= stop_rel^2 ||Y||_F^2 (stop_rel = 0: after
 * min(len, p) steps, or at exactly zero remaining columns); *keff (host)
 * receives the number of steps.  piv (device, min(len, p) ints): the pivot
 * column of each step (first keff written).  RT (device, p x min(len, p)
 * doubles, column-major, leading dimension p; first keff columns written):
 * R^T in the input's column order, RT[r*p + c] = R's entry at row r for
 * input column c (zero for columns pivoted before step r).  Requires
 * len <= 2048, p <= 4096; XTRG_EINVAL otherwise. */
int xtrg_dqrcp(xtrg_ctx ctx, int len, int p, const double* Y, double stop_rel, int* piv, double* RT, int* keff);

#ifdef __cplusplus
}
#endif
#endif /* XTRG_H */
