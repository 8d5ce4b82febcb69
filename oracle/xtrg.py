"""XTRG beta-doubling with variational MPO-product compression (FP64 oracle).

Test infrastructure: see the package docstring.  Follows, in order:

* Sec. II.B, Eqs. (rhoinit) and (rho:scale2): rho_n = rho_{n-1} * rho_{n-1},
  tau_n = 2^n tau0, starting from rho(tau0) at tiny tau0.
* Sec. II.C, Eq. (RhoTau) and App. C.2: rho(tau0) as the truncated
  Maclaurin series sum_k (-tau0)^k/k! H^k; order 1 is I - tau0 H, exact at
  the bond dimension of H; the series start (settn_init) builds H^k by
  compressed products and stops at an expansion error below 1e-15.
* Sec. II.D: truncate by a fixed number of kept states, never by discarded
  weight.
* App. D.1, Eqs. (MPO:prod), (LSEProd), Fig. VMPO: minimise
  ||A*B - C||_F^2 by two-site sweeps.  For C canonical about (i, i+1) the
  local solution is C_i C_{i+1} = C_E, the generalized overlap of A*B with
  the environments of C; the environments are grown in three substeps per
  site (Fig. VMPO(c)); C_E is split by an SVD, U goes to C_i and Lambda V^T
  to C_{i+1} in a left-to-right sweep, Lambda joins U in a right-to-left
  sweep (Fig. VMPO(d)); a few full sweeps suffice.
* Sec. II.B: Z(2 tau_n) = Tr(rho_n^T rho_n) = ||rho_n||_F^2.
* Eq. (ThermalQuan): f, u, c_V.
* Sec. IV.A, Eq. (purif): entanglement of the vectorised MPO.

Readings where the paper is silent (the same rules are used by the GPU
library, implemented independently):
* initial guess of C is rho_n itself (same bonds, right-canonical);
* n_sweeps full sweeps, no tolerance exit; a bond at the end of a
  half-sweep is not optimised twice (its C_E would be identical), it is
  only re-gauged for the next direction;
* keep k <= D states, backing off to the largest k >= D/2 with a relative
  gap sigma_k - sigma_{k+1} > deg_rtol * sigma_k so that a (numerically)
  degenerate multiplet is never split; singular values below
  sv_floor * sigma_1, or below the rounding noise of C_E
  (40 eps sqrt(max dim) ||C_E||_F), count as zero;
* rho_n is stored normalised, rho_n = exp(lambda_n) * rhohat_n with
  ||rhohat_n||_F = 1 and lambda_n in FP64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import mpo as M


# --------------------------------------------------------------------------
# Truncation rule (Sec. II.D: a fixed number of states; multiplet-safe cut)
# --------------------------------------------------------------------------

EPS = 2.220446049250313e-16


def noise_floor(M: np.ndarray) -> float:
    """Rounding-noise level of a matrix: singular values below
    40 eps sqrt(max(m, n)) ||M||_F are resolved to less than ~10% by any
    FP64 factorisation and count as zero (reading of the 'numerically
    zero' case the paper leaves open)."""
    return 40.0 * EPS * float(np.sqrt(max(M.shape))) * float(np.linalg.norm(M))


def keep_count(S: np.ndarray, D: int, deg_rtol: float, sv_floor: float, abs_floor: float = 0.0) -> int:
    """Number of singular values kept out of the descending list S."""
    if S.size == 0 or not S[0] > 0:
        return 1
    r = int(np.count_nonzero(S > max(sv_floor * S[0], abs_floor)))
    r = max(r, 1)
    if r <= D:
        return r
    # a gap separates two multiplets only if it exceeds deg_rtol * S[k-1]
    # plus the absolute rounding noise abs_floor of the values themselves:
    # a split decided by noise would not be reproducible (deg_rtol = 0
    # switches the multiplet protection off: cut at exactly D)
    if deg_rtol <= 0:
        return D
    lo = max(1, (D + 1) // 2)
    for k in range(D, lo - 1, -1):
        if S[k - 1] - S[k] > deg_rtol * S[k - 1] + abs_floor:
            return k
    return D


# --------------------------------------------------------------------------
# Initial state (Eq. RhoTau; App. C.2)
# --------------------------------------------------------------------------

def series_rho(n, bonds, jxy, jz, tau0: float, order: int) -> List[np.ndarray]:
    """Exact MPO of sum_{k<=order} (-tau0)^k/k! H^k.

    The order-fold product of the open automaton has, at its right end,
    the product space of 'start'/'stop' states of each factor; a factor that
    ended in 'start' contributed I, one that ended in 'stop' contributed H.
    Weighting every string with m 'stop' entries by omega_m / C(order, m)
    yields sum_m omega_m H^m (App. B.1 boundary states, App. C.2 for m<=1).
    """
    if order < 1:
        raise ValueError("order >= 1")
    Wopen = M.xxz_automaton(n, bonds, jxy, jz)
    P = Wopen
    for _ in range(order - 1):
        P = M.product(P, Wopen)
    left = np.zeros(2 ** order)
    left[0] = 1.0                                      # all factors in 'start'
    right = np.zeros(2 ** order)
    for idx in range(2 ** order):
        m = bin(idx).count("1")                       # number of 'stop' factors
        omega = (-tau0) ** m / math.factorial(m)
        right[idx] = omega / math.comb(order, m)
    return M.cap(P, left, right)


def init_rho(n, bonds, jxy, jz, tau0: float, order: int, rel_floor: float = 1e-14):
    """rho(tau0) normalised and right-canonical, with lambda_0 = ln||rho||_F.

    The exact series MPO is compressed without loss (QR sweep, then an SVD
    sweep dropping singular values <= rel_floor*sigma_1, i.e. exact zeros)."""
    W = series_rho(n, bonds, jxy, jz, tau0, order)
    W = M.svd_compress(W, D=10 ** 9, rel_floor=rel_floor)
    nrm = float(np.linalg.norm(W[0]))                 # right-canonical: norm on site 0
    W[0] = W[0] / nrm
    return W, math.log(nrm)


def identity(n: int) -> List[np.ndarray]:
    """The identity operator as a normalised, right-canonical MPO of bond 1:
    every site I/sqrt(2), so ||I||_F = 2^(n/2) is carried by the log-norm."""
    return [(np.eye(2) / math.sqrt(2.0)).reshape(1, 2, 2, 1) for _ in range(n)]


def _compress_direct(S: List[np.ndarray], D: int, deg_rtol: float, sv_floor: float) -> List[np.ndarray]:
    """The direct route of App. D.1: left-canonicalise, then a right-to-left
    SVD sweep, each bond cut by the keep rule of the doublings (keep_count:
    at most D values, multiplet-safe, numerically zero values dropped)."""
    W = M.left_canonicalize(S)
    for i in range(len(W) - 1, 0, -1):
        Dl, d1, d2, Dr = W[i].shape
        Mi = W[i].reshape(Dl, d1 * d2 * Dr)
        U, Sv, Vt = np.linalg.svd(Mi, full_matrices=False)
        k = keep_count(Sv, D, deg_rtol, sv_floor, noise_floor(Mi))
        W[i] = Vt[:k].reshape(k, d1, d2, Dr)
        W[i - 1] = np.einsum("astb,bk->astk", W[i - 1], U[:, :k] * Sv[:k])
    return W


def sum_compress(terms: Sequence[List[np.ndarray]], coefs: Sequence[float], D: int,
                 deg_rtol: float = 1e-6, sv_floor: float = 1e-14) -> List[np.ndarray]:
    """sum_k coefs[k] * terms[k] as one MPO of bond <= D, added one term at a
    time: S <- compress(S + coefs[k] terms[k]), each exact sum of two MPOs
    (block-diagonal bonds, App. D.2 Eq. MPO:plus) compressed by the direct
    route (_compress_direct).  Exact when nothing is cut; the exact sums
    stay at bond <= D + bond(terms[k])."""
    S = None
    for W, a in zip(terms, coefs):
        X = [w.copy() for w in W]
        X[0] = X[0] * a
        S = _compress_direct(X if S is None else M.mpo_sum(S, X), D, deg_rtol, sv_floor)
    return S


def settn_init(H: List[np.ndarray], tau0: float, D: int, n_sweeps: int = 2, tol: float = 1e-15,
               k_max: int = 80, deg_rtol: float = 1e-6, sv_floor: float = 1e-14, svd=None):
    """rho(tau0) by the series expansion of Sec. II.C, Eq. (RhoTau), with the
    cutoff order chosen automatically.

    The terms H^k are built one from the other, H^k = H (H^(k-1)), each
    product compressed to bond <= D by product_compress (App. D.1; the same
    sweeps as a doubling, the initial guess the previous term).  The
    recursion starts from H itself, compressed without loss: from the
    identity (bond 1) as the initial guess, the sweeps would only see the
    parts of H whose other sites project onto the identity, and the traceless
    couplings project to zero.  Every term
    is kept normalised with its log-norm l_k, so that
    omega_k H^k = omega_k e^(l_k) Hhat_k with omega_k = (-tau0)^k / k!.  The
    expansion stops at the first order N_c whose term is below tol relative
    to the identity term, |omega_k| e^(l_k - l_0) <= tol (an expansion error
    below 1e-15, as the paper asks; l_0 = ln ||I||_F).  The N_c + 1 terms
    are summed by sum_compress (one term at a time).  Returns (rhohat,
    lambda_0, N_c) with rho(tau0) = e^(lambda_0) rhohat, ||rhohat||_F = 1 and
    rhohat right-canonical."""
    n = len(H)
    l0 = 0.5 * n * math.log(2.0)
    terms, coefs = [identity(n)], [1.0]
    P = M.svd_compress(H, D=10 ** 9, rel_floor=sv_floor)       # H itself, canonical
    h = float(np.linalg.norm(P[0]))
    P[0] = P[0] / h
    l = math.log(h)
    omega = 1.0
    nc = 0
    for k in range(1, k_max + 1):
        if k > 1:
            P, info = product_compress(H, P, D, n_sweeps, deg_rtol, sv_floor, svd=svd)
            l += info.dlog_norm
        omega *= -tau0 / k
        a = omega * math.exp(l - l0)
        terms.append(P)
        coefs.append(a)
        nc = k
        if abs(a) <= tol:
            break
    W = sum_compress(terms, coefs, D, deg_rtol, sv_floor)
    nrm = float(np.linalg.norm(W[0]))
    W[0] = W[0] / nrm
    return W, l0 + math.log(nrm), nc


def taylor_step(H: List[np.ndarray], rho: List[np.ndarray], dtau: float, D: int, n_sweeps: int = 2,
                tol: float = 1e-15, k_max: int = 80, deg_rtol: float = 1e-6, sv_floor: float = 1e-14, svd=None):
    """One pointwise expansion step, Sec. II.C Eq. (Tay):
    rho(tau + dtau) = sum_k (-dtau)^k / k! H^k rho(tau), for the normalised
    right-canonical rhohat of rho(tau).  The terms H^k rhohat = H (H^(k-1)
    rhohat) are compressed products (product_compress, the previous term as
    B and initial guess), each normalised with its log-norm; the expansion
    stops at the first order whose term is at most tol relative to the
    k = 0 term (rhohat, norm 1), and the terms are added one at a time by
    sum_compress.  Returns (rhohat', dlog, N_c) with
    rho(tau + dtau) = e^(lambda + dlog) rhohat' for rho(tau) = e^lambda rhohat."""
    terms, coefs = [[w.copy() for w in rho]], [1.0]
    P, l = terms[0], 0.0
    omega = 1.0
    nc = 0
    for k in range(1, k_max + 1):
        P, info = product_compress(H, P, D, n_sweeps, deg_rtol, sv_floor, svd=svd)
        l += info.dlog_norm
        omega *= -dtau / k
        a = omega * math.exp(l)
        terms.append(P)
        coefs.append(a)
        nc = k
        if abs(a) <= tol:
            break
    W = sum_compress(terms, coefs, D, deg_rtol, sv_floor)
    nrm = float(np.linalg.norm(W[0]))
    W[0] = W[0] / nrm
    return W, math.log(nrm), nc


# --------------------------------------------------------------------------
# Environments (Fig. VMPO(a), (c))
# --------------------------------------------------------------------------

def left_block(L: np.ndarray, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """First two substeps of Fig. VMPO(c): Lb[c,s,a',s'',b'] =
    sum_{a,b,s'} L[c,a,b] A[a,s,s',a'] B[b,s',s'',b']."""
    T1 = np.einsum("cab,astp->cbstp", L, A, optimize=True)        # O(Da^2 Db Dc)
    Lb = np.einsum("cbstp,btuq->cspuq", T1, B, optimize=True)     # O(Da Db^2 Dc)
    return Lb


def left_env(Lb: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Third substep: L'[c',a',b'] = sum_{c,s,s''} Lb[c,s,a',s'',b'] C[c,s,s'',c']."""
    return np.einsum("cspuq,csur->rpq", Lb, C, optimize=True)      # O(Da Db Dc^2)


def right_block(R: np.ndarray, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Mirror of left_block: Rb[a,b,t,t'',c''] =
    sum_{a'',b'',t'} A[a,t,t',a''] B[b,t',t'',b''] R[c'',a'',b'']."""
    U1 = np.einsum("atvp,cpq->atvqc", A, R, optimize=True)
    Rb = np.einsum("atvqc,bvwq->abtwc", U1, B, optimize=True)
    return Rb


def right_env(Rb: np.ndarray, C: np.ndarray) -> np.ndarray:
    """R[c,a,b] = sum_{t,t'',c''} Rb[a,b,t,t'',c''] C[c,t,t'',c'']."""
    return np.einsum("abtwe,ctwe->cab", Rb, C, optimize=True)


def two_site_overlap(Lb: np.ndarray, Rb: np.ndarray) -> np.ndarray:
    """Generalized overlap C_E (Eq. LSEProd, Fig. VMPO(a)) as a matrix with
    rows (c, s, s'') and columns (t, t'', c'')."""
    th = np.einsum("cspuq,pqtwe->csutwe", Lb, Rb, optimize=True)
    c, s, u, t, w, e = th.shape
    return th.reshape(c * s * u, t * w * e)


def sweep_schedule(n: int, n_sweeps: int):
    """Bonds visited by n_sweeps full sweeps: a list of (bond, direction,
    is_last_of_half_sweep).  The bond that ends a half-sweep is not visited
    again at the start of the next one."""
    out = []
    for h in range(2 * n_sweeps):
        if h % 2 == 0:
            bonds = list(range(0 if h == 0 else 1, n - 1))
            d = +1
        else:
            bonds = list(range(n - 3, -1, -1))
            d = -1
        for j, b in enumerate(bonds):
            out.append((b, d, j == len(bonds) - 1))
    return out


@dataclasses.dataclass
class CompressInfo:
    dlog_norm: float
    sv: List[np.ndarray]
    kept: List[int]
    discarded: List[float]
    steps: int
    flops: float
    charges: Optional[List[np.ndarray]] = None   # S^z charge of every bond index (u1 route)

    @property
    def trunc_err_max(self) -> float:
        return max(self.discarded) if self.discarded else 0.0


def square_compress(rho: List[np.ndarray], D: int, n_sweeps: int = 4,
                    deg_rtol: float = 1e-6, sv_floor: float = 1e-14, svd=None, u1: bool = False):
    """One doubling: C ~ rho*rho, compressed variationally to bond <= D.

    ``rho`` must be right-canonical with ||rho||_F = 1.  Returns the new
    normalised right-canonical MPO and a CompressInfo with ln c, where
    c = ||C||_F before normalisation, so lambda_{n+1} = 2 lambda_n + ln c.
    ``svd`` factorises C_E (default: LAPACK gesdd through numpy); the tests
    substitute other factorisations to measure how the result depends on it.
    ``u1``: factorise C_E by charge blocks (block_svd); rho must have
    charge-definite bonds (bond_charges), and so has the result.
    """
    return product_compress(rho, rho, D, n_sweeps, deg_rtol, sv_floor, svd, u1)


def product_compress(A: List[np.ndarray], B: List[np.ndarray], D: int, n_sweeps: int = 4,
                     deg_rtol: float = 1e-6, sv_floor: float = 1e-14, svd=None, u1: bool = False):
    """C ~ A*B compressed variationally to bond <= D (App. D.1, Eq.
    MPO:prod with two different factors): the cross products
    rho_{n,n'} = rho_{n-1} rho_{n'-1} of the interleaved grids (Sec. II.B)
    and the steps H (H^{k-1} rho) of the pointwise expansion (Sec. II.C,
    Eq. Tay).  The initial guess is B, which must be right-canonical (its
    sites 1..L-1 isometric, as every output of this function and of
    init_rho is).  Returns the normalised right-canonical C and a
    CompressInfo with ln c, c = ||C||_F before normalisation.

    With u1, A and B must conserve S^z_tot in charge-definite bond bases
    (bond_charges); C_E is then block-diagonal in the charge of the bond
    being cut, it is factorised block by block (block_svd), and the kept
    singular vectors carry their block's charge into C's bond, so C is
    charge-definite too (info.charges).  The cut is the same keep rule on
    the merged values of all blocks."""
    if svd is None:
        svd = lambda a: np.linalg.svd(a, full_matrices=False)
    n = len(A)
    if n < 2 or len(B) != n:
        raise ValueError("need two MPOs of the same length >= 2")
    C = [w.copy() for w in B]                           # initial guess
    if u1:
        bond_charges(A)                                 # raises unless A conserves S^z in its basis
        qc = bond_charges(B)                            # charges of C's bonds (C = B)
    one = np.ones((1, 1, 1))
    L: List[np.ndarray] = [None] * (n + 1)
    R: List[np.ndarray] = [None] * (n + 2)
    L[0] = one
    R[n] = one
    for j in range(n - 1, 1, -1):                       # R_{n-1} .. R_2
        R[j] = right_env(right_block(R[j + 1], A[j], B[j]), C[j])
    sv = [np.zeros(0)] * (n - 1)
    kept = [1] * (n - 1)
    disc = [0.0] * (n - 1)
    flops = 0.0
    S_last = None
    sched = sweep_schedule(n, n_sweeps)
    for step, (i, d, last) in enumerate(sched):
        Lb = left_block(L[i], A[i], B[i])
        Rb = right_block(R[i + 2], A[i + 1], B[i + 1])
        th = two_site_overlap(Lb, Rb)
        flops += _step_flops(L[i].shape, A[i].shape[3], B[i].shape[3], R[i + 2].shape)
        if u1:
            U, S, Vt, qs = block_svd(th, theta_row_charges(qc[i]), theta_col_charges(qc[i + 2]), svd)
        else:
            U, S, Vt = svd(th)
        k = keep_count(S, D, deg_rtol, sv_floor, noise_floor(th))
        if u1:
            qc[i + 1] = qs[:k].copy()
        tot = float(np.sum(S * S))
        sv[i] = S.copy()
        kept[i] = k
        disc[i] = float(np.sum(S[k:] ** 2) / tot) if tot > 0 else 0.0
        Dc = L[i].shape[0]
        Dc2 = R[i + 2].shape[0]
        go_right = (d > 0) != (last and step != len(sched) - 1)
        if step == len(sched) - 1:
            go_right = False
        if go_right:
            C[i] = U[:, :k].reshape(Dc, 2, 2, k)
            C[i + 1] = (S[:k, None] * Vt[:k]).reshape(k, 2, 2, Dc2)
            L[i + 1] = left_env(Lb, C[i])
        else:
            C[i + 1] = Vt[:k].reshape(k, 2, 2, Dc2)
            C[i] = (U[:, :k] * S[:k]).reshape(Dc, 2, 2, k)
            R[i + 1] = right_env(Rb, C[i + 1])
        S_last = S[:k]
    c = float(np.sqrt(np.sum(S_last * S_last)))
    C[0] = C[0] / c
    return C, CompressInfo(math.log(c), sv, kept, disc, len(sched), flops, qc if u1 else None)


def _step_flops(Lshape, Da2, Db2, Rshape) -> float:
    """Algorithmic flops of one two-site step with the static side built:
    left block (2 substeps), C_E, left/right environment advance.  Uses the
    actual bond dimensions (d = 2)."""
    Dc, Da, Db = Lshape
    Dc2, Da3, Db3 = Rshape
    d = 2
    k1 = 2.0 * Dc * Db * Da * d * d * Da2
    k2 = 2.0 * Dc * d * Da2 * Db * d * d * Db2
    th = 2.0 * (Dc * d * d) * (Da2 * Db2) * (d * d * Dc2)
    k3 = 2.0 * Da2 * Db2 * (Dc * d * d) * Dc
    return k1 + k2 + th + k3


# --------------------------------------------------------------------------
# U(1) charge sectors (Sec. II.A: the models conserve S^z_tot, and the
# paper's tensors are blocked by it; App. B.2).  The tensors stay dense
# here: the charges label the bond indices, and the factorisations run
# block by block.
# --------------------------------------------------------------------------

def bond_charges(W: List[np.ndarray]) -> List[np.ndarray]:
    """S^z charge of every bond index of an MPO whose operator commutes with
    S^z_tot, written in a basis in which every index has a definite charge.

    Site index s = 0 is up (S^z = +1/2), s = 1 down; the entry W[a, s, s', b]
    multiplies |s><s'|, which raises S^z by s' - s.  In a charge-definite
    basis an entry can be non-zero only if q_b = q_a + (s' - s), with q = 0
    at the left end, so the charges follow from the non-zero entries, site
    by site.  An index that no non-zero entry reaches from the left end
    (a state of a redundant MPO that never occurs, such as a product of
    automata in which one factor has stopped before the other started)
    contributes nothing to the operator: its own entries are ignored, and
    it gets charge 0.  Raises ValueError if two entries of one index imply
    different charges (the operator does not conserve S^z, or the basis
    mixes charges)."""
    q = [np.zeros(W[0].shape[0], dtype=np.int64)]
    known = np.ones(W[0].shape[0], dtype=bool)
    for i, w in enumerate(W):
        a, s, t, b = np.nonzero(w)
        use = known[a]
        a, s, t, b = a[use], s[use], t[use], b[use]
        v = q[i][a] + (t - s)
        Dr = w.shape[3]
        lo = np.full(Dr, np.iinfo(np.int64).max)
        hi = np.full(Dr, np.iinfo(np.int64).min)
        np.minimum.at(lo, b, v)
        np.maximum.at(hi, b, v)
        known = hi >= lo
        if np.any(known & (hi != lo)):
            raise ValueError(f"site {i}: a bond index carries two S^z charges")
        q.append(np.where(known, lo, 0))
    return q


def theta_row_charges(q_left: np.ndarray) -> np.ndarray:
    """Charges of the rows (c, s, s'') of C_E: q_c + (s'' - s)."""
    d = np.arange(2)
    return (q_left[:, None, None] + (d[None, None, :] - d[None, :, None])).reshape(-1)


def theta_col_charges(q_right: np.ndarray) -> np.ndarray:
    """Charges of the columns (t, t'', c'') of C_E: the charge a row must
    carry to connect to them, q_c'' - (t'' - t)."""
    d = np.arange(2)
    return (d[:, None, None] - d[None, :, None] + q_right[None, None, :]).reshape(-1)


def block_svd(th: np.ndarray, q_row: np.ndarray, q_col: np.ndarray, svd=None):
    """SVD of a matrix whose entries vanish unless the row and the column
    charge agree.  Sorted by charge it is block-diagonal, so its singular
    triples are those of its blocks, each block factorised on its own.
    Returns U, S, Vt, q: S descending over all blocks (equal values in
    increasing charge), U and Vt zero outside their block, q the charge of
    each triple.  Raises ValueError if an entry between different charges
    is non-zero."""
    if svd is None:
        svd = lambda a: np.linalg.svd(a, full_matrices=False)
    m, n = th.shape
    if np.any(th[q_row[:, None] != q_col[None, :]] != 0):
        raise ValueError("non-zero entry between different S^z charges")
    Us, Ss, Vs, qs = [], [], [], []
    for qv in np.intersect1d(q_row, q_col):
        r = np.nonzero(q_row == qv)[0]
        c = np.nonzero(q_col == qv)[0]
        u, s, vt = svd(th[np.ix_(r, c)])
        U = np.zeros((m, s.size))
        U[r] = u
        V = np.zeros((s.size, n))
        V[:, c] = vt
        Us.append(U)
        Ss.append(s)
        Vs.append(V)
        qs.append(np.full(s.size, qv, dtype=np.int64))
    if not Ss:
        raise ValueError("no charge is shared by the rows and the columns")
    S = np.concatenate(Ss)
    q = np.concatenate(qs)
    order = np.lexsort((q, -S))
    return np.concatenate(Us, axis=1)[:, order], S[order], np.concatenate(Vs, axis=0)[order], q[order]


def canonical_u1(W: List[np.ndarray], rel_floor: float = 1e-14) -> List[np.ndarray]:
    """Lossless canonical form with charge-definite bonds: a left-to-right
    sweep of block SVDs (U stays, S V^T moves right), then a right-to-left
    one (V^T stays, U S moves left), each dropping only the values at or
    below rel_floor * s_1 or the rounding noise (the exact zeros of a
    redundant MPO such as the automaton's).  The result is right-canonical,
    the operator is unchanged."""
    W = [w.copy() for w in W]
    q = bond_charges(W)
    n = len(W)
    for i in range(n - 1):
        Dl, d1, d2, Dr = W[i].shape
        Mi = W[i].reshape(Dl * d1 * d2, Dr)
        U, S, Vt, qs = block_svd(Mi, theta_row_charges(q[i]), q[i + 1])
        k = keep_count(S, 10 ** 9, 0.0, rel_floor, noise_floor(Mi))
        W[i] = U[:, :k].reshape(Dl, d1, d2, k)
        W[i + 1] = np.einsum("kb,bstc->kstc", S[:k, None] * Vt[:k], W[i + 1])
        q[i + 1] = qs[:k]
    for i in range(n - 1, 0, -1):
        Dl, d1, d2, Dr = W[i].shape
        Mi = W[i].reshape(Dl, d1 * d2 * Dr)
        U, S, Vt, qs = block_svd(Mi, q[i], theta_col_charges(q[i + 1]))
        k = keep_count(S, 10 ** 9, 0.0, rel_floor, noise_floor(Mi))
        W[i] = Vt[:k].reshape(k, d1, d2, Dr)
        W[i - 1] = np.einsum("astb,bk->astk", W[i - 1], U[:, :k] * S[:k])
        q[i] = qs[:k]
    return W


def init_rho_u1(n, bonds, jxy, jz, tau0: float, order: int, rel_floor: float = 1e-14):
    """init_rho with charge-definite bonds (canonical_u1 in place of the QR
    and SVD sweeps): the same operator, normalised and right-canonical."""
    W = canonical_u1(series_rho(n, bonds, jxy, jz, tau0, order), rel_floor)
    nrm = float(np.linalg.norm(W[0]))
    W[0] = W[0] / nrm
    return W, math.log(nrm)


# --------------------------------------------------------------------------
# Observables (Eq. ThermalQuan; Sec. II.B for beta = 2 tau_n)
# --------------------------------------------------------------------------

def observables(rho: List[np.ndarray], lam: float, tau: float, H: List[np.ndarray],
                n_sites: int) -> Dict[str, Dict[str, float]]:
    """f, u, c per site at beta = tau (Z = Tr rho) and at beta = 2 tau
    (Z = Tr rho^T rho).  ``rho`` is the normalised MPO, rho_true = e^lam rho.

    Also the invariants of the exact thermal state that the compression
    must keep: herm_resid = ||rho - rho^T||^2 / ||rho||^2, <S^z_tot>, and
    su2_resid = (<(S^x_tot)^2> - <(S^z_tot)^2>) / max(<(S^z_tot)^2>, 1)
    (zero for an SU(2)-symmetric H while no multiplet is split)."""
    n = len(rho)
    SZ = M.local_sum(M.SZ, n)
    SX = M.local_sum(0.5 * (M.SPLUS + M.SMINUS), n)
    out = {}
    rt = M.transpose(rho)
    nrm = M.inner(rho, rho)
    herm = (M.inner(rho, rho) + M.inner(rt, rt) - 2.0 * M.inner(rho, rt)) / nrm
    tr = M.trace(rho)
    e1 = M.trace_of_product(H, rho) / tr
    e2 = M.trace_of_product(H, H, rho) / tr
    z2 = M.trace_of_product(SZ, SZ, rho) / tr
    x2 = M.trace_of_product(SX, SX, rho) / tr
    b = tau
    lnZ = lam + math.log(tr)
    out["tau"] = dict(beta=b, lnZ=lnZ, f=-lnZ / (n_sites * b), u=e1 / n_sites,
                      c=b * b * (e2 - e1 * e1) / n_sites, tr=tr, herm_resid=herm,
                      sz_tot=M.trace_of_product(SZ, rho) / tr, su2_resid=(x2 - z2) / max(z2, 1.0))
    g1 = M.trace_of_product(H, rt, rho) / nrm
    g2 = M.trace_of_product(H, H, rt, rho) / nrm
    z2 = M.trace_of_product(SZ, SZ, rt, rho) / nrm
    x2 = M.trace_of_product(SX, SX, rt, rho) / nrm
    b = 2 * tau
    lnZ = 2 * lam + math.log(nrm)
    out["2tau"] = dict(beta=b, lnZ=lnZ, f=-lnZ / (n_sites * b), u=g1 / n_sites,
                       c=b * b * (g2 - g1 * g1) / n_sites, norm2=nrm, herm_resid=herm,
                       sz_tot=M.trace_of_product(SZ, rt, rho) / nrm, su2_resid=(x2 - z2) / max(z2, 1.0))
    return out


def expectation(rho: List[np.ndarray], ops) -> Dict[str, float]:
    """<O_1 ... O_n> at beta = tau (Tr(O.. rho)/Tr rho) and at beta = 2 tau
    (Tr(O.. rho^T rho)/Tr(rho^T rho), Sec. II.B) by MPO sandwiches."""
    rt = M.transpose(rho)
    return {"tau": M.trace_of_product(*ops, rho) / M.trace(rho),
            "2tau": M.trace_of_product(*ops, rt, rho) / M.inner(rho, rho)}


def binder_ratio(rho: List[np.ndarray]) -> Dict[str, float]:
    """U_4 = <M^2>^2 / <M^4>, M = S^z_tot (Sec. IV.D, Eq. Binder), from the
    exact MPO of M^2 (<M^4> = <M^2 M^2>)."""
    M2 = M.spin_sum_squared(len(rho))
    m2 = expectation(rho, [M2])
    m4 = expectation(rho, [M2, M2])
    return {k: m2[k] ** 2 / m4[k] for k in m2}


def structure_factor(rho: List[np.ndarray], positions, q, center: int) -> Dict[str, float]:
    """Re S(q) = sum_j cos(q . r_0j) <S_0 . S_j> with site 0 = `center`
    (Sec. III.D)."""
    r = np.asarray(positions, dtype=float)
    w = np.cos((r - r[center]) @ np.asarray(q, dtype=float))
    return expectation(rho, [M.correlation(len(rho), center, w)])


def entanglement(rho: List[np.ndarray]) -> np.ndarray:
    """Von Neumann entropy of the normalised superstate |rho> (Eq. purif)
    across every bond: QR sweep left-to-right, then SVD sweep right-to-left;
    the singular values at bond (i-1, i) are the Schmidt coefficients."""
    W = M.left_canonicalize(rho)
    n = len(W)
    out = np.zeros(n - 1)
    for i in range(n - 1, 0, -1):
        Dl, d1, d2, Dr = W[i].shape
        U, S, Vt = np.linalg.svd(W[i].reshape(Dl, d1 * d2 * Dr), full_matrices=False)
        W[i] = Vt.reshape(-1, d1, d2, Dr)
        W[i - 1] = np.einsum("astb,bk->astk", W[i - 1], U * S)
        p = S * S
        p = p / p.sum()
        p = p[p > 0]
        out[i - 1] = float(-np.sum(p * np.log(p)))
    return out


# --------------------------------------------------------------------------
# Driver
# --------------------------------------------------------------------------

def run(n, bonds, jxy, jz, tau0: float, n_doublings: int, D: int, order: int = 1,
        n_sweeps: int = 4, deg_rtol: float = 1e-6, sv_floor: float = 1e-14,
        with_entropy: bool = False, keep_states: bool = False, svd=None, u1: bool = False):
    """Full XTRG run; returns a list of per-doubling records.  u1: the start
    and every doubling keep charge-definite bonds (init_rho_u1, block_svd)."""
    H = M.hamiltonian(n, bonds, jxy, jz)
    rho, lam = (init_rho_u1 if u1 else init_rho)(n, bonds, jxy, jz, tau0, order)
    recs = []
    tau = tau0
    rec = dict(n=0, tau=tau, lam=lam, obs=observables(rho, lam, tau, H, n), bond_dims=M.bond_dims(rho))
    if with_entropy:
        rec["S_E"] = entanglement(rho)
    if keep_states:
        rec["rho"] = rho
    recs.append(rec)
    for k in range(1, n_doublings + 1):
        rho, info = square_compress(rho, D, n_sweeps, deg_rtol, sv_floor, svd=svd, u1=u1)
        lam = 2 * lam + info.dlog_norm
        tau = 2 * tau
        rec = dict(n=k, tau=tau, lam=lam, obs=observables(rho, lam, tau, H, n),
                   bond_dims=M.bond_dims(rho), info=info)
        if with_entropy:
            rec["S_E"] = entanglement(rho)
        if keep_states:
            rec["rho"] = rho
        recs.append(rec)
    return recs
