"""Pins for the oracle's truncation rule: the kept count of Sec. II.D (a
fixed number of states, never a weight threshold), its multiplet-safe
back-off, and the numerical-zero level of the two-site tensor C_E.

The rule decides an integer from floating-point singular values, so the
tests fix it by behaviour: values placed just above and just below every
threshold of the rule, matrices of known exact rank formed in FP64 (their
remaining singular values are pure rounding), and two independent LAPACK
factorisations that must make the same decisions over a whole run.  A wrong
constant, a wrong norm or a dropped term in either threshold fails one of
them.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import xtrg

EPS = 2.220446049250313e-16


# ------------------------------------------------------------ gap test with the noise term

def test_gap_must_exceed_relative_tolerance_plus_noise():
    """A gap between sigma_k and sigma_{k+1} separates two multiplets only if
    it exceeds deg_rtol * sigma_k + eta (eta: the absolute rounding noise of
    the values).  Gaps just below and just above that sum, and the same
    gaps with eta = 0."""
    deg, eta = 1e-6, 1e-5
    base = [1.0, 0.7, 0.4, 0.3]
    thr = deg * 0.3 + eta                               # 1.03e-5 at the cut k = 4
    for gap, want_eta, want_zero in ((0.5 * thr, 3, 4), (0.97 * thr, 3, 4), (1.03 * thr, 4, 4),
                                     (2.0 * thr, 4, 4), (0.5 * deg * 0.3, 3, 3)):
        S = np.array(base + [0.3 - gap, 0.1])
        # D = 4: the search runs over k = 4, 3, 2; the gap after the 0.4 is large
        assert xtrg.keep_count(S, 4, deg, 0.0, eta) == want_eta, gap
        assert xtrg.keep_count(S, 4, deg, 0.0, 0.0) == want_zero, gap


def test_gap_search_keeps_d_when_no_gap_in_range():
    """No gap in [ceil(D/2), D] larger than the tolerance: keep D (a
    multiplet wider than D/2 is split rather than the bond halved)."""
    S = np.array([1.0] + [0.5 - 1e-9 * q for q in range(8)] + [0.1])
    assert xtrg.keep_count(S, 6, 1e-6, 0.0, 0.0) == 6
    assert xtrg.keep_count(S, 6, 0.0, 0.0, 0.0) == 6       # deg_rtol = 0: exactly D
    # a gap at k = 1 lies outside the search range [3, 6]
    assert xtrg.keep_count(S, 6, 1e-6, 0.0, 0.0) != 1


def test_floor_counts_values_strictly_above_both_thresholds():
    """Values above max(sv_floor * sigma_1, eta) count; values at or below
    either threshold are zeros.  Straddle each threshold by 10%."""
    eta = 1e-9
    S = np.array([1.0, 0.3, 1.1 * eta, 0.9 * eta, 0.0])
    assert xtrg.keep_count(S, 10, 1e-6, 0.0, eta) == 3
    assert xtrg.keep_count(S, 10, 1e-6, 0.0, 0.0) == 4
    assert xtrg.keep_count(S, 10, 1e-6, 1.0e-9, 0.0) == 3   # sv_floor * sigma_1 = 1e-9
    assert xtrg.keep_count(S, 10, 1e-6, 1.2e-9, 0.0) == 2
    assert xtrg.keep_count(S, 10, 1e-6, 1e-14, 2e-9) == 2   # the larger threshold decides


# ------------------------------------------------------------ the numerical-zero level

def _with_spectrum(m, n, S, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, len(S))))
    V, _ = np.linalg.qr(rng.standard_normal((n, len(S))))
    return (U * S) @ V.T


@pytest.mark.parametrize("m,n", [(400, 100), (100, 400)])
def test_noise_floor_formula_by_behaviour(m, n):
    """noise_floor(M) = 40 eps sqrt(max(m, n)) ||M||_F.  Two singular values
    placed at 1.1 and 0.9 times that level: exactly one of them counts.  A
    constant 10x larger or smaller, sqrt(min(m, n)) in place of
    sqrt(max(m, n)), or the spectral norm in place of the Frobenius norm
    (here ||M||_F = 1.6 ||M||_2) each move at least one of the two across."""
    big = np.logspace(0, -6, 60)
    f = 40.0 * EPS * math.sqrt(max(m, n)) * float(np.linalg.norm(big))
    S = np.concatenate([big, [1.1 * f, 0.9 * f]])
    A = _with_spectrum(m, n, S, seed=m + 7 * n)
    nf = xtrg.noise_floor(A)
    assert abs(nf / f - 1) < 1e-6
    s = np.linalg.svd(A, compute_uv=False)
    assert xtrg.keep_count(s, 100, 1e-6, 0.0, nf) == 61
    fro, spec = float(np.linalg.norm(A)), float(s[0])
    assert fro > 1.5 * spec
    for wrong in (10 * nf, nf / 10, nf * math.sqrt(min(m, n) / max(m, n)), nf * spec / fro):
        assert xtrg.keep_count(s, 100, 1e-6, 0.0, wrong) != 61


@pytest.mark.parametrize("m,n,r", [(256, 256, 40), (1024, 256, 100), (128, 512, 128), (300, 300, 299)])
def test_exact_rank_matrices_keep_their_rank(m, n, r):
    """M = A B with A m x r and B r x n formed in FP64 has exact rank r; its
    other singular values are rounding noise.  The rule keeps exactly r
    (sv_floor = 0, so only the noise level decides)."""
    rng = np.random.default_rng(r)
    M = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    s = np.linalg.svd(M, compute_uv=False)
    assert xtrg.keep_count(s, 2000, 1e-6, 0.0, xtrg.noise_floor(M)) == r


def test_two_site_shaped_product_keeps_its_rank():
    """The shape of C_E = Lb Rb (App. D.1, Eq. LSEProd): a long inner index
    K = 4096 and a left block of exact rank r.  The product is formed by a
    K-term FP64 sum, and its rank-r content is kept, its noise dropped, with
    the relative scales of a saturated chain's two-site tensor (singular
    values over 12 decades)."""
    rng = np.random.default_rng(5)
    m, n, K, r = 128, 128, 4096, 50
    X = _with_spectrum(m, r, np.logspace(0, -12, r), seed=1)
    Lb = X @ rng.standard_normal((r, K)) / math.sqrt(K)
    th = Lb @ rng.standard_normal((K, n))
    s = np.linalg.svd(th, compute_uv=False)
    assert xtrg.keep_count(s, 2000, 1e-6, 0.0, xtrg.noise_floor(th)) == r


# ------------------------------------------------------------ reproducibility over a whole run

def _gesvd(a):
    import scipy.linalg
    return scipy.linalg.svd(a, full_matrices=False, lapack_driver="gesvd")


def _golden(name):
    import json
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", f"oracle_{name}.json")
    with open(p) as f:
        return json.load(f)


def test_second_lapack_svd_reproduces_the_stored_run():
    """The stored L=10 chain run (gesdd, D = 64, 14 doublings, 4 sweeps) is
    reproduced by the oracle with LAPACK's other SVD driver (gesvd: QR
    iteration instead of divide and conquer): every cut the same, f and u
    at every beta within 1e-12.  With the noise term of the rule the cut
    decisions do not depend on which correct FP64 SVD made the values."""
    g = _golden("chain10_D64")
    wl = W.workload("chain10", g["D"])
    lat = wl.lattice
    recs = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, wl.tau0, wl.n_doublings, wl.D,
                    order=wl.init_order, n_sweeps=g["n_sweeps"], svd=_gesvd)
    for r, s in zip(recs, g["records"]):
        assert r["bond_dims"] == s["bond_dims"], r["n"]
        for key, so in (("tau", s["tau_obs"]), ("2tau", s["two_tau_obs"])):
            o = r["obs"][key]
            assert abs(o["f"] - so["f"]) <= 1e-12 * abs(so["f"]), (r["n"], key)
            assert abs(o["u"] - so["u"]) <= 1e-12 * max(abs(so["u"]), 1e-3), (r["n"], key)


def _gram_svd(a):
    """Factorisation through the Gram matrix of the shorter side: eigenpairs
    of a a^T (or a^T a), sigma = sqrt(eigenvalue), the other side's vectors
    from a.  Exact in exact arithmetic; in FP64 it resolves sigma only down
    to about sqrt(eps) sigma_1."""
    m, n = a.shape
    if m <= n:
        w, U = np.linalg.eigh(a @ a.T)
        o = np.argsort(w)[::-1]
        w, U = w[o], U[:, o]
        S = np.sqrt(np.maximum(w, 0.0))
        Vt = U.T @ a
        nz = S > 0
        Vt[nz] /= S[nz, None]
        return U, S, Vt
    U, S, Vt = _gram_svd(a.T)
    return Vt.T, S, U.T


def test_gram_route_misses_the_fp64_target():
    """Why the truncation is an SVD of C_E and not an eigensolve of its Gram
    matrix: on the stored L=10 chain run the Gram route moves f far beyond
    the 1e-9 FP64 parity target.  The series start leaves components with
    sigma/sigma_1 ~ 1e-8 .. 1e-12 (tau0^2 .. tau0^4 terms) that squaring
    pushes below the rounding level of a a^T."""
    g = _golden("chain10_D64")
    wl = W.workload("chain10", g["D"])
    lat = wl.lattice
    recs = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, wl.tau0, wl.n_doublings, wl.D,
                    order=wl.init_order, n_sweeps=g["n_sweeps"], svd=_gram_svd)
    err = max(abs(r["obs"]["2tau"]["f"] - s["two_tau_obs"]["f"]) / abs(s["two_tau_obs"]["f"])
              for r, s in zip(recs, g["records"]))
    assert err > 1e-6
