"""Oracle pins of the series start (Sec. II.C, Eq. RhoTau), of the
pointwise expansion step (Eq. Tay) and of the compressed MPO sum both end
with (App. D.2, Eq. MPO:plus; App. D.1 direct route).

The series start is exact up to its stopping rule when no term is
truncated, so it is pinned against the dense exponential exp(-tau0 H) of
exact diagonalisation, and its cutoff order against the rule evaluated on
the dense powers of H.
"""
import math

import numpy as np
import scipy.linalg as sl

import workloads as W
from oracle import mpo as M
from oracle import xtrg as OX

EPS = 2.220446049250313e-16


def _h(lat):
    return M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)


def _dense_rho(rho, lam):
    return M.to_dense(rho) * math.exp(lam)


def test_identity_mpo():
    for n in (1, 3, 6):
        W_ = OX.identity(n)
        assert M.bond_dims(W_) == [1] * (n + 1)
        assert np.abs(M.to_dense(W_) * 2.0 ** (n / 2) - np.eye(2 ** n)).max() < 1e-15


def test_sum_compress_is_the_weighted_sum():
    """Three random MPOs (different bonds) with weights: the untruncated
    compressed sum is the dense weighted sum, and its bonds are the rank of
    the sum (not the sum of the bonds)."""
    rng = np.random.default_rng(3)
    n = 5

    def rand(D):
        dims = [1] + [D] * (n - 1) + [1]
        return [rng.standard_normal((dims[i], 2, 2, dims[i + 1])) for i in range(n)]

    A, B, C = rand(3), rand(2), rand(4)
    a = [0.7, -1.3, 2e-3]
    S = OX.sum_compress([A, B, C], a, 10 ** 4)
    want = sum(x * M.to_dense(T) for x, T in zip(a, (A, B, C)))
    assert np.linalg.norm(M.to_dense(S) - want) < 1e-13 * np.linalg.norm(want)
    # a term that is a multiple of another adds no bond dimension
    S2 = OX.sum_compress([A, A], [1.0, 2.0], 10 ** 4)
    assert M.bond_dims(S2) == M.bond_dims(OX.sum_compress([A], [3.0], 10 ** 4))


def test_series_start_equals_the_dense_exponential():
    """Untruncated series start against exp(-tau0 H) from the dense H, for
    small and large tau0 (up to 24 orders), a random-coupling chain, a 2x3
    cylinder and an XXZ chain."""
    cases = [W.random_couplings(W.chain(6), 4), W.square_cylinder(2, 3), W.with_couplings(W.chain(7), 1.0, 1.7)]
    for lat in cases:
        H = _h(lat)
        Hd = M.to_dense(H)
        for tau in (0.05, 0.3, 1.0):
            rho, lam, nc = OX.settn_init(H, tau, 10 ** 4)
            ex = sl.expm(-tau * Hd)
            err = np.linalg.norm(_dense_rho(rho, lam) - ex) / np.linalg.norm(ex)
            assert err < 5e-13, (lat.name, tau, nc, err)
            assert abs(np.linalg.norm(M.to_dense(rho)) - 1.0) < 1e-13


def test_cutoff_order_is_the_first_term_below_tol():
    """N_c is the first k with |(-tau0)^k / k!| ||H^k||_F <= tol ||I||_F,
    evaluated here on the dense powers of H; it grows with tau0 and with the
    number of sites (N_c ~ N tau0)."""
    orders = {}
    for lat in (W.chain(6), W.chain(8)):
        H = _h(lat)
        Hd = M.to_dense(H)
        n = lat.n_sites
        for tau in (0.02, 0.2, 0.8):
            _, _, nc = OX.settn_init(H, tau, 10 ** 4)
            P = np.eye(2 ** n)
            want = None
            for k in range(1, 80):
                P = P @ Hd
                if tau ** k / math.factorial(k) * np.linalg.norm(P) <= 1e-15 * 2.0 ** (n / 2):
                    want = k
                    break
            assert nc == want, (lat.name, tau, nc, want)
            orders[(n, tau)] = nc
    assert orders[(6, 0.02)] < orders[(6, 0.2)] < orders[(6, 0.8)]
    assert orders[(8, 0.8)] > orders[(6, 0.8)]


def test_truncated_series_start_improves_with_D():
    """L = 10 chain at tau0 = 0.5 (19 orders): the terms truncated to D;
    the error against exp(-tau0 H) falls as D grows, and the right-canonical
    form holds (sites 1.. isometric)."""
    lat = W.chain(10)
    H = _h(lat)
    ex = sl.expm(-0.5 * M.to_dense(H))
    errs = []
    for D in (8, 16, 32):
        rho, lam, nc = OX.settn_init(H, 0.5, D)
        errs.append(np.linalg.norm(_dense_rho(rho, lam) - ex) / np.linalg.norm(ex))
        assert max(M.bond_dims(rho)) <= D
        for w in rho[1:]:
            m = w.reshape(w.shape[0], -1)
            assert np.abs(m @ m.T - np.eye(m.shape[0])).max() < 1e-12
    assert errs[0] > errs[1] > errs[2], errs


def test_doublings_from_the_series_start_match_ed():
    """XTRG from rho(tau0) at tau0 = 1/8 (Eq. RhoTau with its cutoff rule
    instead of the linear start): five untruncated doublings of the L = 8
    chain give f within 1e-12 of exact diagonalisation at every beta, where
    the linear start at the same tau0 is off by its tau0^2 error."""
    lat = W.chain(8)
    H = _h(lat)
    E = np.linalg.eigvalsh(M.to_dense(H))
    n = lat.n_sites

    def f_ed(beta):
        e0 = E.min()
        return (e0 - math.log(np.sum(np.exp(-beta * (E - e0)))) / beta) / n

    tau0 = 0.125
    rho, lam, _ = OX.settn_init(H, tau0, 10 ** 4)
    lin, llin = OX.init_rho(lat.n_sites, lat.bonds, lat.jxy, lat.jz, tau0, 1)
    tau = tau0
    worst_settn, worst_lin = 0.0, 0.0
    for _ in range(5):
        rho, info = OX.square_compress(rho, 256, 2)
        lam = 2.0 * lam + info.dlog_norm
        lin, il = OX.square_compress(lin, 256, 2)
        llin = 2.0 * llin + il.dlog_norm
        tau *= 2.0
        for beta, key in ((tau, "tau"), (2 * tau, "2tau")):
            ref = f_ed(beta)
            worst_settn = max(worst_settn, abs(OX.observables(rho, lam, tau, H, n)[key]["f"] - ref) / abs(ref))
            worst_lin = max(worst_lin, abs(OX.observables(lin, llin, tau, H, n)[key]["f"] - ref) / abs(ref))
    assert worst_settn < 1e-12, worst_settn
    assert worst_lin > 1e-4, worst_lin


def test_taylor_steps_follow_the_exponential():
    """Pointwise expansion steps (Eq. Tay) on the exponential grid from the
    series start: rho(0.1) -> rho(0.2) -> ... -> rho(1.6), untruncated,
    equal to exp(-tau H) to 1e-12 at every step on a random-coupling chain
    and a 2x3 cylinder; a step of dtau = 0 returns rho itself."""
    for lat in (W.random_couplings(W.chain(6), 4), W.square_cylinder(2, 3)):
        H = _h(lat)
        Hd = M.to_dense(H)
        rho, lam, _ = OX.settn_init(H, 0.1, 10 ** 4)
        tau = 0.1
        for _ in range(4):
            rho, dl, nc = OX.taylor_step(H, rho, tau, 10 ** 4)
            lam += dl
            tau *= 2.0
            ex = sl.expm(-tau * Hd)
            assert np.linalg.norm(_dense_rho(rho, lam) - ex) < 1e-12 * np.linalg.norm(ex), (lat.name, tau)
        same, dl, nc = OX.taylor_step(H, rho, 0.0, 10 ** 4)
        assert nc == 1 and abs(dl) < 1e-14
        assert np.linalg.norm(M.to_dense(same) - M.to_dense(rho)) < 1e-13
