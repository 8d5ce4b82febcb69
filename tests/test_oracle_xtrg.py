"""Pins for the oracle's initial state, doubling/compression and observables.

Each check compares against something other than the oracle itself:
exact diagonalisation (dense H), brute-force dense products, closed forms
and invariants.  A mistake in an index, a sign or a transposed operand in
the contraction sequence fails the brute-force checks below (the
untruncated doubling must reproduce the dense product exactly).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf
from oracle import ed
from oracle import mpo as M
from oracle import xtrg


def _dense_H(lat):
    return ed.xxz_dense(lat.n_sites, lat.bonds, lat.jxy, lat.jz)


# ---------------------------------------------------------------- init (App. C.2, Eq. RhoTau)

@pytest.mark.parametrize("order", [1, 2, 3])
def test_series_init_is_exact(order):
    lat = W.random_couplings(W.chain(6), 3)
    Hd = _dense_H(lat)
    tau = 0.07
    want = sum((-tau) ** k / math.factorial(k) * np.linalg.matrix_power(Hd, k) for k in range(order + 1))
    rho = xtrg.series_rho(lat.n_sites, lat.bonds, lat.jxy, lat.jz, tau, order)
    assert np.abs(M.to_dense(rho) - want).max() < 1e-13
    rh, lam = xtrg.init_rho(lat.n_sites, lat.bonds, lat.jxy, lat.jz, tau, order)
    assert np.abs(M.to_dense(rh) * math.exp(lam) - want).max() < 1e-12
    assert abs(M.norm(rh) - 1.0) < 1e-13
    for w in rh[1:]:                                   # right-canonical
        m = w.reshape(w.shape[0], -1)
        assert np.abs(m @ m.T - np.eye(w.shape[0])).max() < 1e-13


def test_linear_init_closed_forms():
    lat = W.square_cylinder(3, 3)
    tau = 2.0 ** -10
    rh, lam = xtrg.init_rho(lat.n_sites, lat.bonds, lat.jxy, lat.jz, tau, 1)
    n = lat.n_sites
    tr = M.trace(rh) * math.exp(lam)
    assert abs(tr / cf.linear_init_trace(n) - 1) < 1e-13
    assert abs(math.exp(2 * lam) / cf.linear_init_norm2(n, tau, lat.jxy, lat.jz) - 1) < 1e-13
    # order 1 is exact at the bond dimension of H (App. C.2)
    assert max(M.bond_dims(rh)) <= max(M.automaton_bond_dims(n, lat.bonds))


# ---------------------------------------------------------------- truncation rule

def test_keep_count_rule():
    S = np.array([1.0, 0.5, 0.5, 0.5, 0.1, 0.05, 0.05, 1e-20])
    assert xtrg.keep_count(S, 8, 1e-6, 1e-14) == 7             # floor drops 1e-20
    # D = 3 would split the triplet (0.5, 0.5, 0.5): back off to 1? the
    # search runs over [ceil(D/2), D] = [2, 3]; no gap there -> keep D
    assert xtrg.keep_count(S, 3, 1e-6, 1e-14) == 3
    assert xtrg.keep_count(S, 4, 1e-6, 1e-14) == 4             # gap after the triplet
    assert xtrg.keep_count(S, 6, 1e-6, 1e-14) == 5             # does not split the 0.05 pair
    assert xtrg.keep_count(np.array([0.0, 0.0]), 4, 1e-6, 1e-14) == 1


# ---------------------------------------------------------------- doubling (Eqs. rhoinit, rho:scale2)

def test_untruncated_doubling_equals_dense_square():
    """Brute force: with D above the exact bond dimension the variational
    compression must return rho*rho exactly (App. D.1: exact if D_c = D_a D_b)."""
    lat = W.random_couplings(W.chain(5), 4)
    rh, lam = xtrg.init_rho(lat.n_sites, lat.bonds, lat.jxy, lat.jz, 0.2, 2)
    for _ in range(3):
        R = M.to_dense(rh)
        C, info = xtrg.square_compress(rh, 1000, n_sweeps=2)
        got = M.to_dense(C) * math.exp(info.dlog_norm)
        assert np.linalg.norm(got - R @ R) < 1e-13 * np.linalg.norm(R @ R)
        assert abs(M.norm(C) - 1) < 1e-13
        for w in C[1:]:
            m = w.reshape(w.shape[0], -1)
            assert np.abs(m @ m.T - np.eye(w.shape[0])).max() < 1e-12
        rh = C


def test_exact_doubling_matches_spectrum():
    """T2: untruncated, ln Tr rho_n = ln sum_E p(E)^(2^n) with p the series
    polynomial, and ln ||rho_n||^2 = ln sum_E p(E)^(2^(n+1))."""
    lat = W.chain(6)
    E = ed.spectrum(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    tau0 = 2.0 ** -6
    recs = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, tau0, 7, D=1000, order=2, n_sweeps=1)
    p = 1 - tau0 * E + (tau0 * E) ** 2 / 2
    for r in recs:
        n = r["n"]
        lt = np.log(np.sum(p ** (2 ** n)))
        lf = np.log(np.sum(p ** (2 ** (n + 1))))
        assert abs(r["obs"]["tau"]["lnZ"] - lt) < 1e-11 * max(1, abs(lt))
        assert abs(r["obs"]["2tau"]["lnZ"] - lf) < 1e-11 * max(1, abs(lf))


def _cost(A, B, C):
    AB = M.product(A, B)
    return M.inner(AB, AB) - 2 * M.inner(AB, C) + M.inner(C, C)


def test_variational_not_worse_than_direct_svd():
    """T7 (App. D.1): the variational optimum is at least as good as the
    direct SVD compression of the fused product at the same D."""
    lat = W.random_couplings(W.chain(6), 7)
    rh, lam = xtrg.init_rho(lat.n_sites, lat.bonds, lat.jxy, lat.jz, 0.3, 2)
    rh, _ = xtrg.square_compress(rh, 1000, 2)
    for D in (4, 8, 12):
        # deg_rtol = 0: cut at exactly D, as the direct SVD does (the
        # multiplet-safe back-off may keep fewer states)
        C, info = xtrg.square_compress(rh, D, n_sweeps=4, deg_rtol=0.0)
        Cv = M.scale(C, math.exp(info.dlog_norm))
        Cs = M.svd_compress(M.product(rh, rh), D)
        ev, es = _cost(rh, rh, Cv), _cost(rh, rh, Cs)
        assert max(M.bond_dims(C)) <= D
        assert ev <= es * (1 + 1e-9) + 1e-15


def test_sweeps_monotone():
    """More sweeps never increase the cost (alternating least squares)."""
    lat = W.random_couplings(W.chain(7), 8)
    rh, _ = xtrg.init_rho(lat.n_sites, lat.bonds, lat.jxy, lat.jz, 0.5, 2)
    rh, _ = xtrg.square_compress(rh, 1000, 2)
    costs = []
    for ns in (1, 2, 3):
        C, info = xtrg.square_compress(rh, 6, n_sweeps=ns)
        costs.append(_cost(rh, rh, M.scale(C, math.exp(info.dlog_norm))))
    assert costs[1] <= costs[0] * (1 + 1e-10) and costs[2] <= costs[1] * (1 + 1e-10)


# ---------------------------------------------------------------- observables (Eq. ThermalQuan)

def test_observables_match_ed_untruncated():
    lat = W.random_couplings(W.chain(6), 11)
    Hd = _dense_H(lat)
    E, V = np.linalg.eigh(Hd)
    tau0 = 2.0 ** -8
    recs = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, tau0, 8, D=1000, order=2, n_sweeps=1)
    p = 1 - tau0 * E + (tau0 * E) ** 2 / 2
    n = lat.n_sites
    for r in recs:
        for key, pw in (("tau", 2 ** r["n"]), ("2tau", 2 ** (r["n"] + 1))):
            w = p ** pw
            Z = w.sum()
            e1 = (w * E).sum() / Z
            e2 = (w * E * E).sum() / Z
            b = r["obs"][key]["beta"]
            o = r["obs"][key]
            assert abs(o["u"] - e1 / n) < 1e-11
            assert abs(o["c"] - b * b * (e2 - e1 * e1) / n) < 1e-9 * max(1, b * b)


def test_physical_ed_error_falls_with_D():
    """T3: truncated runs approach the exact result as D grows.  The target
    is rho(tau0)^(2^(n+1)) evaluated on the ED spectrum (p(E)^(2^(n+1)), p the
    series polynomial), which isolates the truncation error; that target is
    itself within the series error of exp(-beta H)."""
    lat = W.chain(8)
    E = ed.spectrum(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    tau0 = 2.0 ** -10
    p = 1 - tau0 * E + (tau0 * E) ** 2 / 2
    errs = []
    for D in (8, 16, 32, 64):
        recs = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, tau0, 14, D=D, order=2, n_sweeps=2)
        o = recs[-1]["obs"]["2tau"]
        lz_series = float(np.log(np.sum(p ** (2 ** 15))))
        errs.append(abs(o["lnZ"] - lz_series) / (lat.n_sites * o["beta"]))
        f_ed = ed.thermo(E, o["beta"], lat.n_sites)[0]
        assert abs(-lz_series / (lat.n_sites * o["beta"]) - f_ed) < 2e-6   # series error
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-7


def test_xy_chain_closed_form():
    """T4: App. F closed form, L = 12, truncated XTRG error falls with D."""
    L = 12
    lat = W.with_couplings(W.chain(L), 1.0, 0.0)
    errs = []
    for D in (8, 16, 32):
        recs = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -8, 11, D=D, order=2, n_sweeps=2)
        o = recs[-1]["obs"]["2tau"]
        errs.append(abs(o["lnZ"] - cf.xy_chain_lnZ(L, 1.0, o["beta"])))
    assert errs[0] > errs[1] > errs[2]


def test_high_temperature_series():
    """T5: ln Z = N ln 2 + beta^2 Tr H^2/(2 Z0) - beta^3 Tr H^3/(6 Z0) + O(beta^4)."""
    lat = W.chain(16)
    tau0 = 2.0 ** -12
    recs = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, tau0, 4, D=64, order=2, n_sweeps=1)
    h3 = abs(cf.h3_per_state(lat.jxy, lat.jz))
    for r in recs:
        b = r["obs"]["2tau"]["beta"]
        ser = cf.high_t_lnZ(lat.n_sites, b, lat.jxy, lat.jz)
        # remaining O(beta^4) term (loose bound N_b beta^4) plus the series
        # start's own error: rho0 misses tau0^3 H^3/6, which after the
        # doublings shifts ln Z by ~ beta tau0^2 Tr(H^3)/(6 Z0)
        tol = lat.n_bonds * b ** 4 + 2 * b * tau0 ** 2 * h3 / 6 + 1e-13 * lat.n_sites
        assert abs(r["obs"]["2tau"]["lnZ"] - ser) < tol
    # and the deviation really is of that size (the beta^2 and beta^3 terms are right)
    b = recs[0]["obs"]["2tau"]["beta"]
    dev = recs[0]["obs"]["2tau"]["lnZ"] - cf.high_t_lnZ(lat.n_sites, b, lat.jxy, lat.jz)
    assert abs(dev) < 0.3 * 0.5 * b * b * cf.h2_per_state(lat.jxy, lat.jz) * b


def _local_sum_mpo(op, n):
    W_ = []
    for i in range(n):
        T = np.zeros((2, 2, 2, 2))
        T[0, :, :, 0] = np.eye(2)
        T[1, :, :, 1] = np.eye(2)
        T[0, :, :, 1] = op
        W_.append(T)
    return M.cap(W_, np.array([1.0, 0.0]), np.array([0.0, 1.0]))


def test_local_sum_mpo_is_the_kronecker_sum():
    """M.local_sum(op, n) == sum_i I x .. x op_i x .. x I (brute force)."""
    n = 5
    for op in (ed.SZ, ed.SX, np.array([[0.3, -1.2], [0.7, 2.0]])):
        want = sum(np.kron(np.kron(np.eye(2 ** i), op), np.eye(2 ** (n - 1 - i))) for i in range(n))
        assert np.abs(M.to_dense(M.local_sum(op, n)) - want).max() < 1e-14


def test_invariant_fields_detect_what_they_measure():
    """The invariant fields of observables() are zero where the symmetry
    holds and measure its breaking where it does not: an XXZ chain
    (jz != jxy) keeps <S^z_tot> = 0 and rho = rho^T but not SU(2); a
    non-symmetric operator gives the closed-form herm_resid."""
    lat = W.with_couplings(W.chain(6), 1.0, 2.0)
    Hd = _dense_H(lat)
    rh, lam = xtrg.init_rho(lat.n_sites, lat.bonds, lat.jxy, lat.jz, 0.5, 2)
    H = M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    o = xtrg.observables(rh, lam, 0.5, H, lat.n_sites)
    R = M.to_dense(rh)
    n = lat.n_sites
    Sz = sum(np.kron(np.kron(np.eye(2 ** i), ed.SZ), np.eye(2 ** (n - 1 - i))) for i in range(n))
    Sx = sum(np.kron(np.kron(np.eye(2 ** i), ed.SX), np.eye(2 ** (n - 1 - i))) for i in range(n))
    for key, Rho in (("tau", R), ("2tau", R.T @ R)):
        tr = np.trace(Rho)
        z2, x2 = np.trace(Sz @ Sz @ Rho) / tr, np.trace(Sx @ Sx @ Rho) / tr
        assert abs(o[key]["sz_tot"]) < 1e-13
        assert abs(o[key]["su2_resid"] - (x2 - z2) / max(z2, 1.0)) < 1e-12
        assert abs(o[key]["su2_resid"]) > 1e-3            # XXZ: no SU(2)
        assert o[key]["herm_resid"] < 1e-14
    # a non-symmetric operator: rho' = rho (I + a Sz S+) has
    # ||rho' - rho'^T||^2 / ||rho'||^2 computed densely
    X = R @ (np.eye(2 ** n) + 0.3 * Sz @ np.kron(np.array([[0.0, 1.0], [0.0, 0.0]]), np.eye(2 ** (n - 1))))
    A = M.svd_compress(_dense_to_mpo(X, n), 10 ** 6)
    nrm = M.inner(A, A)
    o2 = xtrg.observables(M.scale(A, 1 / math.sqrt(nrm)), 0.0, 0.5, H, n)
    Xd = M.to_dense(A)
    want = np.linalg.norm(Xd - Xd.T) ** 2 / np.linalg.norm(Xd) ** 2
    assert abs(o2["tau"]["herm_resid"] - want) < 1e-12 and want > 1e-3


def _dense_to_mpo(X, n):
    """Exact MPO of a dense 2^n x 2^n operator (successive reshapes and SVDs)."""
    T = X.reshape([2] * (2 * n))
    T = T.transpose([x for i in range(n) for x in (i, n + i)])   # (s0 s0' s1 s1' ...)
    W = []
    left = 1
    rest = T.reshape(1, -1)
    for i in range(n - 1):
        rest = rest.reshape(left * 4, -1)
        U, S, Vt = np.linalg.svd(rest, full_matrices=False)
        k = int(np.sum(S > 1e-14 * S[0]))
        W.append(U[:, :k].reshape(left, 2, 2, k))
        rest = S[:k, None] * Vt[:k]
        left = k
    W.append(rest.reshape(left, 2, 2, 1))
    return W


def test_invariants_truncated():
    """T6: Tr rho > 0, Hermiticity, SU(2): <(Sx_tot)^2> = <(Sz_tot)^2>
    when no multiplet is split, <Sz_tot> = 0."""
    lat = W.chain(8)
    recs = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -8, 11, D=24, order=2,
                    n_sweeps=2, keep_states=True)
    sx = _local_sum_mpo(ed.SX, lat.n_sites)
    sz = _local_sum_mpo(ed.SZ, lat.n_sites)
    for r in recs:
        rh = r["rho"]
        assert M.trace(rh) > 0
        rt = M.transpose(rh)
        herm = M.inner(rh, rh) + M.inner(rt, rt) - 2 * M.inner(rh, rt)
        assert herm < 1e-10
        tr = M.trace(rh)
        x2 = M.trace_of_product(sx, sx, rh) / tr
        z2 = M.trace_of_product(sz, sz, rh) / tr
        assert abs(x2 - z2) < 1e-8 * max(1.0, z2)
        assert abs(M.trace_of_product(sz, rh) / tr) < 1e-12
        o = r["obs"]
        for key in ("tau", "2tau"):
            assert o[key]["herm_resid"] < 1e-10
            assert abs(o[key]["sz_tot"]) < 1e-12
            assert abs(o[key]["su2_resid"]) < 1e-8


def test_entanglement_brute_force_and_high_t():
    """Eq. (purif): S_E equals the entropy of the Schmidt values of the
    vectorised operator (brute force via dense reshapes), and it grows like
    beta^2 at high temperature (gamma -> 2)."""
    lat = W.chain(6)
    recs = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -10, 10, D=1000, order=2,
                    n_sweeps=1, keep_states=True, with_entropy=True)
    n = lat.n_sites
    for r in recs[::3]:
        Rd = M.to_dense(r["rho"])
        psi = Rd.reshape([2] * (2 * n))
        # reorder to (s0 s0' s1 s1' ...)
        perm = [x for i in range(n) for x in (i, n + i)]
        psi = psi.transpose(perm)
        for cut in range(1, n):
            s = np.linalg.svd(psi.reshape(4 ** cut, -1), compute_uv=False)
            p = s * s / np.sum(s * s)
            p = p[p > 0]
            assert abs(-np.sum(p * np.log(p)) - r["S_E"][cut - 1]) < 1e-10
    se = [r["S_E"][n // 2 - 1] for r in recs]
    assert all(b >= a for a, b in zip(se, se[1:]))           # grows with beta
    # S ~ beta^2 up to a log (S ~ -p ln p with p ~ beta^2): the log-slope
    # gamma between beta and 2 beta is below 2 and tends to 2 as beta -> 0
    gam = []
    for tau0 in (2.0 ** -8, 2.0 ** -14, 2.0 ** -20):
        rr = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, tau0, 1, D=1000, order=2,
                      n_sweeps=1, with_entropy=True)
        gam.append(math.log(rr[1]["S_E"][n // 2 - 1] / rr[0]["S_E"][n // 2 - 1]) / math.log(2.0))
    assert 1.7 < gam[0] < gam[1] < gam[2] < 2.0
    assert gam[2] > 1.9
