"""Pins for the small-MPO sandwiches: the Binder ratio (Sec. IV.D, Eq.
Binder) and the static structure factor (Sec. III.D), checked against dense
operators and exact diagonalisation."""
import math

import numpy as np

import workloads as W
from oracle import ed
from oracle import mpo as M
from oracle import xtrg


def _site_op(op, i, n):
    return np.kron(np.kron(np.eye(2 ** i), op), np.eye(2 ** (n - 1 - i)))


def test_spin_sum_squared_is_dense_square():
    n = 5
    Mz = sum(_site_op(ed.SZ, i, n) for i in range(n))
    assert np.abs(M.to_dense(M.spin_sum_squared(n)) - Mz @ Mz).max() < 1e-14
    assert max(M.bond_dims(M.spin_sum_squared(n))) == 3


def test_correlation_mpo_is_dense_sum():
    n = 5
    rng = np.random.default_rng(2)
    for c in (0, 2, 4):
        w = rng.standard_normal(n)
        S = [np.array([[0, .5], [.5, 0]]), None, ed.SZ]
        want = 0.75 * w[c] * np.eye(2 ** n)
        for j in range(n):
            if j == c:
                continue
            for a in (ed.SX, ed.SZ):
                want = want + w[j] * _site_op(a, c, n) @ _site_op(a, j, n)
            # S^y S^y = -(S+ - S-)(S+ - S-)/4, real as a product of two imaginary factors
            Ay = np.array([[0, 1], [-1, 0]]) / 2.0
            want = want - w[j] * _site_op(Ay, c, n) @ _site_op(Ay, j, n)
        assert np.abs(M.to_dense(M.correlation(n, c, w)) - want).max() < 1e-13


def test_binder_ratio_and_structure_factor_match_ed():
    """Untruncated XTRG on the L=8 chain: U_4 and S(q) at both estimators
    against the exact operator p(H)^(2^n) (p the second-order series of the
    start) built from the ED spectrum."""
    lat = W.chain(8)
    n = lat.n_sites
    Hd = ed.xxz_dense(n, lat.bonds, lat.jxy, lat.jz)
    E, V = np.linalg.eigh(Hd)
    tau0 = 2.0 ** -10
    recs = xtrg.run(n, lat.bonds, lat.jxy, lat.jz, tau0, 10, D=10 ** 4, order=2, n_sweeps=1,
                    keep_states=True)
    p = 1 - tau0 * E + (tau0 * E) ** 2 / 2
    Mz = sum(_site_op(ed.SZ, i, n) for i in range(n))
    pos = np.arange(n, dtype=float)[:, None]
    q = np.array([math.pi])
    c = n // 2
    Ssum = 0.0
    for r in recs[-3:]:
        for key, pw in (("tau", 2 ** r["n"]), ("2tau", 2 ** (r["n"] + 1))):
            rho = (V * (p / p[0]) ** pw) @ V.T
            z = np.trace(rho)
            m2 = np.trace(Mz @ Mz @ rho) / z
            m4 = np.trace(Mz @ Mz @ Mz @ Mz @ rho) / z
            u4 = xtrg.binder_ratio(r["rho"])[key]
            assert abs(u4 - m2 * m2 / m4) < 1e-10 * abs(u4)
            w = np.cos((pos - pos[c]) @ q)
            O = 0.75 * w[c] * np.eye(2 ** n)
            for j in range(n):
                if j != c:
                    for a in (ed.SX, ed.SZ):
                        O = O + w[j] * _site_op(a, c, n) @ _site_op(a, j, n)
                    Ay = np.array([[0, 1], [-1, 0]]) / 2.0
                    O = O - w[j] * _site_op(Ay, c, n) @ _site_op(Ay, j, n)
            sq = np.trace(O @ rho) / z
            got = xtrg.structure_factor(r["rho"], pos, q, c)[key]
            assert abs(got - sq) < 1e-10 * max(1.0, abs(sq))
            Ssum = max(Ssum, abs(sq))
    assert Ssum > 0.5                       # antiferromagnetic peak at q = pi
