"""Pins for the oracle's compression of a product of two different MPOs,
C ~ A*B (App. D.1, Eq. MPO:prod): the cross products rho_{n,n'} of the
interleaved temperature grids (Sec. II.B) and the steps H (H^{k-1} rho) of
the pointwise expansion (Sec. II.C, Eq. Tay).  Checked against the dense
product (brute force), the direct SVD compression of the exact product
(App. D.1), and the commutation of two functions of the same H."""
import math

import numpy as np

import workloads as W
from oracle import mpo as M
from oracle import xtrg


def _pair(lat, t1, t2, order=2):
    a, la = xtrg.init_rho(lat.n_sites, lat.bonds, lat.jxy, lat.jz, t1, order)
    b, lb = xtrg.init_rho(lat.n_sites, lat.bonds, lat.jxy, lat.jz, t2, order)
    return a, b


def test_untruncated_cross_product_is_the_dense_product():
    """rho(t1) rho(t2) with t1 != t2, and H rho, compressed with a budget
    above the exact bond dimension: the dense operator A B exactly."""
    lat = W.random_couplings(W.chain(5), 6)
    a, b = _pair(lat, 0.3, 0.11)
    H = M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    for A, B in ((a, b), (b, a), (H, b)):
        want = M.to_dense(A) @ M.to_dense(B)
        C, info = xtrg.product_compress(A, B, 10 ** 4, n_sweeps=2)
        got = M.to_dense(C) * math.exp(info.dlog_norm)
        assert np.linalg.norm(got - want) < 1e-13 * np.linalg.norm(want)
        assert abs(M.norm(C) - 1) < 1e-13
        for w in C[1:]:                                    # right-canonical
            m = w.reshape(w.shape[0], -1)
            assert np.abs(m @ m.T - np.eye(w.shape[0])).max() < 1e-12


def test_square_is_the_product_with_itself():
    lat = W.chain(6)
    a, _ = _pair(lat, 0.2, 0.2)
    C1, i1 = xtrg.square_compress(a, 8, 2)
    C2, i2 = xtrg.product_compress(a, a, 8, 2)
    assert i1.dlog_norm == i2.dlog_norm
    for x, y in zip(C1, C2):
        assert np.array_equal(x, y)


def test_truncated_cross_product_not_worse_than_direct_svd():
    """At a budget below the exact bond dimension the variational optimum
    is at least as close to A B as the direct SVD compression of the exact
    product MPO (App. D.1)."""
    lat = W.random_couplings(W.chain(7), 9)
    a, b = _pair(lat, 0.4, 0.25)
    a, _ = xtrg.square_compress(a, 1000, 2)
    AB = M.product(a, b)
    for D in (4, 8, 12):
        C, info = xtrg.product_compress(a, b, D, n_sweeps=4, deg_rtol=0.0)
        Cv = M.scale(C, math.exp(info.dlog_norm))
        Cs = M.svd_compress(AB, D)
        ev = M.inner(AB, AB) - 2 * M.inner(AB, Cv) + M.inner(Cv, Cv)
        es = M.inner(AB, AB) - 2 * M.inner(AB, Cs) + M.inner(Cs, Cs)
        assert max(M.bond_dims(C)) <= D
        assert ev <= es * (1 + 1e-9) + 1e-15


def test_functions_of_one_hamiltonian_commute():
    """rho(t1) and rho(t2) are polynomials in the same H: A B = B A, and
    the compressed products in either order agree (untruncated: exactly;
    truncated at D = 12: to the truncation error)."""
    lat = W.chain(6)
    a, b = _pair(lat, 0.5, 0.17)
    C1, i1 = xtrg.product_compress(a, b, 10 ** 4, 2)
    C2, i2 = xtrg.product_compress(b, a, 10 ** 4, 2)
    d1 = M.to_dense(C1) * math.exp(i1.dlog_norm)
    d2 = M.to_dense(C2) * math.exp(i2.dlog_norm)
    assert np.linalg.norm(d1 - d2) < 1e-13 * np.linalg.norm(d1)
    C1, i1 = xtrg.product_compress(a, b, 12, 2)
    C2, i2 = xtrg.product_compress(b, a, 12, 2)
    d1 = M.to_dense(C1) * math.exp(i1.dlog_norm)
    d2 = M.to_dense(C2) * math.exp(i2.dlog_norm)
    assert np.linalg.norm(d1 - d2) < 1e-5 * np.linalg.norm(d1)
