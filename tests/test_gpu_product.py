"""xtrg_product_compress (C ~ A B, App. D.1 Eq. MPO:prod with two different
factors: the cross products rho_{n,n'} of Sec. II.B and H (H^{k-1} rho) of
Eq. Tay) against the oracle's product_compress and the dense product."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import mpo as M
from oracle import xtrg as OX

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1801_00142_amd import Context
    c = Context(0)
    yield c
    c.close()


def _rho(ctx, lat, tau, order=2, doublings=0, D=1000):
    H = ctx.hamiltonian_xxz(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    r, _ = ctx.init_rho(H, tau, order)
    for _ in range(doublings):
        r, _ = ctx.square_compress(r, D, 2)
    return r, H


def test_product_with_itself_is_the_doubling(ctx):
    lat = W.chain(8)
    r, _ = _rho(ctx, lat, 2.0 ** -4, doublings=2, D=16)
    a, ia = ctx.square_compress(r, 16, 2)
    b, ib = ctx.product_compress(r, r, 16, 2)
    assert ia["dlog_norm"] == ib["dlog_norm"]
    for x, y in zip(a.to_host(), b.to_host()):
        assert np.array_equal(x, y)


def test_untruncated_products_are_exact(ctx):
    """rho(t1) rho(t2), rho(t2) rho(t1) and H rho with a budget above the
    exact bond dimension: the dense product (brute force)."""
    lat = W.random_couplings(W.chain(6), 4)
    a, H = _rho(ctx, lat, 0.3)
    b, _ = _rho(ctx, lat, 0.11)
    for A, B in ((a, b), (b, a), (H, b)):
        want = M.to_dense(A.to_host()) @ M.to_dense(B.to_host())
        C, info = ctx.product_compress(A, B, 10 ** 4, 2)
        got = M.to_dense(C.to_host()) * math.exp(info["dlog_norm"])
        assert np.linalg.norm(got - want) < 1e-13 * np.linalg.norm(want)


@pytest.mark.parametrize("case", [
    dict(lat=W.chain(10), ta=2.0 ** -6, tb=2.0 ** -6 * 2 ** 0.5, da=3, db=3, D=24),
    dict(lat=W.with_couplings(W.chain(9), 1.0, 1.5), ta=2.0 ** -5, tb=2.0 ** -4, da=2, db=1, D=20),
], ids=["chain10_cross", "xxz9_cross"])
def test_truncated_cross_product_matches_oracle(ctx, case):
    """rho_{n,n'}: two runs on different temperature grids (z-shifted, or
    different doubling counts), multiplied and truncated to D: the same
    bonds, ln c within 1e-12, and the normalised operators' overlap with
    the oracle's result 1 within 1e-11 (computed on the host by MPO
    contraction)."""
    lat, D = case["lat"], case["D"]
    ga, H = _rho(ctx, lat, case["ta"], doublings=case["da"], D=D)
    gb, _ = _rho(ctx, lat, case["tb"], doublings=case["db"], D=D)
    A, B = ga.to_host(), gb.to_host()
    C, info = ctx.product_compress(ga, gb, D, 2)
    Co, io = OX.product_compress(A, B, D, 2)
    Cg = C.to_host()
    assert M.bond_dims(Cg) == M.bond_dims(Co)
    assert abs(info["dlog_norm"] - io.dlog_norm) < 1e-12 * max(1.0, abs(io.dlog_norm))
    assert abs(1.0 - M.inner(Cg, Co)) < 1e-11
    # H rho: the first step of the pointwise expansion (Eq. Tay)
    Hh = H.to_host()
    C2, i2 = ctx.product_compress(H, gb, D, 2)
    C2o, i2o = OX.product_compress(Hh, B, D, 2)
    assert M.bond_dims(C2.to_host()) == M.bond_dims(C2o)
    assert abs(i2["dlog_norm"] - i2o.dlog_norm) < 1e-12 * max(1.0, abs(i2o.dlog_norm))
    assert abs(1.0 - M.inner(C2.to_host(), C2o)) < 1e-11


def test_product_rejects_mismatched_factors(ctx):
    from paper_1801_00142_amd import XtrgError
    a, _ = _rho(ctx, W.chain(6), 0.1)
    b, _ = _rho(ctx, W.chain(7), 0.1)
    with pytest.raises(XtrgError):
        ctx.product_compress(a, b, 8, 2)


# ---------------------------------------------------------------- small-MPO sandwiches (Sec. IV.D, III.D)

def test_operator_mpos_match_oracle(ctx):
    """xtrg_spin_sum_mpo (powers 1, 2) and xtrg_correlation_mpo against the
    oracle's MPOs as dense operators (L = 6, every centre)."""
    n = 6
    M1 = ctx.spin_sum_mpo(n, 1)
    M2 = ctx.spin_sum_mpo(n, 2)
    Mz = M.to_dense(M.local_sum(M.SZ, n))
    assert np.abs(M.to_dense(M1.to_host()) - Mz).max() < 1e-15
    assert np.abs(M.to_dense(M2.to_host()) - M.to_dense(M.spin_sum_squared(n))).max() < 1e-14
    assert max(M2.bond_dims) == 3
    w = np.random.default_rng(1).standard_normal(n)
    for c in range(n):
        O = ctx.correlation_mpo(n, c, w)
        assert max(O.bond_dims) == 5
        assert np.abs(M.to_dense(O.to_host()) - M.to_dense(M.correlation(n, c, w))).max() < 1e-13


def test_binder_ratio_and_structure_factor_match_oracle(ctx):
    """U_4 and Re S(q) of truncated runs (chain L=10, D=24; 3x3 cylinder
    D=30) at both estimators against the oracle's run, to 1e-9."""
    from paper_1801_00142_amd import run
    for lat, D, q in ((W.chain(10), 24, [math.pi]), (W.square_cylinder(3, 3), 30, [math.pi, 2 * math.pi / 3])):
        args = (lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -8, 8, D)
        ora = OX.run(*args, order=1, n_sweeps=2, keep_states=True)
        H = ctx.hamiltonian_xxz(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
        rho, lam = ctx.init_rho(H, 2.0 ** -8, 1)
        W_ = lat.n_sites // 3 if len(q) == 2 else 1
        pos = (np.array([[i // W_, i % W_] for i in range(lat.n_sites)], dtype=float) if len(q) == 2
               else np.arange(lat.n_sites, dtype=float)[:, None])
        c = lat.n_sites // 2
        for k in range(9):
            if k > 0:
                new, _ = ctx.square_compress(rho, D, 2)
                rho.close()
                rho = new
            o = ora[k]["rho"]
            assert rho.bond_dims == M.bond_dims(o)
            u_g = ctx.binder_ratio(rho)
            u_o = OX.binder_ratio(o)
            s_g = ctx.structure_factor(rho, pos, q, c)
            s_o = OX.structure_factor(o, pos, q, c)
            for j, key in enumerate(("tau", "2tau")):
                assert abs(u_g[j] - u_o[key]) < 1e-9 * abs(u_o[key]), (k, key)
                assert abs(s_g[j] - s_o[key]) < 1e-9 * max(1.0, abs(s_o[key])), (k, key)
