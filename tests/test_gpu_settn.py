"""xtrg_settn_init (the series start of Sec. II.C, Eq. RhoTau, with the
automatic cutoff order) and xtrg_taylor_step (the pointwise expansion of
Eq. Tay) against the dense exponential and the oracle, through the C ABI."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

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


def _h(ctx, lat):
    return ctx.hamiltonian_xxz(lat.n_sites, lat.bonds, lat.jxy, lat.jz)


@pytest.mark.parametrize("lat", [W.random_couplings(W.chain(6), 4), W.square_cylinder(2, 3),
                                 W.with_couplings(W.chain(7), 1.0, 1.7)], ids=["chain6_rand", "cyl2x3", "xxz7"])
def test_untruncated_series_start_is_the_exponential(ctx, lat):
    """Budget above every bond: rho(tau0) equals exp(-tau0 H) of the dense
    H for tau0 = 0.05, 0.3, 1.0 (9 to 24 orders), with the cutoff order of
    the oracle.  Bound 2e-12 relative: every compression may drop values
    below its noise floor, 40 eps sqrt(4D) ||M|| ~ 1.4e-13 of each term at
    the bonds here, and up to ~20 terms and the sum are compressed (the
    oracle's LAPACK run lands at 1e-13, the GPU's Jacobi at 8e-13)."""
    H = _h(ctx, lat)
    Hd = M.to_dense(M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz))
    Ho = M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    for tau in (0.05, 0.3, 1.0):
        rho, lam, nc = ctx.settn_init(H, tau, 10 ** 4)
        _, _, nco = OX.settn_init(Ho, tau, 10 ** 4)
        assert nc == nco, (tau, nc, nco)
        ex = sl.expm(-tau * Hd)
        got = M.to_dense(rho.to_host()) * math.exp(lam)
        assert np.linalg.norm(got - ex) < 2e-12 * np.linalg.norm(ex), tau


@pytest.mark.parametrize("D", [16, 32])
def test_truncated_series_start_matches_oracle(ctx, D):
    """L = 10 chain at tau0 = 0.5 with every power truncated to D: the same
    cutoff order and bond dimensions as the oracle, ln of the norm within
    1e-12, and the normalised operators' overlap 1 within 1e-10."""
    lat = W.chain(10)
    H = _h(ctx, lat)
    Ho = M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    rho, lam, nc = ctx.settn_init(H, 0.5, D)
    ro, lo, nco = OX.settn_init(Ho, 0.5, D)
    g = rho.to_host()
    assert nc == nco
    assert M.bond_dims(g) == M.bond_dims(ro)
    assert abs(lam - lo) < 1e-12 * abs(lo)
    assert abs(1.0 - M.inner(g, ro)) < 1e-10


def test_doublings_from_the_series_start_match_ed(ctx):
    """XTRG through the library from the series start at tau0 = 1/8: five
    untruncated doublings of the L = 8 chain, f within 5e-12 of exact
    diagonalisation at both estimators of every doubling.  The bound: the
    ~10 terms are added one at a time and every partial sum is compressed,
    each time to the FP64 noise floor (~1e-13 of the sum), so rho(tau0)
    carries ~1e-12; an error delta in rho(tau0) reaches f = -ln Z/(N beta)
    as about delta / (N tau0) at every doubling (Z ~ rho(tau0)^(2^n)),
    i.e. ~1e-12 here (measured 1.6e-12)."""
    lat = W.chain(8)
    H = _h(ctx, lat)
    E = np.linalg.eigvalsh(M.to_dense(M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)))
    n = lat.n_sites

    def f_ed(beta):
        e0 = E.min()
        return (e0 - math.log(np.sum(np.exp(-beta * (E - e0)))) / beta) / n

    rho, lam, _ = ctx.settn_init(H, 0.125, 10 ** 4)
    tau = 0.125
    for _ in range(5):
        new, info = ctx.square_compress(rho, 256, 2)
        rho.close()
        rho = new
        lam = 2.0 * lam + info["dlog_norm"]
        tau *= 2.0
        obs = ctx.observables(rho, lam, tau, H, n, entropy=False)
        for beta, key in ((tau, "tau"), (2 * tau, "2tau")):
            ref = f_ed(beta)
            assert abs(obs[key]["f"] - ref) < 5e-12 * abs(ref), (tau, key)


def test_series_start_in_run_and_serving(ctx):
    """run(..., series_tol) and a served request with "series_tol" start from
    the same rho(tau0) and give the same records bit for bit; f matches ED
    to 5e-12 at tau0 = 1/4 after four doublings (the bound of the test
    above; the linear start would be off by its tau0^2 error)."""
    from paper_1801_00142_amd import Context, run
    from paper_1801_00142_amd.serve import Server, Solve
    lat = W.chain(8)
    recs = run(ctx, lat.n_sites, lat.bonds, lat.jxy, lat.jz, 0.25, 4, 256, n_sweeps=2, series_tol=1e-15)
    with Context(0) as c2:
        served = Server(c2).run([Solve(0, lat.n_sites, lat.bonds, lat.jxy, lat.jz, 0.25, 4, 256,
                                       series_tol=1e-15)])[0]
    assert served["status"] == 0, served["error"]
    for a, b in zip(recs, served["records"]):
        assert a["lam"] == b["lam"] and a["bond_dims"] == b["bond_dims"]
        assert a["obs"]["tau"]["f"] == b["f_tau"] and a["obs"]["2tau"]["f"] == b["f_2tau"]
    E = np.linalg.eigvalsh(M.to_dense(M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)))
    e0 = E.min()
    beta = 2 * recs[-1]["tau"]
    ref = (e0 - math.log(np.sum(np.exp(-beta * (E - e0)))) / beta) / lat.n_sites
    assert abs(recs[-1]["obs"]["2tau"]["f"] - ref) < 5e-12 * abs(ref)


@pytest.mark.parametrize("lat", [W.random_couplings(W.chain(6), 4), W.square_cylinder(2, 3)],
                         ids=["chain6_rand", "cyl2x3"])
def test_taylor_steps_follow_the_exponential(ctx, lat):
    """Pointwise expansion steps on the exponential grid from the series
    start, rho(0.1) -> ... -> rho(1.6), untruncated: exp(-tau H) of the
    dense H to 2e-12 at every step (the bound of the series start: the
    compressions' noise floors over ~20 terms)."""
    H = _h(ctx, lat)
    Hd = M.to_dense(M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz))
    rho, lam, _ = ctx.settn_init(H, 0.1, 10 ** 4)
    tau = 0.1
    for _ in range(4):
        new, dl, nc = ctx.taylor_step(H, rho, tau, 10 ** 4)
        rho.close()
        rho = new
        lam += dl
        tau *= 2.0
        ex = sl.expm(-tau * Hd)
        got = M.to_dense(rho.to_host()) * math.exp(lam)
        assert np.linalg.norm(got - ex) < 2e-12 * np.linalg.norm(ex), tau


def test_truncated_taylor_step_matches_oracle(ctx):
    """L = 10 chain: from the series start rho(0.25) at D = 24, one step of
    dtau = 0.25 truncated to D = 24 on both sides: the same cutoff order and
    bond dimensions, the log-norm increment within 1e-12, the normalised
    operators' overlap 1 within 1e-10."""
    lat = W.chain(10)
    H = _h(ctx, lat)
    Ho = M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    rho, lam, _ = ctx.settn_init(H, 0.25, 24)
    ro = rho.to_host()
    new, dl, nc = ctx.taylor_step(H, rho, 0.25, 24)
    no, dlo, nco = OX.taylor_step(Ho, ro, 0.25, 24)
    g = new.to_host()
    assert nc == nco
    assert M.bond_dims(g) == M.bond_dims(no)
    assert abs(dl - dlo) < 1e-12 * max(1.0, abs(dlo))
    assert abs(1.0 - M.inner(g, no)) < 1e-10


def test_series_start_rejects_bad_arguments(ctx):
    from paper_1801_00142_amd import XtrgError
    H = _h(ctx, W.chain(4))
    for args in ((0.0, 8), (-0.1, 8), (0.1, 0)):
        with pytest.raises(XtrgError):
            ctx.settn_init(H, *args)
    with pytest.raises(XtrgError):
        ctx.settn_init(H, 0.1, 8, tol=0.0)
    # a large tau0 with many orders: the terms are added one at a time, so
    # the sums stay within the sweeps' limits (L = 8, tau0 = 1, 28 orders
    # of centre bond up to 256 would be a one-shot sum of bond ~5400)
    H8 = _h(ctx, W.chain(8))
    rho, lam, nc = ctx.settn_init(H8, 1.0, 256)
    assert nc > 20 and max(rho.bond_dims) <= 256
    with pytest.raises(XtrgError):
        ctx.taylor_step(H, rho, 0.1, 8)                  # H of 4 sites, rho of 8
    with pytest.raises(XtrgError):
        ctx.taylor_step(H8, rho, float("nan"), 8)
