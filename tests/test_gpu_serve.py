"""Serving through the C ABI (xtrg_serve_submit / xtrg_serve_poll) and the
per-chain independence of the batched doubling.

The runs of a z-shift average are independent (Sec. II.B, Eq. zshift), so
a failure of one must not touch the others: a run with non-finite
couplings, or one whose memory estimate exceeds the budget, fails alone,
and every other run's records equal those of the same run served alone.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1801_00142_amd import Context
    c = Context(0)
    yield c
    c.close()


def _solves():
    from paper_1801_00142_amd import XTRG_FP32
    from paper_1801_00142_amd.serve import Solve
    out = []
    lats = [W.chain(6), W.square_cylinder(2, 3), W.with_couplings(W.chain(7), 1.0, 1.5),
            W.random_couplings(W.chain(5), 3), W.chain(8)]
    for q, (lat, D, arr) in enumerate(zip(lats, [8, 12, 16, 6, 10], [0.0, 0.0, 0.0, 0.0, 0.1])):
        out.append(Solve(q, lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -6 * 2 ** (q / 4), 6, D,
                         arrival_s=arr, precision=XTRG_FP32 if q == 2 else 0, beta_mix=0.1, u1=q == 4))
    return out


def _serve(budget, solves):
    from paper_1801_00142_amd import Context
    from paper_1801_00142_amd.serve import Server
    with Context(0, hbm_budget=budget) as c:
        return Server(c).run(solves)


def _same_records(a, b):
    assert len(a["records"]) == len(b["records"])
    for x, y in zip(a["records"], b["records"]):
        assert x["bond_dims"] == y["bond_dims"]
        for key in ("lam", "f_tau", "u_tau", "c_tau", "f_2tau", "u_2tau", "c_2tau"):
            assert x[key] == y[key], (x["n"], key)


def test_serve_results_equal_alone():
    """Continuous batching in the library: five runs (one with FP32
    contractions from beta_mix on, one with U(1) charge blocks, the others
    FP64 dense factorisations) arriving at different
    times under a budget that holds two at once.  Some wait for memory; each
    run's records (bond dimensions, lambda, f, u, c at every doubling) are
    bit-identical to the run served alone."""
    import dataclasses
    from paper_1801_00142_amd.serve import footprint_bytes, shared_bytes
    solves = _solves()
    budget = 2 * max(footprint_bytes(s.n_sites, s.D) for s in solves) + shared_bytes(max(s.D for s in solves))
    mixed = _serve(budget, solves)
    assert sorted(mixed) == [s.rid for s in solves]
    for s in solves:
        r = mixed[s.rid]
        assert r["status"] == 0, r["error"]
        assert r["doublings"] == s.n_doublings and len(r["records"]) == s.n_doublings + 1
        assert r["latency_s"] >= r["finished_s"] - r["admitted_s"] >= 0
    waited = [mixed[s.rid]["admitted_s"] - mixed[s.rid]["submitted_s"] for s in solves]
    assert max(waited) > 0.05                                 # some runs waited for memory
    for s in solves:
        alone = _serve(budget, [dataclasses.replace(s, arrival_s=0.0)])[s.rid]
        _same_records(alone, mixed[s.rid])


def test_serve_lanes_overlap_and_keep_results():
    """Two lanes: a large run (chain L = 12, D = 48) and two small ones
    (D = 8, about 400 times less work per doubling) submitted together.  The
    small runs go to the second lane and finish while the large one is
    still doubling; with one lane all three advance in lockstep.  Every
    run's records are bit-identical either way."""
    from paper_1801_00142_amd.serve import Solve
    big = W.chain(12)
    small = [W.chain(6), W.with_couplings(W.chain(6), 1.0, 1.3)]
    solves = [Solve(0, big.n_sites, big.bonds, big.jxy, big.jz, 2.0 ** -6, 8, 48)]
    for q, lat in enumerate(small, start=1):
        solves.append(Solve(q, lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -6 * 2 ** (q / 4), 8, 8))
    from paper_1801_00142_amd import Context
    from paper_1801_00142_amd.serve import Server
    out = {}
    for lanes in (1, 2):
        with Context(0) as c:
            out[lanes] = Server(c, lanes=lanes).run(solves)
    for s in solves:
        for lanes in (1, 2):
            assert out[lanes][s.rid]["status"] == 0, out[lanes][s.rid]["error"]
        _same_records(out[1][s.rid], out[2][s.rid])
    two = out[2]
    assert max(two[q]["finished_s"] for q in (1, 2)) < 0.5 * two[0]["finished_s"]
    one = out[1]
    assert min(one[q]["finished_s"] for q in (1, 2)) > 0.9 * one[0]["finished_s"]


def test_serve_set_lanes_rejects_bad_counts(ctx):
    from paper_1801_00142_amd import XtrgError
    for n in (0, 5):
        with pytest.raises(XtrgError):
            ctx.serve_set_lanes(n)
    ctx.serve_set_lanes(2)


def test_serve_failures_stay_with_their_run():
    """T10: a run with a NaN coupling fails with XTRG_ENUMERIC and a run
    whose memory estimate exceeds the budget fails with XTRG_ENOMEM; the
    runs beside them finish with the records they have alone."""
    import dataclasses
    from paper_1801_00142_amd.serve import Solve, footprint_bytes, shared_bytes
    good = _solves()[:2]
    lat = W.chain(6)
    nan = Solve(10, lat.n_sites, lat.bonds, [1.0, math.nan] + [1.0] * (lat.n_bonds - 2), lat.jz, 2.0 ** -6, 6, 8)
    big = Solve(11, 40, W.chain(40).bonds, [1.0] * 39, [1.0] * 39, 2.0 ** -6, 6, 4096)
    budget = 2 * max(footprint_bytes(s.n_sites, s.D) for s in good) + shared_bytes(max(s.D for s in good))
    assert footprint_bytes(big.n_sites, big.D) > budget
    res = _serve(budget, good + [nan, big])
    assert res[10]["status"] == -4 and res[10]["error"]
    assert res[11]["status"] == -2 and "budget" in res[11]["error"]
    for s in good:
        assert res[s.rid]["status"] == 0
        alone = _serve(budget, [dataclasses.replace(s, arrival_s=0.0)])[s.rid]
        _same_records(alone, res[s.rid])


def test_serve_rejects_malformed_requests(ctx):
    from paper_1801_00142_amd import XtrgError
    for bad in ({"n_sites": 4}, {"n_sites": 4, "bonds": [[0, 9]], "jxy": 1, "jz": 1, "tau0": 0.1,
                                 "n_doublings": 2, "D": 4},
                {"n_sites": 4, "bonds": [[0, 1]], "jxy": 1, "jz": 1, "tau0": -1, "n_doublings": 2, "D": 4},
                {"n_sites": 4, "bonds": [[0, 1]], "jxy": [1, 2], "jz": 1, "tau0": 0.1, "n_doublings": 2,
                 "D": 4},
                {"n_sites": 4, "bonds": [[0, 1]], "jxy": 1, "jz": 1, "tau0": 0.1, "n_doublings": 2, "D": 4,
                 "precision": "fp8"}):
        with pytest.raises(XtrgError):
            ctx.serve_submit(bad)


def test_serve_matches_run(ctx):
    """A served run reproduces run() through the single-chain calls: lambda,
    f, u and c at every doubling, bit for bit."""
    from paper_1801_00142_amd import run
    from paper_1801_00142_amd.serve import Solve
    lat = W.chain(8)
    s = Solve(0, lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -6, 6, 12)
    got = _serve(0, [s])[0]
    ref = run(ctx, lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -6, 6, 12, n_sweeps=2)
    for x, r in zip(got["records"], ref):
        assert x["bond_dims"] == r["bond_dims"]
        assert x["lam"] == r["lam"]
        for key, est in (("tau", "tau"), ("2tau", "2tau")):
            for q in ("f", "u", "c"):
                assert x[f"{q}_{key}"] == r["obs"][est][q]


def test_serve_u1_matches_run(ctx):
    """A served run with "u1": true reproduces run(u1=True) bit for bit; a
    u1 request with the series start is refused."""
    import json
    from paper_1801_00142_amd import run
    from paper_1801_00142_amd.serve import Solve
    from paper_1801_00142_amd.xtrg import XtrgError
    lat = W.with_couplings(W.square_cylinder(2, 4), 1.0, 1.5)
    s = Solve(0, lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -6, 6, 12, u1=True)
    got = _serve(0, [s])[0]
    assert got["status"] == 0, got["error"]
    ref = run(ctx, lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -6, 6, 12, n_sweeps=2, u1=True)
    for x, r in zip(got["records"], ref):
        assert x["bond_dims"] == r["bond_dims"]
        assert x["lam"] == r["lam"]
        for key, est in (("tau", "tau"), ("2tau", "2tau")):
            for q in ("f", "u", "c"):
                assert x[f"{q}_{key}"] == r["obs"][est][q]
    bad = dict(s.request(), series_tol=1e-12)
    with pytest.raises(XtrgError):
        ctx.serve_submit(bad)


def test_batched_chain_with_nan_fails_alone(ctx):
    """xtrg_square_compress_batched: a chain whose input holds a NaN stops
    with XTRG_ENUMERIC and no handle; the chains beside it return exactly
    what they return alone."""
    lat = W.chain(8)
    H = ctx.hamiltonian_xxz(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    rhos = [ctx.init_rho(H, t, 1)[0] for t in (2.0 ** -5, 2.0 ** -4, 2.0 ** -3)]
    for _ in range(2):
        outs, _ = ctx.square_compress_batched(rhos, 16, 2)
        rhos = outs
    sites = rhos[1].to_host()
    sites[3] = sites[3].copy()
    sites[3].flat[5] = math.nan
    bad = ctx.mpo_from_host(sites)
    outs, infos = ctx.square_compress_batched([rhos[0], bad, rhos[2]], 16, 2, sv_stride=4)
    assert outs[1] is None and infos[1]["status"] == -4
    for q in (0, 2):
        assert infos[q]["status"] == 0
        new, info = ctx.square_compress(rhos[q], 16, 2, sv_stride=4)
        assert new.bond_dims == outs[q].bond_dims
        for a, b in zip(new.to_host(), outs[q].to_host()):
            assert np.array_equal(a, b)
        assert info["dlog_norm"] == infos[q]["dlog_norm"]
    # the single-chain call reports the same failure as an error
    from paper_1801_00142_amd import XtrgError
    with pytest.raises(XtrgError):
        ctx.square_compress(bad, 16, 2)


def test_invariant_fields_match_oracle(ctx):
    """herm_resid, <S^z_tot> and the SU(2) residual of xtrg_observables
    against the oracle's, on a Heisenberg and an XXZ run."""
    from oracle import xtrg as OX
    from paper_1801_00142_amd import run
    for lat in (W.chain(8), W.with_couplings(W.chain(8), 1.0, 1.7)):
        args = (lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -8, 8, 16)
        gpu = run(ctx, *args, order=2, n_sweeps=2)
        ora = OX.run(*args, order=2, n_sweeps=2)
        for g, o in zip(gpu, ora):
            for key in ("tau", "2tau"):
                go, oo = g["obs"][key], o["obs"][key]
                assert abs(go["herm_resid"] - oo["herm_resid"]) < 1e-12
                assert abs(go["sz_tot"] - oo["sz_tot"]) < 1e-12
                assert abs(go["su2_resid"] - oo["su2_resid"]) < 1e-9 * max(1.0, abs(oo["su2_resid"]))
