"""Oracle pins of the U(1) charge-sector route (Sec. II.A: the XXZ models
conserve S^z_tot; App. B.2): charge inference from the exact zeros of an
MPO, the block SVD of a charge-conserving matrix, the charge-preserving
canonical form of the start, and doublings that factorise C_E by charge
blocks.

What fixes them from outside the route:
* the block SVD against LAPACK's SVD of the whole matrix;
* the charge counts and the per-charge singular values of every bond
  against the operator-space rank and values, per charge, of the dense rho
  at that cut (dense linear algebra only);
* untruncated doublings against the closed form sum_E (1 - tau0 E)^(2^n)
  of the linear start;
* truncated doublings against the stored run of the dense-SVD oracle
  (tests/golden/oracle_chain10_D64.json, written by make_golden.py);
* the multiplet-safe cut: SU(2) multiplets span charges -j..j, so the kept
  charge counts of the Heisenberg chain are symmetric and non-increasing
  in |q| at every bond.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import mpo as M
from oracle import xtrg as OX

HERE = os.path.dirname(os.path.abspath(__file__))


def _h(lat):
    return M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)


def _random_charged(rng, m, n, qmax=2):
    qr = rng.integers(-qmax, qmax + 1, m)
    qc = rng.integers(-qmax, qmax + 1, n)
    th = rng.standard_normal((m, n)) * (qr[:, None] == qc[None, :])
    return th, qr, qc


def test_block_svd_is_the_svd_of_the_whole_matrix():
    """Random charge-conserving matrices (rows and columns with charges in
    -2..2, some charges on one side only): the merged singular values are
    LAPACK's values of the whole matrix, U S V^T is the matrix, U and V are
    orthonormal and zero outside their block, and an entry planted between
    two charges is refused."""
    rng = np.random.default_rng(11)
    for m, n in ((40, 30), (17, 64), (64, 64)):
        th, qr, qc = _random_charged(rng, m, n)
        U, S, Vt, q = OX.block_svd(th, qr, qc)
        ref = np.linalg.svd(th, compute_uv=False)
        r = min(S.size, ref.size)
        assert np.all(np.diff(S) <= 0)
        assert np.abs(S[:r] - ref[:r]).max() < 1e-13 * ref[0]
        assert np.all(ref[r:] < 1e-13 * ref[0]) and np.all(S[r:] < 1e-13 * ref[0])
        assert np.abs((U * S) @ Vt - th).max() < 1e-13 * ref[0]
        assert np.abs(U.T @ U - np.eye(S.size)).max() < 1e-13
        assert np.abs(Vt @ Vt.T - np.eye(S.size)).max() < 1e-13
        assert np.all(U[qr[:, None] != q[None, :]] == 0)
        assert np.all(Vt[q[:, None] != qc[None, :]] == 0)
        bad = th.copy()
        i, j = np.argwhere(qr[:, None] != qc[None, :])[0]
        bad[i, j] = 1e-3
        with pytest.raises(ValueError):
            OX.block_svd(bad, qr, qc)


def test_charges_of_the_hamiltonian_and_of_non_conserving_mpos():
    """The automaton MPO of the XXZ chain and of a 2x3 cylinder: every
    index has a definite charge in -1..1 (the pending S+, S- and S^z
    strings), and the dense H commutes with S^z_tot.  A transverse field
    (not U(1)-symmetric) and a gauge rotation that mixes two indices of
    different charge (same operator) are refused."""
    for lat in (W.with_couplings(W.chain(6), 1.0, 1.7), W.square_cylinder(2, 3)):
        H = _h(lat)
        q = OX.bond_charges(H)
        assert all(set(v.tolist()) <= {-1, 0, 1} for v in q)
        n = lat.n_sites
        sz = np.array([sum(0.5 - ((k >> (n - 1 - j)) & 1) for j in range(n)) for k in range(2 ** n)])
        Hd = M.to_dense(H)
        assert np.abs(Hd * sz[None, :] - sz[:, None] * Hd).max() < 1e-14
    lat = W.chain(6)
    H = _h(lat)
    Sx = np.array([[0.0, 0.5], [0.5, 0.0]])
    with pytest.raises(ValueError):
        OX.bond_charges(M.mpo_sum(H, M.local_sum(Sx, lat.n_sites)))
    q = OX.bond_charges(H)
    i = 2
    a, b = int(np.argmax(q[i + 1] == 1)), int(np.argmax(q[i + 1] == 0))
    G = np.eye(H[i].shape[3])
    G[a, b] = G[b, a] = 0.3
    Hr = [w.copy() for w in H]
    Hr[i] = np.einsum("astb,bc->astc", H[i], G)
    Hr[i + 1] = np.einsum("cb,bstd->cstd", np.linalg.inv(G), H[i + 1])
    assert np.abs(M.to_dense(Hr) - M.to_dense(H)).max() < 1e-13
    with pytest.raises(ValueError):
        OX.bond_charges(Hr)


def _sector_values(O, n, cut):
    """Operator-space singular values of the dense operator O (2^n x 2^n)
    across the cut after `cut` sites, per charge sum_{j<cut} (s'_j - s_j)
    of the left part, relative to ||O||_F."""
    T = O.reshape([2] * (2 * n))
    left = [ax for j in range(cut) for ax in (j, n + j)]
    right = [ax for j in range(cut, n) for ax in (j, n + j)]
    Mx = T.transpose(left + right).reshape(4 ** cut, 4 ** (n - cut))
    idx = np.arange(4 ** cut)
    q = np.zeros(4 ** cut, dtype=int)
    for j in range(cut):
        s = (idx >> (2 * (cut - 1 - j) + 1)) & 1
        t = (idx >> (2 * (cut - 1 - j))) & 1
        q += t - s
    nrm = np.linalg.norm(Mx)
    return {int(v): np.linalg.svd(Mx[q == v], compute_uv=False) / nrm for v in np.unique(q)}


def _sector_ranks(O, n, cut, rel=1e-11):
    """The number of bond indices of each charge in a minimal MPO of O: the
    rank of each charge block of _sector_values."""
    vals = _sector_values(O, n, cut)
    top = max(v[0] for v in vals.values() if v.size)
    return {q: int(np.sum(v > rel * top)) for q, v in vals.items() if np.sum(v > rel * top)}


def _counts(q):
    v, c = np.unique(q, return_counts=True)
    return {int(a): int(b) for a, b in zip(v, c)}


@pytest.mark.parametrize("lat", [W.chain(6), W.square_cylinder(2, 3)], ids=["chain6", "cyl2x3"])
def test_charge_counts_are_the_sector_ranks_of_the_dense_operator(lat):
    """The charge-preserving start (second-order series): at every cut, the
    number of bond indices of charge q is the rank of the dense rho0
    reshaped across the cut, restricted to left charge q.  Three untruncated
    u1 doublings: they are the dense squares, and at every cut the singular
    values the last sweep reports for the indices of charge q are the dense
    operator-space values of that charge (all above 1e-10 of the largest,
    to 1e-12; the squares also hold values down to the noise floor, which
    no fixed rank tolerance separates from zero)."""
    n = lat.n_sites
    rho, lam = OX.init_rho_u1(n, lat.bonds, lat.jxy, lat.jz, 0.05, 2)
    Hd = M.to_dense(_h(lat))
    want = np.eye(2 ** n) - 0.05 * Hd + 0.00125 * Hd @ Hd
    assert np.linalg.norm(M.to_dense(rho) * math.exp(lam) - want) < 1e-13 * np.linalg.norm(want)
    q = OX.bond_charges(rho)
    for cut in range(1, n):
        assert _counts(q[cut]) == _sector_ranks(want, n, cut), cut
    for k in range(1, 4):
        rho, info = OX.square_compress(rho, 10 ** 4, 2, u1=True)
        lam = 2 * lam + info.dlog_norm
        want = want @ want
        q = info.charges
        got = M.to_dense(rho) * math.exp(lam)
        assert np.linalg.norm(got - want) < 1e-12 * np.linalg.norm(want), k
        # the reported charges are those the tensors carry
        assert all(np.array_equal(a, b) for a, b in zip(q, OX.bond_charges(rho)))
        for cut in range(1, n):
            sv = info.sv[cut - 1][:q[cut].size]
            sv = sv / math.sqrt(np.sum(info.sv[cut - 1] ** 2))
            dense = _sector_values(want, n, cut)
            top = sv[0]
            for v in set(dense) | set(q[cut].tolist()):
                mine = np.sort(sv[q[cut] == v])[::-1]
                ref = dense.get(v, np.zeros(0))
                mine, ref = mine[mine > 1e-10 * top], ref[ref > 1e-10 * top]
                assert mine.size == ref.size, (k, cut, v)
                assert np.abs(mine - ref).max(initial=0.0) < 1e-12, (k, cut, v)


def test_untruncated_u1_doublings_follow_the_closed_form():
    """Linear start rho0 = I - tau0 H (L = 8 chain, tau0 = 1/16), six u1
    doublings without truncation: ln Tr rho_n = ln sum_E (1 - tau0 E)^(2^n)
    and ln ||rho_n||_F^2 = ln sum_E (1 - tau0 E)^(2^(n+1)) to 1e-12."""
    lat = W.chain(8)
    n = lat.n_sites
    E = np.linalg.eigvalsh(M.to_dense(_h(lat)))
    tau0 = 1.0 / 16
    rho, lam = OX.init_rho_u1(n, lat.bonds, lat.jxy, lat.jz, tau0, 1)
    p = 1.0 - tau0 * E
    for k in range(1, 7):
        rho, info = OX.square_compress(rho, 10 ** 4, 2, u1=True)
        lam = 2 * lam + info.dlog_norm
        ln_tr = lam + math.log(M.trace(rho))
        assert abs(ln_tr - math.log(np.sum(p ** (2 ** k)))) < 1e-12 * abs(ln_tr)
        assert abs(2 * lam - math.log(np.sum(p ** (2 ** (k + 1))))) < 1e-12 * abs(2 * lam)


@pytest.fixture(scope="module")
def chain10_u1():
    wl = W.workload("chain10", 64)
    lat = wl.lattice
    return OX.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, wl.tau0, wl.n_doublings, wl.D, order=wl.init_order,
                  n_sweeps=4, u1=True)


def test_u1_doublings_reproduce_the_stored_dense_run(chain10_u1):
    """The L = 10 chain workload (second-order start at tau0 = 2^-10, 14
    doublings, D = 64, 4 sweeps) by charge blocks against the stored run of
    the dense-SVD oracle: the same bond dimensions after every doubling, f
    and u within 1e-11 (measured 7e-13), c within 5e-9 (measured 9e-10: c
    is a difference of two nearly equal terms at low temperature)."""
    with open(os.path.join(HERE, "golden", "oracle_chain10_D64.json")) as fh:
        g = json.load(fh)
    assert len(chain10_u1) == len(g["records"])
    for r, gr in zip(chain10_u1, g["records"]):
        assert r["bond_dims"] == gr["bond_dims"], r["n"]
        for key, gk in (("tau", "tau_obs"), ("2tau", "two_tau_obs")):
            for o, tol in (("f", 1e-11), ("u", 1e-11), ("c", 5e-9)):
                ref = gr[gk][o]
                assert abs(r["obs"][key][o] - ref) <= tol * abs(ref), (r["n"], key, o)


def test_u1_cut_keeps_su2_multiplets(chain10_u1):
    """Heisenberg chain (SU(2)): a multiplet of spin j holds one state of
    each charge -j..j, so a cut that keeps multiplets whole leaves charge
    counts n_q = n_-q, non-increasing in |q|, at every bond of every
    truncated doubling."""
    saw_cut = False
    for r in chain10_u1[1:]:
        info = r["info"]
        saw_cut |= max(info.discarded) > 0
        for q in info.charges[1:-1]:
            c = _counts(q)
            top = max(abs(v) for v in c)
            for v in range(0, top + 1):
                assert c.get(v, 0) == c.get(-v, 0), (r["n"], c)
                assert c.get(v, 0) >= c.get(v + 1, 0), (r["n"], c)
    assert saw_cut
