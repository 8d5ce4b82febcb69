"""The library's host-side decision rules (paper_1801_00142_amd/csrc/
host_rules.h, compiled here with g++ for the host) against the oracle, on
the CPU: the truncation rule (Sec. II.D; the multiplet-safe cut and the
noise floor), the sweep schedule and its gauge (App. D.1), the S^z charges
read from an MPO's non-zero entries and the grouping of a tensor's rows and
columns by charge (Sec. II.A; App. B.2), and the order in which the values
of charge blocks are merged.  These rules take integer decisions (a kept
count, a bond, a side, a charge, an order), so library and oracle must
agree exactly."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import mpo as M
from oracle import xtrg as OX

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp("host_rules") / "libhost_rules.so")
    subprocess.run([gxx, "-O2", "-std=c++17", "-shared", "-fPIC",
                    "-I", os.path.join(ROOT, "paper_1801_00142_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host_rules_shim.cpp"), "-o", out], check=True)
    h = C.CDLL(out)
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
    h.hr_keep_count.restype = C.c_int
    h.hr_keep_count.argtypes = [dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double]
    h.hr_infer_charges.restype = C.c_int
    h.hr_infer_charges.argtypes = [C.c_int, ip, dp, ip]
    h.hr_merge.restype = None
    h.hr_merge.argtypes = [C.c_int, ip, ip, dp, dp, ip, ip, ip]
    h.hr_schedule.restype = C.c_int
    h.hr_schedule.argtypes = [C.c_int, C.c_int, ip, ip, ip, ip]
    h.hr_charge_blocks.restype = C.c_int
    h.hr_charge_blocks.argtypes = [C.c_int, ip, C.c_int, ip, ip, ip, ip, ip, ip]
    return h


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _graded(rng, n):
    """Descending values over 14 decades with planted near-degenerate
    groups: gaps of 0.5, 0.97, 1.03 and 2 times 1e-6 relative, and exact
    ties."""
    S = np.sort(10.0 ** rng.uniform(-14, 0, n))[::-1].copy()
    for _ in range(n // 8):
        i = rng.integers(1, n)
        f = rng.choice([0.0, 0.5e-6, 0.97e-6, 1.03e-6, 2e-6])
        S[i] = S[i - 1] * (1.0 - f)
    return np.sort(S)[::-1].copy()


def test_keep_count_matches_the_oracle(lib):
    """Random graded spectra (up to 700 values), budgets from 1 to past the
    rank, the multiplet protection on and off, with and without the noise
    term: the library keeps exactly the oracle's count every time."""
    rng = np.random.default_rng(7)
    cases = 0
    for _ in range(400):
        n = int(rng.integers(1, 700))
        S = _graded(rng, n)
        for D in {1, max(1, n // 3), max(1, n // 2), n, n + 5}:
            for deg in (0.0, 1e-6):
                for eta in (0.0, 40 * 2.2e-16 * np.sqrt(n) * np.sqrt(np.sum(S * S)), 1e-7):
                    want = OX.keep_count(S, D, deg, 1e-14, eta)
                    got = lib.hr_keep_count(_dp(S), n, D, deg, 1e-14, eta)
                    assert got == want, (n, D, deg, eta)
                    cases += 1
    # zero and empty spectra keep one value
    z = np.zeros(5)
    assert lib.hr_keep_count(_dp(z), 5, 3, 1e-6, 1e-14, 0.0) == OX.keep_count(z, 3, 1e-6, 1e-14) == 1
    assert cases > 4000


def _random_charged_mpo(rng, L, qmax=2, dmax=6, density=0.5):
    dims = [1] + [int(rng.integers(1, dmax + 1)) for _ in range(L - 1)] + [1]
    q = [np.zeros(1, dtype=int)] + [rng.integers(-qmax, qmax + 1, dims[i]) for i in range(1, L)] + [np.zeros(1, dtype=int)]
    sites = []
    for i in range(L):
        w = np.zeros((dims[i], 2, 2, dims[i + 1]))
        for a in range(dims[i]):
            for s in range(2):
                for t in range(2):
                    for b in range(dims[i + 1]):
                        if q[i + 1][b] == q[i][a] + (t - s) and rng.random() < density:
                            w[a, s, t, b] = rng.standard_normal()
        sites.append(w)
    return sites, dims


def _reached(sites):
    """Bond indices reached from the left end through non-zero entries."""
    r = [np.ones(1, dtype=bool)]
    for w in sites:
        r.append(np.any(w[r[-1]] != 0, axis=(0, 1, 2)))
    return r


def _infer(lib, sites, dims):
    L = len(sites)
    d = np.array(dims, dtype=np.int32)
    flat = np.concatenate([w.reshape(-1) for w in sites])
    out = np.zeros(int(d.sum()), dtype=np.int32)
    rc = lib.hr_infer_charges(L, _ip(d), _dp(flat), _ip(out))
    if rc != 0:
        return None
    return np.split(out.astype(np.int64), np.cumsum(dims)[:-1])


def test_charges_match_the_oracle(lib):
    """Random charge-conserving MPOs (charges -2..2, half the allowed entries
    set, so some indices are never reached), the oracle's charge-definite
    starts and u1 doublings, and the automaton Hamiltonian: the library reads
    the same charge for every bond index as the oracle; MPOs with one entry
    that breaks the charge rule are refused by both."""
    rng = np.random.default_rng(3)
    for _ in range(60):
        L = int(rng.integers(2, 7))
        sites, dims = _random_charged_mpo(rng, L)
        got = _infer(lib, sites, dims)
        want = OX.bond_charges(sites)
        assert got is not None
        for g, w in zip(got, want):
            assert np.array_equal(g, w)
    lat = W.chain(8)
    rho, _ = OX.init_rho_u1(lat.n_sites, lat.bonds, lat.jxy, lat.jz, 2.0 ** -4, 2)
    rho, _ = OX.square_compress(rho, 24, 2, u1=True)
    H = M.hamiltonian(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    for mpo in (rho, H):
        got = _infer(lib, mpo, [w.shape[0] for w in mpo] + [1])
        for g, w in zip(got, OX.bond_charges(mpo)):
            assert np.array_equal(g, w)
    # one entry between indices whose charges the other entries already fix
    broken = 0
    for _ in range(40):
        sites, dims = _random_charged_mpo(rng, 4, density=0.9)
        q = OX.bond_charges(sites)
        reach = _reached(sites)
        i = int(rng.integers(1, 4))
        cand = [(a, s, t, b) for a in range(dims[i]) for s in range(2) for t in range(2) for b in range(dims[i + 1])
                if sites[i][a, s, t, b] == 0 and reach[i][a] and reach[i + 1][b]
                and q[i + 1][b] != q[i][a] + (t - s)]
        if not cand:
            continue
        a, s, t, b = cand[int(rng.integers(len(cand)))]
        sites[i][a, s, t, b] = 1.0
        with pytest.raises(ValueError):
            OX.bond_charges(sites)
        assert _infer(lib, sites, dims) is None
        broken += 1
    assert broken > 10


def test_merge_order_matches_the_oracle_block_svd(lib):
    """The merged order of the values of charge blocks: descending, equal
    values in increasing charge, each block's own order kept; the same
    values, charges and order as the oracle's block_svd, whose triples are
    LAPACK's SVD of each block, on random charge-conserving matrices with
    degenerate blocks (two charges holding the same block)."""
    rng = np.random.default_rng(5)
    for _ in range(30):
        qs = np.arange(-2, 3)
        blocks = {}
        for qv in qs:
            m, n = int(rng.integers(1, 9)), int(rng.integers(1, 9))
            blocks[int(qv)] = rng.standard_normal((m, n))
        blocks[1] = blocks[-1].copy()                  # exact ties across charges
        rows = np.concatenate([np.full(b.shape[0], qv) for qv, b in blocks.items()])
        cols = np.concatenate([np.full(b.shape[1], qv) for qv, b in blocks.items()])
        th = np.zeros((rows.size, cols.size))
        r0 = c0 = 0
        for b in blocks.values():
            th[r0:r0 + b.shape[0], c0:c0 + b.shape[1]] = b
            r0 += b.shape[0]
            c0 += b.shape[1]
        perm_r, perm_c = rng.permutation(rows.size), rng.permutation(cols.size)
        th, rows, cols = th[np.ix_(perm_r, perm_c)], rows[perm_r], cols[perm_c]
        _, S_ref, _, q_ref = OX.block_svd(th, rows, cols)
        # the library merges per-block value lists (blocks in increasing charge)
        per = [np.linalg.svd(th[np.ix_(rows == qv, cols == qv)], full_matrices=False)[1] for qv in sorted(blocks)]
        q = np.array(sorted(blocks), dtype=np.int32)
        r = np.array([p.size for p in per], dtype=np.int32)
        vals = np.concatenate(per)
        S = np.zeros(vals.size)
        qo, fr, rk = (np.zeros(vals.size, dtype=np.int32) for _ in range(3))
        lib.hr_merge(len(per), _ip(q), _ip(r), _dp(vals), _dp(S), _ip(qo), _ip(fr), _ip(rk))
        assert np.array_equal(S, S_ref)
        assert np.array_equal(qo, q_ref)
        for j in range(vals.size):                  # each value's block and rank point back to it
            assert per[fr[j]][rk[j]] == S[j]


def test_sweep_schedule_and_gauge_match_the_oracle(lib):
    """The bonds of every two-site step, their direction, the end of each
    half-sweep, and which side keeps the isometry (the gauge the split
    takes), for chains of 2 to 70 sites and 1 to 5 sweeps: the library's
    schedule is the oracle's step for step."""
    for n in list(range(2, 12)) + [48, 64, 70]:
        for ns in range(1, 6):
            m = 2 * ns * max(n - 1, 1)
            bond, d, last, gauge = (np.zeros(m, dtype=np.int32) for _ in range(4))
            k = lib.hr_schedule(n, ns, _ip(bond), _ip(d), _ip(last), _ip(gauge))
            ref = OX.sweep_schedule(n, ns)
            assert k == len(ref)
            for j, (b, dr, ls) in enumerate(ref):
                go_right = (dr > 0) != (ls and j != len(ref) - 1)
                if j == len(ref) - 1:
                    go_right = False
                assert (bond[j], d[j], bool(last[j]), bool(gauge[j])) == (b, dr, ls, go_right), (n, ns, j)


def test_charge_blocks_match_the_oracle(lib):
    """The grouping of rows and columns by charge that the block
    factorisation uses: the same charges (present on both sides, increasing)
    and the same rows and columns per block as the oracle's block_svd
    (charges drawn from -3..3, some on one side only)."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        nl, npc = int(rng.integers(1, 80)), int(rng.integers(1, 80))
        ql = rng.integers(-3, 4, nl).astype(np.int32)
        qp = rng.integers(-2, 3, npc).astype(np.int32)
        q, nr, nc = (np.zeros(16, dtype=np.int32) for _ in range(3))
        rows, cols = np.zeros(nl, dtype=np.int32), np.zeros(npc, dtype=np.int32)
        nb = lib.hr_charge_blocks(nl, _ip(ql), npc, _ip(qp), _ip(q), _ip(nr), _ip(nc), _ip(rows), _ip(cols))
        shared = np.intersect1d(ql, qp)
        assert nb == shared.size and np.array_equal(q[:nb], shared)
        orr = oc = 0
        for t, qv in enumerate(shared):
            r_ref, c_ref = np.nonzero(ql == qv)[0], np.nonzero(qp == qv)[0]
            assert np.array_equal(rows[orr:orr + nr[t]], r_ref) and np.array_equal(cols[oc:oc + nc[t]], c_ref)
            orr += nr[t]
            oc += nc[t]
