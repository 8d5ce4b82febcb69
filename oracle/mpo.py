"""MPO construction and plain MPO algebra (test infrastructure).

An MPO is a Python list of real FP64 site tensors W[i] of shape
(Dl, d, d, Dr), indices [alpha, sigma, sigma', alpha'] with
W[., s, s', .] = <s| . |s'> (row = output / bra, column = input / ket),
the layout of App. B.1 ("rank-4 tensor T_{alpha alpha' sigma sigma'}",
reordered).  The outermost bonds have dimension 1.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

I2 = np.eye(2)
SPLUS = np.array([[0.0, 1.0], [0.0, 0.0]])
SMINUS = SPLUS.T.copy()
SZ = np.diag([0.5, -0.5])

# Operators opened at the first site of a bond, the operator that closes
# it at the second site, and the coupling that multiplies the closing one:
# S+S- and S-S+ with jxy/2, Sz Sz with jz (real form, App. F and App. B.1).
_OPEN = (SPLUS, SMINUS, SZ)
_CLOSE = (SMINUS, SPLUS, SZ)


def pending_sites(n: int, bonds: Sequence) -> List[List[int]]:
    """For every cut p (between sites p and p+1), the sorted list of sites
    i <= p that still have a bond partner j > p.  These are the interaction
    terms that must be carried across the cut (App. B.1, m_int)."""
    out = []
    for p in range(n - 1):
        out.append(sorted({i for i, j in bonds if i <= p < j}))
    return out


def automaton_bond_dims(n: int, bonds: Sequence) -> List[int]:
    """Virtual dimensions 2 + 3 * (#pending sites) at every internal cut
    (start, stop, and one channel per pending site and operator)."""
    return [2 + 3 * len(P) for P in pending_sites(n, bonds)]


def xxz_automaton(n: int, bonds: Sequence, jxy: Sequence, jz: Sequence):
    """Automaton MPO of the XXZ Hamiltonian on an arbitrary bond list
    (App. B.1).  Returns the *open* list of site tensors whose outermost
    bonds are the full 2-dimensional {start, stop} spaces; cap them with
    ``cap`` to obtain an operator.

    Channel layout at each cut: 0 = start, 1 = stop, 2 + 3k + a = operator a
    (S+, S-, Sz) opened at the k-th pending site.
    """
    coup = {}
    for (i, j), a, b in zip(bonds, jxy, jz):
        i, j = min(i, j), max(i, j)
        ca, cb = coup.get((i, j), (0.0, 0.0))
        coup[(i, j)] = (ca + a, cb + b)
    pend = pending_sites(n, list(coup.keys()))
    dims = [2] + [2 + 3 * len(P) for P in pend] + [2]

    def chan(cut, site, a):
        return 2 + 3 * pend[cut].index(site) + a

    W = []
    for p in range(n):
        Dl, Dr = dims[p], dims[p + 1]
        T = np.zeros((Dl, 2, 2, Dr))
        T[0, :, :, 0] = I2                      # start stays start
        T[1, :, :, 1] = I2                      # stop stays stop
        if p < n - 1 and p in pend[p]:          # open a term at site p
            for a in range(3):
                T[0, :, :, chan(p, p, a)] = _OPEN[a]
        if p > 0:
            for i in pend[p - 1]:
                if p < n - 1 and i in pend[p]:  # carry the pending operator
                    for a in range(3):
                        T[chan(p - 1, i, a), :, :, chan(p, i, a)] = I2
                if (i, p) in coup:               # close the term at site p
                    ja, jzz = coup[(i, p)]
                    cf = (0.5 * ja, 0.5 * ja, jzz)
                    for a in range(3):
                        T[chan(p - 1, i, a), :, :, 1] += cf[a] * _CLOSE[a]
        W.append(T)
    return W


def cap(W_open: List[np.ndarray], left: np.ndarray, right: np.ndarray) -> List[np.ndarray]:
    """Contract boundary vectors into the outermost virtual bonds.
    left = e_start gives the automaton its start state; right = c0 e_start
    + c1 e_stop yields the operator c0*I + c1*H (App. B.1, App. C.2)."""
    W = [w.copy() for w in W_open]
    W[0] = np.einsum("a,asti->sti", left, W[0])[None]
    W[-1] = np.einsum("asti,i->ast", W[-1], right)[..., None]
    return W


def hamiltonian(n, bonds, jxy, jz) -> List[np.ndarray]:
    """MPO of H: start state on the left, stop state on the right."""
    return cap(xxz_automaton(n, bonds, jxy, jz), np.array([1.0, 0.0]), np.array([0.0, 1.0]))


def local_sum(op: np.ndarray, n: int) -> List[np.ndarray]:
    """MPO of sum_i op_i (op a single-site 2 x 2 operator) by the automaton
    of App. B.1 with one operator per term: start -> start (I), start ->
    stop (op), stop -> stop (I)."""
    W = []
    for _ in range(n):
        T = np.zeros((2, 2, 2, 2))
        T[0, :, :, 0] = I2
        T[1, :, :, 1] = I2
        T[0, :, :, 1] = op
        W.append(T)
    return cap(W, np.array([1.0, 0.0]), np.array([0.0, 1.0]))


def spin_sum_squared(n: int) -> List[np.ndarray]:
    """MPO of (sum_i S^z_i)^2 (Sec. IV.D: the D = 3 MPO of the Binder
    ratio) as the automaton start -> (one S^z placed) -> done: sum over
    ordered pairs i < j twice, plus the diagonal (S^z_i)^2 = I/4."""
    W = []
    for _ in range(n):
        T = np.zeros((3, 2, 2, 3))
        for a in range(3):
            T[a, :, :, a] = I2
        T[0, :, :, 1] = 2.0 * SZ
        T[1, :, :, 2] = SZ
        T[0, :, :, 2] = SZ @ SZ
        W.append(T)
    return cap(W, np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0]))


def correlation(n: int, center: int, w) -> List[np.ndarray]:
    """MPO of sum_j w_j S_center . S_j (Sec. III.D, the structure factor's
    sum) as the sum of the automaton Hamiltonians of the bonds (center, j),
    j != center, with couplings w_j, plus 3/4 w_center times the identity:
    built from the Hamiltonian automaton and exact MPO sums, not compact."""
    bonds = [(min(center, j), max(center, j)) for j in range(n) if j != center]
    cj = [float(w[j]) for j in range(n) if j != center]
    Hq = hamiltonian(n, bonds, cj, cj) if bonds else None
    ident = [np.eye(2).reshape(1, 2, 2, 1).copy() for _ in range(n)]
    ident[0] = ident[0] * (0.75 * float(w[center]))
    return mpo_sum(Hq, ident) if Hq is not None else ident


def mpo_sum(A: List[np.ndarray], B: List[np.ndarray]) -> List[np.ndarray]:
    """Exact MPO of A + B (block-diagonal bonds, App. D.2 Eq. MPO:plus)."""
    n = len(A)
    out = []
    for i, (a, b) in enumerate(zip(A, B)):
        la, _, _, ra = a.shape
        lb, _, _, rb = b.shape
        if n == 1:
            out.append(a + b)
        elif i == 0:
            T = np.zeros((1, 2, 2, ra + rb))
            T[..., :ra] = a
            T[..., ra:] = b
            out.append(T)
        elif i == n - 1:
            T = np.zeros((la + lb, 2, 2, 1))
            T[:la] = a
            T[la:] = b
            out.append(T)
        else:
            T = np.zeros((la + lb, 2, 2, ra + rb))
            T[:la, :, :, :ra] = a
            T[la:, :, :, ra:] = b
            out.append(T)
    return out


def to_dense(W: List[np.ndarray]) -> np.ndarray:
    """Contract an MPO into a dense 2^n x 2^n matrix (brute force)."""
    T = W[0]                                     # (1, s, s', D)
    T = T.reshape(T.shape[1], T.shape[2], T.shape[3])
    for w in W[1:]:
        # T[(S), (S'), a] x w[a, s, s', b] -> T[(S s), (S' s'), b]
        T = np.einsum("xya,astb->xsytb", T, w)
        x, s, y, t, b = T.shape
        T = T.reshape(x * s, y * t, b)
    return T[:, :, 0]


def product(A: List[np.ndarray], B: List[np.ndarray]) -> List[np.ndarray]:
    """Exact MPO of the operator product A*B with fused bonds (a,b)
    (App. D.1, 'fat' index of dimension Da*Db)."""
    return [_fuse_product(a, b) for a, b in zip(A, B)]


def _fuse_product(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    # C[(a,b), s, u, (a',b')] = sum_t A[a,s,t,a'] B[b,t,u,b']
    c = np.einsum("asti,btuj->absuij", a, b)
    Da, Db, d1, d2, Da2, Db2 = c.shape
    return c.reshape(Da * Db, d1, d2, Da2 * Db2)


def scale(W: List[np.ndarray], x: float) -> List[np.ndarray]:
    out = [w.copy() for w in W]
    out[0] = out[0] * x
    return out


def inner(A: List[np.ndarray], B: List[np.ndarray]) -> float:
    """Frobenius inner product Tr(A^T B) = sum_{s,s'} A[s,s'] B[s,s']."""
    E = np.ones((1, 1))
    for a, b in zip(A, B):
        # E[x, y] a[x, s, t, x'] b[y, s, t, y'] -> E'[x', y']
        T = np.tensordot(E, a, axes=([0], [0]))          # [y, s, t, p]
        E = np.tensordot(T, b, axes=([0, 1, 2], [0, 1, 2]))  # [p, q]
    return float(E[0, 0])


def trace(W: List[np.ndarray]) -> float:
    """Tr of the operator: contract sigma = sigma' on every site."""
    v = np.ones((1,))
    for w in W:
        v = v @ np.einsum("asst->at", w)
    return float(v[0])


def trace_of_product(*mpos: List[np.ndarray]) -> float:
    """Tr(M1 M2 ... Mk) of MPOs by a transfer-matrix contraction (no dense
    operator is formed).  Used for Tr(H rho), Tr(H rho^T rho) etc.

    The running environment E has one axis per MPO (its bond at the current
    cut).  At each site the input index of M_j is contracted with the output
    index of M_{j+1}, and the input of M_k with the output of M_1 (trace)."""
    k = len(mpos)
    n = len(mpos[0])
    E = np.ones([1] * k)
    for i in range(n):
        W1 = mpos[0][i]
        T = np.tensordot(E, W1, axes=([0], [0]))       # [a2..ak, s1, s2, b1]
        T = np.moveaxis(T, -2, -1)                       # [a2..ak, s1, b1, s2]
        for j in range(1, k):
            Wj = mpos[j][i]                              # [a, x, y, b]
            T = np.tensordot(T, Wj, axes=([0, T.ndim - 1], [0, 1]))
            T = np.moveaxis(T, -2, -1)                   # [..., s1, b1..b_j+1, y]
        E = np.trace(T, axis1=0, axis2=T.ndim - 1)      # [b1..bk]
    return float(E.reshape(-1)[0])


def transpose(W: List[np.ndarray]) -> List[np.ndarray]:
    """MPO of the transposed operator (swap sigma and sigma')."""
    return [w.transpose(0, 2, 1, 3).copy() for w in W]


def norm(W: List[np.ndarray]) -> float:
    return float(np.sqrt(max(inner(W, W), 0.0)))


def bond_dims(W: List[np.ndarray]) -> List[int]:
    return [W[0].shape[0]] + [w.shape[3] for w in W]


def left_canonicalize(W: List[np.ndarray]) -> List[np.ndarray]:
    """Left-to-right QR sweep: sites 0..n-2 left-isometric."""
    W = [w.copy() for w in W]
    for i in range(len(W) - 1):
        Dl, d1, d2, Dr = W[i].shape
        Q, R = np.linalg.qr(W[i].reshape(Dl * d1 * d2, Dr))
        k = Q.shape[1]
        W[i] = Q.reshape(Dl, d1, d2, k)
        W[i + 1] = np.einsum("kb,bstc->kstc", R, W[i + 1])
    return W


def svd_compress(W: List[np.ndarray], D: int, rel_floor: float = 1e-14) -> List[np.ndarray]:
    """Direct SVD compression (App. D.1, the 'direct SVD' route): left-
    canonicalise with QR, then sweep right-to-left keeping at most D
    singular values per bond.  Optimal per bond for a canonical MPO."""
    W = left_canonicalize(W)
    for i in range(len(W) - 1, 0, -1):
        Dl, d1, d2, Dr = W[i].shape
        M = W[i].reshape(Dl, d1 * d2 * Dr)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        noise = 40.0 * 2.220446049250313e-16 * np.sqrt(max(M.shape)) * np.linalg.norm(M)
        k = min(D, int(np.sum(S > max(rel_floor * S[0], noise)))) if S[0] > 0 else 1
        k = max(k, 1)
        W[i] = Vt[:k].reshape(k, d1, d2, Dr)
        W[i - 1] = np.einsum("astb,bk->astk", W[i - 1], U[:, :k] * S[:k])
    return W
