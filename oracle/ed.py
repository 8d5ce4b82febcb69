"""Exact diagonalisation of the spin-1/2 XXZ model (test infrastructure).

The dense Hamiltonian is built directly as a sum of Kronecker products of
2x2 spin matrices, independently of any MPO.  Basis: site 0 is the most
significant tensor factor; local basis (|up>, |down>).
"""
from __future__ import annotations

import numpy as np

SX = np.array([[0.0, 0.5], [0.5, 0.0]])
SZ = np.array([[0.5, 0.0], [0.0, -0.5]])
# Sy is imaginary; Sx Sx + Sy Sy = (S+ S- + S- S+)/2 is real.
SPLUS = np.array([[0.0, 1.0], [0.0, 0.0]])
SMINUS = SPLUS.T.copy()


def site_op(op: np.ndarray, i: int, n: int) -> np.ndarray:
    """Dense operator acting as ``op`` on site i of an n-site chain."""
    out = np.ones((1, 1))
    for k in range(n):
        out = np.kron(out, op if k == i else np.eye(2))
    return out


def xxz_dense(n: int, bonds, jxy, jz) -> np.ndarray:
    """H = sum_b jxy_b/2 (S+_i S-_j + S-_i S+_j) + jz_b Sz_i Sz_j (dense)."""
    dim = 2 ** n
    H = np.zeros((dim, dim))
    for (i, j), a, b in zip(bonds, jxy, jz):
        H += 0.5 * a * (site_op(SPLUS, i, n) @ site_op(SMINUS, j, n)
                        + site_op(SMINUS, i, n) @ site_op(SPLUS, j, n))
        H += b * (site_op(SZ, i, n) @ site_op(SZ, j, n))
    return H


def total_op(op: np.ndarray, n: int) -> np.ndarray:
    return sum(site_op(op, i, n) for i in range(n))


def spectrum(n: int, bonds, jxy, jz) -> np.ndarray:
    return np.linalg.eigvalsh(xxz_dense(n, bonds, jxy, jz))


def lnZ(E: np.ndarray, beta: float) -> float:
    """ln Tr exp(-beta H) from the spectrum, shifted for stability."""
    e0 = E.min()
    return float(-beta * e0 + np.log(np.sum(np.exp(-beta * (E - e0)))))


def thermo(E: np.ndarray, beta: float, n_sites: int):
    """(f, u, c) per site at inverse temperature beta (Eq. ThermalQuan)."""
    e0 = E.min()
    w = np.exp(-beta * (E - e0))
    Z = w.sum()
    em = (w * E).sum() / Z
    e2 = (w * E * E).sum() / Z
    lz = -beta * e0 + np.log(Z)
    f = -lz / (n_sites * beta)
    u = em / n_sites
    c = beta * beta * (e2 - em * em) / n_sites
    return f, u, c
