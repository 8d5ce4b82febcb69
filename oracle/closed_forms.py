"""Closed forms used to pin the oracle (test infrastructure).

* App. F: open XY chain, H = (J/2) sum (S+S- + S-S+), maps to free fermions
  with eps_k = J cos(k pi/(L+1)); Z = prod_k (1 + exp(-beta eps_k)).
* High-temperature expansion (Sec. III.B, next to the c_V ~ 1/T^2 fit):
  with Z0 = Tr I and Tr H = 0, ln Z = N ln 2 + beta^2 Tr(H^2)/(2 Z0)
  - beta^3 Tr(H^3)/(6 Z0) + O(beta^4).  For spin-1/2 XXZ bonds,
  Tr(h_b^2)/4 = (2 jxy^2 + jz^2)/16 per bond and distinct bonds are
  trace-orthogonal, so Tr(H^2)/Z0 = sum_b (2 jxy_b^2 + jz_b^2)/16.
* Linear start (App. C.2): Tr(I - tau H) = 2^N (Tr H = 0) and
  ||I - tau H||_F^2 = 2^N (1 + tau^2 Tr(H^2)/Z0).
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np


def xy_chain_lnZ(L: int, J: float, beta: float) -> float:
    """ln Z of the open XY chain (App. F)."""
    k = np.arange(1, L + 1)
    eps = J * np.cos(k * np.pi / (L + 1))
    return float(np.sum(np.logaddexp(0.0, -beta * eps)))


def h2_per_state(jxy: Sequence[float], jz: Sequence[float]) -> float:
    """Tr(H^2)/2^N for the XXZ model."""
    return float(sum((2.0 * a * a + b * b) / 16.0 for a, b in zip(jxy, jz)))


def h3_per_state(jxy: Sequence[float], jz: Sequence[float]) -> float:
    """Tr(H^3)/2^N for the XXZ model on a lattice WITHOUT triangles.

    A bond h = jxy (SxSx + SySy) + jz SzSz has eigenvalues jz/4 (twice),
    jxy/2 - jz/4 and -jxy/2 - jz/4, so Tr(h^3)/4 follows from them.  Any
    product of two or three different bonds contains a site that appears
    linearly (no closed loop), whose spin operator is traceless."""
    tot = 0.0
    for a, b in zip(jxy, jz):
        ev = (b / 4.0, b / 4.0, a / 2.0 - b / 4.0, -a / 2.0 - b / 4.0)
        tot += sum(e ** 3 for e in ev) / 4.0
    return float(tot)


def high_t_lnZ(n_sites: int, beta: float, jxy: Sequence[float], jz: Sequence[float]) -> float:
    """ln Z through third order in beta (cumulant expansion with Tr H = 0):
    N ln 2 + beta^2 Tr(H^2)/(2 Z0) - beta^3 Tr(H^3)/(6 Z0); triangle-free."""
    return (n_sites * math.log(2.0) + 0.5 * beta * beta * h2_per_state(jxy, jz)
            - beta ** 3 / 6.0 * h3_per_state(jxy, jz))


def linear_init_trace(n_sites: int) -> float:
    return 2.0 ** n_sites


def linear_init_norm2(n_sites: int, tau: float, jxy, jz) -> float:
    return 2.0 ** n_sites * (1.0 + tau * tau * h2_per_state(jxy, jz))
