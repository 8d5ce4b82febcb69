"""Seeded, synthetic workload descriptions shared by the oracle and the GPU path.

This module holds *inputs only*: lattice geometries (as 1D-ordered bond
lists), coupling constants, imaginary-time grids and the request mix of the
batched workload.  It contains none of the method's arithmetic (no operator,
no tensor, no contraction), so that the FP64 oracle and the HIP library can
both consume it without sharing any computation.

Geometries follow the paper's models: the spin-1/2 Heisenberg / XXZ chain
(Sec. III.B, "Heisenberg chain"), the square lattice (Sec. III.C) mapped to a 1D snake
(Sec. II.A: range up to 2W-1, D_H = 3W+2 with open boundaries) and
triangular-lattice YC cylinders (Sec. III.D).  Cylinder embeddings where the
paper only shows a figure are a stated reading: column-major site index
j = x*W + y with y periodic.
"""
from __future__ import annotations

import dataclasses
import math
import random
from typing import List, Sequence, Tuple

Bond = Tuple[int, int]


@dataclasses.dataclass(frozen=True)
class Lattice:
    """A spin-1/2 lattice as an ordered 1D site list plus a bond list.

    ``bonds`` holds pairs (i, j) with i < j in the 1D (MPO) ordering;
    ``jxy`` / ``jz`` are the per-bond XXZ couplings of
    H = sum_b jxy_b (Sx Sx + Sy Sy) + jz_b Sz Sz.
    """
    name: str
    n_sites: int
    bonds: Tuple[Bond, ...]
    jxy: Tuple[float, ...]
    jz: Tuple[float, ...]

    @property
    def n_bonds(self) -> int:
        return len(self.bonds)


def _normalise(bonds: Sequence[Bond]) -> List[Bond]:
    out = sorted({(min(i, j), max(i, j)) for i, j in bonds if i != j})
    return out


def chain(L: int, jxy: float = 1.0, jz: float = 1.0, pbc: bool = False) -> Lattice:
    """Open (or periodic) chain with nearest-neighbour bonds."""
    bonds = [(i, i + 1) for i in range(L - 1)]
    if pbc and L > 2:
        bonds.append((0, L - 1))
    bonds = _normalise(bonds)
    return Lattice(f"chain_L{L}{'_pbc' if pbc else ''}", L, tuple(bonds),
                   tuple([jxy] * len(bonds)), tuple([jz] * len(bonds)))


def square_snake_obc(W: int, L: int, jxy: float = 1.0, jz: float = 1.0) -> Lattice:
    """W x L open square lattice, boustrophedon ("snake") 1D ordering.

    Column x holds sites x*W .. x*W+W-1, running up for even x and down for
    odd x, so that the 1D path is connected.  Longest bond: 2W-1.
    """
    def idx(x, y):
        return x * W + (y if x % 2 == 0 else W - 1 - y)
    bonds = []
    for x in range(L):
        for y in range(W):
            if y + 1 < W:
                bonds.append((idx(x, y), idx(x, y + 1)))
            if x + 1 < L:
                bonds.append((idx(x, y), idx(x + 1, y)))
    bonds = _normalise(bonds)
    return Lattice(f"square_obc_W{W}_L{L}", W * L, tuple(bonds),
                   tuple([jxy] * len(bonds)), tuple([jz] * len(bonds)))


def square_cylinder(W: int, L: int, jxy: float = 1.0, jz: float = 1.0) -> Lattice:
    """Square-lattice cylinder, periodic in y (width W), open in x (length L).

    Column-major 1D ordering j = x*W + y.
    """
    def idx(x, y):
        return x * W + (y % W)
    bonds = []
    for x in range(L):
        for y in range(W):
            if W > 2 or y + 1 < W:
                bonds.append((idx(x, y), idx(x, y + 1)))
            if x + 1 < L:
                bonds.append((idx(x, y), idx(x + 1, y)))
    bonds = _normalise(bonds)
    return Lattice(f"square_yc_W{W}_L{L}", W * L, tuple(bonds),
                   tuple([jxy] * len(bonds)), tuple([jz] * len(bonds)))


def triangular_yc(W: int, L: int, jxy: float = 1.0, jz: float = 1.0) -> Lattice:
    """Triangular-lattice YC cylinder of width W, length L.

    Column-major ordering j = x*W + y, y periodic.  Bonds of each site:
    (x,y)-(x,y+1), (x,y)-(x+1,y), (x,y)-(x+1,y-1), y taken mod W.
    """
    def idx(x, y):
        return x * W + (y % W)
    bonds = []
    for x in range(L):
        for y in range(W):
            if W > 2 or y + 1 < W:
                bonds.append((idx(x, y), idx(x, y + 1)))
            if x + 1 < L:
                bonds.append((idx(x, y), idx(x + 1, y)))
                bonds.append((idx(x, y), idx(x + 1, y - 1)))
    bonds = _normalise(bonds)
    return Lattice(f"triangular_yc_W{W}_L{L}", W * L, tuple(bonds),
                   tuple([jxy] * len(bonds)), tuple([jz] * len(bonds)))


def with_couplings(lat: Lattice, jxy: float, jz: float) -> Lattice:
    return dataclasses.replace(lat, name=f"{lat.name}_jxy{jxy:g}_jz{jz:g}",
                               jxy=tuple([jxy] * lat.n_bonds), jz=tuple([jz] * lat.n_bonds))


def random_couplings(lat: Lattice, seed: int, lo: float = 0.5, hi: float = 1.5) -> Lattice:
    """Seeded disordered couplings (used only by tests that want no symmetry)."""
    rng = random.Random(seed)
    jxy = tuple(rng.uniform(lo, hi) for _ in lat.bonds)
    jz = tuple(rng.uniform(lo, hi) for _ in lat.bonds)
    return dataclasses.replace(lat, name=f"{lat.name}_rand{seed}", jxy=jxy, jz=jz)


# --------------------------------------------------------------------------
# The five workloads (imaginary-time grids of the doubling scheme: tau_n = 2^n tau0)
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    lattice: Lattice
    tau0: float
    n_doublings: int
    D: int
    init_order: int
    n_sweeps: int = 4


def workload(name: str, D: int | None = None) -> Workload:
    """The named synthetic workloads.

    chain10   : Heisenberg chain L=10, tau0=2^-10, 2nd-order series start,
                14 doublings (beta = 16), D = 64.
    chain12   : Heisenberg chain L=12, tau0=2^-8, linear start, 11 doublings
                (beta = 8, 16 via the Frobenius estimator); its centre bonds
                saturate at D = 128 or 256 (parity case at full tensor shape).
    chain64   : Heisenberg chain L=64, tau0=2^-12, 18 doublings (beta = 64),
                D = 128 or 256.
    square4x12: square YC W=4, L=12 (48 sites), tau0=2^-10, 15 doublings
                (beta = 32), D = 256.
    tri6x12   : triangular YC W=6, L=12 (72 sites), tau0=2^-10, 15 doublings,
                D = 512.
    """
    if name == "chain10":
        return Workload(name, chain(10), 2.0 ** -10, 14, D or 64, 2)
    if name == "chain12":
        return Workload(name, chain(12), 2.0 ** -8, 11, D or 256, 1)
    if name == "chain64":
        return Workload(name, chain(64), 2.0 ** -12, 18, D or 256, 1)
    if name == "square4x12":
        return Workload(name, square_cylinder(4, 12), 2.0 ** -10, 15, D or 256, 1)
    if name == "tri6x12":
        return Workload(name, triangular_yc(6, 12), 2.0 ** -10, 15, D or 512, 1)
    raise KeyError(name)


@dataclasses.dataclass(frozen=True)
class Request:
    """One thermal solve of the batched workload."""
    rid: int
    lattice: Lattice
    tau0: float
    n_doublings: int
    D: int
    arrival_s: float


def serve_requests(n: int = 64, seed: int = 0, rate_hz: float = 1.0, widths=(4, 6), lengths=(8, 16),
                   Ds=(64, 128, 256), n_doublings: int = 15) -> List[Request]:
    """Seeded request mix: XXZ square cylinders W in {4,6}, L ~ U{8..16},
    Delta = Jz/Jxy ~ U[1,2], D in {64,128,256}, tau0 = 2^-10 * 2^(k/4)
    (k = 0..3, interleaved z-shift grids), 15 doublings, Poisson arrivals.
    The widths, length range, bond budgets and doublings can be scaled down
    (same distributions otherwise)."""
    rng = random.Random(seed)
    out = []
    t = 0.0
    for r in range(n):
        W = rng.choice(list(widths))
        L = rng.randint(lengths[0], lengths[1])
        delta = rng.uniform(1.0, 2.0)
        D = rng.choice(list(Ds))
        k = rng.randint(0, 3)
        t += rng.expovariate(rate_hz)
        lat = with_couplings(square_cylinder(W, L), 1.0, delta)
        out.append(Request(r, lat, 2.0 ** -10 * 2.0 ** (k / 4.0), n_doublings, D, t))
    return out


def zshift_tau0(tau0: float, n_z: int) -> List[float]:
    """Interleaved initial tau0 * 2^(i/n_z), i = 0..n_z-1 (z-shifts)."""
    return [tau0 * 2.0 ** (i / n_z) for i in range(n_z)]


def betas(tau0: float, n_doublings: int) -> List[float]:
    """tau_n = 2^n tau0 for n = 0..n_doublings."""
    return [tau0 * 2.0 ** n for n in range(n_doublings + 1)]


def log2_exact(x: float) -> float:
    return math.log2(x)
