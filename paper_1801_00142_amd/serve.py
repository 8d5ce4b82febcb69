"""Continuous batching of thermal solves on one GPU.

Requests (a lattice, tau0, number of doublings, bond budget) arrive over
time.  The server keeps every admitted solve's MPO resident and advances
all of them together, one doubling per step, through the batched doubling
(xtrg_square_compress_batched: the Jacobi rounds of all chains run as one
grouped launch).  A request that arrives while others run is admitted at the
next step if its device-memory estimate fits the budget; a finished one
leaves the batch at once.  Each result is identical to the same solve run
alone (the batched doubling returns what the single-chain call does).
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

from .xtrg import XTRG_FP64, Context


@dataclasses.dataclass
class Solve:
    rid: int
    n_sites: int
    bonds: Sequence
    jxy: Sequence[float]
    jz: Sequence[float]
    tau0: float
    n_doublings: int
    D: int
    arrival_s: float = 0.0
    n_sweeps: int = 2
    order: int = 1
    precision: int = XTRG_FP64


def footprint_bytes(n_sites: int, D: int) -> int:
    """Device bytes one chain holds during a doubling at bond budget D (FP64):
    the per-site environment blocks 4 D^3 (L - 1), the warm-start bases
    (4D)(4D + 32) (L - 1), sites and their copies 4 x 4 D^2 L, environments,
    the two-site overlap, SVD workspaces, those of the QR route of first
    visits and the Jacobi's closing check (Z^T Z)."""
    L = n_sites
    blocks = 4.0 * D ** 3 * (L - 1)
    warm = (4.0 * D) * (4.0 * D + 32) * (L - 1)
    sites = 4 * 4.0 * D * D * L
    envs = 2.0 * D ** 3 + 4.0 * D ** 3
    svd = 4 * (4.0 * D) * (4.0 * D + 32)
    qr = 6 * (4.0 * D) * (4.0 * D + 32)      # factor, [R^T; I] and its Jacobi, Q [W S; 0], Gram check
    check = (4.0 * D + 32) ** 2
    return int(8 * (blocks + warm + sites + envs + svd + qr + check))


@dataclasses.dataclass
class _Active:
    req: Solve
    H: object
    rho: object
    lam: float
    tau: float
    done: int = 0
    admitted_s: float = 0.0
    records: List[dict] = dataclasses.field(default_factory=list)


class Server:
    def __init__(self, ctx: Context, hbm_budget: Optional[int] = None, max_chains: int = 64):
        self.ctx = ctx
        if hbm_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.85 * free)
        self.budget = hbm_budget
        self.max_chains = max_chains

    def _admit(self, r: Solve, now: float) -> _Active:
        c = self.ctx
        H = c.hamiltonian_xxz(r.n_sites, r.bonds, r.jxy, r.jz)
        rho, lam = c.init_rho(H, r.tau0, r.order)
        a = _Active(r, H, rho, lam, r.tau0, admitted_s=now)
        a.records.append(self._record(a, None))
        return a

    def _record(self, a: _Active, info) -> dict:
        r = a.req
        obs = self.ctx.observables(a.rho, a.lam, a.tau, a.H, r.n_sites, entropy=False)
        rec = dict(n=a.done, tau=a.tau, lam=a.lam, bond_dims=a.rho.bond_dims, f_tau=obs["tau"]["f"],
                   f_2tau=obs["2tau"]["f"], u_2tau=obs["2tau"]["u"], c_2tau=obs["2tau"]["c"])
        if info is not None:
            rec["trunc_err_max"] = info["trunc_err_max"]
        return rec

    def run(self, solves: Sequence[Solve], clock: Callable[[], float] = time.perf_counter,
            log: Optional[Callable[[str], None]] = None) -> Dict[int, dict]:
        """Serve all requests (arrival_s relative to the start); returns per
        request its records and timings (arrival, admission, finish, latency)."""
        pending = sorted(solves, key=lambda r: r.arrival_s)
        active: List[_Active] = []
        out: Dict[int, dict] = {}
        t0 = clock()
        steps = 0
        while pending or active:
            now = clock() - t0
            used = sum(footprint_bytes(a.req.n_sites, a.req.D) for a in active)
            while pending and pending[0].arrival_s <= now and len(active) < self.max_chains:
                need = footprint_bytes(pending[0].n_sites, pending[0].D)
                if active and used + need > self.budget:
                    break                                   # wait for memory to free up
                r = pending.pop(0)
                active.append(self._admit(r, now))
                used += need
                if log:
                    log(f"t={now:.2f}s admit request {r.rid} (L={r.n_sites}, D={r.D}); {len(active)} active")
            if not active:
                time.sleep(max(0.0, min(pending[0].arrival_s - now, 0.05)))
                continue
            news, infos = self.ctx.square_compress_batched(
                [a.rho for a in active], [a.req.D for a in active], [a.req.n_sweeps for a in active],
                precision=active[0].req.precision if len({a.req.precision for a in active}) == 1 else XTRG_FP64)
            steps += 1
            still = []
            for a, new, info in zip(active, news, infos):
                a.rho.close()
                a.rho = new
                a.lam = 2 * a.lam + info["dlog_norm"]
                a.tau *= 2
                a.done += 1
                a.records.append(self._record(a, info))
                if a.done >= a.req.n_doublings:
                    fin = clock() - t0
                    out[a.req.rid] = dict(records=a.records, arrival_s=a.req.arrival_s, admitted_s=a.admitted_s,
                                          finished_s=fin, latency_s=fin - a.req.arrival_s)
                    a.rho.close()
                    a.H.close()
                    if log:
                        log(f"t={fin:.2f}s finish request {a.req.rid}; latency {fin - a.req.arrival_s:.2f}s")
                else:
                    still.append(a)
            if len(still) < len(active):
                self.ctx.trim()                            # workspaces sized for the departed chains
            active = still
        return out


def percentile(xs: Sequence[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    ys = sorted(xs)
    if not ys:
        return math.nan
    k = max(1, math.ceil(q / 100.0 * len(ys)))
    return ys[k - 1]
