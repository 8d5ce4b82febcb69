"""Client of the library's serving loop (xtrg_serve_submit / xtrg_serve_poll).

The continuous batching itself runs inside libxtrg.so: worker threads (one
per lane; a solve's lane follows its size) admit queued thermal solves as
device memory allows, advance their admitted solves by one doubling per
batch step through the batched doubling, keep lambda and the observables of
every doubling, and retire finished solves (include/xtrg.h).  This module only submits requests at their arrival times
and polls for results.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

from .xtrg import Context

_PREC = {0: "fp64", 1: "fp32", 2: "bf16x3"}


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
    precision: int = 0          # XTRG_FP64, XTRG_FP32 or XTRG_BF16X3
    beta_mix: float = 1.0
    series_tol: float = 0.0     # > 0: the series start (xtrg_settn_init) to this expansion error
    u1: bool = False            # S^z charges on the bonds, C_E factorised by charge blocks

    def request(self) -> dict:
        r = dict(n_sites=self.n_sites, bonds=[list(b) for b in self.bonds], jxy=list(self.jxy),
                 jz=list(self.jz), tau0=self.tau0, n_doublings=self.n_doublings, D=self.D,
                 n_sweeps=self.n_sweeps, order=self.order, precision=_PREC[self.precision],
                 beta_mix=self.beta_mix)
        if self.series_tol > 0:
            r["series_tol"] = self.series_tol
        if self.u1:
            r["u1"] = True
        return r


def footprint_bytes(n_sites: int, D: int) -> int:
    """The library's admission estimate of one solve's device memory (FP64):
    environment blocks 4 D^3 (L-1), warm bases (4D)(4D+32)(L-1), sites and
    copies 16 D^2 L, environments 6 D^3, two-site tensor and SVD workspaces
    4 (4D)(4D+32), QR route 6 (4D)(4D+32), closing check (4D+32)^2, plus
    4 MiB of grouped-launch descriptors and Gram partials."""
    L, d = n_sites, float(D)
    m, mc = 4 * d, 4 * d + 32
    elems = (4 * d ** 3 * (L - 1) + m * mc * (L - 1) + 16 * d * d * L + 6 * d ** 3 + 4 * m * mc + 6 * m * mc
             + mc * mc)
    return int(8 * elems) + (4 << 20)


def shared_bytes(D_max: int) -> int:
    """What the library reserves for the context's shared workspaces before
    admitting runs: 64 MiB plus the split-K partials 16 (4D)^2 doubles."""
    return (64 << 20) + int(8 * 16 * (4.0 * D_max) ** 2)


class Server:
    """Submits solves at their arrival times to the library's serving loop
    on `ctx` (whose hbm_budget, if set, is the admission budget; `lanes`, if
    given, sets the number of concurrent lanes) and collects the results."""

    def __init__(self, ctx: Context, poll_s: float = 0.005, lanes: Optional[int] = None):
        self.ctx = ctx
        self.poll_s = poll_s
        if lanes is not None:
            ctx.serve_set_lanes(lanes)

    def run(self, solves: Sequence[Solve], clock: Callable[[], float] = time.perf_counter,
            log: Optional[Callable[[str], None]] = None) -> Dict[int, dict]:
        """Serve all requests (arrival_s relative to the start); returns per
        request the library's result (records, status, error, submit /
        admit / finish times on the library's clock, latency)."""
        pending = sorted(solves, key=lambda r: r.arrival_s)
        ids: Dict[int, int] = {}
        out: Dict[int, dict] = {}
        progress: Dict[int, int] = {}
        t0 = clock()
        while pending or len(out) < len(ids):
            now = clock() - t0
            while pending and pending[0].arrival_s <= now:
                r = pending.pop(0)
                ids[r.rid] = self.ctx.serve_submit(r.request())
                if log:
                    log(f"t={now:.2f}s submit request {r.rid} (L={r.n_sites}, D={r.D})")
            for rid, lid in ids.items():
                if rid in out:
                    continue
                res = self.ctx.serve_poll(lid)
                if res is not None and res.get("busy"):
                    if log and res["doublings"] != progress.get(rid):
                        progress[rid] = res["doublings"]
                        log(f"t={clock() - t0:.2f}s request {rid}: {res['state']}, {res['doublings']} doublings done")
                    continue
                if res is not None:
                    res["arrival_s"] = next(s.arrival_s for s in solves if s.rid == rid)
                    out[rid] = res
                    if log:
                        log(f"t={clock() - t0:.2f}s request {rid} done (status {res['status']}); "
                            f"latency {res['latency_s']:.2f}s")
            time.sleep(self.poll_s)
        return out


def percentile(xs: Sequence[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    ys = sorted(xs)
    if not ys:
        return math.nan
    k = max(1, math.ceil(q / 100.0 * len(ys)))
    return ys[k - 1]
