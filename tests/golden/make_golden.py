"""Write the stored oracle results used by the GPU parity tests.

Runs only the FP64 oracle (oracle/) on the seeded workloads of workloads.py
and stores f, u, c, ln Z at every beta of the doubling grid, plus the bond
dimensions, as JSON.  Usage:  python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import xtrg  # noqa: E402

CASES = {
    # the L=10 chain workload: 2nd-order start at tau0 = 2^-10, 14 doublings, D = 64
    "chain10_D64": dict(workload="chain10", D=64, n_sweeps=4),
    # L=12 chains whose centre bonds saturate at D = 128 and D = 256 (two-site
    # tensors of 512 x 512 and 1024 x 1024, the shapes of the L=64 chain at
    # those budgets): linear start at tau0 = 2^-8, 11 doublings, 2 sweeps
    "chain12_D128": dict(workload="chain12", D=128, n_sweeps=2),
    "chain12_D256": dict(workload="chain12", D=256, n_sweeps=2),
    # the same runs with charge-definite bonds: the start by block SVD sweeps,
    # every C_E factorised by S^z charge blocks (oracle u1 route)
    "chain10_D64_u1": dict(workload="chain10", D=64, n_sweeps=4, u1=True),
    "chain12_D128_u1": dict(workload="chain12", D=128, n_sweeps=2, u1=True),
    "chain12_D256_u1": dict(workload="chain12", D=256, n_sweeps=2, u1=True),
}


def main(names):
    for name in names:
        cfg = CASES[name]
        wl = W.workload(cfg["workload"], cfg["D"])
        lat = wl.lattice
        t0 = time.time()
        recs = xtrg.run(lat.n_sites, lat.bonds, lat.jxy, lat.jz, wl.tau0, wl.n_doublings, wl.D,
                        order=wl.init_order, n_sweeps=cfg["n_sweeps"], u1=cfg.get("u1", False))
        out = dict(case=name, workload=cfg["workload"], D=wl.D, n_sweeps=cfg["n_sweeps"], u1=cfg.get("u1", False),
                   tau0=wl.tau0,
                   order=wl.init_order, n_doublings=wl.n_doublings, n_sites=lat.n_sites,
                   seconds=time.time() - t0, records=[])
        for r in recs:
            out["records"].append(dict(n=r["n"], tau=r["tau"], lam=r["lam"], bond_dims=r["bond_dims"],
                                       tau_obs=r["obs"]["tau"], two_tau_obs=r["obs"]["2tau"]))
        with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, f"{out['seconds']:.1f}s")


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
