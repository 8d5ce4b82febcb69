"""Throughput of the XTRG doubling step on one MI355X.

One step = one beta-doubling of the L = 64 Heisenberg chain (tau0 = 2^-12,
linear start) at bond dimension D = 256, i.e. the whole hot path: the
static right blocks, n_sweeps two-site sweeps (left/right blocks, the
two-site overlap C_E, SVD truncation, projection, environment advance) and
the normalisation.  The untimed warm-up doublings grow the bonds from the
start state until they reach D (plus --warmup more, leaving at least the
workload's last doubling), so every timed step runs at the saturated bond
dimension; the timed steps stay within the workload's 18 doublings (beta up
to 64): once its last doubling is done, the state after the warm-up is
restored between two timed steps.  The metric counts the algorithmic
flops of the contractions (64 D^4 per uniform two-site step, counted with
the actual bond dimensions) divided by the wall time of the timed steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--D 256] [--sweeps 4] [--batch N]

--batch N runs N independent chains with interleaved temperature grids
(tau0 * 2^(i/N), the z-shifts of Sec. II.B) through the batched doubling;
the value is then the whole batch's flops over its wall time.

Prints one JSON line.  Only one GPU is used: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
PEAK_FP32_MFMA_TFLOPS = 157.3  # dense FP32 matrix
PEAK_BF16_MFMA_TFLOPS = 2500.0  # dense bf16 matrix
PEAK_HBM_GBS = 8000.0
# HBM bytes per Jacobi round of a 1024 x 1024 SVD in the row-sliced form
# (Gram + rotate launches, 32 block pairs x 4 slices), from rocprofv3
# FETCH_SIZE + WRITE_SIZE scaled by a plain 1 GiB copy (FETCH x2.0, WRITE
# x1.0); see the counters summary in profiles/.  Valid for the kernels as
# measured: reset to None when they change.
JACOBI_ROUND_TRAFFIC_1024 = 26.82e6
JACOBI_ROUND_BYTES_1024 = 16.0 * 1024 * 1024   # algorithmic: every column read and written once
# The same for the one-launch round (jacobi_round<0>, the round of the S^z
# charge blocks, a few hundred rows each at D = 256), measured on a 320 x 320
# SVD (570 rounds): FETCH 502.66 KiB x 2.0 + WRITE 688.55 KiB x 1.0 per
# round, against 16 * 320 * 320 algorithmic bytes.
JACOBI_ROUND0_TRAFFIC = (502.655 * 2.0 + 688.550) * 1024.0
JACOBI_ROUND0_BYTES = 16.0 * 320 * 320


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="chain64")
    ap.add_argument("--D", type=int, default=256)
    ap.add_argument("--sweeps", type=int, default=4, help="full sweeps per doubling (the default of the method)")
    ap.add_argument("--side-sweeps", type=int, default=2,
                    help="also time this many doublings at 2 sweeps (0: skip)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the accuracy legs (stored-oracle parity run, SVD of a centre two-site tensor)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--batch-leg", type=int, default=4,
                    help="after the single-chain figures, also time one saturated doubling of this many "
                         "z-shifted chains through the batched doubling (0: skip)")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16x3"], default="fp64",
                    help="contraction precision of the doublings that reach beta >= --beta-mix")
    ap.add_argument("--beta-mix", type=float, default=1.0)
    ap.add_argument("--mixed-leg", type=int, default=2,
                    help="with FP64 contractions: this many doublings timed again with FP32 contractions "
                         "(the same doubling of the workload, the state restored first), with their accuracy")
    ap.add_argument("--dense", action="store_true",
                    help="factorise every two-site tensor as one dense matrix (default: U(1) charge sectors, "
                         "a charge-definite start and every two-site tensor factorised by S^z charge blocks)")
    ap.add_argument("--serve", type=int, default=0,
                    help="serve N requests of the scaled-down mixed workload instead (p50/p99 latency)")
    ap.add_argument("--serve-rate", type=float, default=2.0)
    ap.add_argument("--serve-slice", default=None,
                    help="a:b: serve only requests a..b-1 of the seeded stream, their arrivals shifted so that "
                         "request a arrives at 0 (a long stream in parts; per-request latencies are printed)")
    ap.add_argument("--serve-lanes", type=int, default=2,
                    help="concurrent lanes of the serving loop (requests grouped by size)")
    ap.add_argument("--serve-full", action="store_true",
                    help="the serving workload at its stated size: W in {4,6}, L in [8,16], D in {64,128,256}, "
                         "15 doublings (default: a scaled-down mix that finishes in about a minute)")
    a = ap.parse_args()
    a.u1 = not a.dense
    return a


def batch_leg(ctx, H, wl, args, mixed):
    """One saturated doubling of n z-shifted chains (tau0 2^(i/n), Sec. II.B)
    through the batched doubling: the chains are grown to the bond budget in
    the batched path, then one doubling is timed (whole-batch flops over its
    wall time)."""
    import torch
    from paper_1801_00142_amd import XTRG_FP64
    n = args.batch_leg
    taus = [wl.tau0 * 2.0 ** (i / n) for i in range(n)]
    rhos = [ctx.init_rho(H, t, wl.init_order, u1=args.u1)[0] for t in taus]
    tau = wl.tau0
    done = 0

    def step():
        nonlocal rhos, tau
        prec = mixed if 4 * tau >= args.beta_mix else XTRG_FP64
        tau *= 2
        news, infos = ctx.square_compress_batched(rhos, args.D, args.sweeps, precision=prec, u1=args.u1)
        for r in rhos:
            r.close()
        rhos = news
        return infos

    while done < wl.n_doublings:
        infos = step()
        done += 1
        dmin = min(i["D_kept_max"] for i in infos)
        print(f"batch leg warm-up doubling {done}: smallest max bond {dmin}", file=sys.stderr, flush=True)
        if dmin >= args.D:
            break
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flops = sum(i["flops"] for i in infos)
    print("batch leg timed doubling done", file=sys.stderr, flush=True)
    for r in rhos:
        r.close()
    return {"chains": n, "value": round(flops / dt / 1e12, 4), "unit": "TFLOP/s", "ms_per_step": round(dt * 1e3, 3),
            "warmup_doublings": done, "note": "one saturated doubling of the z-shifted chains through the "
                                              "batched doubling (grouped GEMM launches, grouped Jacobi rounds)"}


def theta_roofline(prec, achieved, launches, avg_s, flops):
    """The two-site overlap C_E against the matrix-core peak of the precision
    it ran in (the last timed doubling's): FP64, FP32, or bf16x3, whose three
    bf16 products per multiply-add are priced against the dense bf16 peak."""
    from paper_1801_00142_amd import XTRG_BF16X3, XTRG_FP32
    if prec == XTRG_FP32:
        kern, peak, work = "gemm_kernel<128,128,...,1,float,double>", PEAK_FP32_MFMA_TFLOPS, achieved
    elif prec == XTRG_BF16X3:
        kern, peak, work = "gemm_bf3_kernel<128,128,...,1,double>", PEAK_BF16_MFMA_TFLOPS, 3.0 * achieved
    else:
        kern, peak, work = "gemm_kernel<128,128,...,1,double,double>", PEAK_FP64_TFLOPS, achieved
    return {"bound": "mfma", "kernel": f"two-site overlap C_E ({kern})", "achieved": round(achieved, 3),
            "peak": peak, "unit": "TFLOP/s", "frac": round(work / peak, 4), "launches": launches,
            "avg_launch_ms": round(avg_s * 1e3, 4), "flops_per_launch": flops}


def cpu_baseline(sites, D, n_steps):
    """Time the FP64 oracle's two-site step (left block, right block, C_E,
    SVD, environment advance) on a bounded sample: n_steps steps at the
    centre bond of the saturated MPO, with seeded environments of the
    shapes the step sees.  Returns (TFLOP/s, seconds, flops, threads)."""
    import numpy as np
    from oracle import xtrg as OX

    L = len(sites)
    i = L // 2 - 1
    A_i, A_j = sites[i], sites[i + 1]
    Dl, Dm, Dr = A_i.shape[0], A_i.shape[3], A_j.shape[3]
    rng = np.random.default_rng(0)
    E = rng.standard_normal((min(D, Dl), Dl, Dl))
    R = rng.standard_normal((min(D, Dr), Dr, Dr))
    flops = 0.0
    t0 = time.perf_counter()
    for _ in range(n_steps):
        Lb = OX.left_block(E, A_i, A_i)
        Rb = OX.right_block(R, A_j, A_j)
        th = OX.two_site_overlap(Lb, Rb)
        U, S, Vt = np.linalg.svd(th, full_matrices=False)
        k = min(D, U.shape[1])
        C_i = U[:, :k].reshape(E.shape[0], 2, 2, k)
        OX.left_env(Lb, C_i)
        flops += OX._step_flops(E.shape, Dm, Dm, R.shape)
    dt = time.perf_counter() - t0
    threads = os.environ.get("OPENBLAS_NUM_THREADS") or os.environ.get("OMP_NUM_THREADS") or "default"
    return flops / dt / 1e12, dt, flops, threads, (th, S)


def svd_accuracy(ctx, th, S_ref, D):
    """The GPU's truncated SVD of the oracle's two-site tensor (both routes:
    the Jacobi on the tensor, and the pivoted QR + Jacobi of first visits)
    against LAPACK's values of the same tensor: max |d sigma| / sigma_1 over
    the resolved values, and whether the cut rule keeps the same count."""
    import numpy as np
    import torch
    from oracle import xtrg as OX
    m, n = th.shape
    dY = torch.from_numpy(np.ascontiguousarray(th)).to("cuda")     # row-major m x n = column-major n x m
    nf = OX.noise_floor(th)
    k_ref = OX.keep_count(S_ref, D, 1e-6, 1e-14, nf)
    out = {"shape": [m, n], "k_lapack": k_ref}
    for route in ("jacobi", "qr"):
        sig = torch.zeros(m, dtype=torch.float64, device="cuda")
        if route == "jacobi":
            ctx.dsvd_left(n, m, dY.data_ptr(), sig.data_ptr(), 0, None)
            keff = min(m, n)
        else:
            keff = ctx.dsvd_left_qr(n, m, dY.data_ptr(), sig.data_ptr(), 0, None)
        torch.cuda.synchronize()
        s = sig.cpu().numpy()[:min(m, n)]
        r = min(keff, len(S_ref))
        out[route] = {"max_dsigma_rel": float(np.abs(s[:r] - S_ref[:r]).max() / S_ref[0]),
                      "k": OX.keep_count(s, D, 1e-6, 1e-14, nf), "resolved": int(keff)}
    return out


def parity_leg(ctx, name="chain12_D256", precision=0, beta_mix=1.0, u1=False):
    """The stored FP64 oracle run of the L=12 chain at D=256 (two-site
    tensors of 1024 x 1024, 11 doublings, 2 sweeps) rerun through the
    library in the bench's contraction precision and schedule: largest
    relative deviation of f, u, c over both estimators and every beta, and
    whether every doubling kept the same bond dimensions."""
    import json
    import workloads as W
    from paper_1801_00142_amd import run
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.json")
    ref = json.load(open(path))
    lat = W.workload(ref["workload"], ref["D"]).lattice
    t0 = time.perf_counter()
    gpu = run(ctx, lat.n_sites, lat.bonds, lat.jxy, lat.jz, ref["tau0"], ref["n_doublings"], ref["D"],
              order=ref["order"], n_sweeps=ref["n_sweeps"], precision=precision, beta_mix=beta_mix, u1=u1)
    dt = time.perf_counter() - t0
    err = {"f": 0.0, "u": 0.0, "c": 0.0}
    same = True
    for g, o in zip(gpu, ref["records"]):
        same &= g["bond_dims"] == o["bond_dims"]
        for key, okey in (("tau", "tau_obs"), ("2tau", "two_tau_obs")):
            for q, floor in (("f", 0.0), ("u", 1e-3), ("c", 1e-3)):
                vo = o[okey][q]
                err[q] = max(err[q], abs(g["obs"][key][q] - vo) / max(abs(vo), floor))
    pname = {0: "FP64", 1: "FP32", 2: "bf16x3"}[precision]
    return {"workload": f"{name}: chain L=12, D={ref['D']}, {ref['n_doublings']} doublings, "
                        f"{ref['n_sweeps']} sweeps, {pname} contractions"
                        + (f" from beta >= {beta_mix}" if precision else "")
                        + (", U(1) charge blocks" if u1 else "") + ", vs the stored FP64 oracle run",
            "max_rel_df": err["f"], "max_rel_du": err["u"], "max_rel_dc": err["c"],
            "bond_dims_equal": bool(same), "seconds": round(dt, 2)}


def serve_main(args):
    """Continuous batching of a mixed request stream: square XXZ cylinders
    W in {2,3}, L in [4,8], Delta in [1,2], D in {16,32,64}, tau0 = 2^-10
    2^(k/4), 10 doublings, Poisson arrivals (the serving workload's
    distributions at a scale that finishes in about a minute)."""
    import workloads as W
    from paper_1801_00142_amd import Context
    from paper_1801_00142_amd.serve import Server, Solve, percentile
    if args.serve_full:
        reqs = W.serve_requests(args.serve, seed=0, rate_hz=args.serve_rate)
        mix = "square XXZ cylinders W 4/6, L 8-16, D 64/128/256, 15 doublings"
    else:
        reqs = W.serve_requests(args.serve, seed=0, rate_hz=args.serve_rate, widths=(2, 3), lengths=(4, 8),
                                Ds=(16, 32, 64), n_doublings=10)
        mix = "square XXZ cylinders W 2-3, L 4-8, D 16/32/64, 10 doublings"
    n_stream = len(reqs)
    if args.serve_slice:
        a, b = (int(x) for x in args.serve_slice.split(":"))
        t_a = reqs[a].arrival_s
        reqs = [dataclasses.replace(r, arrival_s=r.arrival_s - t_a) for r in reqs[a:b]]
    solves = [Solve(r.rid, r.lattice.n_sites, r.lattice.bonds, r.lattice.jxy, r.lattice.jz, r.tau0,
                    r.n_doublings, r.D, arrival_s=r.arrival_s) for r in reqs]
    ctx = Context(0)
    t0 = time.perf_counter()
    res = Server(ctx, lanes=args.serve_lanes).run(solves, log=lambda m: print(m, file=sys.stderr, flush=True))
    dt = time.perf_counter() - t0
    failed = [k for k, v in res.items() if v["status"] != 0]
    if failed:
        print(f"requests that failed: {failed}", file=sys.stderr)
    lat = [v["latency_s"] for v in res.values()]
    flops = sum(v.get("flops", 0.0) for v in res.values())
    out = {
        "metric": "TFLOP/s in MPO product-compression sweeps at D=256; p50/p99 serve latency",
        "value": round(flops / dt / 1e12, 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": len(solves),
        "warmup": 0, "ms_per_step": round(dt / len(solves) * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(solves)} mixed requests: {mix}, Poisson arrivals {args.serve_rate}/s"
                               + (f", requests {args.serve_slice} of a stream of {n_stream}" if args.serve_slice else "")
                               + f", {args.serve_lanes} lane(s)"},
        "serve": {"p50_latency_s": round(percentile(lat, 50), 3), "p99_latency_s": round(percentile(lat, 99), 3),
                  "solves_per_s": round(len(solves) / dt, 4), "wall_s": round(dt, 2), "failed": len(failed)},
    }
    if args.serve_slice:
        out["serve"]["latencies_s"] = {str(k): round(v["latency_s"], 3) for k, v in sorted(res.items())}
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); independent chains would shard "
              "across GPUs without communication", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    from paper_1801_00142_amd import Context
    if args.serve > 0:
        return serve_main(args)

    wl = W.workload(args.workload, args.D)
    lat = wl.lattice
    nb = max(args.batch, 1)
    taus = W.zshift_tau0(wl.tau0, nb)
    ctx = Context(0)
    H = ctx.hamiltonian_xxz(lat.n_sites, lat.bonds, lat.jxy, lat.jz)
    rhos = [ctx.init_rho(H, t, wl.init_order, u1=args.u1)[0] for t in taus]

    from paper_1801_00142_amd import XTRG_BF16X3, XTRG_FP32, XTRG_FP64
    mixed = {"fp64": XTRG_FP64, "fp32": XTRG_FP32, "bf16x3": XTRG_BF16X3}[args.precision]
    tau = [wl.tau0]

    last_prec = [XTRG_FP64]
    mode = {"mixed": mixed}

    def doubling(n_sweeps):
        nonlocal rhos
        # the result reaches beta = 2 tau_{n+1} = 4 tau_n (the schedule of run())
        prec = mode["mixed"] if 4 * tau[0] >= args.beta_mix else XTRG_FP64
        if prec != last_prec[0]:
            ctx.trim()              # the FP64 workspaces of the early doublings are not reused
            last_prec[0] = prec
        tau[0] *= 2
        if nb == 1:
            new, info = ctx.square_compress(rhos[0], args.D, n_sweeps, precision=prec, u1=args.u1)
            news, infos = [new], [info]
        else:
            news, infos = ctx.square_compress_batched(rhos, args.D, n_sweeps, precision=prec, u1=args.u1)
        for r in rhos:
            r.close()
        rhos = news
        return infos

    # warm-up: grow the bonds to D, then --warmup more doublings, leaving
    # at least one doubling of the workload for the timed region
    n_done = 0
    saturated_at = None
    while True:
        infos = doubling(args.sweeps)
        n_done += 1
        dmax = min(i["D_kept_max"] for i in infos)
        if saturated_at is None and dmax >= args.D:
            saturated_at = n_done
        print(f"warm-up doubling {n_done}: max bond {dmax}", file=sys.stderr, flush=True)
        if saturated_at is not None and n_done >= saturated_at + args.warmup:
            break
        if n_done >= wl.n_doublings - 1:
            break

    # The timed doublings stay within the workload's temperature range: once
    # its last doubling is done, the state after the warm-up is restored
    # (outside the timed windows) and the doublings continue from there.
    snap = ([r.to_host() for r in rhos], tau[0], n_done)
    state = {"n": n_done, "restores": 0}

    def restore():
        nonlocal rhos
        for r in rhos:
            r.close()
        rhos = [ctx.mpo_from_host(x) for x in snap[0]]
        if args.u1:
            for r in rhos:
                r.label_charges()
        tau[0] = snap[1]
        state["n"] = snap[2]
        state["restores"] += 1

    def timed(n_steps, n_sweeps, label):
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_report()                       # reset
        flops = 0.0
        steps_2site = 0
        dt = 0.0
        for _ in range(n_steps):
            if state["n"] >= wl.n_doublings:
                restore()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = doubling(n_sweeps)
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            state["n"] += 1
            flops += sum(i["flops"] for i in infos)
            steps_2site += sum(i["steps"] for i in infos)
            print(f"{label} doubling {state['n']} done: {steps_2site} two-site steps", file=sys.stderr, flush=True)
        prof = ctx.profile_report()
        ctx.profile(False)
        return flops, steps_2site, dt, prof

    # the timed steps' window on the kernel tracer's clock (CLOCK_BOOTTIME),
    # for per-kernel statistics of exactly these steps from a trace
    torch.cuda.synchronize()
    win0 = time.clock_gettime_ns(time.CLOCK_BOOTTIME)
    flops, steps_2site, dt, prof = timed(args.steps, args.sweeps, "timed")
    win1 = time.clock_gettime_ns(time.CLOCK_BOOTTIME)
    value = flops / dt / 1e12
    main_prec = last_prec[0]          # the contraction precision of the timed doublings
    side = None
    if args.side_sweeps > 0 and args.sweeps != 2:
        f2, s2, d2, _ = timed(args.side_sweeps, 2, "2-sweep")
        side = {"value": round(f2 / d2 / 1e12, 4), "n_sweeps": 2, "doublings": args.side_sweeps,
                "ms_per_step": round(d2 / args.side_sweeps * 1e3, 3)}
    mixed_leg = None
    if args.mixed_leg > 0 and mixed == XTRG_FP64:
        # the same doubling with FP32 contractions (FP64 SVD, cut and
        # normalisation), timed after the state is restored
        restore()
        mode["mixed"] = XTRG_FP32
        fm, sm, dm, _ = timed(args.mixed_leg, args.sweeps, "fp32")
        mode["mixed"] = mixed
        mixed_leg = {"precision": "f32 contractions, f64 svd", "value": round(fm / dm / 1e12, 4),
                     "unit": "TFLOP/s", "doublings": args.mixed_leg, "ms_per_step": round(dm / args.mixed_leg * 1e3, 3),
                     "solves_per_s_vs_fp64": round((dt / args.steps) / (dm / args.mixed_leg), 4)}

    svd_calls = prof.pop("svd_calls", 0)
    svd_sweeps = prof.pop("svd_sweeps", 0)
    warm_stats = {k: prof.pop(k, 0) for k in ("warm_built", "warm_rejected", "warm_used", "warm_m")}
    qr_stats = {k: prof.pop(k, 0) for k in ("qr_calls", "qr_rows", "qr_sweeps", "qr_used", "qr_rejected")}
    rounds = prof.pop("svd_rounds")                 # sliced rounds: a Gram and a rotate launch each
    rounds_fused = prof.pop("svd_rounds_fused")
    th = prof["theta_gemm"]
    th_avg_s = th["ms"] / max(th["calls"], 1) / 1e3
    th_flops = th["flops"] / max(th["calls"], 1)
    th_achieved = th_flops / th_avg_s / 1e12 if th_avg_s > 0 else 0.0
    # the dominant kernel: the Jacobi round, timed by event pairs around
    # each sweep's launches; algorithmic bytes: every active column read and
    # written once per round.  Dense 1024-row tensors take the round split
    # over row slices (a Gram launch and a rotate launch back to back); the
    # charge blocks (a few hundred rows) take the one-launch round, all
    # blocks of a two-site tensor in one grouped launch.
    sliced = rounds["ms"] >= rounds_fused["ms"]
    rr = rounds if sliced else rounds_fused
    n_rounds = max(rr["calls"] // (2 if sliced else 1), 1)
    round_us = rr["ms"] / n_rounds * 1e3
    round_bytes = rr["bytes"] / n_rounds
    round_gbs = round_bytes / (round_us * 1e-6) / 1e9 if round_us > 0 else 0.0
    total_ms = sum(v["ms"] for v in prof.values())
    shares = {k: round(v["ms"] / total_ms, 4) if total_ms else 0.0 for k, v in prof.items()}
    svd_ms = prof["svd"]["ms"] + prof.get("qr_start", {"ms": 0.0})["ms"]
    shares["svd_rounds_of_svd"] = round((rounds["ms"] + rounds_fused["ms"]) / svd_ms, 4) if svd_ms else 0.0

    # observables of the saturated state (what the serving loop evaluates
    # after every doubling), timed once
    torch.cuda.synchronize()
    t_obs = time.perf_counter()
    obs = ctx.observables(rhos[0], 0.0, tau[0], H, lat.n_sites, entropy=False)
    torch.cuda.synchronize()
    obs_s = time.perf_counter() - t_obs
    # properties of the exact state that hold at any size: a check of the
    # final compressed state where no oracle run reaches (beta = 2 tau_n)
    inv = {k: obs["2tau"][k] for k in ("herm_resid", "sz_tot", "su2_resid")}
    inv["beta"] = obs["2tau"]["beta"]

    wl_name = (f"{lat.name} {'Heisenberg' if set(lat.jz) == set(lat.jxy) == {1.0} else 'XXZ'}, "
               f"tau0=2^{math.log2(wl.tau0):g}, D={args.D}, {args.sweeps} sweeps/doubling")
    if nb > 1:
        wl_name += f", {nb} z-shifted chains batched"
    if args.u1:
        wl_name += ", U(1) charge sectors (two-site tensors factorised by S^z blocks)"
    # the headline metric (its serve-latency half is measured by --serve N --serve-full)
    metric = ("TFLOP/s in MPO product-compression sweeps at D=256; p50/p99 serve latency" if args.D == 256
              else f"TFLOP/s in MPO product-compression sweeps at D={args.D}")
    out = {
        "metric": metric,
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 contractions, f64 svd", "bf16x3": "bf16x3 contractions, f64 svd"}[
            args.precision],
        "data": "synthetic",
        "config": {"workload": wl_name, "L": lat.n_sites, "D": args.D, "n_sweeps": args.sweeps,
                   "chains": nb, "two_site_steps_per_doubling": steps_2site // max(args.steps, 1),
                   "warmup_doublings": n_done, "saturated_after": saturated_at,
                   "doublings_in_workload": wl.n_doublings, "state_restores": state["restores"]},
        "timed_window_ns": [win0, win1],
        "sweeps_per_s": round(nb * args.steps * args.sweeps / dt, 4),
        "observables_s": round(obs_s, 3),
        "invariants": inv,
        "phase_share": shares,
        "svd_sweeps_avg": round(svd_sweeps / max(svd_calls, 1), 2),
        "svd_warm": {"calls": svd_calls, "warm_started": warm_stats["warm_used"],
                     "bases_built": warm_stats["warm_built"], "bases_rejected": warm_stats["warm_rejected"],
                     "mean_completion": round(warm_stats["warm_m"] /
                                              max(warm_stats["warm_built"] + warm_stats["warm_rejected"], 1), 1)},
        # first visits: column-pivoted QR, then the Jacobi on [R^T; I] (none on the tensor itself)
        "svd_qr_start": {"factorizations": qr_stats["qr_calls"], "used": qr_stats["qr_used"],
                         "rejected": qr_stats["qr_rejected"],
                         "mean_rows": round(qr_stats["qr_rows"] / max(qr_stats["qr_calls"], 1), 1),
                         "rt_sweeps_avg": round(qr_stats["qr_sweeps"] / max(qr_stats["qr_used"], 1), 2)},
        "roofline": {"bound": "hbm",
                     "kernel": ("jacobi_round<1> + jacobi_round<2> (one block-Jacobi SVD round split over row "
                                "slices: Gram launch, rotate launch)") if sliced else
                               ("jacobi_round<0> (one block-Jacobi SVD round in one launch; every S^z charge "
                                "block of the two-site tensor is a problem of the grouped launch)"),
                     "achieved": round(round_gbs, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(round_gbs / PEAK_HBM_GBS, 4),
                     "traffic": (JACOBI_ROUND_TRAFFIC_1024 * round_bytes / JACOBI_ROUND_BYTES_1024 if sliced else
                                 JACOBI_ROUND0_TRAFFIC * round_bytes / JACOBI_ROUND0_BYTES
                                 if JACOBI_ROUND0_TRAFFIC else None),
                     "traffic_note": ("rocprofv3 FETCH_SIZE + WRITE_SIZE of the " +
                                      ("1024-column sliced round" if sliced else "one-launch round of the charge "
                                       "blocks") + ", copy-scaled, scaled to this run's mean algorithmic bytes "
                                      "per round"),
                     "rounds": n_rounds, "avg_round_us": round(round_us, 3), "bytes_per_round": round_bytes},
        "roofline_theta": theta_roofline(main_prec, th_achieved, th["calls"], th_avg_s, th_flops),
    }
    if side:
        out["value_2_sweeps"] = side
    if mixed_leg:
        out["mixed_leg"] = mixed_leg
    sites = None
    if not args.no_cpu_baseline or not args.no_accuracy:
        sites = rhos[0].to_host()
    if not args.no_accuracy:
        print("accuracy: stored-oracle parity run", file=sys.stderr, flush=True)
        out["accuracy"] = {"parity": parity_leg(ctx, "chain12_D256_u1" if args.u1 else "chain12_D256",
                                                precision=mixed, beta_mix=args.beta_mix, u1=args.u1)}
        if mixed_leg:
            mixed_leg["accuracy"] = parity_leg(ctx, "chain12_D256_u1" if args.u1 else "chain12_D256",
                                               precision=XTRG_FP32, beta_mix=args.beta_mix, u1=args.u1)
    if not args.no_cpu_baseline:
        tf, cdt, cfl, threads, (th_c, S_c) = cpu_baseline(sites, args.D, args.cpu_steps)
        out["cpu_baseline"] = {"value": round(tf, 5), "unit": "TFLOP/s",
                               "cores": len(os.sched_getaffinity(0)), "blas_threads": threads,
                               "kind": "oracle", "seconds": round(cdt, 2),
                               "sample": f"{args.cpu_steps} two-site steps (left/right block, C_E, LAPACK SVD, "
                                         f"environment) at the centre bond of the saturated D={args.D} MPO, "
                                         "seeded environments"}
        if not args.no_accuracy:
            print("accuracy: SVD of the centre two-site tensor", file=sys.stderr, flush=True)
            out["accuracy"]["svd_centre"] = svd_accuracy(ctx, th_c, S_c, args.D)
    for r in rhos:
        r.close()
    if args.batch_leg > 1 and nb == 1:
        ctx.trim()                  # the single chain's workspaces
        out["batch_leg"] = batch_leg(ctx, H, wl, args, mixed)
    H.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
