"""Kernel micro-benchmarks of the library (for profiling runs).

    python -m paper_1801_00142_amd.microbench svd N DECADES [REPS]
        one-sided Jacobi SVD (xtrg_dsvd_left) of an N x N matrix with a
        graded spectrum sigma_k = 10^(-DECADES k/(N-1)) and random orthogonal
        factors (seeded); prints the time and Jacobi sweeps per call.
    python -m paper_1801_00142_amd.microbench qr N [REPS]
        column-pivoted QR (xtrg_dqrcp, triangular factor, no early stop) of a
        seeded Gaussian N x N matrix: N Householder steps, one launch each;
        prints the time per call and per step.
    python -m paper_1801_00142_amd.microbench copy GIB
        one device-to-device copy of GIB GiB: the reference for scaling the
        HBM byte counters (FETCH_SIZE, WRITE_SIZE) of other kernels.
    python -m paper_1801_00142_amd.microbench gemm M N K [REPS]
        the library's FP64 GEMM (xtrg_dgemm, A M x K and B K x N row-major,
        seeded uniform entries) REPS times; prints TFLOP/s.  M = N = 1024,
        K = 65536 is the two-site overlap C_E at D = 256.
    python -m paper_1801_00142_amd.microbench peaks [N]
        measured ceilings beside the published peaks: the library's N x N x N
        GEMM in FP64, FP32 and bf16x3 (xtrg_dgemm, xtrg_sgemm,
        xtrg_gemm_bf16x3; N = 8192 by default) and a timed 4 GiB
        device-to-device copy (read + write bytes over its time).
"""
import sys
import time

import numpy as np


def svd(n: int, decades: float, reps: int = 2) -> None:
    import torch
    from . import Context
    rng = np.random.default_rng(0)
    U0, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V0, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s0 = 10.0 ** -np.linspace(0, decades, n)
    Y = (U0 * s0) @ V0.T
    ctx = Context(0)
    dY = torch.from_numpy(Y.T.copy()).cuda()
    sig = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.profile(True)
    ctx.profile_report()
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.dsvd_left(n, n, dY.data_ptr(), sig.data_ptr(), 0, None)
        torch.cuda.synchronize()
        print(f"svd {n}x{n}, {decades} decades: {time.perf_counter() - t:.4f} s", flush=True)
    r = ctx.profile_report()
    print(f"sweeps per call {r['svd_sweeps'] / max(r['svd_calls'], 1):.1f}; "
          f"max |sigma - sigma_exact| / sigma_1 = {np.abs(sig.cpu().numpy() - s0).max():.2e}", flush=True)
    # algorithmic bytes per round (every active column read and written once),
    # for scaling the HBM counters of the round kernels
    for key, per in (("svd_rounds_fused", 1), ("svd_rounds", 2)):
        q = r.get(key, {})
        if q.get("calls"):
            n = q["calls"] // per
            print(f"{key}: {n} rounds, {q['bytes'] / n:.1f} algorithmic bytes per round, "
                  f"{q['ms'] / n * 1e3:.3f} us per round", flush=True)
    ctx.close()


def qr(n: int, reps: int = 3) -> None:
    import torch
    from . import Context
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((n, n))
    ctx = Context(0)
    dY = torch.from_numpy(Y.T.copy()).cuda()
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    RT = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        k = ctx.dqrcp(n, n, dY.data_ptr(), 0.0, piv.data_ptr(), RT.data_ptr())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        print(f"qr {n}x{n}: {dt:.4f} s, {k} steps, {dt / max(k, 1) * 1e6:.2f} us per step", flush=True)
    ctx.close()


def copy(gib: float) -> None:
    import torch
    n = int(gib * 2 ** 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {n * 8} bytes", flush=True)


def gemm(m: int, n: int, k: int, reps: int = 5) -> None:
    import torch
    from . import Context
    ctx = Context(0)
    g = torch.Generator(device="cpu").manual_seed(0)
    A = torch.rand((m, k), generator=g, dtype=torch.float64).cuda()
    B = torch.rand((k, n), generator=g, dtype=torch.float64).cuda()
    C = torch.empty((m, n), dtype=torch.float64, device="cuda")
    ctx.dgemm(m, n, k, 0, 0, A.data_ptr(), k, B.data_ptr(), n, C.data_ptr(), n)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        ctx.dgemm(m, n, k, 0, 0, A.data_ptr(), k, B.data_ptr(), n, C.data_ptr(), n)
    torch.cuda.synchronize()
    print(f"dgemm {m}x{n}x{k}: {reps * 2.0 * m * n * k / (time.perf_counter() - t) / 1e12:.1f} TFLOP/s", flush=True)
    ctx.close()


def peaks(n: int = 8192) -> None:
    import torch
    from . import Context
    ctx = Context(0)
    g = torch.Generator(device="cpu").manual_seed(0)
    A = torch.rand((n, n), generator=g, dtype=torch.float64).cuda()
    B = torch.rand((n, n), generator=g, dtype=torch.float64).cuda()
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    A32, B32 = A.float(), B.float()
    flops = 2.0 * n ** 3
    calls = [("fp64", 78.6, lambda: ctx.dgemm(n, n, n, 0, 0, A.data_ptr(), n, B.data_ptr(), n, C.data_ptr(), n)),
             ("fp32", 157.3, lambda: ctx.sgemm(n, n, n, 0, 0, A32.data_ptr(), n, B32.data_ptr(), n, C.data_ptr(), n)),
             ("bf16x3", 2500.0 / 3, lambda: ctx.gemm_bf16x3(n, n, n, 0, 0, A32.data_ptr(), n, B32.data_ptr(), n,
                                                          C.data_ptr(), n))]
    for name, peak, f in calls:
        f()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        tf = 3 * flops / (time.perf_counter() - t) / 1e12
        print(f"gemm {name} {n}^3: {tf:.1f} TFLOP/s (published dense peak {peak:.1f}{' / 3 products' if name == 'bf16x3' else ''}, "
              f"{tf / peak:.2f})", flush=True)
    m = (4 << 30) // 8
    a = torch.ones(m, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    gbs = 5 * 2 * m * 8 / (time.perf_counter() - t) / 1e9
    print(f"copy 4 GiB: {gbs:.0f} GB/s read + write (published HBM peak 8000, {gbs / 8000:.2f})", flush=True)
    ctx.close()


if __name__ == "__main__":
    if len(sys.argv) >= 4 and sys.argv[1] == "svd":
        svd(int(sys.argv[2]), float(sys.argv[3]), int(sys.argv[4]) if len(sys.argv) > 4 else 2)
    elif len(sys.argv) >= 3 and sys.argv[1] == "qr":
        qr(int(sys.argv[2]), int(sys.argv[3]) if len(sys.argv) > 3 else 3)
    elif len(sys.argv) == 3 and sys.argv[1] == "copy":
        copy(float(sys.argv[2]))
    elif len(sys.argv) >= 5 and sys.argv[1] == "gemm":
        gemm(int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4]), int(sys.argv[5]) if len(sys.argv) > 5 else 5)
    elif len(sys.argv) >= 2 and sys.argv[1] == "peaks":
        peaks(int(sys.argv[2]) if len(sys.argv) > 2 else 8192)
    else:
        print(__doc__)
        sys.exit(2)
