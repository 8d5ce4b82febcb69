"""bench.py's command-line contract, checked without a GPU: one GPU only
(more exits with a message before touching a device), and the options the
measurement runs use parse."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, timeout=120):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=timeout, cwd=ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = _bench("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_options_parse():
    sys.path.insert(0, ROOT)
    import bench
    old = sys.argv
    try:
        sys.argv = ["bench.py", "--steps", "20", "--warmup", "5", "--precision", "fp32", "--beta-mix", "0",
                    "--workload", "tri6x12", "--D", "512", "--batch-leg", "0", "--serve", "64", "--serve-full",
                    "--serve-rate", "0.025", "--serve-slice", "0:11", "--serve-lanes", "2"]
        a = bench.parse()
    finally:
        sys.argv = old
    assert (a.steps, a.warmup, a.precision, a.D, a.serve, a.serve_slice, a.serve_lanes) == \
        (20, 5, "fp32", 512, 64, "0:11", 2)
    assert a.sweeps == 4 and a.gpus == 1 and a.batch_leg == 0
    assert a.u1 and a.mixed_leg == 2                       # U(1) charge blocks and the FP32 leg by default
    old = sys.argv
    try:
        sys.argv = ["bench.py", "--dense", "--mixed-leg", "0"]
        b = bench.parse()
    finally:
        sys.argv = old
    assert not b.u1 and b.mixed_leg == 0
