"""xtrg_dgemm_noalloc: the split-K DGEMM with its partial products in the
library's fixed device scratch instead of an allocated workspace.  Two
calls in a row (the second smaller), each compared bit for bit with
xtrg_dgemm on the same inputs; no device memory allocated by the call;
shapes whose partials exceed the scratch rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_noalloc_dgemm_equals_dgemm_twice():
    import torch
    from paper_1801_00142_amd import Context
    from paper_1801_00142_amd.xtrg import _lib
    rng = np.random.default_rng(7)
    with Context(0) as ctx:
        # shapes that take the split-K path (few output tiles, long K); the
        # second call is smaller and leaves the first call's partials behind
        for (M, N, K, tA, tB) in [(256, 192, 30000, 0, 1), (96, 130, 5000, 1, 0)]:
            A = rng.standard_normal((K, M) if tA else (M, K))
            B = rng.standard_normal((N, K) if tB else (K, N))
            dA, dB = _dev(A), _dev(B)
            ref = torch.zeros((M, N), dtype=torch.float64, device="cuda")
            ctx.dgemm(M, N, K, tA, tB, dA.data_ptr(), A.shape[1], dB.data_ptr(), B.shape[1], ref.data_ptr(), N)
            torch.cuda.synchronize()
            before = ctx.bytes
            got = torch.full((M, N), np.nan, dtype=torch.float64, device="cuda")
            ctx.dgemm_noalloc(M, N, K, tA, tB, dA.data_ptr(), A.shape[1], dB.data_ptr(), B.shape[1],
                              got.data_ptr(), N)
            torch.cuda.synchronize()
            assert ctx.bytes == before                    # the context allocated nothing
            assert torch.equal(got, ref)
            want = (A.T if tA else A) @ (B.T if tB else B)
            assert np.abs(got.cpu().numpy() - want).max() < 1e-12 * np.abs(want).max() * np.sqrt(K)


def test_noalloc_dgemm_rejects_oversized_partials():
    import torch
    from paper_1801_00142_amd import Context, XtrgError
    with Context(0) as ctx:
        # 1024 x 1024 output, K = 65536: 16 split-K slices of 1 Mi doubles
        # each need 16 Mi doubles, twice the fixed scratch
        M = N = 1024
        buf = torch.zeros(8, dtype=torch.float64, device="cuda")
        with pytest.raises(XtrgError, match="split-K partials"):
            ctx.dgemm_noalloc(M, N, 65536, 0, 0, buf.data_ptr(), 65536, buf.data_ptr(), N, buf.data_ptr(), N)
