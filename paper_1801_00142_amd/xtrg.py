"""ctypes binding of libxtrg.so (argument marshalling only).

Every tensor operation runs in the HIP library; this module converts Python
and NumPy arguments to the C ABI of include/xtrg.h and back.  It raises
immediately if the compiled library is absent: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import weakref
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libxtrg.so")
_lib = None

XTRG_FP64 = 0
XTRG_FP32 = 1
XTRG_BF16X3 = 2


class XtrgError(RuntimeError):
    pass


class CompressOpts(C.Structure):
    _fields_ = [("D_max", C.c_int), ("n_sweeps", C.c_int), ("precision", C.c_int),
                ("degen_rtol", C.c_double), ("sv_floor", C.c_double), ("no_warm_start", C.c_int),
                ("no_qr_start", C.c_int), ("u1", C.c_int)]


class CompressInfo(C.Structure):
    _fields_ = [("dlog_norm", C.c_double), ("trunc_err_max", C.c_double), ("sweeps_done", C.c_int),
                ("D_kept_max", C.c_int), ("steps", C.c_int), ("flops", C.c_double),
                ("sv", C.POINTER(C.c_double)), ("sv_stride", C.c_int), ("status", C.c_int)]


class Obs(C.Structure):
    _fields_ = [("beta", C.c_double), ("lnZ", C.c_double), ("f", C.c_double), ("u", C.c_double),
                ("c", C.c_double), ("tr_rho", C.c_double), ("S_E_center", C.c_double),
                ("S_E_max", C.c_double), ("herm_resid", C.c_double), ("sz_tot", C.c_double),
                ("su2_resid", C.c_double)]


def load_library(path: Optional[str] = None):
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        raise XtrgError(f"{p} is missing: build it with `python -m paper_1801_00142_amd.build`")
    # One HIP runtime per process: PyTorch ships its own copy of the runtime
    # library under the same soname.  Loaded after it, libxtrg.so binds to
    # that copy, so torch's streams and device pointers are valid in the
    # library; loaded first, a second runtime would come up beside torch's
    # and torch would find no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(p)
    vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
    sig = {
        "xtrg_ctx_create": (C.c_int, [C.c_int, vp, C.c_size_t, C.POINTER(vp)]),
        "xtrg_ctx_destroy": (C.c_int, [vp]),
        "xtrg_last_error": (C.c_char_p, [vp]),
        "xtrg_ctx_bytes": (C.c_size_t, [vp]),
        "xtrg_ctx_trim": (C.c_int, [vp]),
        "xtrg_hamiltonian_xxz": (C.c_int, [vp, C.c_int, C.c_int, ip, dp, dp, C.POINTER(vp)]),
        "xtrg_mpo_from_host": (C.c_int, [vp, C.c_int, C.c_int, ip, C.POINTER(dp), C.POINTER(vp)]),
        "xtrg_mpo_shape": (C.c_int, [vp, ip, ip]),
        "xtrg_mpo_to_host": (C.c_int, [vp, C.POINTER(dp)]),
        "xtrg_mpo_destroy": (C.c_int, [vp]),
        "xtrg_init_rho": (C.c_int, [vp, vp, C.c_double, C.c_int, C.c_int, C.POINTER(vp), dp]),
        "xtrg_init_rho_u1": (C.c_int, [vp, vp, C.c_double, C.c_int, C.c_int, C.POINTER(vp), dp]),
        "xtrg_mpo_label_charges": (C.c_int, [vp]),
        "xtrg_mpo_charges": (C.c_int, [vp, ip]),
        "xtrg_square_compress": (C.c_int, [vp, vp, C.POINTER(CompressOpts), C.POINTER(vp),
                                           C.POINTER(CompressInfo)]),
        "xtrg_product_compress": (C.c_int, [vp, vp, vp, C.POINTER(CompressOpts), C.POINTER(vp),
                                            C.POINTER(CompressInfo)]),
        "xtrg_square_compress_batched": (C.c_int, [vp, C.c_int, C.POINTER(vp), C.POINTER(CompressOpts),
                                                   C.POINTER(vp), C.POINTER(CompressInfo)]),
        "xtrg_observables": (C.c_int, [vp, vp, C.c_double, C.c_double, vp, C.c_int, C.POINTER(Obs),
                                       C.POINTER(Obs), dp]),
        "xtrg_dgemm": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp, C.c_long, vp,
                                 C.c_long, vp, C.c_long]),
        "xtrg_dgemm_noalloc": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp, C.c_long, vp,
                                         C.c_long, vp, C.c_long]),
        "xtrg_sgemm": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp, C.c_long, vp,
                                 C.c_long, vp, C.c_long, C.c_int]),
        "xtrg_gemm_bf16x3": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp, C.c_long, vp,
                                       C.c_long, vp, C.c_long, C.c_int]),
        "xtrg_dsvd_left": (C.c_int, [vp, C.c_int, C.c_int, vp, vp, C.c_int, vp]),
        "xtrg_dsvd_left_qr": (C.c_int, [vp, C.c_int, C.c_int, vp, vp, C.c_int, vp, ip]),
        "xtrg_dqrcp": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_double, vp, vp, ip]),
        "xtrg_spin_sum_mpo": (C.c_int, [vp, C.c_int, C.c_int, C.POINTER(vp)]),
        "xtrg_correlation_mpo": (C.c_int, [vp, C.c_int, C.c_int, dp, C.POINTER(vp)]),
        "xtrg_expectation": (C.c_int, [vp, vp, C.c_int, C.POINTER(vp), dp, dp]),
        "xtrg_serve_submit": (C.c_int, [vp, C.c_char_p, C.POINTER(C.c_ulonglong)]),
        "xtrg_serve_poll": (C.c_int, [vp, C.c_ulonglong, C.c_char_p, C.c_size_t]),
        "xtrg_serve_set_lanes": (C.c_int, [vp, C.c_int]),
        "xtrg_settn_init": (C.c_int, [vp, vp, C.c_double, C.c_int, C.c_int, C.c_double, C.POINTER(vp), dp, ip]),
        "xtrg_taylor_step": (C.c_int, [vp, vp, vp, C.c_double, C.c_int, C.c_int, C.c_double, C.POINTER(vp), dp,
                                       ip]),
        "xtrg_profile_enable": (C.c_int, [vp, C.c_int]),
        "xtrg_profile_report": (C.c_int, [vp, C.c_char_p, C.c_size_t]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> List[str]:
    return ["xtrg_ctx_create", "xtrg_ctx_destroy", "xtrg_last_error", "xtrg_ctx_bytes", "xtrg_ctx_trim",
            "xtrg_hamiltonian_xxz", "xtrg_mpo_from_host", "xtrg_mpo_shape", "xtrg_mpo_to_host",
            "xtrg_mpo_destroy", "xtrg_init_rho", "xtrg_init_rho_u1", "xtrg_mpo_label_charges", "xtrg_mpo_charges",
            "xtrg_square_compress", "xtrg_product_compress", "xtrg_square_compress_batched", "xtrg_observables",
            "xtrg_dgemm", "xtrg_dgemm_noalloc", "xtrg_sgemm", "xtrg_gemm_bf16x3", "xtrg_dsvd_left", "xtrg_dsvd_left_qr", "xtrg_dqrcp", "xtrg_spin_sum_mpo", "xtrg_correlation_mpo", "xtrg_expectation", "xtrg_serve_submit", "xtrg_serve_poll", "xtrg_serve_set_lanes", "xtrg_settn_init", "xtrg_taylor_step", "xtrg_profile_enable",
            "xtrg_profile_report"]


class MPO:
    def __init__(self, ctx: "Context", handle):
        self.ctx = ctx
        self.h = handle
        ctx._live.add(self)

    def shape(self):
        L = C.c_int()
        _check(self.ctx, _lib.xtrg_mpo_shape(self.h, C.byref(L), None))
        dims = (C.c_int * (L.value + 1))()
        _check(self.ctx, _lib.xtrg_mpo_shape(self.h, None, dims))
        return L.value, list(dims)

    @property
    def bond_dims(self):
        return self.shape()[1]

    def to_host(self) -> List[np.ndarray]:
        L, dims = self.shape()
        arrs = [np.empty((dims[i], 2, 2, dims[i + 1]), dtype=np.float64) for i in range(L)]
        ptrs = (C.POINTER(C.c_double) * L)(*[a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs])
        _check(self.ctx, _lib.xtrg_mpo_to_host(self.h, ptrs))
        return arrs

    def charges(self) -> List[np.ndarray]:
        """S^z charge of every bond index (L+1 arrays), for MPOs with
        charge-definite bonds (xtrg_init_rho_u1, label_charges, u1 doublings)."""
        L, dims = self.shape()
        buf = (C.c_int * sum(dims))()
        _check(self.ctx, _lib.xtrg_mpo_charges(self.h, buf))
        flat = np.frombuffer(buf, dtype=np.int32).astype(np.int64)
        return list(np.split(flat, np.cumsum(dims)[:-1]))

    def label_charges(self):
        """Read the charges of the bond indices from the non-zero entries."""
        _check(self.ctx, _lib.xtrg_mpo_label_charges(self.h))
        return self

    def close(self):
        # an MPO is released before its context; after Context.close() the
        # handle is already gone
        if self.h and self.ctx.h:
            _lib.xtrg_mpo_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check(ctx, rc):
    if rc != 0:
        msg = _lib.xtrg_last_error(ctx.h if ctx is not None else None)
        raise XtrgError(f"xtrg error {rc}: {msg.decode() if msg else ''}")


class Context:
    def __init__(self, device: int = 0, stream: Optional[int] = None, hbm_budget: int = 0):
        load_library()
        h = C.c_void_p()
        rc = _lib.xtrg_ctx_create(device, C.c_void_p(stream) if stream else None, hbm_budget, C.byref(h))
        if rc != 0:
            raise XtrgError(f"xtrg_ctx_create failed ({rc})")
        self.h = h
        self._live = weakref.WeakSet()

    def close(self):
        if self.h:
            for m in list(self._live):
                m.close()
            _lib.xtrg_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def bytes(self) -> int:
        return int(_lib.xtrg_ctx_bytes(self.h))

    def trim(self):
        """Release the workspaces (kept at their largest size between calls)."""
        _check(self, _lib.xtrg_ctx_trim(self.h))

    def hamiltonian_xxz(self, n_sites: int, bonds: Sequence, jxy: Sequence[float], jz: Sequence[float]) -> MPO:
        b = np.ascontiguousarray(np.array(bonds, dtype=np.int32).reshape(-1))
        a = np.ascontiguousarray(np.array(jxy, dtype=np.float64))
        z = np.ascontiguousarray(np.array(jz, dtype=np.float64))
        h = C.c_void_p()
        _check(self, _lib.xtrg_hamiltonian_xxz(self.h, n_sites, len(a), b.ctypes.data_as(C.POINTER(C.c_int)),
                                               a.ctypes.data_as(C.POINTER(C.c_double)),
                                               z.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)))
        return MPO(self, h)

    def mpo_from_host(self, sites: Sequence[np.ndarray]) -> MPO:
        sites = [np.ascontiguousarray(s, dtype=np.float64) for s in sites]
        L = len(sites)
        dims = (C.c_int * (L + 1))(*([sites[0].shape[0]] + [s.shape[3] for s in sites]))
        ptrs = (C.POINTER(C.c_double) * L)(*[s.ctypes.data_as(C.POINTER(C.c_double)) for s in sites])
        h = C.c_void_p()
        _check(self, _lib.xtrg_mpo_from_host(self.h, L, 2, dims, ptrs, C.byref(h)))
        return MPO(self, h)

    def init_rho(self, H: MPO, tau0: float, order: int = 1, D0_max: int = 0, u1: bool = False):
        h = C.c_void_p()
        lam = C.c_double()
        f = _lib.xtrg_init_rho_u1 if u1 else _lib.xtrg_init_rho
        _check(self, f(self.h, H.h, tau0, order, D0_max, C.byref(h), C.byref(lam)))
        return MPO(self, h), lam.value

    def settn_init(self, H: MPO, tau0: float, D_max: int, n_sweeps: int = 2, tol: float = 1e-15):
        """rho(tau0) by the series expansion with automatic cutoff order:
        (rho_hat, log_norm, cutoff order)."""
        h = C.c_void_p()
        lam = C.c_double()
        nt = C.c_int()
        _check(self, _lib.xtrg_settn_init(self.h, H.h, tau0, D_max, n_sweeps, tol, C.byref(h), C.byref(lam),
                                          C.byref(nt)))
        return MPO(self, h), lam.value, nt.value

    def taylor_step(self, H: MPO, rho: MPO, dtau: float, D_max: int, n_sweeps: int = 2, tol: float = 1e-15):
        """rho(tau + dtau) by the pointwise expansion (Eq. Tay):
        (rho_hat', dlog_norm, cutoff order)."""
        h = C.c_void_p()
        dl = C.c_double()
        nt = C.c_int()
        _check(self, _lib.xtrg_taylor_step(self.h, H.h, rho.h, dtau, D_max, n_sweeps, tol, C.byref(h), C.byref(dl),
                                           C.byref(nt)))
        return MPO(self, h), dl.value, nt.value

    def square_compress(self, rho: MPO, D_max: int, n_sweeps: int = 4, degen_rtol: float = 1e-6,
                        sv_floor: float = 1e-14, sv_stride: int = 0, precision: int = XTRG_FP64,
                        warm_start: bool = True, qr_start: bool = True, u1: bool = False):
        o = CompressOpts(D_max, n_sweeps, precision, degen_rtol, sv_floor, int(not warm_start),
                         int(not qr_start), int(u1))
        info = CompressInfo()
        L = rho.shape()[0]
        buf = None
        if sv_stride > 0:
            buf = np.zeros((L - 1, sv_stride))
            info.sv = buf.ctypes.data_as(C.POINTER(C.c_double))
            info.sv_stride = sv_stride
        h = C.c_void_p()
        _check(self, _lib.xtrg_square_compress(self.h, rho.h, C.byref(o), C.byref(h), C.byref(info)))
        out = dict(dlog_norm=info.dlog_norm, trunc_err_max=info.trunc_err_max, sweeps=info.sweeps_done,
                   D_kept_max=info.D_kept_max, steps=info.steps, flops=info.flops)
        if buf is not None:
            out["sv"] = buf
        return MPO(self, h), out

    def product_compress(self, A: MPO, B: MPO, D_max: int, n_sweeps: int = 4, degen_rtol: float = 1e-6,
                         sv_floor: float = 1e-14, precision: int = XTRG_FP64, warm_start: bool = True,
                         qr_start: bool = True, u1: bool = False):
        """out ~ A B / c (B: the right-canonical initial guess); returns (MPO, info)."""
        o = CompressOpts(D_max, n_sweeps, precision, degen_rtol, sv_floor, int(not warm_start), int(not qr_start),
                         int(u1))
        info = CompressInfo()
        h = C.c_void_p()
        _check(self, _lib.xtrg_product_compress(self.h, A.h, B.h, C.byref(o), C.byref(h), C.byref(info)))
        return MPO(self, h), dict(dlog_norm=info.dlog_norm, trunc_err_max=info.trunc_err_max,
                                  sweeps=info.sweeps_done, D_kept_max=info.D_kept_max, steps=info.steps,
                                  flops=info.flops)

    def square_compress_batched(self, rhos: Sequence[MPO], D_max, n_sweeps=4,
                                degen_rtol: float = 1e-6, sv_floor: float = 1e-14, sv_stride: int = 0,
                                precision=XTRG_FP64, warm_start: bool = True, qr_start: bool = True,
                                u1: bool = False):
        """One doubling of every chain in `rhos` together.  D_max, n_sweeps and
        precision are one value for all chains or a sequence with one per
        chain.  Returns ([new MPO per chain], [info dict per chain]).  A chain
        that the library stopped (non-finite tensors, memory refused by the
        budget) has None in place of its MPO and its code in info["status"];
        the other chains' results are unaffected."""
        n = len(rhos)

        def per(v, name):
            out = list(v) if isinstance(v, (list, tuple)) else [v] * n
            if len(out) != n:
                raise ValueError(f"one {name} per chain")
            return out
        Ds, Ss, Ps = per(D_max, "D_max"), per(n_sweeps, "n_sweeps"), per(precision, "precision")
        o = (CompressOpts * n)(*[CompressOpts(Ds[q], Ss[q], Ps[q], degen_rtol, sv_floor, int(not warm_start),
                                              int(not qr_start), int(u1))
                               for q in range(n)])
        infos = (CompressInfo * n)()
        bufs = []
        for q, r in enumerate(rhos):
            if sv_stride > 0:
                b = np.zeros((r.shape()[0] - 1, sv_stride))
                infos[q].sv = b.ctypes.data_as(C.POINTER(C.c_double))
                infos[q].sv_stride = sv_stride
                bufs.append(b)
        hin = (C.c_void_p * n)(*[r.h for r in rhos])
        hout = (C.c_void_p * n)()
        rc = _lib.xtrg_square_compress_batched(self.h, n, hin, o, hout, infos)
        if rc != 0 and not any(hout[q] for q in range(n)) and not any(infos[q].status for q in range(n)):
            _check(self, rc)                     # the whole call failed
        err = _lib.xtrg_last_error(self.h).decode() if rc != 0 else ""
        outs, dicts = [], []
        for q in range(n):
            st = infos[q].status
            outs.append(MPO(self, C.c_void_p(hout[q])) if hout[q] else None)
            d = dict(status=st)
            if st == 0:
                d.update(dlog_norm=infos[q].dlog_norm, trunc_err_max=infos[q].trunc_err_max,
                         sweeps=infos[q].sweeps_done, D_kept_max=infos[q].D_kept_max, steps=infos[q].steps,
                         flops=infos[q].flops)
                if bufs:
                    d["sv"] = bufs[q]
            else:
                d["error"] = err
            dicts.append(d)
        return outs, dicts

    def observables(self, rho: MPO, log_norm: float, tau: float, H: MPO, n_sites: int,
                    entropy: bool = True) -> Dict[str, Dict[str, float]]:
        a, b = Obs(), Obs()
        L = rho.shape()[0]
        se = np.zeros(max(L - 1, 1)) if entropy else None
        _check(self, _lib.xtrg_observables(self.h, rho.h, log_norm, tau, H.h, n_sites, C.byref(a), C.byref(b),
                                           se.ctypes.data_as(C.POINTER(C.c_double)) if entropy else None))
        fa = {k: getattr(a, k) for k, _ in Obs._fields_}
        fb = {k: getattr(b, k) for k, _ in Obs._fields_}
        fa["tr"] = fa.pop("tr_rho")
        fb["norm2"] = fb.pop("tr_rho")
        out = {"tau": fa, "2tau": fb}
        if entropy:
            out["S_E"] = se[: L - 1]
        return out

    # small operator MPOs and expectation values (Binder ratio, structure factor)
    def spin_sum_mpo(self, L: int, power: int = 1) -> MPO:
        h = C.c_void_p()
        _check(self, _lib.xtrg_spin_sum_mpo(self.h, L, power, C.byref(h)))
        return MPO(self, h)

    def correlation_mpo(self, L: int, center: int, weights: Sequence[float]) -> MPO:
        w = np.ascontiguousarray(np.array(weights, dtype=np.float64))
        if w.shape != (L,):
            raise ValueError("one weight per site")
        h = C.c_void_p()
        _check(self, _lib.xtrg_correlation_mpo(self.h, L, center, w.ctypes.data_as(C.POINTER(C.c_double)),
                                               C.byref(h)))
        return MPO(self, h)

    def expectation(self, rho: MPO, ops: Sequence[MPO]):
        """(<O_1..O_n> at beta = tau_n, at beta = 2 tau_n) for n = 1 or 2 operators."""
        arr = (C.c_void_p * len(ops))(*[o.h for o in ops])
        a, b = C.c_double(), C.c_double()
        _check(self, _lib.xtrg_expectation(self.h, rho.h, len(ops), arr, C.byref(a), C.byref(b)))
        return a.value, b.value

    def binder_ratio(self, rho: MPO):
        """U_4 = <M^2>^2 / <M^4> of M = S^z_tot (Eq. Binder) at beta = tau_n and 2 tau_n."""
        L = rho.shape()[0]
        M2 = self.spin_sum_mpo(L, 2)
        m2 = self.expectation(rho, [M2])
        m4 = self.expectation(rho, [M2, M2])
        M2.close()
        return tuple(x * x / y for x, y in zip(m2, m4))

    def structure_factor(self, rho: MPO, positions, q, center: int):
        """Re S(q) = sum_j cos(q . (r_j - r_center)) <S_center . S_j> (Sec. III.D)
        at beta = tau_n and 2 tau_n; positions: one coordinate vector per site."""
        r = np.asarray(positions, dtype=np.float64)
        w = np.cos((r - r[center]) @ np.asarray(q, dtype=np.float64))
        O = self.correlation_mpo(len(r), center, w)
        out = self.expectation(rho, [O])
        O.close()
        return out

    # serving: the library's continuous-batching loop (include/xtrg.h)
    def serve_set_lanes(self, n: int) -> None:
        """Lanes of the serving loop (1 to 4; not while a lane has work)."""
        _check(self, _lib.xtrg_serve_set_lanes(self.h, int(n)))

    def serve_submit(self, request: dict) -> int:
        """Queue one XTRG run (the JSON fields of xtrg_serve_submit); returns its id."""
        import json
        rid = C.c_ulonglong()
        _check(self, _lib.xtrg_serve_submit(self.h, json.dumps(request).encode(), C.byref(rid)))
        return rid.value

    def serve_poll(self, rid: int, cap: int = 1 << 20):
        """The run's result dict once it is finished (or failed); while it is
        queued or running, {"busy": True, "state", "doublings"} (its progress)."""
        import json
        buf = C.create_string_buffer(cap)
        rc = _lib.xtrg_serve_poll(self.h, rid, buf, cap)
        if rc == -5:                               # XTRG_EBUSY: queued or running
            d = json.loads(buf.value.decode()) if buf.value else {}
            return {"busy": True, "state": d.get("state", "queued"), "doublings": d.get("doublings", 0)}
        if rc != 0 and cap < (1 << 26):
            return self.serve_poll(rid, cap * 8)   # grow the buffer for long runs
        _check(self, rc)
        return json.loads(buf.value.decode())

    def profile(self, on: bool = True):
        _check(self, _lib.xtrg_profile_enable(self.h, int(on)))

    def profile_report(self) -> Dict[str, Dict[str, float]]:
        import json
        buf = C.create_string_buffer(4096)
        _check(self, _lib.xtrg_profile_report(self.h, buf, 4096))
        return json.loads(buf.value.decode())

    # kernel-level entry points (device pointers as Python ints)
    def dgemm(self, M, N, K, transA, transB, A, lda, B, ldb, Cp, ldc):
        _check(self, _lib.xtrg_dgemm(self.h, M, N, K, int(transA), int(transB), C.c_void_p(A), lda,
                                     C.c_void_p(B), ldb, C.c_void_p(Cp), ldc))

    def dgemm_noalloc(self, M, N, K, transA, transB, A, lda, B, ldb, Cp, ldc):
        """xtrg_dgemm without device allocation (enqueued; does not wait)."""
        _check(self, _lib.xtrg_dgemm_noalloc(self.h, M, N, K, int(transA), int(transB), C.c_void_p(A), lda,
                                             C.c_void_p(B), ldb, C.c_void_p(Cp), ldc))

    def sgemm(self, M, N, K, transA, transB, A, lda, B, ldb, Cp, ldc, c_double=True):
        _check(self, _lib.xtrg_sgemm(self.h, M, N, K, int(transA), int(transB), C.c_void_p(A), lda,
                                     C.c_void_p(B), ldb, C.c_void_p(Cp), ldc, int(c_double)))

    def gemm_bf16x3(self, M, N, K, transA, transB, A, lda, B, ldb, Cp, ldc, c_double=True):
        _check(self, _lib.xtrg_gemm_bf16x3(self.h, M, N, K, int(transA), int(transB), C.c_void_p(A), lda,
                                           C.c_void_p(B), ldb, C.c_void_p(Cp), ldc, int(c_double)))

    def dsvd_left(self, length, p, Y, sigma, k=0, U=None):
        _check(self, _lib.xtrg_dsvd_left(self.h, length, p, C.c_void_p(Y), C.c_void_p(sigma), k,
                                         C.c_void_p(U) if U else None))

    def dsvd_left_qr(self, length, p, Y, sigma, k=0, U=None):
        """The first-visit route (pivoted QR, Jacobi on [R^T; I]); returns keff."""
        ke = C.c_int()
        _check(self, _lib.xtrg_dsvd_left_qr(self.h, length, p, C.c_void_p(Y), C.c_void_p(sigma), k,
                                            C.c_void_p(U) if U else None, C.byref(ke)))
        return ke.value

    def dqrcp(self, length, p, Y, stop_rel, piv, RT):
        """Column-pivoted QR (triangular factor) of the device matrix Y; returns keff."""
        k = C.c_int()
        _check(self, _lib.xtrg_dqrcp(self.h, length, p, C.c_void_p(Y), stop_rel, C.c_void_p(piv),
                                     C.c_void_p(RT), C.byref(k)))
        return k.value


def run(ctx: Context, n_sites: int, bonds, jxy, jz, tau0: float, n_doublings: int, D: int, order: int = 1,
        n_sweeps: int = 4, degen_rtol: float = 1e-6, sv_floor: float = 1e-14, observe: bool = True,
        entropy: bool = False, precision: int = XTRG_FP64, beta_mix: float = 1.0, series_tol: float = 0.0,
        u1: bool = False):
    """Full XTRG run through the library: rho(tau0), then n_doublings doublings;
    returns per-doubling records (observables at beta = tau_n and 2 tau_n).

    rho(tau0) is the fixed-order start of xtrg_init_rho (order 1 or 2), or,
    with series_tol > 0, the series start of xtrg_settn_init to an expansion
    error below series_tol (bond <= D), which permits a larger tau0.

    precision != XTRG_FP64 applies from the doubling whose result reaches
    beta = 2 tau_{n+1} >= beta_mix; earlier doublings run in FP64.  The
    relative error a doubling leaves in ln Z enters f = -ln Z/(N beta) divided
    by beta, so the high-temperature doublings need the most precision.

    u1: charge-definite bonds throughout (xtrg_init_rho_u1, and every
    doubling factorises its two-site tensors by S^z charge blocks)."""
    H = ctx.hamiltonian_xxz(n_sites, bonds, jxy, jz)
    if series_tol > 0:
        rho, lam, _ = ctx.settn_init(H, tau0, D, 2, series_tol)
    else:
        rho, lam = ctx.init_rho(H, tau0, order, u1=u1)
    tau = tau0
    recs = []

    def rec(n, info=None):
        r = dict(n=n, tau=tau, lam=lam, bond_dims=rho.bond_dims)
        if observe:
            r["obs"] = ctx.observables(rho, lam, tau, H, n_sites, entropy=entropy)
        if info is not None:
            r["info"] = info
        return r

    recs.append(rec(0))
    for n in range(1, n_doublings + 1):
        prec = precision if 4 * tau >= beta_mix else XTRG_FP64
        new, info = ctx.square_compress(rho, D, n_sweeps, degen_rtol, sv_floor, precision=prec, u1=u1)
        rho.close()
        rho = new
        lam = 2 * lam + info["dlog_norm"]
        tau = 2 * tau
        recs.append(rec(n, info))
    rho.close()
    H.close()
    return recs
