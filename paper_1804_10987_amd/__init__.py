"""MI355X-native batched decentralized precoding (PD / FD Wiener-filter and ZF).

Thin Python binding over the C ABI of ``libprecode.so`` (include/precode.h).
PyTorch provides device memory and streams only; every step of the method
runs in the library's HIP kernels.  There is no CPU fallback: if the library
is not built, importing the binding's entry points raises.

Tensors: H [n_sc, B, U], s [K, n_sc, U], x [K, n_sc, B], all complex64 on the
GPU, contiguous.  ``rho`` is the WF regularizer kappa = U N0 / rho^2 of
Theorem 1 (ignored for ZF).
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

from . import _lib
from ._lib import (ARCH_FD, ARCH_PD, IMPL_AUTO, IMPL_FUSED, IMPL_PLAIN, PREC_FP32, PREC_FP64,  # noqa: F401
                   PREC_SPLIT_BF16, PREC_SPLIT_FP16, ST_FAIL, ST_FP64, ST_OK, WF, ZF, PrecodeError)

__all__ = ["Context", "Frame", "pd", "fd", "params", "default_context"]

_PREC = {"fp32": PREC_FP32, "split_fp16": PREC_SPLIT_FP16, "split_bf16": PREC_SPLIT_BF16, "fp64": PREC_FP64}
_IMPL = {"auto": IMPL_AUTO, "fused": IMPL_FUSED, "plain": IMPL_PLAIN}


def params(power: float = 1.0, Es: float = 1.0, tau: float = 0.125, precision="fp32", refine_steps: int = 0,
           fp64_ratio: float = 0.5, impl="auto", tau_c=None, power_c=None) -> _lib.Params:
    """Call parameters.  tau_c / power_c: optional per-cluster tau_c and
    budgets rho_c^2 (summing to power) for FD and MRT (Sec. III-C)."""
    p = _lib.Params()
    _lib.load().precode_params_init(ctypes.byref(p))
    p.power, p.Es, p.tau = power, Es, tau
    p.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    p.refine_steps = refine_steps
    p.fp64_ratio = fp64_ratio
    p.impl = _IMPL[impl] if isinstance(impl, str) else int(impl)
    keep = []
    for name, vals in (("cluster_tau", tau_c), ("cluster_power", power_c)):
        if vals is not None:
            arr = (ctypes.c_float * len(vals))(*[float(v) for v in vals])
            keep.append(arr)
            setattr(p, name, ctypes.cast(arr, ctypes.POINTER(ctypes.c_float)))
    p._keep = keep  # the host arrays live as long as the parameters
    return p


def _torch():
    import torch

    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _sizes(sizes: Sequence[int]):
    arr = (ctypes.c_int * len(sizes))(*[int(v) for v in sizes])
    return arr, len(sizes)


def _mode(mode) -> int:
    if isinstance(mode, str):
        return {"zf": ZF, "wf": WF}[mode.lower()]
    return int(mode)


def _check_tensor(t, name, shape):
    torch = _torch()
    if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous complex64 CUDA tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


class Frame:
    """Resident per-frame state (factorization, beta / weights) of one cell."""

    def __init__(self, ctx: "Context", handle: int, arch: int, H, n_sc: int, B: int, U: int, C: int):
        self.ctx, self.handle, self.arch, self.H = ctx, handle, arch, H
        self.n_sc, self.B, self.U, self.C = n_sc, B, U, C

    def symbols(self, s, x=None, stream=None):
        torch = _torch()
        nk = s.shape[0]
        _check_tensor(s, "s", (nk, self.n_sc, self.U))
        if x is None:
            x = torch.empty((nk, self.n_sc, self.B), dtype=torch.complex64, device=s.device)
        _lib.check(_lib.load().precode_frame_symbols(self.ctx.handle, self.handle, _ptr(s), nk, _ptr(x),
                                                     _stream(stream)), "precode_frame_symbols")
        return x

    def factors(self, stream=None):
        torch = _torch()
        n = self.n_sc if self.arch == ARCH_PD else self.n_sc * self.C
        scale = torch.empty(n, dtype=torch.float32, device=self.H.device)
        status = torch.empty(n, dtype=torch.int32, device=self.H.device)
        _lib.check(_lib.load().precode_frame_factors(self.ctx.handle, self.handle, _ptr(scale), _ptr(status),
                                                     _stream(stream)), "precode_frame_factors")
        if self.arch == ARCH_FD:
            scale, status = scale.view(self.n_sc, self.C), status.view(self.n_sc, self.C)
        return scale, status

    def release(self):
        if self.handle:
            _lib.check(_lib.load().precode_frame_release(self.ctx.handle, self.handle), "precode_frame_release")
            self.handle = None


class Context:
    """A library context on one device (workspace under an HBM budget)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(lib.precode_ctx_create(int(device), int(budget_bytes), ctypes.byref(h)), "precode_ctx_create")
        self.handle = h.value
        self.device = device

    def close(self):
        if self.handle:
            _lib.load().precode_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def bytes_held(self) -> int:
        return _lib.load().precode_ctx_bytes(self.handle)

    @property
    def last_impl(self) -> str:
        return {0: "none", IMPL_FUSED: "fused", IMPL_PLAIN: "plain"}[_lib.load().precode_ctx_last_impl(self.handle)]

    @property
    def last_waves(self) -> int:
        """Waves per workgroup (1, 2 or 4) of the last fused launch (autotuned shape)."""
        return _lib.load().precode_ctx_last_waves(self.handle)

    def _run(self, arch, H, s, rho, sizes, mode, prm, x, scale, status, stream, noalloc=False):
        torch = _torch()
        n_sc, B, U = H.shape
        K = s.shape[0]
        _check_tensor(H, "H", (n_sc, B, U))
        _check_tensor(s, "s", (K, n_sc, U))
        C = len(sizes)
        if x is None:
            x = torch.empty((K, n_sc, B), dtype=torch.complex64, device=H.device)
        _check_tensor(x, "x", (K, n_sc, B))
        n_scale = n_sc if arch == ARCH_PD else n_sc * C
        if scale is None:
            scale = torch.empty(n_scale, dtype=torch.float32, device=H.device)
        if status is None:
            status = torch.empty(n_scale, dtype=torch.int32, device=H.device)
        arr, C = _sizes(sizes)
        prm = prm if prm is not None else params()
        name = "precode_pd_noalloc" if noalloc else ("precode_pd" if arch == ARCH_PD else "precode_fd")
        fn = getattr(_lib.load(), name)
        _lib.check(fn(self.handle, _ptr(H), _ptr(s), float(rho), arr, C, _mode(mode), B, U, n_sc, K,
                      ctypes.byref(prm), _ptr(x), _ptr(scale), _ptr(status), _stream(stream)), name)
        if arch == ARCH_FD:
            scale, status = scale.view(n_sc, C), status.view(n_sc, C)
        return x, scale, status

    def pd(self, H, s, rho, sizes, mode="wf", prm=None, x=None, beta=None, status=None, stream=None):
        """PD precoding (Sec. III-B).  Returns (x, beta [n_sc], status [n_sc])."""
        return self._run(ARCH_PD, H, s, rho, sizes, mode, prm, x, beta, status, stream)

    def pd_noalloc(self, H, s, rho, sizes, mode="wf", prm=None, x=None, beta=None, status=None, stream=None):
        """precode_pd_noalloc: PD precoding whose workspace comes from the
        library's fixed per-GPU array (no device allocation by the call)."""
        return self._run(ARCH_PD, H, s, rho, sizes, mode, prm, x, beta, status, stream, noalloc=True)

    def fd(self, H, s, rho, sizes, mode="wf", prm=None, x=None, weights=None, status=None, stream=None):
        """FD precoding (Sec. III-C).  Returns (x, weights [n_sc, C], status [n_sc, C])."""
        return self._run(ARCH_FD, H, s, rho, sizes, mode, prm, x, weights, status, stream)

    def central(self, H, s, rho, prm=None, x=None, beta=None, status=None, stream=None):
        """Centralized WF in the B x B form of Theorem 1 (rho = kappa > 0).
        Returns (x, beta [n_sc], status [n_sc])."""
        torch = _torch()
        n_sc, B, U = H.shape
        K = s.shape[0]
        _check_tensor(H, "H", (n_sc, B, U))
        _check_tensor(s, "s", (K, n_sc, U))
        x = torch.empty((K, n_sc, B), dtype=torch.complex64, device=H.device) if x is None else x
        _check_tensor(x, "x", (K, n_sc, B))
        beta = torch.empty(n_sc, dtype=torch.float32, device=H.device) if beta is None else beta
        status = torch.empty(n_sc, dtype=torch.int32, device=H.device) if status is None else status
        prm = prm if prm is not None else params()
        _lib.check(_lib.load().precode_central(self.handle, _ptr(H), _ptr(s), float(rho), B, U, n_sc, K,
                                               ctypes.byref(prm), _ptr(x), _ptr(beta), _ptr(status),
                                               _stream(stream)), "precode_central")
        return x, beta, status

    def mrt(self, H, s, sizes, prm=None, x=None, weights=None, status=None, stream=None):
        """MRT with per-cluster power normalization (one cluster: centralized).
        Returns (x, weights [n_sc, C], status [n_sc, C])."""
        torch = _torch()
        n_sc, B, U = H.shape
        K = s.shape[0]
        _check_tensor(H, "H", (n_sc, B, U))
        _check_tensor(s, "s", (K, n_sc, U))
        arr, C = _sizes(sizes)
        x = torch.empty((K, n_sc, B), dtype=torch.complex64, device=H.device) if x is None else x
        _check_tensor(x, "x", (K, n_sc, B))
        weights = torch.empty(n_sc * C, dtype=torch.float32, device=H.device) if weights is None else weights
        status = torch.empty(n_sc * C, dtype=torch.int32, device=H.device) if status is None else status
        prm = prm if prm is not None else params()
        _lib.check(_lib.load().precode_mrt(self.handle, _ptr(H), _ptr(s), arr, C, B, U, n_sc, K,
                                           ctypes.byref(prm), _ptr(x), _ptr(weights), _ptr(status),
                                           _stream(stream)), "precode_mrt")
        return x, weights.view(n_sc, C), status.view(n_sc, C)

    def frame(self, arch, H, rho, sizes, mode="wf", prm=None, stream=None) -> Frame:
        """Per-frame part (Gram, factorization, beta / weights) kept resident."""
        n_sc, B, U = H.shape
        _check_tensor(H, "H", (n_sc, B, U))
        arr, C = _sizes(sizes)
        prm = prm if prm is not None else params()
        arch = {"pd": ARCH_PD, "fd": ARCH_FD}.get(arch, arch)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().precode_frame_prepare(self.handle, arch, _ptr(H), float(rho), arr, C, _mode(mode),
                                                     B, U, n_sc, ctypes.byref(prm), ctypes.byref(h),
                                                     _stream(stream)), "precode_frame_prepare")
        return Frame(self, h.value, arch, H, n_sc, B, U, C)

    def _job_struct(self, j, keep):
        torch = _torch()
        H, s = j["H"], j["s"]
        n_sc, B, U = H.shape
        K = s.shape[0]
        arch = {"pd": ARCH_PD, "fd": ARCH_FD}.get(j.get("arch", "pd"), j.get("arch", "pd"))
        sizes = list(j["sizes"])
        C = len(sizes)
        x = j.get("x")
        if x is None:
            x = torch.empty((K, n_sc, B), dtype=torch.complex64, device=H.device)
        ns = n_sc if arch == ARCH_PD else n_sc * C
        sc = j.get("scale")
        if sc is None:
            sc = torch.empty(ns, dtype=torch.float32, device=H.device)
        st = j.get("status")
        if st is None:
            st = torch.empty(ns, dtype=torch.int32, device=H.device)
        sz = (ctypes.c_int * C)(*sizes)
        keep.append(sz)
        a = _lib.Job()
        a.arch, a.mode, a.B, a.U, a.n_sc, a.K, a.C = arch, _mode(j.get("mode", "wf")), B, U, n_sc, K, C
        a.cluster_sizes = ctypes.cast(sz, ctypes.POINTER(ctypes.c_int))
        a.rho = float(j["rho"])
        a.power, a.Es, a.tau = float(j.get("power", 1.0)), float(j.get("Es", 1.0)), float(j.get("tau", 0.125))
        a.H, a.s, a.x, a.scale, a.status = _ptr(H), _ptr(s), _ptr(x), _ptr(sc), _ptr(st)
        return a, (x, sc, st)

    def serve(self, jobs, arrivals, symbol_period_s=1e-3 / 14, max_active=16, n_streams=4, precision="fp32",
              slab_bytes=1 << 30, impl="auto"):
        """Continuous-batching serving loop (precode_serve).  jobs: list of job
        dicts as for batch(); arrivals: arrival time (s) of each job.  Returns
        (outputs [(x, scale, status)], per-symbol latencies [list of arrays],
        stats dict)."""
        import numpy as np

        keep = []
        arr = (_lib.ServeJob * len(jobs))()
        outs = []
        for i, j in enumerate(jobs):
            a, o = self._job_struct(j, keep)
            arr[i].job = a
            arr[i].arrival_s = float(arrivals[i])
            arr[i].symbol_period_s = float(symbol_period_s)
            outs.append(o)
        cfg = _lib.ServeConfig()
        cfg.max_active, cfg.n_streams = int(max_active), int(n_streams)
        cfg.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
        cfg.slab_bytes = int(slab_bytes)
        cfg.impl = _IMPL[impl] if isinstance(impl, str) else int(impl)
        total = sum(int(j["s"].shape[0]) for j in jobs)
        lat = np.zeros(max(total, 1), np.float64)
        stats = _lib.ServeStats()
        _lib.check(_lib.load().precode_serve(self.handle, arr, len(jobs), ctypes.byref(cfg),
                                             lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             ctypes.byref(stats)), "precode_serve")
        per_job, o = [], 0
        for j in jobs:
            k = int(j["s"].shape[0])
            per_job.append(lat[o:o + k].copy())
            o += k
        sd = {f: getattr(stats, f) for f, _ in _lib.ServeStats._fields_}
        return outs, per_job, sd

    def _job_array(self, jobs):
        keep = []
        arr = (_lib.Job * len(jobs))()
        outs = []
        for i, j in enumerate(jobs):
            a, o = self._job_struct(j, keep)
            arr[i] = a
            outs.append(o)
        return arr, outs, keep

    def batch(self, jobs, precision="fp32", stream=None):
        """Heterogeneous batch: jobs is a list of dicts with keys arch, mode,
        H, s, rho, sizes and optional x, scale, status, power, Es, tau.
        Outputs are allocated when absent; returns the list of (x, scale, status)."""
        arr, outs, keep = self._job_array(jobs)
        prec = _PREC[precision] if isinstance(precision, str) else int(precision)
        _lib.check(_lib.load().precode_batch(self.handle, arr, len(jobs), prec, _stream(stream)), "precode_batch")
        return outs

    def batch_plan(self, jobs, precision="fp32"):
        """Records the batch's launches into a HIP graph (precode_batch_plan_*);
        returns a BatchPlan whose launch(stream) replays it with the same
        buffers.  Outputs are allocated when absent (plan.outputs)."""
        arr, outs, keep = self._job_array(jobs)
        prec = _PREC[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().precode_batch_plan_create(self.handle, arr, len(jobs), prec, ctypes.byref(h)),
                   "precode_batch_plan_create")
        return BatchPlan(self, h.value, jobs, outs)


class BatchPlan:
    """A recorded batch (HIP graph); keeps the job tensors alive."""

    def __init__(self, ctx, handle, jobs, outputs):
        self.ctx, self.handle, self.jobs, self.outputs = ctx, handle, jobs, outputs

    @property
    def launches(self):
        return _lib.load().precode_batch_plan_launches(self.handle)

    @property
    def fused_jobs(self):
        """Jobs with n_sc > 0 the plan runs on the fused kernels."""
        return _lib.load().precode_batch_plan_fused_jobs(self.handle)

    def launch(self, stream=None):
        _lib.check(_lib.load().precode_batch_plan_launch(self.handle, _stream(stream)), "precode_batch_plan_launch")

    def destroy(self):
        if self.handle:
            _lib.check(_lib.load().precode_batch_plan_destroy(self.handle), "precode_batch_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def autotune_reset():
    """precode_autotune_reset: forget the process's tuned launch shapes; the
    next call of each problem shape reads the tuning cache file again."""
    _lib.load().precode_autotune_reset()


_default = {}


def default_context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def pd(H, s, rho, sizes, mode="wf", **kw):
    """PD precoding with the device's default context.  See Context.pd."""
    prm = kw.pop("prm", None)
    if prm is None and kw:
        prm = params(**{k: kw.pop(k) for k in list(kw) if k in params.__code__.co_varnames})
    return default_context(H.device.index or 0).pd(H, s, rho, sizes, mode, prm, **kw)


def fd(H, s, rho, sizes, mode="wf", **kw):
    """FD precoding with the device's default context.  See Context.fd."""
    prm = kw.pop("prm", None)
    if prm is None and kw:
        prm = params(**{k: kw.pop(k) for k in list(kw) if k in params.__code__.co_varnames})
    return default_context(H.device.index or 0).fd(H, s, rho, sizes, mode, prm, **kw)


# ---------------------------------------------------------------------------
# The UE side of the uncoded-BER link (precode_qam_map, precode_ue_receive,
# precode_ue_gain, precode_qam_errors)
# ---------------------------------------------------------------------------
def _check_labels(t, name):
    torch = _torch()
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous int32 CUDA tensor" % name)


def qam_map(labels, order: int, s=None, stream=None):
    """Gray-labelled unit-energy square QAM points of int32 labels (any shape)."""
    torch = _torch()
    _check_labels(labels, "labels")
    s = torch.empty(labels.shape, dtype=torch.complex64, device=labels.device) if s is None else s
    _check_tensor(s, "s", tuple(labels.shape))
    _lib.check(_lib.load().precode_qam_map(_ptr(labels), labels.numel(), int(order), _ptr(s), _stream(stream)),
               "precode_qam_map")
    return s


def ue_receive(H, x, noise=None, N0: float = 0.0, scale=None, s_hat=None, stream=None):
    """s_hat [K, n_sc, U] = scale[n] (H_dl x + sqrt(N0) noise), H_dl = H^H."""
    torch = _torch()
    n_sc, B, U = H.shape
    K = x.shape[0]
    _check_tensor(H, "H", (n_sc, B, U))
    _check_tensor(x, "x", (K, n_sc, B))
    if noise is not None:
        _check_tensor(noise, "noise", (K, n_sc, U))
    if scale is not None and (scale.dtype != torch.float32 or tuple(scale.shape) != (n_sc,) or not scale.is_cuda):
        raise ValueError("scale must be a float32 CUDA tensor [n_sc]")
    s_hat = torch.empty((K, n_sc, U), dtype=torch.complex64, device=H.device) if s_hat is None else s_hat
    _check_tensor(s_hat, "s_hat", (K, n_sc, U))
    _lib.check(_lib.load().precode_ue_receive(_ptr(H), _ptr(x), _ptr(noise), float(N0), _ptr(scale), B, U, n_sc,
                                              K, _ptr(s_hat), _stream(stream)), "precode_ue_receive")
    return s_hat


def ue_gain(y_pilot, N0: float, Es: float = 1.0, beta=None, stream=None):
    """Joint MSE-optimal UE factor [n_sc] from noise-free pilot responses [U, n_sc, U]."""
    torch = _torch()
    U, n_sc, U2 = y_pilot.shape
    _check_tensor(y_pilot, "y_pilot", (U, n_sc, U))
    beta = torch.empty(n_sc, dtype=torch.float32, device=y_pilot.device) if beta is None else beta
    _lib.check(_lib.load().precode_ue_gain(_ptr(y_pilot), float(N0), float(Es), U, n_sc, _ptr(beta),
                                           _stream(stream)), "precode_ue_gain")
    return beta


def qam_errors(s_hat, labels, order: int, count=None, labels_out=None, stream=None):
    """Adds the bit errors of the nearest-point decisions of s_hat against
    labels to the int64 device counter `count` (created zeroed if None);
    returns (count, labels_out)."""
    torch = _torch()
    _check_labels(labels, "labels")
    _check_tensor(s_hat, "s_hat", tuple(labels.shape))
    if count is None:
        count = torch.zeros(1, dtype=torch.int64, device=labels.device)
    if labels_out is not None:
        _check_labels(labels_out, "labels_out")
    _lib.check(_lib.load().precode_qam_errors(_ptr(s_hat), _ptr(labels), labels.numel(), int(order),
                                              _ptr(labels_out), _ptr(count), _stream(stream)), "precode_qam_errors")
    return count, labels_out
