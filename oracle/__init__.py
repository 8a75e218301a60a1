"""FP64 CPU oracle for feedforward decentralized precoding (arXiv:1804.10987).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of ``bench.py``; never by the product library, which shares
no code with it.

``oracle.c`` holds the plain-loop FP64 implementation of PD (Sec. III-B) and
FD (Sec. III-C) precoding; this module compiles it with gcc and wraps it with
ctypes.  ``exact.py`` holds an exact Gaussian-rational brute force used to pin
the C oracle on tiny integer inputs.

Conventions (see oracle.c): H is [n_sc][B][U] (Hermitian transpose of the
paper's U x B downlink channel), s is [K][n_sc][U], x is [K][n_sc][B].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc -O2 -fopenmp, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                        "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_pd.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ip, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, dp, dp, ip, dp, dp]
        lib.oracle_pd.restype = ctypes.c_int
        lib.oracle_fd.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ip, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, ip, dp, dp]
        lib.oracle_fd.restype = ctypes.c_int
        lib.oracle_central.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       dp, dp, ip]
        lib.oracle_central.restype = ctypes.c_int
        lib.oracle_mrt.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   dp, dp, ip, dp]
        lib.oracle_mrt.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _prep(H, s, sizes):
    H = np.ascontiguousarray(np.asarray(H), dtype=np.complex128)
    s = np.ascontiguousarray(np.asarray(s), dtype=np.complex128)
    if H.ndim == 2:
        H = H[None]
    if s.ndim == 1:
        s = s[None, None]
    elif s.ndim == 2:
        s = s[:, None] if H.shape[0] == 1 else s[None]
    n_sc, B, U = H.shape
    K = s.shape[0]
    assert s.shape == (K, n_sc, U), (s.shape, H.shape)
    sizes = np.ascontiguousarray(np.asarray(sizes if sizes is not None else [B], dtype=np.int32))
    return H, s, sizes, n_sc, B, U, K


def pd(H, s, kappa, sizes=None, zf=False, power=1.0, Es=1.0, threads=None, intermediates=False):
    """PD-WF (zf=False) or PD-ZF precoding in FP64 (Sec. III-B, Thm. 1, Lemma 1).

    Returns (x [K][n_sc][B] complex128, beta [n_sc], status [n_sc]) and, with
    intermediates=True, also (G, A^-1) each [n_sc][U][U].
    """
    H, s, sizes, n_sc, B, U, K = _prep(H, s, sizes)
    x = np.zeros((K, n_sc, B), np.complex128)
    beta = np.zeros(n_sc, np.float64)
    status = np.zeros(n_sc, np.int32)
    G = np.zeros((n_sc, U, U), np.complex128) if intermediates else None
    Ai = np.zeros((n_sc, U, U), np.complex128) if intermediates else None
    rc = _load().oracle_pd(_dptr(H.view(np.float64)), _dptr(s.view(np.float64)), B, U, n_sc, K,
                           _iptr(sizes), len(sizes), float(kappa), int(bool(zf)), float(power),
                           float(Es), int(threads or os.cpu_count() or 1),
                           _dptr(x.view(np.float64)), _dptr(beta), _iptr(status),
                           _dptr(None if G is None else G.view(np.float64)),
                           _dptr(None if Ai is None else Ai.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle_pd: cluster sizes do not sum to B")
    if intermediates:
        return x, beta, status, G, Ai
    return x, beta, status


def _per_cluster(v, C, what):
    if v is None:
        return None
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    if a.shape != (C,):
        raise ValueError("%s: one value per cluster expected" % what)
    return a


def fd(H, s, kappa, sizes, zf=False, tau=0.125, power=1.0, Es=1.0, threads=None, tau_c=None, power_c=None):
    """FD-WF (zf=False) or FD-ZF precoding in FP64 (Sec. III-C).

    tau_c / power_c: optional per-cluster tau_c and budgets rho_c^2 (sum rho^2).
    Returns (x [K][n_sc][B] complex128, weights [n_sc][C], status [n_sc][C]).
    """
    H, s, sizes, n_sc, B, U, K = _prep(H, s, sizes)
    C = len(sizes)
    tc = _per_cluster(tau_c, C, "tau_c")
    pc = _per_cluster(power_c, C, "power_c")
    if pc is not None and (not (pc > 0).all() or abs(pc.sum() - power) > 1e-9 * power):
        raise ValueError("power_c: positive budgets summing to power expected")
    x = np.zeros((K, n_sc, B), np.complex128)
    w = np.zeros((n_sc, C), np.float64)
    status = np.zeros((n_sc, C), np.int32)
    rc = _load().oracle_fd(_dptr(H.view(np.float64)), _dptr(s.view(np.float64)), B, U, n_sc, K,
                           _iptr(sizes), C, float(kappa), int(bool(zf)), float(tau), float(power),
                           float(Es), int(threads or os.cpu_count() or 1),
                           _dptr(x.view(np.float64)), _dptr(w), _iptr(status), _dptr(tc), _dptr(pc))
    if rc != 0:
        raise ValueError("oracle_fd: cluster sizes do not sum to B")
    return x, w, status


def central(H, s, kappa, power=1.0, Es=1.0, threads=None):
    """Centralized WF precoding in the B x B form of Theorem 1 (eq.
    originalQmatrix, eq. precodingfactor), FP64.  kappa > 0.

    Returns (x [K][n_sc][B] complex128, beta [n_sc], status [n_sc]).
    """
    H, s, _, n_sc, B, U, K = _prep(H, s, None)
    x = np.zeros((K, n_sc, B), np.complex128)
    beta = np.zeros(n_sc, np.float64)
    status = np.zeros(n_sc, np.int32)
    rc = _load().oracle_central(_dptr(H.view(np.float64)), _dptr(s.view(np.float64)), B, U, n_sc, K,
                                float(kappa), float(power), float(Es), int(threads or os.cpu_count() or 1),
                                _dptr(x.view(np.float64)), _dptr(beta), _iptr(status))
    if rc != 0:
        raise ValueError("oracle_central: kappa must be positive")
    return x, beta, status


def mrt(H, s, sizes=None, power=1.0, Es=1.0, threads=None, power_c=None):
    """MRT with per-cluster power normalization (C = 1: centralized), FP64.

    Returns (x [K][n_sc][B] complex128, weights [n_sc][C], status [n_sc][C]).
    """
    H, s, sizes, n_sc, B, U, K = _prep(H, s, sizes)
    C = len(sizes)
    pc = _per_cluster(power_c, C, "power_c")
    x = np.zeros((K, n_sc, B), np.complex128)
    w = np.zeros((n_sc, C), np.float64)
    status = np.zeros((n_sc, C), np.int32)
    rc = _load().oracle_mrt(_dptr(H.view(np.float64)), _dptr(s.view(np.float64)), B, U, n_sc, K,
                            _iptr(sizes), C, float(power), float(Es), int(threads or os.cpu_count() or 1),
                            _dptr(x.view(np.float64)), _dptr(w), _iptr(status), _dptr(pc))
    if rc != 0:
        raise ValueError("oracle_mrt: cluster sizes do not sum to B")
    return x, w, status
