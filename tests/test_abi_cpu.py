"""Host-side checks of the C ABI: the library loads, exports every entry
point that include/precode.h declares, and validates arguments with the
documented return codes without touching a device."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "precode.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|void|size_t|char)\s*\*?\s*(precode_\w+)\s*\(",
                                 text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1804_10987_amd import _lib
    return _lib.load()


def test_header_declares_entry_points():
    names = _declared()
    for n in ("precode_pd", "precode_fd", "precode_frame_prepare", "precode_frame_symbols", "precode_batch",
              "precode_ctx_create", "precode_validate", "precode_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_1804_10987_amd import _lib
    assert set(_declared()) == set(_lib.SIGNATURES)


def test_params_defaults(lib):
    from paper_1804_10987_amd import _lib
    p = _lib.Params()
    lib.precode_params_init(ctypes.byref(p))
    assert p.power == 1.0 and p.Es == 1.0 and p.tau == 0.125
    assert p.precision == _lib.PREC_FP32 and p.refine_steps == 0 and p.impl == _lib.IMPL_AUTO
    assert abs(p.fp64_ratio - 0.5) < 1e-7


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -99):
        assert lib.precode_strerror(code)


def _validate(lib, arch=0, rho=0.8, sizes=(32, 32), mode=1, B=64, U=8, n_sc=64, K=14, prm=None):
    arr = (ctypes.c_int * len(sizes))(*sizes)
    return lib.precode_validate(arch, rho, arr, len(sizes), mode, B, U, n_sc, K,
                                ctypes.byref(prm) if prm is not None else None)


@pytest.mark.parametrize("arch", [0, 1])
def test_validate_accepts_paper_shapes(lib, arch):
    assert _validate(lib, arch) == 0
    assert _validate(lib, arch, sizes=(32,) * 8, B=256, U=16, n_sc=1200) == 0
    assert _validate(lib, arch, sizes=(32,) * 16, B=512, U=32, n_sc=3300) == 0
    assert _validate(lib, arch, n_sc=0) == 0 and _validate(lib, arch, K=0) == 0
    assert _validate(lib, arch, mode=0, rho=float("nan")) == 0  # rho ignored for ZF


@pytest.mark.parametrize("kw,code", [
    (dict(sizes=(32, 31)), -1),                 # sum != B
    (dict(sizes=(64, 0), B=64), -1),            # empty cluster
    (dict(sizes=(16, 16, 32, 0)), -1),
    (dict(U=0), -1), (dict(B=0, sizes=(1,)), -1), (dict(n_sc=-1), -1), (dict(K=-1), -1),
    (dict(rho=-0.1), -1), (dict(rho=float("nan")), -1), (dict(rho=float("inf")), -1),
    (dict(mode=2), -1), (dict(arch=3), -1),
    (dict(U=65), -2), (dict(B=8192, sizes=(8192,)), -2), (dict(K=5000), -2),
    (dict(sizes=(1,) * 300, B=300), -2),
])
def test_validate_rejects(lib, kw, code):
    assert _validate(lib, **kw) == code


def test_validate_params(lib):
    from paper_1804_10987_amd import _lib
    for field, bad in [("power", 0.0), ("power", float("nan")), ("Es", -1.0), ("tau", -0.5),
                       ("precision", 7), ("refine_steps", 2), ("fp64_ratio", float("inf")), ("impl", 9)]:
        p = _lib.Params()
        lib.precode_params_init(ctypes.byref(p))
        setattr(p, field, bad)
        assert _validate(lib, prm=p) == -1, field


def test_null_context_rejected(lib):
    arr = (ctypes.c_int * 2)(32, 32)
    assert lib.precode_pd(None, None, None, 0.8, arr, 2, 1, 64, 8, 64, 14, None, None, None, None, None) == -1
    assert lib.precode_fd(None, None, None, 0.8, arr, 2, 1, 64, 8, 64, 14, None, None, None, None, None) == -1
    out = ctypes.c_void_p()
    assert lib.precode_frame_symbols(None, None, None, 1, None, None) == -1
    assert lib.precode_ctx_create(0, 0, None) == -1
    assert lib.precode_batch(None, None, 0, 0, None) == -1
    assert out.value is None


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes mirror has the size and field offsets the C compiler gives
    the header's struct (a host C program prints them)."""
    import subprocess

    from paper_1804_10987_amd import _lib

    structs = {"precode_params": _lib.Params, "precode_job": _lib.Job, "precode_serve_job": _lib.ServeJob,
               "precode_serve_config": _lib.ServeConfig, "precode_serve_stats": _lib.ServeStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "precode.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname + " size"]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[cname + "." + f]) == getattr(py, f).offset, (cname, f)
