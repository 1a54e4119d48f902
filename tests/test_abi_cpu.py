"""CPU-only checks of the C-ABI library: it builds for gfx950, loads without a
GPU, and exports every function include/gabp.h declares (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(gabp_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    # build.py by path: importing the package would load the library first
    import importlib.util
    path = os.path.join(ROOT, "paper_0810_1119_amd", "build.py")
    spec = importlib.util.spec_from_file_location("gabp_hip_build", path)
    build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(build)
    if not os.path.exists(build.LIB):
        build.build()
    return ctypes.CDLL(build.LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("gabp_solve", "gabp_solve_batched", "gabp_residual", "gabp_plan_create"):
        assert required in names, required


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_default_opts_without_gpu(lib):
    lib.gabp_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.gabp_version()
    from paper_0810_1119_amd import gabp_default_opts
    o = gabp_default_opts()
    assert o.msg_fp32 == 1 and o.tol == 1e-8 and o.check_every == 0  # automatic interval
