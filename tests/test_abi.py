"""The C-ABI library loads, exports every symbol include/se2n.h declares, and
rejects bad arguments on the host (no GPU work is issued by these calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "se2n.h")
LIB = os.path.join(ROOT, "paper_1304_2062_amd", "libse2n.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(se2n_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is not built (run python -m paper_1304_2062_amd.build)")
    L = ctypes.CDLL(LIB)
    L.se2n_last_error.restype = ctypes.c_char_p
    L.se2n_workspace_bytes.restype = ctypes.c_size_t
    L.se2n_workspace_bytes.argtypes = [ctypes.c_void_p]
    return L


def test_header_declares_the_paper_calls():
    names = _declared()
    for want in ("se2n_plan_create", "se2n_plan_destroy", "se2n_workspace_bytes", "se2n_precompute",
                 "se2n_orient", "se2n_lift", "se2n_diffuse", "se2n_project", "se2n_inpaint",
                 "se2n_last_error"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(se2n_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        getattr(lib, n)


@pytest.mark.parametrize("M,N,dt,code", [
    (100, 16, 0, -1), (8, 16, 0, -1), (8192, 16, 0, -1), (18, 16, 0, -1), (54, 16, 0, -1), (64, 2, 0, -1),
    (64, 66, 0, -1), (64, 65, 0, -1), (64, 3, 0, -1), (64, 16, 7, -1),
])
def test_plan_create_rejects_bad_sizes(lib, M, N, dt, code):
    h = ctypes.c_void_p()
    rc = lib.se2n_plan_create(ctypes.byref(h), M, N, dt)
    assert rc == code
    assert lib.se2n_last_error().decode()
    assert h.value is None


def test_null_arguments_are_rejected(lib):
    assert lib.se2n_plan_create(None, 64, 16, 0) == -1
    assert lib.se2n_plan_destroy(None) == -1
    assert lib.se2n_workspace_bytes(None) == 0
    null = ctypes.c_void_p()
    d = ctypes.c_double
    assert lib.se2n_precompute(null, d(1.0), d(1.0), 10, 0, null) == -1
    assert b"NULL" in lib.se2n_last_error()
    assert lib.se2n_diffuse(null, null, d(1.0), d(1.0), 10, 0, null, null) == -1
    assert lib.se2n_inpaint(null, null, null, d(2.0), d(1.0), d(1.0), 10, 0, 0, null, null, null, null, null) == -1
    assert lib.se2n_orient(null, null, null, d(2.0), null, null, null) == -1
    assert lib.se2n_lift(null, null, null, null, null, null) == -1
    assert lib.se2n_project(null, null, 0, null, null) == -1


def test_error_message_is_cleared_by_a_good_call(lib):
    lib.se2n_plan_create(None, 64, 16, 0)
    assert lib.se2n_last_error().decode() != ""
    lib.se2n_version.restype = ctypes.c_char_p
    assert lib.se2n_version().startswith(b"se2n")
