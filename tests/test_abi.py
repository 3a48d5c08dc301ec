"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and its host-only helpers behave as documented."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(kc_[a-z0-9_]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2301_00061_amd import _lib
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"kc_lower_bound", "kc_objective", "kc_tighten", "kc_reduce"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), f"libkc.so does not export {n}"
    from paper_2301_00061_amd import _lib
    assert set(_lib.EXPORTS) == names


def test_margins(lib):
    for d in range(1, 17):
        u = 2.0 ** -24
        g = (d + 3) * u / (1 - (d + 3) * u)
        assert lib.kc_rel_margin(d) == g
        assert lib.kc_abs_margin(d) == (d + 3) * 2.0 ** -126
    # every margin of the workloads is below the 1e-6 relative gap tolerance
    assert lib.kc_rel_margin(5) < 1e-6


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    rc = lib.kc_create(C.byref(h), 0, None)
    assert rc != 0 and not h.value
    lib.kc_destroy(None)
    assert lib.kc_last_error(None) == b"null handle"


def test_calls_reject_null_handle(lib):
    from paper_2301_00061_amd import _lib
    P = _lib.Points(0, 10, 16, 2, 0)
    assert lib.kc_lower_bound(None, C.byref(P), None, None, None, None, None, None) == _lib.KC_EINVAL
    assert lib.kc_objective(None, C.byref(P), 1, 1, None, 32, None, None, None) == _lib.KC_EINVAL
