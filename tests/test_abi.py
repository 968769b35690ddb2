"""CPU checks of the boundary: the built library loads and exports every entry point
that include/dnqs.h declares, and host-side argument checks need no GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dnqs.h")
LIB = os.path.join(ROOT, "paper_2601_21310_amd", "libdnqs.so")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dnqs_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2601_21310_amd import build
        build.build()
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 15
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB], text=True)
    exported = set(re.findall(r"\b(dnqs_[a-z0-9_]+)\b", out))
    missing = [s for s in syms if s not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for s in syms:
        getattr(lib, s)


def test_param_count_host_only(lib):
    from paper_2601_21310_amd._native import Net
    lib.dnqs_param_count.argtypes = [C.POINTER(Net), C.c_int, C.c_int, C.c_int]
    lib.dnqs_param_count.restype = C.c_int64
    for widths, M, na, nb, want in [((16, 64, 64, 128), 8, 4, 4, 13696), ((32, 256, 256, 320), 16, 5, 5, 156800),
                                    ((56, 512, 512, 512, 784), 28, 7, 7, 957472),
                                    ((112, 1024, 1024, 2688), 56, 12, 12, 3923200)]:
        net = Net.from_widths(widths)
        assert lib.dnqs_param_count(C.byref(net), M, na, nb) == want
    bad = Net.from_widths((16, 64, 64, 127))
    assert lib.dnqs_param_count(C.byref(bad), 8, 4, 4) == -1
    assert lib.dnqs_param_count(C.byref(Net.from_widths((16, 64, 128))), 65, 4, 4) == -1


def test_null_context_is_rejected(lib):
    lib.dnqs_set_integrals.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                       C.c_double]
    assert lib.dnqs_set_integrals(None, 0, 4, 2, 2, None, None, 0.0) == -1
    lib.dnqs_last_error.restype = C.c_char_p
    lib.dnqs_last_error.argtypes = [C.c_void_p]
    assert isinstance(lib.dnqs_last_error(None), bytes)
