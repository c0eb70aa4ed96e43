"""The C-ABI library loads and exports every function include/*.h
declares; calls that need no GPU behave (no compute is run here)."""
import ctypes as C
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
LIB = os.path.join(ROOT, "paper_2604_13880_amd", "libcg.so")


def declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(cg_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2604_13880_amd import build
        build.build()
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(HEADERS) >= 2 and len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_abi():
    from paper_2604_13880_amd import binding
    assert sorted(binding.exported_symbols()) == declared()


def test_inim_size_and_argument_checks_without_gpu(lib):
    f = lib.cg_inim_size
    f.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    p, tb, mb = C.c_int64(), C.c_size_t(), C.c_size_t()
    assert f(1024, 0, C.byref(p), C.byref(tb), C.byref(mb)) == 0
    assert p.value >= 1025 and p.value % 64 == 0
    assert tb.value == 4 * 1025 * p.value and mb.value == 4 * 2049
    assert f(1024, 2, C.byref(p), C.byref(tb), C.byref(mb)) == 0 and tb.value == 8 * 1025 * p.value
    assert f(1000, 0, C.byref(p), C.byref(tb), C.byref(mb)) == -1      # not a power of two
    assert f(8, 0, None, None, None) == -1                               # below 16
    assert f(16384, 0, None, None, None) == -1                           # above 8192
    assert f(64, 3, None, None, None) == 0                               # double accumulation, float tables
    assert f(64, 4, None, None, None) == -1                              # bad precision


def test_create_fails_cleanly_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = C.c_void_p()
    lib.cg_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
    assert lib.cg_create(0, C.byref(h)) != 0 and not h.value
