"""The C ABI library loads and exports every symbol include/rqlp.h declares;
argument checks that need no GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2209_12464_amd import build, rqlp
    if not os.path.exists(rqlp.LIB_PATH):
        build.build()
    return rqlp._lib()


def _declared():
    text = open(os.path.join(ROOT, "include", "rqlp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rqlp_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_2209_12464_amd import rqlp
    assert sorted(rqlp.exported_symbols()) == _declared()


def test_status_strings(lib):
    for code in range(6):
        s = lib.rqlp_status_string(code)
        assert isinstance(s, bytes) and len(s) > 3
    assert lib.rqlp_status_string(99) == b"unknown status"


def test_workspace_size_argument_checks(lib):
    assert lib.rqlp_workspace_size(8000, 8000, 200, 10, 1, 1) > 0
    assert lib.rqlp_workspace_size(8000, 8000, 0, 10, 1, 1) == 0        # k < 1
    assert lib.rqlp_workspace_size(100, 50, 45, 10, 0, 1) == 0          # d > min(m, n)
    assert lib.rqlp_workspace_size(1000, 1000, 250, 10, 0, 1) > 0       # d = 260: wide tiles
    assert lib.rqlp_workspace_size(2000, 2000, 540, 5, 0, 1) == 0       # d > 544
    assert lib.rqlp_workspace_size_csr(1000, 1000, 5000, 250, 10, 0, 1) == 0  # CSR: d > 256
    assert lib.rqlp_workspace_size(100, 50, 5, 1, -1, 1) == 0           # q < 0
    assert lib.rqlp_workspace_size(100, 50, 5, 1, 0, 7) == 0            # bad precision
    # bfloat16 products: dense only, and the workspace adds the bf16 copies of A and A^T
    bf = lib.rqlp_workspace_size(1000, 800, 20, 5, 0, 2)
    f32 = lib.rqlp_workspace_size(1000, 800, 20, 5, 0, 1)
    assert bf >= f32 + 2 * 1000 * 800 * 2
    assert lib.rqlp_workspace_size_csr(1000, 800, 5000, 20, 5, 0, 2) == 0
    small = lib.rqlp_workspace_size(1000, 800, 20, 5, 0, 0)
    big = lib.rqlp_workspace_size(2000, 800, 20, 5, 0, 0)
    assert 0 < small < big
    assert lib.rqlp_workspace_size_csr(100000, 50000, 5000000, 100, 10, 1, 1) > 0
    assert lib.rqlp_workspace_size_csr(100, 50, -1, 5, 1, 0, 1) == 0


def test_null_context_is_rejected(lib):
    nul = ctypes.c_void_p(0)
    st = lib.rqlp_decompose(nul, ctypes.c_void_p(16), 10, 10, 10, 2, 1, 0, 1, 0, ctypes.c_void_p(16),
                            ctypes.c_void_p(16), ctypes.c_void_p(16), nul, 0, nul)
    assert st == 1
    st = lib.rqlp_decompose_csr(nul, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 10, 10, 5,
                                2, 1, 0, 1, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                nul, 0, nul)
    assert st == 1
    st = lib.rqlp_decompose_noalloc(nul, ctypes.c_void_p(16), 10, 10, 10, 2, 1, 0, 1, 0, ctypes.c_void_p(16),
                                    ctypes.c_void_p(16), ctypes.c_void_p(16), nul)
    assert st == 1
    assert lib.rqlp_create(None, 0) == 1
    assert lib.rqlp_destroy(nul) == 0
    assert lib.rqlp_set_timing(nul, 1) == 1
