"""The C-ABI library loads and exports every entry point include/adef2.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adef2.h")
LIB = os.path.join(ROOT, "paper_2606_17971_amd", "libadef2.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adef2_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2606_17971_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ("adef2_set_reference", "adef2_restrict", "adef2_solve", "adef2_solve_batched",
                 "adef2_compact", "adef2_create", "adef2_destroy", "adef2_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (adef2_\w+)", out))
    assert set(declared()) <= exported
    # nothing beyond the header is exported under the library prefix
    assert exported <= set(declared())


def test_binding_covers_the_header():
    import paper_2606_17971_amd.binding as b
    assert set(b.EXPORTS) == set(declared())


def test_defaults_without_gpu(lib):
    import paper_2606_17971_amd.binding as b
    o = b.default_opts()
    assert o.tau_cond == 1e10 and o.maxit == 100000 and o.precision == b.FP64
    assert abs(o.drop_rel - 1e-6) < 1e-20 and o.check_every > 0


def test_null_context_errors_without_gpu(lib):
    import paper_2606_17971_amd.binding as b
    assert b._lib.adef2_destroy(None) == b.E_ARG
    assert b._lib.adef2_solve(None, None, None, 1e-8, None, None, None, None) == b.E_ARG
