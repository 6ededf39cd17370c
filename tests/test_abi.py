"""Host-side checks of the C ABI: the built library loads and exports every function
that include/rb.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rb.h")
LIB = os.path.join(ROOT, "paper_1804_06363_amd", "librb.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rb_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("rb_solve_batch", "rb_offline_build", "rb_solve_multi",
                     "rb_basis_from_host", "rb_problem_create_stencil", "rb_ctx_create"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librb.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librb.so not built")
def test_binding_lists_match_header():
    from paper_1804_06363_amd import rb
    assert sorted(rb.EXPORTED) == declared_functions()
    assert rb.rb_version().decode().startswith("rb ")
