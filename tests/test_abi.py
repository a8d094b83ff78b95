"""The C-ABI library loads and exports every function include/bsim.h
declares (no GPU needed: nothing is called)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsim.h")
LIB = os.path.join(ROOT, "paper_2111_12493_amd", "libbsim.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bsim_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("bsim_ctx_create", "bsim_summarize", "bsim_apply_updates",
                     "bsim_batch_summarize", "bsim_result_free", "bsim_state_free"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbsim.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbsim.so not built")
def test_binding_declares_the_same_symbols():
    from paper_2111_12493_amd import binding
    assert sorted(binding.EXPORTS) == declared_functions()
