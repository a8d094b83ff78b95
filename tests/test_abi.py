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


def header_constants():
    text = open(HEADER).read()
    out = {}
    for name, val in re.findall(r"#define\s+(BSIM_[A-Z0-9_]+)\s+\(?(-?\d+)u?\)?", text):
        out[name] = int(val)
    return out


def test_binding_constants_match_the_header():
    from paper_2111_12493_amd import binding
    h = header_constants()
    pairs = {"BSIM_OK": binding.OK, "BSIM_E_INVALID": binding.E_INVALID, "BSIM_E_RANGE": binding.E_RANGE,
             "BSIM_E_NOMEM": binding.E_NOMEM, "BSIM_E_DEVICE": binding.E_DEVICE,
             "BSIM_E_UNSUPPORTED": binding.E_UNSUPPORTED, "BSIM_E_BUSY": binding.E_BUSY, "BSIM_E_IO": binding.E_IO,
             "BSIM_MEM_HOST": binding.MEM_HOST, "BSIM_MEM_DEVICE": binding.MEM_DEVICE,
             "BSIM_STOP_AT_FIXPOINT": binding.STOP_AT_FIXPOINT, "BSIM_KEEP_LEVELS": binding.KEEP_LEVELS,
             "BSIM_UNTYPED": binding.UNTYPED, "BSIM_RESULT_ON_HOST": binding.RESULT_ON_HOST,
             "BSIM_NO_SUMMARY_EDGES": binding.NO_SUMMARY_EDGES, "BSIM_BACKWARD": binding.BACKWARD,
             "BSIM_BOTH_DIRECTIONS": binding.BOTH_DIRECTIONS, "BSIM_PREV_LEVEL_EDGES": binding.PREV_LEVEL_EDGES}
    for name, val in pairs.items():
        assert h.get(name) == val, (name, h.get(name), val)
    flags = [h[n] for n in pairs if n.startswith("BSIM_") and not n.startswith(("BSIM_E_", "BSIM_OK", "BSIM_MEM"))]
    # flag bits are distinct single bits
    assert all(f and (f & (f - 1)) == 0 for f in flags) and len(set(flags)) == len(flags)
