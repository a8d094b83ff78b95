"""Table capacities at the sizes where 32-bit slot arithmetic ends (CPU).

The library sizes its open-addressing tables (class tables, the edge-triple
tables of change detection) as powers of two with 32-bit slot masks.  A
helper that returned the power of two in 32 bits would turn 2^32 into 0 and
build an empty table; these cases pin the helpers instead: 2^32 slots is the
largest table, anything larger is refused with BSIM_E_UNSUPPORTED (-5).  The
check is a host-only program compiled from the library's own header, so no
GPU is involved."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def results():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    out_dir = os.path.join(ROOT, "_build")
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "table_slots_check_%d" % os.getpid())  # one per test process
    src = os.path.join(ROOT, "tests", "native", "table_slots_check.cpp")
    subprocess.run([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2111_12493_amd", "csrc"),
                    src, "-o", exe], check=True, capture_output=True)
    lines = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    return dict((ln.split(" ", 1)[0], ln.split(" ", 1)[1]) for ln in lines if ln.strip())


def test_next_pow2_is_64_bit(results):
    assert results["next_pow2_2e32p1"] == str(1 << 33)


@pytest.mark.parametrize("case,want", [
    ("diff_m_0", 64),
    ("diff_m_2e30", 1 << 32),        # the 2^30-edge workload: 2^32 slots, not 0
    ("diff_m_2e31m2", 1 << 32),
    ("diff_m_2e31m1", 1 << 32),
    ("diff_m_2e31", None),
    ("split_n_0", 64),
    ("split_n_2e27", 1 << 28),
    ("split_n_1431655765", 1 << 31),
    ("split_n_1431655766", 1 << 32),  # once fell back to a 64-slot table
    ("split_n_2863311530", 1 << 32),
    ("split_n_2863311531", None),
    ("split_n_4294967294", None),
])
def test_table_slots(results, case, want):
    if want is None:
        assert results[case] == "unsupported -5"
    else:
        assert results[case] == str(want)
