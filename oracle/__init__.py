"""CPU oracle for hash-based labeled forward k-bisimulation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package.  It shares no code with
the GPU library (`paper_2111_12493_amd`) and imports nothing from it; the
graphs both sides consume come from the separate input-generator module.

Contents
  bsim_oracle.c  -- the step-by-step hash-spec oracle (plain C, single thread)
  oracle.py      -- ctypes wrapper around it
  exact.py       -- hash-free exact refinement and definition-level brute force
                    (pure Python), used to pin the oracle's partitions
"""
