"""CPU oracle for hash-based labeled forward k-bisimulation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package.  It shares no code with
the GPU library: nothing here loads libbsim or its binding.  The one thing
it takes from the package directory is the input-generator module
(`paper_2111_12493_amd.graphgen`: the `Graph` container and seeded
generators, none of the method's arithmetic), whose graphs both sides
consume.

Contents
  bsim_oracle.c  -- the step-by-step hash-spec oracle (plain C, single thread)
  oracle.py      -- ctypes wrapper around it
  exact.py       -- hash-free exact refinement and definition-level brute force
                    (pure Python), used to pin the oracle's partitions
"""
