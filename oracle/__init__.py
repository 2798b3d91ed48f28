"""CPU oracle for the state-vector path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never touches it, and it never touches the product path.

Contents:
  oracle.c   plain complex128 gate-by-gate simulator (Eq. 1-4 of the paper),
             readouts (probabilities, Pauli expectations, MaxCut cost),
             QAOA cost layer; built into liboracle.so by build().
  sim.py     ctypes wrapper plus small numpy helpers around it.
  mlp.py     FP64 numpy forward/backward/Adam for the 48-128-128-1 MLP cost
             model (parity unpinned against the paper, which has no MLP;
             pinned by central finite differences).

Every function cites the passage of the paper it follows; where the paper
is silent, the reading taken is named in the function's docstring.
"""
