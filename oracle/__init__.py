"""FP64 CPU oracle for cut-circuit reconstruction -- TEST INFRASTRUCTURE.

A plain, slow, obviously correct implementation of what the reconstruction
library computes, written from the paper ("Cutting Quantum Circuits to Run on
Quantum and Classical Platforms", Tang & Martonosi):

* ``statevector``  -- state-vector simulation (Section 2) of whole circuits
  and of every subcircuit variant (Section 3.1: each Pauli assignment of the
  cuts initialises and measures the subcircuits differently).
* ``attribution``  -- variant probabilities -> entry vectors p_{i,k}.
* ``reconstruct``  -- Eq. 1, the Kronecker sum over all 4^K cut labelings,
  as a literal loop, per output bin, and as one einsum contraction.
* ``dd``           -- dynamic definition, Algorithm 1, and the breadth-first
  query.
* ``shots``        -- finite-shot emulation and the chi-square loss of Eq. 3.
* ``cutfind``      -- exhaustive cut search with the objective of Section 4.1.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library and must never
serve as a fallback for it.  numpy float64 throughout.

Every function that has no independent pin would say "parity unpinned" in
its docstring; none does: all functions here are pinned by
tests/test_oracle_*.py and tests/test_cutfind.py (``shots.philox4x32_10`` by
the published Philox4x32-10 known-answer vectors, the list handling of
``dd.run`` and ``dd.run_bfs`` by a case worked by hand from Algorithm 1).
"""
