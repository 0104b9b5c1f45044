"""CPU oracle for deterministic-walk optimal T-count synthesis (Di Matteo & Mosca,
"Parallelizing quantum circuit synthesis", arXiv:1606.07413).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
re-statement of what the walk step computes, written from the paper's
definitions with exact integer arithmetic (Python ints; numpy int64 only where a
bound check proves it cannot overflow).  Only the test-suite, the smoke check
and the benchmark's CPU-baseline leg may import it.  It shares no code with the
HIP library and never imports it.

Modules
  pauli      n-qubit Paulis in binary symplectic form (Sec. 4.1)
  cyclotomic exact arithmetic in Z[omega]/2^d, omega = e^{i pi/4} (for the trace formula)
  zmat       exact channel representations over Z[1/sqrt2] (Sec. 4.1, channel rep)
  walk       the walk function f(x, b) = z_b(x), trails, distinguished points (Sec. 2, 3)
  search     distinguished-point table, trail backtracking, claw check, search driver (Sec. 3)
  bfs        brute-force T-count by breadth-first search over Clifford cosets (Sec. 3, brute force)
  mlp        float64 reference for the depth-order network (forward + backward)

Parity pins: every function is pinned by tests in tests/test_oracle_*.py
against closed forms, textbook matrices, invariants or brute force.  The hash
constants and key streams are this project's reading of the paper's unspecified
"known hash function"; the walk step and trails are therefore pinned only by
their mathematical properties (coset invariance, the planted-claw identity,
determinism, merging), not by values printed in the paper.
"""
