"""FP64 CPU oracle for layered-medium multi-particle scattering (Lai, Kobayashi,
Greengard, "A fast solver for multi-particle scattering in a layered medium").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
restatement of what the paper computes, written with numpy/scipy in double
precision.  Only the test-suite, the package smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code, tables or helpers with the
HIP library, and the HIP library never calls it.

Modules
-------
mie        single dielectric disk, Section 3.1, eqs. (17)-(18)
star       scattering matrix of a smooth star by Mueller's second-kind
           integral equations, Section 4, eqs. (31)-(32) and (35)
contour    three-segment Sommerfeld contour, Section 5.1 eq. (37), Section 6
layered    per-node 4x4 interface system A_lambda, Section 2 eq. (10)
operators  M2L (Section 3.2, Lemma 3.1), M2S (Section 5.3, Theorem 5.1),
           S2L (Section 5.2.1, Lemma 5.1 / eq. (40)), rotated S (Section 4.1)
system     Schur-complement system (Section 5.4, eq. (49)), dense LU solve,
           matrix-free matvec and GMRES, field evaluation (eq. (36))
stack      the same system for any number of layers (interface conditions
           (8)-(9) at every interface), TM or TE
Every module that depends on the interface conditions takes pol = "TM" (the
paper's case) or "TE" ((1/k^2) du/dn continuous instead of du/dn).

Parity status of every function is listed in its docstring; the pins live in
``tests/test_oracle_*.py``.
"""

__all__ = ["mie", "star", "contour", "layered", "operators", "system", "stack"]
