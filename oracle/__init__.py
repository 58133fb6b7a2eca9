"""FP64 CPU oracle for the refinement-free Calderon-preconditioned EFIE
(Adrian, Andriulli, Eibert, arXiv:1803.08333).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links
or executes this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use it.  It shares no code with the HIP
library (no kernels, headers, tables or helpers); the two meet only on the
seeded inputs produced by ``synth``.

Plain, slow and written to be checked against the paper by eye:
  quadrature  -- the 7-point degree-5 triangle rule of the quadrature spec
  topology    -- RWG edges, star matrix Sigma, loop matrix Lambda (Sec. 2)
  grams       -- G_ll (P1 mass), G_pp, the closed-form mixed Gram G_tp (Sec. 3)
  singular    -- closed-form 1/R and (r'-r)/R triangle potentials
  assembly    -- dense T_A and V blocks of the EFIE (Sec. 2), complex128
  rhs         -- plane-wave excitation vector e (Sec. 2)
  rfcmp       -- projectors, the preconditioned system of eq. (NewFormulation),
                 CG, power-iteration scalings (Sec. 4), recovery j = P_o i
  mie         -- PEC-sphere surface current from the Mie series (pin only)

Every function cites the passage of the paper it follows.
"""

from . import quadrature, topology, grams, singular, assembly, rhs, rfcmp  # noqa: F401
