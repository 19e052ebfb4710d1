"""FP64 CPU oracle for the openQ*D Wilson-clover / C* / SAP-GCR hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library and its Python
binding never do, and it shares no code with them.

Everything is complex128 numpy, vectorised over lattice sites only, with the
formulas written in the paper's notation (Campos et al., "openQ*D simulation
code for QCD+QED", Lattice 2017):

  lattice.py  extended lattice, C* shifted boundaries, neighbours  (Sec. 2.1)
  fields.py   orbifold gauge field, U(1) phases, clover, Pauli term (Sec. 2.1,
              Sec. 2.3)
  dirac.py    gamma matrices, D = m0 + Dw + dDsw, even-odd blocks and the
              Schur complement D^ (Sec. 2.3, Sec. 2.4)
  solvers.py  GCR on D^, minimal-residual block solver, Schwarz alternating
              procedure, flexible GCR, defect correction (solvers named in the
              abstract and Sec. 2; the steps follow the literature the paper
              builds on, see each docstring)
  rational.py multi-shift CG on D^dag D^ + mu^2 and rational functions of it
              (Sec. 2.4, Table 2)
  deflation.py  local deflation of the SAP-GCR: deflation subspace, little
              Dirac operator, deflated preconditioner (abstract, Sec. 2,
              Appendix A; steps from the published method the paper cites)
  dense.py    dense matrices and brute-force tools for tiny lattices

Parity status: every function is pinned by a CPU test against closed forms,
identities of the paper or brute force (the open time boundary by closed forms
of the boundary clover: a field whose only non-trivial links are the cut ones,
and a uniform flux whose boundary leaves are half missing), except the solver
iteration counts (the paper prints none).
"""

from .lattice import Lattice  # noqa: F401
