"""Plain FP64 CPU oracle for the adaptive multiscale finite volume (MSFV)
method of Wu Fung & Ruthotto, "A Multiscale Method for Model Order Reduction
in PDE Parameter Estimation" (arXiv:1707.07598).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: it exists so that the tests, the package's smoke check and
the benchmark's CPU-baseline leg can check the HIP path against a slow,
obviously correct implementation written from the paper.  It shares no code
with the HIP path (no kernels, headers, helpers, tables or generators); only
the seeded input generators in ``workloads`` serve both.

Everything is FP64 NumPy/SciPy with direct solves:

* ``geometry``  -- fine grid, coarse vertices, segments and entities
  (Sec. 3.2, step 1: the nested coarse partition).
* ``operator``  -- sigma = exp(m) (Sec. 2.1), harmonic-averaged two-point
  fluxes, the fine operator A(m) (Sec. 2.2) and its derivative terms.
* ``basis``     -- the parameter-dependent prolongation S_k(m) built entity
  by entity (Sec. 3.2, eq. multiscaleBasis_step3), its tangent and its
  reverse-mode derivative (Sec. 4.5, eq. reducedDiscreteMSBasisPDE).
* ``reduced``   -- reduced forward F_k(m) (eq. fwdProbRed, eq. reducedPDE),
  the adaptive sensitivities J_k (eq. sensred, Sec. 4.3) in forward and
  transposed form, the fixed-basis sensitivities (eq. senssimple), the
  fine-mesh reference (eq. forwardProbFine, eq. sens) and the SSD misfit.

Parity unpinned: none.  Every function is pinned by a ``-m "not gpu"`` test
in ``tests/test_oracle_*.py`` against closed forms, invariants, special cases
or finite differences (see each test module's header for the list).
"""
from .geometry import Geometry  # noqa: F401
from .operator import conductivity, fine_operator, fine_faces  # noqa: F401
from .basis import Basis, build_basis  # noqa: F401
from . import reduced  # noqa: F401
