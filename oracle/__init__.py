"""FP64 CPU oracle for the real-time Kohn-Sham step (TEST INFRASTRUCTURE ONLY).

This package is the slow, plain reference that the HIP library is checked
against.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the library never calls it and never falls back to it.
It shares no code with the HIP path: it reads the seeded inputs of ``synth`` and
recomputes everything from the definitions, in complex128 with numpy.

Contents, each function citing the passage it follows:

* ``fd``          finite-difference weights of the second and first derivative;
* ``hamiltonian`` H(A) psi of Eq. 3 (atomic units) with the nonlocal term as
                  the two products of Sec. V.B.5, and a dense assembly for tiny grids;
* ``propagate``   the fourth-order Taylor step as an explicit power sum, with
                  the vector potential taken at the step midpoint (Eq. 2);
* ``observables`` density, local current, energy and overlap;
* ``adjoint``     the gradient of the absorbed energy w.r.t. the samples A_k;
* ``split``       hi+lo rounding of operands (BF16 / FP16), the mixed-precision
                  products of Sec. VI.C evaluated exactly in FP64.

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` (closed forms, dense eigendecomposition, library
expm, torch autograd, brute-force finite differences).  The paper prints no
numerical result of this path, so no pin uses a printed value.
"""
from . import fd, hamiltonian, propagate, observables, adjoint, split  # noqa: F401
