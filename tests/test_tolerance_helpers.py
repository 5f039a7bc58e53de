"""The FP32 operator tolerance of the GPU parity tests (helpers.fp32_operator_tol)
rests on |H||u|, the sum of the magnitudes of every term of H u.  These checks
keep that sum honest: it bounds |H u| element by element (triangle
inequality), it is exactly |H u| where no two terms can cancel, and the
condition numbers it gives do not depend on the scale of u."""
import numpy as np

from helpers import fp32_operator_tol, magnitude_h
from oracle import hamiltonian as H
from synth import Domain, make_domain


def test_magnitude_sum_bounds_every_element():
    dom = make_domain(11, (9, 8, 10), 5, 2, proj_per_atom=8, h=0.4, fd_order=6)
    A = np.array([0.3, -0.2, 0.1])
    hu = H.apply_h(dom, A, dom.psi)
    M = magnitude_h(dom, A, dom.psi)
    assert np.all(M >= np.abs(hu) * (1 - 1e-12))
    assert np.all(M > 0)


def test_magnitude_sum_is_exact_without_cancellation():
    # a delta function at one point, a positive constant potential, A = 0 and
    # no projectors: at the delta's own point H u has two terms of the same
    # sign (the kinetic centre weight and the potential), so the magnitude
    # sum equals |H u| there; at a nearest neighbour there is one term only
    dom = make_domain(12, (7, 7, 7), 1, 1, proj_per_atom=4, h=0.5, fd_order=2)
    u = np.zeros((dom.n_grid, 1), np.complex128)
    u[100, 0] = 1.0 + 2.0j
    loc = Domain(dom.shape, dom.h, dom.fd_order, u, np.full(dom.n_grid, 0.7),
                 np.zeros((dom.n_grid, 0), np.complex128), np.zeros(0), dom.occ)
    hu = H.apply_h(loc, np.zeros(3), u)
    M = magnitude_h(loc, np.zeros(3), u)
    assert np.isclose(M[100, 0], np.abs(hu[100, 0]), rtol=1e-12)
    assert np.isclose(M[101, 0], np.abs(hu[101, 0]), rtol=1e-12)


def test_tolerance_is_scale_free():
    dom = make_domain(13, (9, 9, 9), 4, 1, proj_per_atom=8, h=0.4, fd_order=4)
    A = np.array([0.0, 0.0, 0.2])
    hu = H.apply_h(dom, A, dom.psi)
    t1 = fp32_operator_tol(dom, A, dom.psi, hu, occ_scale=False)
    t2 = fp32_operator_tol(dom, A, 3.0 * dom.psi, 3.0 * hu, occ_scale=False)
    # the occupation factors scale the magnitudes and the reference alike
    t3 = fp32_operator_tol(dom, A, dom.psi, hu * dom.occ[None, :], occ_scale=True)
    assert np.allclose(t1, t2, rtol=1e-12)
    assert np.allclose(t1, t3, rtol=1e-12)
    assert all(x > 0 for x in t1)
