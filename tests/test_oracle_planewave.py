"""Closed-form pins: plane waves exp(i k.r)/sqrt(L^3) on the periodic mesh are
exact eigenvectors of the finite-difference H with V constant and no
projectors, with
    eps(k, A) = 1/2 sum_d K2(k_d) + sum_d A_d K1(k_d) + 1/2 |A|^2 + V,
    K2(k) = -(1/h^2)(c0 + 2 sum_m c_m cos(m k h)),  K1(k) = (2/h) sum_m a_m sin(m k h).
The step multiplies each one by T4(-i dt eps); density, current and energy
follow in closed form.  A plane-wave projector column with the orbital's k
shifts eps by its D.
"""
import math

import numpy as np
import pytest

from oracle import adjoint as ADJ
from oracle import fd
from oracle import hamiltonian as H
from oracle import observables as O
from oracle import propagate as P
from synth import Domain

SHAPE = (8, 10, 12)          # distinct edges catch axis mix-ups
HS = 0.5
MODES = [(1, 0, 0), (0, 2, -1), (-1, 1, 3), (2, -3, 1)]


def K2(k, h, order):
    c = fd.second(order)
    return -(c[0] + 2 * sum(c[m] * np.cos(m * k * h) for m in range(1, len(c)))) / h ** 2


def K1(k, h, order):
    a = fd.first(order)
    return 2 * sum(a[m - 1] * np.sin(m * k * h) for m in range(1, len(a) + 1)) / h


def _kvec(mode):
    L = np.array(SHAPE) * HS
    return 2 * np.pi * np.array(mode) / L


def _plane_domain(order, v0=0.0, proj_modes=(), d=(), occ=None):
    nx, ny, nz = SHAPE
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = HS * np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    vol = np.prod(SHAPE) * HS ** 3
    psi = np.stack([np.exp(1j * r @ _kvec(m)) / np.sqrt(vol) for m in MODES], axis=1)
    if proj_modes:
        proj = np.stack([np.exp(1j * (r @ _kvec(m) + 0.7 * i)) / np.sqrt(vol)
                         for i, m in enumerate(proj_modes)], axis=1)
    else:
        proj = np.zeros((psi.shape[0], 0), np.complex128)
    occ = np.array([2.0, 1.5, 1.0, 0.5]) if occ is None else occ
    return Domain(SHAPE, HS, order, psi, np.full(psi.shape[0], v0), proj,
                  np.asarray(d, dtype=np.float64), occ)


def _eps(order, A, v0=0.0):
    out = []
    for m in MODES:
        k = _kvec(m)
        out.append(0.5 * sum(K2(k[i], HS, order) for i in range(3))
                   + sum(A[i] * K1(k[i], HS, order) for i in range(3))
                   + 0.5 * float(np.dot(A, A)) + v0)
    return np.array(out)


def _t4(z):
    return sum(z ** k / math.factorial(k) for k in range(5))


@pytest.mark.parametrize("order", [2, 4, 6])
def test_plane_waves_are_eigenvectors(order):
    A = np.array([0.11, -0.23, 0.37])
    dom = _plane_domain(order, v0=-0.3)
    hpsi = H.apply_h(dom, A, dom.psi)
    eps = _eps(order, A, -0.3)
    assert np.abs(hpsi - dom.psi * eps[None, :]).max() < 1e-12


@pytest.mark.parametrize("order", [4, 6])
def test_multi_step_phase_is_product_of_taylor_factors(order):
    rng = np.random.default_rng(3)
    a_mid = rng.uniform(-0.2, 0.2, size=(6, 3))
    dt = 0.05
    dom = _plane_domain(order)
    psi, _ = P.propagate(dom, a_mid, dt, dom.psi)
    fac = np.ones(len(MODES), complex)
    for A in a_mid:
        fac *= _t4(-1j * dt * _eps(order, A))
    assert np.abs(psi - dom.psi * fac[None, :]).max() < 1e-12
    # and within the truncation bound of the exact phase
    phase = np.exp(-1j * dt * sum(_eps(order, A) for A in a_mid))
    x = dt * max(np.abs(_eps(order, A)).max() for A in a_mid)
    assert np.abs(fac - phase).max() <= len(a_mid) * x ** 5 / 120 * 1.01


@pytest.mark.parametrize("order", [2, 6])
def test_density_current_energy_closed_forms(order):
    A = np.array([0.05, -0.1, 0.2])
    dom = _plane_domain(order, v0=0.4)
    vol = np.prod(SHAPE) * HS ** 3
    rho = O.density(dom, dom.psi)
    assert np.abs(rho - dom.occ.sum() / vol).max() < 1e-14
    j = O.current(dom, A, dom.psi)
    for d in range(3):
        jd = sum(dom.occ[n] * (K1(_kvec(m)[d], HS, order) + A[d]) for n, m in enumerate(MODES)) / vol
        assert np.abs(j[:, d] - jd).max() < 1e-13
    e = O.energy(dom, A, dom.psi)
    assert abs(e - float(dom.occ @ _eps(order, A, 0.4))) < 1e-12


def test_plane_wave_projector_shifts_eigenvalue_by_d():
    A = np.array([0.0, 0.0, 0.2])
    d = [0.7, -0.4]
    # first projector matches orbital 1's k, the second orbital 3's, with phases
    dom = _plane_domain(4, proj_modes=(MODES[1], MODES[3]), d=d)
    hpsi = H.apply_h(dom, A, dom.psi)
    eps = _eps(4, A)
    eps[1] += d[0]
    eps[3] += d[1]
    assert np.abs(hpsi - dom.psi * eps[None, :]).max() < 1e-12


def test_plane_wave_gradient_closed_form():
    """L = sum f eps0 (prod_j |T4_j|^2 - 1);
    dL/dA_k,z = sum f eps0 prod_{j!=k} |T4_j|^2 (-x^5/12 + x^7/72) dt (K1(k_z) + A_k,z),
    x = dt eps(k, A_k)."""
    order = 4
    dt = 0.3                  # large enough for |T4| != 1 to matter
    rng = np.random.default_rng(7)
    a_mid = np.zeros((5, 3))
    a_mid[:, 2] = rng.uniform(-0.3, 0.3, size=5)
    dom = _plane_domain(order)
    loss, grad = ADJ.loss_and_grad(dom, a_mid, dt, dom.psi, dirs=(2,))
    eps0 = _eps(order, np.zeros(3))
    mod2 = np.array([[abs(_t4(-1j * dt * e)) ** 2 for e in _eps(order, A)] for A in a_mid])
    l_ref = float(dom.occ @ (eps0 * (mod2.prod(axis=0) - 1)))
    assert abs(loss - l_ref) < 1e-12 * max(1.0, abs(l_ref))
    kz = np.array([_kvec(m)[2] for m in MODES])
    for k in range(len(a_mid)):
        x = dt * _eps(order, a_mid[k])
        dmod = (-x ** 5 / 12 + x ** 7 / 72) * dt * (K1(kz, HS, order) + a_mid[k, 2])
        others = np.prod(np.delete(mod2, k, axis=0), axis=0)
        g_ref = float(dom.occ @ (eps0 * others * dmod))
        assert abs(grad[k, 2] - g_ref) < 1e-10 * max(1e-6, abs(g_ref)) + 1e-14
