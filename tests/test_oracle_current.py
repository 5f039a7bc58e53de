"""Pins of the current / Maxwell oracle:

* the nonlocal current equals the expectation of i[V_nl, r] formed with dense
  matrices, r measured from each atom (the commutator written out, not the
  projector-pair sum);
* under H = V_nl alone, d<r>/dt (central differences of the exact evolution
  from numpy.linalg.eigh) equals the nonlocal current: the sign and factor of
  the commutator as a velocity;
* real orbitals with real projectors carry no nonlocal current;
* a uniform electron gas (one constant orbital) with an initial kick of the
  field oscillates at the plasma frequency omega^2 = 4 pi n in the exact
  discrete form a_k = dt b0 sin(k theta) / sin(theta), cos theta = 1 - omega^2 dt^2 / 2;
* with no electrons the induced field stays zero and the coupled step reduces
  to the plain step with the averaged external field.
"""
import math

import numpy as np

from oracle import current as CUR
from oracle import hamiltonian as H
from oracle import propagate as P
from synth import Domain, make_domain, projector_moments


def _dom(seed=51, n_atoms=2, per=4, shape=(7, 8, 9)):
    return make_domain(seed, shape, 3, n_atoms, proj_per_atom=per, h=0.45, fd_order=4)


def _positions(dom, centre):
    nx, ny, nz = dom.shape
    L = np.array(dom.shape) * dom.h
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = dom.h * np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1) - centre
    return r - L * np.round(r / L)


def _dense_vnl(dom, cols):
    b = dom.proj[:, cols]
    return dom.h ** 3 * (b * dom.d[cols][None, :]) @ b.conj().T


def test_nonlocal_current_matches_dense_commutator():
    dom = _dom()
    rng = np.random.default_rng(2)
    psi = dom.psi + 0.3 * (rng.standard_normal(dom.psi.shape) + 1j * rng.standard_normal(dom.psi.shape))
    per = dom.n_proj // len(dom.atoms)
    want = np.zeros(3)
    for a in range(len(dom.atoms)):
        v = _dense_vnl(dom, slice(a * per, (a + 1) * per))
        x = _positions(dom, dom.atoms[a])
        for d in range(3):
            c = 1j * (v * x[None, :, d] - x[:, d, None] * v)        # i [V_a, X_d]
            want[d] += np.real(dom.h ** 3 * np.einsum("gn,gk,kn,n->", psi.conj(), c, psi, dom.occ))
    got = CUR.nonlocal_current(dom, psi, projector_moments(dom))
    assert np.abs(got - want).max() < 1e-12 * max(1.0, np.abs(want).max())
    assert np.abs(want).max() > 1e-3                                 # not a vacuous zero


def test_nonlocal_velocity_is_the_time_derivative_of_position():
    dom = _dom(seed=52, n_atoms=1, per=8)
    v = _dense_vnl(dom, slice(0, dom.n_proj))
    lam, u = np.linalg.eigh(v)
    x = _positions(dom, dom.atoms[0])
    rng = np.random.default_rng(3)
    psi = dom.psi + 0.2 * (rng.standard_normal(dom.psi.shape) + 1j * rng.standard_normal(dom.psi.shape))

    def mean_r(t):
        pt = u @ (np.exp(-1j * t * lam)[:, None] * (u.conj().T @ psi))
        return np.array([dom.h ** 3 * np.sum(dom.occ * np.sum(np.abs(pt) ** 2 * x[:, d:d + 1], axis=0))
                         for d in range(3)])

    delta = 1e-5
    fd = (mean_r(delta) - mean_r(-delta)) / (2 * delta)
    got = CUR.nonlocal_current(dom, psi, projector_moments(dom))
    assert np.abs(got - fd).max() < 1e-6 * max(1.0, np.abs(fd).max())
    assert np.abs(fd).max() > 1e-3


def test_real_state_has_no_nonlocal_current():
    dom = _dom(seed=53)
    k = np.argmax(np.abs(dom.proj), axis=0)
    ph = dom.proj[k, np.arange(dom.n_proj)] / np.abs(dom.proj[k, np.arange(dom.n_proj)])
    proj = (dom.proj / ph[None, :]).real.astype(np.complex128)
    psi = dom.psi.real.astype(np.complex128)
    real = Domain(dom.shape, dom.h, dom.fd_order, psi, dom.v_loc, proj, dom.d, dom.occ, dom.atoms)
    j = CUR.nonlocal_current(real, psi, projector_moments(real))
    assert np.abs(j).max() < 1e-13


def _uniform_gas(shape=(6, 7, 8), h=0.5):
    n_g = int(np.prod(shape))
    vol = n_g * h ** 3
    psi = np.full((n_g, 1), 1.0 / math.sqrt(vol), dtype=np.complex128)
    return Domain(shape, h, 4, psi, np.zeros(n_g), np.zeros((n_g, 0), np.complex128), np.zeros(0),
                  np.array([2.0])), 2.0 / vol


def test_uniform_gas_oscillates_at_the_plasma_frequency():
    dom, nbar = _uniform_gas()
    n, dt, b0 = 60, 0.05, np.array([0.0, 0.0, 0.01])
    psi, a_ind, b, cur, mids = CUR.maxwell_propagate(dom, np.zeros((n + 1, 3)), dt, dom.psi, b=b0)
    w2 = 4 * math.pi * nbar
    theta = math.acos(1 - w2 * dt ** 2 / 2)
    k = np.arange(n + 1)
    a = dt * b0[2] * np.sin(k * theta) / math.sin(theta)
    assert abs(a_ind[2] - a[n]) < 1e-12
    # J_k = nbar a_k (diamagnetic only), the step fields are the averages
    assert np.abs(cur[:, 2] - nbar * a[:n]).max() < 1e-12
    assert np.abs(mids[:, 2] - 0.5 * (a[:n] + a[1:])).max() < 1e-12
    assert np.abs(cur[:, :2]).max() == 0.0 and abs(a_ind[0]) + abs(a_ind[1]) == 0.0


def test_no_electrons_reduces_to_the_prescribed_field():
    dom = _dom(seed=54)
    empty = Domain(dom.shape, dom.h, dom.fd_order, dom.psi, dom.v_loc, dom.proj, dom.d,
                   np.zeros_like(dom.occ), dom.atoms)
    rng = np.random.default_rng(4)
    a_ext = rng.uniform(-0.2, 0.2, size=(5, 3))
    psi, a_ind, b, cur, mids = CUR.maxwell_propagate(empty, a_ext, 0.03, empty.psi, projector_moments(empty))
    ref, _ = P.propagate(empty, 0.5 * (a_ext[:-1] + a_ext[1:]), 0.03, empty.psi)
    assert np.abs(a_ind).max() == 0.0 and np.abs(cur).max() == 0.0
    assert np.abs(psi - ref).max() == 0.0
