"""Pins of the occupation oracle (f_s and n_exc from the cross overlap with the
reference orbitals):

* a permutation of the reference orbitals moves each occupation to its image
  (fixes the index order of S and the sum over n);
* a unitary mixing inside the reference span keeps equal occupations and gives
  n_exc = 0;
* a rotation of each orbital out of the span by theta_n gives
  f_s = f_s cos^2(theta_s) and n_exc = sum_n f_n sin^2(theta_n);
* plane waves propagated by Taylor-4 steps keep n_exc = 0 while their norms
  shrink, and f_s = f_s prod_k |T4(-i dt eps_s(A_k))|^2 in closed form;
* a brute-force triple loop over grid points on a tiny grid.
"""
import numpy as np

from oracle import occupations as OC
from oracle import propagate as P
from synth import make_domain
from test_oracle_planewave import MODES, _eps, _plane_domain, _t4

SHAPE = (6, 7, 8)


def _dom(occ):
    dom = make_domain(41, SHAPE, len(occ), 2, proj_per_atom=4, h=0.45, fd_order=4)
    dom.occ = np.asarray(occ, dtype=np.float64)
    return dom


def _complement(dom, psi0, k, rng):
    """k orbitals orthonormal (h^3 metric) and orthogonal to psi0."""
    x = rng.standard_normal((psi0.shape[0], k)) + 1j * rng.standard_normal((psi0.shape[0], k))
    basis = psi0 * np.sqrt(dom.h ** 3)
    x = x - basis @ (basis.conj().T @ x)
    q, _ = np.linalg.qr(x)
    return q / np.sqrt(dom.h ** 3)


def test_reference_state_is_fully_occupied_at_start():
    dom = _dom([2.0, 1.0, 0.5, 0.25])
    f, n_exc = OC.occupations(dom, dom.psi, dom.psi)
    assert np.abs(f - dom.occ).max() < 1e-11
    assert abs(n_exc) < 1e-11


def test_permutation_moves_occupations_to_the_image():
    dom = _dom([2.0, 1.5, 1.0, 0.5, 0.25])
    perm = [2, 0, 4, 1, 3]                     # psi_n(t) = psi_{perm[n]}(0), no involution
    psi = dom.psi[:, perm]
    f, n_exc = OC.occupations(dom, dom.psi, psi)
    want = np.zeros(5)
    want[perm] = dom.occ
    assert np.abs(f - want).max() < 1e-11
    assert abs(n_exc) < 1e-11


def test_unitary_mixing_inside_the_span():
    dom = _dom([2.0] * 5)
    rng = np.random.default_rng(3)
    q, _ = np.linalg.qr(rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5)))
    psi = dom.psi @ q
    f, n_exc = OC.occupations(dom, dom.psi, psi)
    assert np.abs(f - 2.0).max() < 1e-11
    assert abs(n_exc) < 1e-11


def test_rotation_out_of_the_span():
    occ = np.array([2.0, 1.5, 1.0, 0.5])
    dom = _dom(occ)
    rng = np.random.default_rng(4)
    chi = _complement(dom, dom.psi, 4, rng)
    theta = np.array([0.1, 0.7, 1.2, np.pi / 2])
    phase = np.exp(1j * rng.uniform(0, 2 * np.pi, 4))
    psi = dom.psi * np.cos(theta) + chi * (np.sin(theta) * phase)
    f, n_exc = OC.occupations(dom, dom.psi, psi)
    assert np.abs(f - occ * np.cos(theta) ** 2).max() < 1e-11
    assert abs(n_exc - float(occ @ np.sin(theta) ** 2)) < 1e-11
    # invariant under phases of the reference columns
    f2, n2 = OC.occupations(dom, dom.psi * np.exp(1j * np.arange(4)), psi)
    assert np.abs(f2 - f).max() < 1e-13 and abs(n2 - n_exc) < 1e-11


def test_plane_waves_keep_zero_excitation_while_norms_shrink():
    order, dt = 4, 0.2                        # |T4| visibly below 1, inside the stability bound
    rng = np.random.default_rng(8)
    a_mid = rng.uniform(-0.3, 0.3, size=(5, 3))
    dom = _plane_domain(order)
    psi, _ = P.propagate(dom, a_mid, dt, dom.psi)
    f, n_exc = OC.occupations(dom, dom.psi, psi)
    mod2 = np.ones(len(MODES))
    for A in a_mid:
        mod2 *= np.abs(_t4(-1j * dt * _eps(order, A))) ** 2
    assert mod2.min() < 1 - 1e-4               # the norm change is not negligible
    assert mod2.max() <= 1.0
    assert np.abs(f - dom.occ * mod2).max() < 1e-11
    assert abs(n_exc) < 1e-11


def test_brute_force_tiny_grid():
    dom = _dom([2.0, 1.0, 0.5])
    rng = np.random.default_rng(9)
    psi = dom.psi @ (np.eye(3) * 0.8) + 0.05 * (rng.standard_normal(dom.psi.shape)
                                                + 1j * rng.standard_normal(dom.psi.shape))
    f, n_exc = OC.occupations(dom, dom.psi, psi)
    n_g = dom.psi.shape[0]
    f_bf = [0.0] * 3
    tot = 0.0
    for n in range(3):
        col = 0.0
        for s in range(3):
            acc = 0j
            for g in range(n_g):
                acc += dom.psi[g, s].conjugate() * psi[g, n]
            acc *= dom.h ** 3
            f_bf[s] += dom.occ[n] * abs(acc) ** 2
            col += abs(acc) ** 2
        nrm = dom.h ** 3 * sum(abs(psi[g, n]) ** 2 for g in range(n_g))
        tot += dom.occ[n] * (nrm - col)
    assert np.abs(f - np.array(f_bf)).max() < 1e-11
    assert abs(n_exc - tot) < 1e-11
