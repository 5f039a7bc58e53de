"""Pins of the oracle's H and Taylor step on tiny grids against dense linear
algebra: the assembled matrix is Hermitian, the matrix-free power sum equals
the same polynomial applied through numpy's eigendecomposition, and it stays
within the truncation bound of scipy's matrix exponential."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import hamiltonian as H
from oracle import observables as O
from oracle import propagate as P
from synth import make_domain

CASES = [
    dict(shape=(7, 6, 8), order=4, n_orb=3, n_atoms=2, ppa=4, A=(0.3, -0.2, 0.5)),
    dict(shape=(8, 8, 8), order=6, n_orb=2, n_atoms=2, ppa=8, A=(0.0, 0.0, 0.4)),
    dict(shape=(5, 7, 6), order=2, n_orb=4, n_atoms=1, ppa=4, A=(-0.1, 0.25, 0.0)),
]


def _dom(c, seed=11):
    return make_domain(seed, c["shape"], c["n_orb"], c["n_atoms"], proj_per_atom=c["ppa"],
                       h=0.45, fd_order=c["order"])


def _t4(z):
    return sum(z ** k / math.factorial(k) for k in range(5))


@pytest.mark.parametrize("c", CASES)
def test_dense_h_is_hermitian(c):
    dom = _dom(c)
    hm = H.dense(dom, np.array(c["A"]))
    assert np.abs(hm - hm.conj().T).max() < 1e-12 * np.abs(hm).max()


@pytest.mark.parametrize("c", CASES)
def test_matrix_free_matches_dense_columns(c):
    dom = _dom(c)
    A = np.array(c["A"])
    hm = H.dense(dom, A)
    ref = hm @ dom.psi
    assert np.abs(H.apply_h(dom, A, dom.psi) - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("c", CASES)
def test_taylor_step_equals_eigendecomposition(c):
    dom = _dom(c)
    A = np.array(c["A"])
    dt = 0.05
    hm = H.dense(dom, A)
    lam, v = np.linalg.eigh(hm)
    ref = v @ (_t4(-1j * dt * lam)[:, None] * (v.conj().T @ dom.psi))
    got = P.taylor4_step(dom, A, dt, dom.psi)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("c", CASES)
def test_taylor_within_truncation_bound_of_expm(c):
    dom = _dom(c)
    A = np.array(c["A"])
    dt = 0.02
    hm = H.dense(dom, A)
    x = dt * np.linalg.norm(hm, 2)
    psi = dom.psi
    exact = scipy.linalg.expm(-1j * dt * hm) @ psi
    got = P.taylor4_step(dom, A, dt, psi)
    bound = math.exp(x) * x ** 5 / 120
    err = np.sqrt(dom.h ** 3 * np.sum(np.abs(got - exact) ** 2, axis=0))
    assert np.all(err <= bound * 1.0001 + 1e-14)
    # sharper: the difference is the first dropped term -(-i dt H)^5 psi / 5!
    # up to the remainder of the next order
    lead = psi.copy()
    for _ in range(5):
        lead = -1j * dt * (hm @ lead)
    resid = np.sqrt(dom.h ** 3 * np.sum(np.abs((exact - got) - lead / 120) ** 2, axis=0))
    assert np.all(resid <= math.exp(x) * x ** 6 / 720 * 1.0001 + 1e-14)
    assert np.sqrt(dom.h ** 3 * np.sum(np.abs(lead) ** 2, axis=0)).max() / 120 > 10 * resid.max()


def test_forward_then_backward_returns_state():
    c = CASES[0]
    dom = _dom(c)
    A = np.array(c["A"])
    dt = 0.02
    hm = H.dense(dom, A)
    x = dt * np.linalg.norm(hm, 2)
    back = P.taylor4_step(dom, A, -dt, P.taylor4_step(dom, A, dt, dom.psi))
    err = np.sqrt(dom.h ** 3 * np.sum(np.abs(back - dom.psi) ** 2, axis=0))
    assert err.max() <= x ** 5 / 10 + 1e-14


@pytest.mark.parametrize("c", CASES)
def test_energy_matches_dense_quadratic_form(c):
    dom = _dom(c)
    A = np.array(c["A"])
    hm = H.dense(dom, A)
    e_ref = sum(dom.occ[n] * dom.h ** 3 * np.real(dom.psi[:, n].conj() @ hm @ dom.psi[:, n])
                for n in range(dom.n_orb))
    assert abs(O.energy(dom, A, dom.psi) - e_ref) < 1e-12 * abs(e_ref)
    e_loc, e_nl = O.energy_parts(dom, A, dom.psi)
    assert abs(e_loc + e_nl - e_ref) < 1e-12 * abs(e_ref)
