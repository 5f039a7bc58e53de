"""Invariants of the method that hold for any input: norm and energy drift
within the Taylor-4 bound, orthonormal start, zero current for real orbitals
at A = 0, invariance under projector column phases, particle count."""
import math

import numpy as np
import pytest

from oracle import hamiltonian as H
from oracle import observables as O
from oracle import propagate as P
from synth import config, make_domain


@pytest.fixture(scope="module")
def c1():
    return config(1)


def test_overlap_is_identity_at_start(c1):
    dom = c1.domains[0]
    assert np.abs(O.overlap(dom, dom.psi) - np.eye(dom.n_orb)).max() < 1e-13


def test_particle_count(c1):
    dom = c1.domains[0]
    assert abs(dom.h ** 3 * O.density(dom, dom.psi).sum() - dom.occ.sum()) < 1e-12


def test_norm_and_energy_drift_bound(c1):
    """|T4(-ix)|^2 = 1 - x^6/72 + x^8/576 per eigencomponent, so over n steps the
    norm and the energy move by at most n (dt lambda_max)^6 / 72 (relative)."""
    dom = c1.domains[0]
    A = np.zeros(3)
    # lambda_max of H from power iteration on the matrix-free operator
    rng = np.random.default_rng(0)
    v = rng.standard_normal((dom.n_grid, 1)) + 0j
    for _ in range(60):
        v = H.apply_h(dom, A, v)
        v /= np.linalg.norm(v)
    lam = abs(np.vdot(v, H.apply_h(dom, A, v)))
    x = c1.dt * lam * 1.05
    assert x ** 2 <= 8.0                       # inside the stability bound
    psi, obs = P.propagate(dom, c1.a_mid, c1.dt, dom.psi, want_energy=True)
    n = c1.n_steps
    norms = dom.h ** 3 * np.sum(np.abs(psi) ** 2, axis=0)
    assert np.all(norms <= 1 + 1e-13)
    assert np.all(1 - norms <= n * x ** 6 / 72)
    e = obs["energy"]
    e_end = O.energy(dom, A, psi)
    scale = dom.occ.sum() * lam
    assert abs(e_end - e[0]) <= n * x ** 6 / 72 * scale


def test_real_orbitals_carry_no_current():
    dom = make_domain(3, (9, 8, 10), 3, 2, proj_per_atom=4, h=0.4, fd_order=6)
    dom.psi = np.ascontiguousarray(dom.psi.real.astype(np.complex128))
    j = O.current(dom, np.zeros(3), dom.psi)
    assert np.abs(j).max() < 1e-15


def test_current_diamagnetic_part():
    dom = make_domain(4, (9, 8, 10), 3, 2, proj_per_atom=4, h=0.4, fd_order=4)
    A = np.array([0.1, 0.2, -0.3])
    j0 = O.current(dom, np.zeros(3), dom.psi)
    j1 = O.current(dom, A, dom.psi)
    rho = O.density(dom, dom.psi)
    assert np.abs(j1 - j0 - rho[:, None] * A[None, :]).max() < 1e-14


def test_projector_phase_invariance():
    dom = make_domain(5, (8, 9, 7), 3, 3, proj_per_atom=8, h=0.4, fd_order=6)
    A = np.array([0.0, 0.1, 0.2])
    ref = P.taylor4_step(dom, A, 0.03, dom.psi)
    rng = np.random.default_rng(1)
    dom2 = make_domain(5, (8, 9, 7), 3, 3, proj_per_atom=8, h=0.4, fd_order=6)
    dom2.proj = dom2.proj * np.exp(1j * rng.uniform(0, 2 * np.pi, dom2.n_proj))[None, :]
    got = P.taylor4_step(dom2, A, 0.03, dom2.psi)
    assert np.abs(got - ref).max() < 1e-13
    # while a projector actually acts: D = 0 gives a different result
    dom2.d = np.zeros_like(dom2.d)
    assert np.abs(P.taylor4_step(dom2, A, 0.03, dom2.psi) - ref).max() > 1e-6


def test_orbitals_propagate_independently():
    """The step is column-wise: propagating a subset of orbitals gives the same columns."""
    dom = make_domain(6, (8, 8, 9), 4, 2, proj_per_atom=4, h=0.4, fd_order=4)
    A = np.array([0.0, 0.0, 0.3])
    full = P.taylor4_step(dom, A, 0.02, dom.psi)
    sub = P.taylor4_step(dom, A, 0.02, dom.psi[:, [1, 3]].copy())
    assert np.abs(full[:, [1, 3]] - sub).max() < 1e-14


def test_midpoint_pulse_samples():
    from synth import pulse_midpoints
    a = pulse_midpoints(200, 0.02, 200)
    t = (np.arange(200) + 0.5) * 0.02
    ref = 0.05 * np.sin(0.1 * t) * np.sin(np.pi * t / 4.0) ** 2
    assert np.allclose(a[:, 2], ref, rtol=0, atol=1e-17)
    assert np.all(a[:, :2] == 0)
    assert math.isclose(a[:, 2].max(), ref.max())
