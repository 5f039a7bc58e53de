"""Pins of the oracle's Eq. 2 / Eq. 5 step (normalised nonlocal half-steps in
the reference-orbital space around the local propagator): it reduces to the
local Taylor step for v_nl = 0, keeps every orbital at unit norm, multiplies a
reference orbital by the closed-form phase ((1-delta)/|1-delta|)^2, and gives
the closed form for plane waves."""
import math

import numpy as np

from oracle import propagate as P
from synth import Domain, make_domain


def _dom():
    return make_domain(81, (9, 10, 8), 4, 2, proj_per_atom=4, h=0.45, fd_order=4)


def test_reduces_to_local_step_without_nonlocal_term():
    d = _dom()
    A = np.array([0.1, 0.0, -0.2])
    loc = Domain(d.shape, d.h, d.fd_order, d.psi, d.v_loc, np.zeros((d.n_grid, 0), complex), np.zeros(0), d.occ)
    ref = P.taylor4_step(loc, A, 0.02, d.psi)
    got = P.eq2_step(d, A, 0.02, d.psi, d.psi, 0.0)
    # both normalisations act on norms that the local step changes by < dt^6
    norms = np.sqrt(d.h ** 3 * np.sum(np.abs(ref) ** 2, axis=0))
    assert np.abs(got - ref / norms).max() < 1e-14


def test_unit_norm_after_each_step():
    d = _dom()
    rng = np.random.default_rng(1)
    psi = d.psi + 0.1 * (rng.standard_normal(d.psi.shape) + 1j * rng.standard_normal(d.psi.shape))
    out = P.eq2_step(d, np.array([0, 0, 0.3]), 0.05, psi, d.psi, 0.7)
    assert np.abs(d.h ** 3 * np.sum(np.abs(out) ** 2, axis=0) - 1).max() < 1e-13


def test_reference_orbitals_pick_up_the_half_step_phase():
    d = _dom()
    delta = 0.5j * 0.05 * 0.9
    out = P.nonlocal_half_step(d, d.psi, d.psi, delta)
    phase = (1 - delta) / abs(1 - delta)
    assert np.abs(out - phase * d.psi).max() < 1e-13


def test_plane_wave_closed_form():
    shape, h = (8, 6, 10), 0.5
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = h * np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    L = np.array(shape) * h
    modes = [(1, 0, 0), (0, 1, -1), (2, -1, 1)]
    psi = np.stack([np.exp(1j * r @ (2 * np.pi * np.array(m) / L)) for m in modes], 1) / math.sqrt(np.prod(L))
    d = Domain(shape, h, 4, psi, np.zeros(len(r)), np.zeros((len(r), 0), complex), np.zeros(0), np.ones(3))
    A = np.array([0.0, 0.2, 0.1])
    dt, v = 0.04, 1.3
    c = (-5 / 2, 4 / 3, -1 / 12)
    a = (2 / 3, -1 / 12)
    eps = []
    for m in modes:
        k = 2 * np.pi * np.array(m) / L
        K2 = [-(c[0] + 2 * (c[1] * np.cos(kk * h) + c[2] * np.cos(2 * kk * h))) / h ** 2 for kk in k]
        K1 = [2 * (a[0] * np.sin(kk * h) + a[1] * np.sin(2 * kk * h)) / h for kk in k]
        eps.append(0.5 * sum(K2) + sum(A[i] * K1[i] for i in range(3)) + 0.5 * A @ A)
    t4 = lambda zz: sum(zz ** j / math.factorial(j) for j in range(5))
    delta = 0.5j * dt * v
    ph = ((1 - delta) / abs(1 - delta)) ** 2
    expect = psi * np.array([ph * t4(-1j * dt * e) / abs(t4(-1j * dt * e)) for e in eps])[None, :]
    got = P.eq2_step(d, A, dt, psi, psi, v)
    assert np.abs(got - expect).max() < 1e-12
