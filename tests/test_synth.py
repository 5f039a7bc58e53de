"""The seeded input generator: deterministic, orthonormal orbitals, normalised
projector columns, the batched workload's shape draws."""
import hashlib

import numpy as np

from synth import batched_domain, batched_domain_shapes, make_domain


def _digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_seeded_generation_is_deterministic():
    a = make_domain(7, (9, 10, 11), 5, 3, proj_per_atom=8, fd_order=6)
    b = make_domain(7, (9, 10, 11), 5, 3, proj_per_atom=8, fd_order=6)
    assert _digest(a.psi, a.v_loc, a.proj, a.d) == _digest(b.psi, b.v_loc, b.proj, b.d)
    c = make_domain(8, (9, 10, 11), 5, 3, proj_per_atom=8, fd_order=6)
    assert _digest(a.psi) != _digest(c.psi)


def test_orthonormal_orbitals_and_normalised_projectors():
    d = make_domain(9, (12, 11, 10), 6, 3, proj_per_atom=8)
    s = d.h ** 3 * d.psi.conj().T @ d.psi
    assert np.abs(s - np.eye(6)).max() < 1e-13
    n = d.h ** 3 * np.sum(np.abs(d.proj) ** 2, axis=0)
    assert np.abs(n - 1).max() < 1e-13
    assert d.proj.shape == (12 * 11 * 10, 24)
    assert np.all(d.v_loc < 0) and np.all((d.d >= -1) & (d.d <= 1))


def test_batched_shapes():
    shapes = batched_domain_shapes()
    assert len(shapes) == 512
    edges = np.array([s[0] for s in shapes])
    orbs = np.array([s[1] for s in shapes])
    assert edges.min() >= 20 and edges.max() <= 40
    assert orbs.min() >= 16 and orbs.max() <= 96
    assert all(s[2] == s[1] // 4 for s in shapes)
    d = batched_domain(3)
    assert d.shape == (shapes[3][0],) * 3 and d.n_orb == shapes[3][1]
    assert d.n_proj == 8 * shapes[3][2]
