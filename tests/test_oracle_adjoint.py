"""Pins of the oracle gradient: the adjoint step is the transpose of the step
(dot-product test), the gradient matches central finite differences of the
FP64 loss, and it matches torch's complex128 autograd through a dense Taylor
loop assembled independently of the oracle's matrix-free operator."""
import math

import numpy as np
import pytest
import torch

from oracle import adjoint as ADJ
from oracle import fd
from oracle import propagate as P
from synth import make_domain, pulse_midpoints


def _small(seed=21, shape=(7, 8, 6), order=4):
    return make_domain(seed, shape, 3, 2, proj_per_atom=4, h=0.45, fd_order=order)


def test_dot_product_test():
    dom = _small()
    A = np.array([0.1, -0.2, 0.3])
    rng = np.random.default_rng(2)
    lam = rng.standard_normal(dom.psi.shape) + 1j * rng.standard_normal(dom.psi.shape)
    v = rng.standard_normal(dom.psi.shape) + 1j * rng.standard_normal(dom.psi.shape)
    lhs = ADJ.inner(dom, ADJ.taylor4_adjoint(dom, A, 0.04, lam), v)
    rhs = ADJ.inner(dom, lam, P.taylor4_step(dom, A, 0.04, v))
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


@pytest.mark.parametrize("order", [4, 6])
def test_gradient_matches_central_differences(order):
    dom = _small(order=order, shape=(7, 7, 8))
    n = 6
    a_mid = pulse_midpoints(n, 0.05, n) * 4.0
    a_mid[:, 0] = 0.03
    dt = 0.05
    loss, grad = ADJ.loss_and_grad(dom, a_mid, dt, dom.psi)
    eps = 1e-5
    for k in (0, 2, 5):
        for d in (0, 2):
            ap, am = a_mid.copy(), a_mid.copy()
            ap[k, d] += eps
            am[k, d] -= eps
            fd_g = (ADJ.absorbed_energy(dom, ap, dt, dom.psi)[0]
                    - ADJ.absorbed_energy(dom, am, dt, dom.psi)[0]) / (2 * eps)
            assert abs(grad[k, d] - fd_g) <= 1e-6 * max(abs(fd_g), 1e-4), (k, d, grad[k, d], fd_g)


def _dense_ops_torch(dom):
    """-1/2 Lap, the three first-derivative matrices and V + v_nl, built with
    explicit index arithmetic (no np.roll) as torch complex128 matrices."""
    nx, ny, nz = dom.shape
    n = nx * ny * nz
    c, a = fd.second(dom.fd_order), fd.first(dom.fd_order)
    lap = np.zeros((n, n))
    d1 = [np.zeros((n, n)) for _ in range(3)]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                g = (z * ny + y) * nx + x
                lap[g, g] += 3 * c[0] / dom.h ** 2
                for axis, (ex, ey, ez) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    for m in range(1, len(c)):
                        for s in (1, -1):
                            gg = (((z + s * m * ez) % nz) * ny + (y + s * m * ey) % ny) * nx + (x + s * m * ex) % nx
                            lap[g, gg] += c[m] / dom.h ** 2
                            d1[axis][g, gg] += s * a[m - 1] / dom.h
    vnl = dom.proj @ np.diag(dom.d) @ dom.proj.conj().T * dom.h ** 3
    t = lambda m: torch.tensor(m, dtype=torch.complex128)
    return t(-0.5 * lap), [t(m) for m in d1], t(np.diag(dom.v_loc) + vnl)


def test_gradient_matches_torch_autograd():
    dom = _small(seed=22, shape=(5, 6, 5), order=2)
    n_steps, dt = 5, 0.06
    rng = np.random.default_rng(9)
    a_mid = rng.uniform(-0.3, 0.3, size=(n_steps, 3))
    kin, d1, rest = _dense_ops_torch(dom)
    ident = torch.eye(dom.n_grid, dtype=torch.complex128)
    a_t = torch.tensor(a_mid, dtype=torch.float64, requires_grad=True)
    psi0 = torch.tensor(dom.psi)
    occ = torch.tensor(dom.occ, dtype=torch.float64)
    h3 = dom.h ** 3

    def ham(A):
        m = kin + rest
        for d in range(3):
            m = m - 1j * A[d].to(torch.complex128) * d1[d]
        return m + 0.5 * (A @ A).to(torch.complex128) * ident

    def e0(psi):
        hp = ham(torch.zeros(3, dtype=torch.float64)) @ psi
        return (h3 * (psi.conj() * hp).sum(0).real * occ).sum()

    psi = psi0
    for k in range(n_steps):
        hm = ham(a_t[k])
        term, acc = psi, psi
        for m in range(1, 5):
            term = (-1j * dt / m) * (hm @ term)
            acc = acc + term
        psi = acc
    loss = e0(psi) - e0(psi0)
    loss.backward()
    ref = a_t.grad.numpy()
    l_or, g_or = ADJ.loss_and_grad(dom, a_mid, dt, dom.psi)
    assert abs(l_or - loss.item()) < 1e-12 * max(1.0, abs(loss.item()))
    assert np.abs(g_or - ref).max() < 1e-10 * max(1e-8, np.abs(ref).max())
