"""Gradient of the absorbed energy w.r.t. the vector-potential samples
(oracle; test infrastructure only).

Loss: the field-free energy gained over the run,
    L = E0[psi_N] - E0[psi_0],   E0[psi] = h^3 sum_n f_n <psi_n | H(A=0) psi_n>.
With psi_{k+1} = U_k psi_k, U_k = T4(-i dt H(A_k)) and H Hermitian,
    dL/dA_{k,d} = 2 Re <lambda_{k+1}, (dU_k/dA_{k,d}) psi_k>,
    lambda_N = f o H(0) psi_N,   lambda_k = U_k^H lambda_{k+1} = T4(+i dt H(A_k)) lambda_{k+1},
where <a, b> = h^3 sum_{g,n} conj(a) b.  (dU_k/dA) psi_k is obtained here by
forward-mode differentiation of the explicit power sum,
    d phi_m = (-i dt / m) [ (dH/dA) phi_{m-1} + H d phi_{m-1} ],
with dH/dA_d = -i D1_d + A_d (Eq. 3: only the kinetic term depends on A).
"""
import numpy as np

from . import hamiltonian as H
from . import observables as O
from .propagate import taylor4_step


def inner(dom, a, b):
    """<a, b> = h^3 sum conj(a) b over grid and orbitals."""
    return dom.h ** 3 * np.vdot(a, b)


def taylor4_adjoint(dom, A, dt, lam):
    """U^H lam = sum_m (+i dt H)^m / m! lam."""
    phi = lam
    out = lam.copy()
    for m in range(1, 5):
        phi = (1j * dt / m) * H.apply_h(dom, A, phi)
        out = out + phi
    return out


def dstep(dom, A, dt, psi, d):
    """(dU/dA_d) psi by forward-mode differentiation of the power sum."""
    phi = psi
    dphi = np.zeros_like(psi)
    out = np.zeros_like(psi)
    for m in range(1, 5):
        c = -1j * dt / m
        dphi = c * (H.dh_da(dom, A, phi, d) + H.apply_h(dom, A, dphi))
        phi = c * H.apply_h(dom, A, phi)
        out = out + dphi
    return out


def absorbed_energy(dom, a_mid, dt, psi0):
    psi = psi0
    for k in range(len(a_mid)):
        psi = taylor4_step(dom, a_mid[k], dt, psi)
    zero = np.zeros(3)
    return O.energy(dom, zero, psi) - O.energy(dom, zero, psi0), psi


def adjoint_step(dom, A, dt, psi_k, lam_next, dirs=(0, 1, 2)):
    """Returns (lambda_k, g_k) with g_k[d] = 2 Re <lambda_{k+1}, dU/dA_d psi_k>."""
    g = np.zeros(3)
    for d in dirs:
        g[d] = 2.0 * np.real(inner(dom, lam_next, dstep(dom, A, dt, psi_k, d)))
    return taylor4_adjoint(dom, A, dt, lam_next), g


def loss_and_grad(dom, a_mid, dt, psi0, dirs=(0, 1, 2)):
    """(L, dL/dA [n_steps, 3]) by a full forward sweep and the adjoint sweep."""
    a_mid = np.asarray(a_mid, dtype=np.float64)
    states = [psi0]
    for k in range(len(a_mid)):
        states.append(taylor4_step(dom, a_mid[k], dt, states[-1]))
    zero = np.zeros(3)
    loss = O.energy(dom, zero, states[-1]) - O.energy(dom, zero, psi0)
    lam = O.occupied_h(dom, zero, states[-1])
    grad = np.zeros((len(a_mid), 3))
    for k in range(len(a_mid) - 1, -1, -1):
        lam, grad[k] = adjoint_step(dom, a_mid[k], dt, states[k], lam, dirs)
    return loss, grad
