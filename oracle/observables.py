"""Density, current, energy and overlap (oracle; test infrastructure only).

* rho(r)  = sum_n f_n |psi_n(r)|^2                       (so h^3 sum rho = sum f);
* j_d(r)  = sum_n f_n [Im(conj(psi_n) D1_d psi_n) + A_d |psi_n|^2]
  the local particle current of the kinetic term of Eq. 3 (paramagnetic plus
  diamagnetic part; the nonlocal commutator term is not included);
* E       = h^3 sum_n f_n <psi_n | H(A) psi_n>, real part, in FP64;
* S       = h^3 Psi^H Psi, the orbital overlap (Sec. V.B.5's Psi^H Psi form).
"""
import numpy as np

from . import hamiltonian as H


def density(dom, psi):
    return np.abs(psi) ** 2 @ dom.occ


def current(dom, A, psi):
    A = np.asarray(A, dtype=np.float64)
    u4 = H.grid4(psi, dom.shape)
    w = np.abs(psi) ** 2 @ dom.occ
    j = np.empty((psi.shape[0], 3))
    for d in range(3):
        g = H.derivative(u4, dom.h, dom.fd_order, d).reshape(psi.shape)
        j[:, d] = np.imag(np.conj(psi) * g) @ dom.occ + A[d] * w
    return j


def energy(dom, A, psi):
    hpsi = H.apply_h(dom, A, psi)
    return float(np.real(dom.h ** 3 * np.sum(np.conj(psi) * hpsi, axis=0) @ dom.occ))


def energy_parts(dom, A, psi):
    """(local, nonlocal) parts of the energy."""
    hl = H.apply_hloc(dom, A, psi)
    e_loc = float(np.real(dom.h ** 3 * np.sum(np.conj(psi) * hl, axis=0) @ dom.occ))
    if dom.n_proj == 0:
        return e_loc, 0.0
    p = H.project(dom, psi)
    e_nl = float(np.real((dom.d[:, None] * np.abs(p) ** 2).sum(axis=0) @ dom.occ))
    return e_loc, e_nl


def overlap(dom, psi):
    return dom.h ** 3 * (psi.conj().T @ psi)


def occupied_h(dom, A, psi):
    """f_n H(A) psi_n for every orbital."""
    return H.apply_h(dom, A, psi) * dom.occ[None, :]
