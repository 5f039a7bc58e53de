"""Occupations of the reference orbitals and the number of excited electrons
(oracle; test infrastructure only).

The local field dynamics hands the atomic dynamics the occupation numbers
f_s of the domain's Kohn-Sham states and, from them, the number of
photo-excited electrons n_exc (Sec. V.A.3 and V.A.8).  The paper gives no
formula; the projection reading is taken here.  The reference states are the
orbitals Psi(0) that also define Eq. 5's nonlocal operator:

    S_sn  = h^3 <psi_s(0) | psi_n(t)>                  (cross overlap)
    f_s   = sum_n f_n |S_sn|^2                         (weight of reference state s)
    n_exc = sum_n f_n (h^3 <psi_n(t)|psi_n(t)> - sum_s |S_sn|^2)

n_exc is the occupation-weighted norm of the part of each orbital outside the
span of orthonormal reference orbitals.  It does not count the small norm change
of a truncated Taylor step as excitation: sum_s f_s + n_exc = sum_n f_n |psi_n|^2.
"""
import numpy as np


def cross_overlap(dom, psi0, psi):
    """S = h^3 Psi0^H Psi, [n_ref][n_orb]."""
    return dom.h ** 3 * (psi0.conj().T @ psi)


def occupations(dom, psi0, psi):
    """(f [n_ref], n_exc) of the orbitals psi with occupations dom.occ."""
    s2 = np.abs(cross_overlap(dom, psi0, psi)) ** 2
    f = s2 @ dom.occ
    norms = dom.h ** 3 * np.sum(np.abs(psi) ** 2, axis=0)
    n_exc = float(dom.occ @ (norms - s2.sum(axis=0)))
    return f, n_exc
