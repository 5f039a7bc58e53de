"""Macroscopic current and its coupling to the Maxwell equation for the
vector potential (oracle; test infrastructure only).

The particle velocity of H(A) (Eq. 3, e/c folded into A) is v = i[H, r] =
-i grad + A + i[V_nl, r].  Its local part gives the current density j of the
observables module; the nonlocal commutator contributes, per orbital,
<psi| i[V_nl, r_d] |psi> = -2 Im <psi| V_nl r_d |psi>, which with
V_nl = sum_p |b_p> D_p <b_p| becomes a sum over projector pairs (the
electric-current half of Sec. V.B.5's GEMMification):

    J_nl,d = -2 sum_{n,p} f_n D_p Im( conj(P_pn) R_d,pn ),
    P = h^3 B^H Psi,  R_d = h^3 B_d^H Psi,  B_d = (r - R_atom)_d B,

r measured from each projector's own atom (the commutator of a projector
with a constant vanishes, so any per-projector origin gives the same result).
The macroscopic current density is J = (h^3 sum_g j(g) + J_nl) / Omega.

A uniform vector potential obeys Ampere's law with no curl term; for the
particle current of electrons (charge -1, atomic units) the induced part obeys
d^2 A_ind / dt^2 = -4 pi J.  It is advanced by a leapfrog with A_ind at step
times and its rate b at half steps (the reading taken for the Maxwell update):

    J_k     = J(psi_k, A_ext(t_k) + A_ind,k)
    b       <- b - 4 pi dt J_k
    A_ind,k+1 = A_ind,k + dt b
    psi_k+1 = T4(-i dt H(A_mid)) psi_k,  A_mid = average of A_ext and A_ind over t_k, t_k+1.
"""
import numpy as np

from . import hamiltonian as H
from . import observables as O
from . import propagate as P


def nonlocal_current(dom, psi, proj_r):
    """J_nl [3], the occupation-weighted nonlocal commutator current (not / Omega)."""
    if dom.n_proj == 0:
        return np.zeros(3)
    p = H.project(dom, psi)                                   # h^3 B^H psi
    out = np.zeros(3)
    for d in range(3):
        r = dom.h ** 3 * (psi.conj().T @ proj_r[d]).conj().T  # h^3 B_d^H psi
        out[d] = -2.0 * np.sum(dom.occ[None, :] * dom.d[:, None] * np.imag(np.conj(p) * r))
    return out


def local_current(dom, A, psi):
    """h^3 sum_g j(g) [3] (paramagnetic plus diamagnetic, not / Omega)."""
    return dom.h ** 3 * O.current(dom, A, psi).sum(axis=0)


def macroscopic_current(dom, A, psi, proj_r=None):
    vol = dom.n_grid * dom.h ** 3
    j = local_current(dom, A, psi)
    if proj_r is not None:
        j = j + nonlocal_current(dom, psi, proj_r)
    return j / vol


def maxwell_propagate(dom, a_ext, dt, psi, proj_r=None, a_ind=None, b=None):
    """n = len(a_ext) - 1 steps of the coupled scheme; a_ext [n+1, 3] at the
    step times.  Returns (psi, a_ind, b, currents [n, 3], step fields [n, 3])."""
    a_ext = np.asarray(a_ext, dtype=np.float64)
    a_ind = np.zeros(3) if a_ind is None else np.array(a_ind, dtype=np.float64)
    b = np.zeros(3) if b is None else np.array(b, dtype=np.float64)
    cur, mids = [], []
    for k in range(len(a_ext) - 1):
        j = macroscopic_current(dom, a_ext[k] + a_ind, psi, proj_r)
        b = b - 4.0 * np.pi * dt * j
        a_new = a_ind + dt * b
        a_mid = 0.5 * (a_ext[k] + a_ext[k + 1]) + 0.5 * (a_ind + a_new)
        psi = P.taylor4_step(dom, a_mid, dt, psi)
        a_ind = a_new
        cur.append(j)
        mids.append(a_mid)
    return psi, a_ind, b, np.array(cur).reshape(-1, 3), np.array(mids).reshape(-1, 3)
