"""Fourth-order Taylor propagation (oracle; test infrastructure only).

The step psi <- exp(-i dt H) psi is approximated by the truncated series
    psi_{k+1} = sum_{m=0}^{4} phi_m,   phi_0 = psi_k,   phi_m = (-i dt / m) H(A_k) phi_{m-1},
i.e. the explicit power sum (the library uses a nested form; this one is kept
deliberately different).  The vector potential of step k is the value at the
step midpoint t_k + dt/2, the midpoint rule of Eq. 2.

Per-step observables refer to the state entering step k, evaluated with that
step's field A_k.
"""
import numpy as np

from . import hamiltonian as H
from . import observables as O


def taylor4_step(dom, A, dt, psi):
    phi = psi
    out = psi.copy()
    for m in range(1, 5):
        phi = (-1j * dt / m) * H.apply_h(dom, A, phi)
        out = out + phi
    return out


def propagate(dom, a_mid, dt, psi, n_steps=None, want_rho=False, want_j=False,
              want_energy=False):
    """Run ``n_steps`` steps; returns (psi, dict of per-step observables)."""
    a_mid = np.asarray(a_mid, dtype=np.float64)
    n_steps = len(a_mid) if n_steps is None else n_steps
    obs = {"rho": [], "j": [], "energy": []}
    for k in range(n_steps):
        A = a_mid[k]
        if want_rho:
            obs["rho"].append(O.density(dom, psi))
        if want_j:
            obs["j"].append(O.current(dom, A, psi))
        if want_energy:
            obs["energy"].append(O.energy(dom, A, psi))
        psi = taylor4_step(dom, A, dt, psi)
    return psi, {k: np.array(v) for k, v in obs.items() if v}


def nonlocal_half_step(dom, psi, psi0, delta):
    """Eq. 2's nonlocal factor with the nonlocal operator in the space of the
    reference orbitals (Eq. 5): psi <- psi - delta Psi0 (h^3 Psi0^H psi), then each
    orbital rescaled to unit norm (the normaliser of Eq. 2)."""
    p = dom.h ** 3 * (psi.conj().T @ psi0).conj().T        # h^3 Psi0^H psi
    out = psi - delta * (psi0 @ p)
    norms = np.sqrt(dom.h ** 3 * np.sum(np.abs(out) ** 2, axis=0))
    return out / norms[None, :]


def eq2_step(dom, A, dt, psi, psi0, v_nl):
    """One step of Eq. 2: N exp(-i dt h_loc(A)) N with N the normalised
    half-step 1 - i dt v_nl / 2 of the reference-orbital projector v_nl
    |Psi0><Psi0| (delta = i dt v_nl / 2 in Eq. 5), and the local propagator
    taken as the fourth-order Taylor series of h_loc alone."""
    from synth import Domain
    loc = Domain(dom.shape, dom.h, dom.fd_order, dom.psi, dom.v_loc,
                 np.zeros((dom.n_grid, 0), np.complex128), np.zeros(0), dom.occ)
    delta = 0.5j * dt * v_nl
    psi = nonlocal_half_step(dom, psi, psi0, delta)
    psi = taylor4_step(loc, A, dt, psi)
    return nonlocal_half_step(dom, psi, psi0, delta)


def eq2_propagate(dom, a_mid, dt, psi, psi0, v_nl, n_steps=None):
    a_mid = np.asarray(a_mid, dtype=np.float64)
    n_steps = len(a_mid) if n_steps is None else n_steps
    for k in range(n_steps):
        psi = eq2_step(dom, a_mid[k], dt, psi, psi0, v_nl)
    return psi
