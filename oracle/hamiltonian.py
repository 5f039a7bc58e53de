"""H(A) psi for one domain (oracle; test infrastructure only).

Eq. 3 in atomic units (hbar = m = 1, e/c folded into A):
    h = 1/2 (-i grad + A)^2 + v_loc + v_nl
      = -1/2 Lap - i A.grad + 1/2 |A|^2 + v_loc + v_nl,
with grad and Lap replaced by periodic central finite differences (Sec. V.A.5)
and the nonlocal part written as projector products in the spirit of Sec. V.B.5:
    v_nl psi = B (D o P),   P = h^3 B^H psi   (<a|b> = h^3 sum_g conj(a_g) b_g).

Orbitals are handled as a 4-D array [nz, ny, nx, N_o] so that np.roll along an
axis gives the neighbour at +-m mesh points.
"""
import numpy as np

from . import fd

_AXIS = {0: 2, 1: 1, 2: 0}     # Cartesian direction d -> array axis of [nz, ny, nx, N_o]


def grid4(u, shape):
    """View [N_g, N_o] as [nz, ny, nx, N_o]."""
    nx, ny, nz = shape
    return u.reshape(nz, ny, nx, -1)


def laplacian(u4, h, order):
    """Periodic finite-difference Laplacian of every orbital."""
    c = fd.second(order)
    out = 3.0 * c[0] * u4
    for d in range(3):
        ax = _AXIS[d]
        for m in range(1, len(c)):
            out = out + c[m] * (np.roll(u4, -m, axis=ax) + np.roll(u4, m, axis=ax))
    return out / h ** 2


def derivative(u4, h, order, d):
    """Periodic finite-difference first derivative along Cartesian direction d."""
    a = fd.first(order)
    ax = _AXIS[d]
    out = np.zeros_like(u4)
    for m in range(1, len(a) + 1):
        out = out + a[m - 1] * (np.roll(u4, -m, axis=ax) - np.roll(u4, m, axis=ax))
    return out / h


def apply_hloc(dom, A, u):
    """Local part: (-1/2 Lap - i A.grad + v_loc + 1/2 |A|^2) u, u of shape [N_g, N_o]."""
    A = np.asarray(A, dtype=np.float64)
    u4 = grid4(u, dom.shape)
    y = -0.5 * laplacian(u4, dom.h, dom.fd_order)
    for d in range(3):
        if A[d] != 0.0:
            y = y - 1j * A[d] * derivative(u4, dom.h, dom.fd_order, d)
    y = y.reshape(u.shape)
    return y + (dom.v_loc + 0.5 * float(A @ A))[:, None] * u


def project(dom, u):
    """P = h^3 B^H u, shape [N_p, N_o], evaluated as h^3 (u^H B)^H so that the
    (large) projector array is never copied."""
    return dom.h ** 3 * (u.conj().T @ dom.proj).conj().T


def apply_vnl(dom, u):
    """Nonlocal part B (D o P)."""
    if dom.n_proj == 0:
        return np.zeros_like(u)
    return dom.proj @ (dom.d[:, None] * project(dom, u))


def apply_h(dom, A, u):
    """Full H(A) u."""
    return apply_hloc(dom, A, u) + apply_vnl(dom, u)


def dh_da(dom, A, u, d):
    """(dH/dA_d) u = -i D1_d u + A_d u (only the kinetic term depends on A)."""
    u4 = grid4(u, dom.shape)
    return (-1j * derivative(u4, dom.h, dom.fd_order, d)).reshape(u.shape) + A[d] * u


def dense(dom, A):
    """Assemble H(A) as an N_g x N_g matrix by applying it to unit vectors
    (tiny grids only)."""
    n = dom.n_grid
    return apply_h(dom, A, np.eye(n, dtype=np.complex128))
