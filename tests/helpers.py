"""Shared test helpers: moving seeded synth domains onto the GPU and error
metrics.  (Not a test module.)"""
import os
from typing import NamedTuple, Optional

import numpy as np


def to_device(dom, precision, device="cuda"):
    """synth.Domain (FP64 numpy) -> paper_2509_00966_amd.Domain on the GPU."""
    import torch
    from paper_2509_00966_amd import Domain, complex_dtype, real_dtype

    cd, rd = complex_dtype(precision), real_dtype(precision)

    def t(x, dt):
        return torch.from_numpy(np.ascontiguousarray(x)).to(device=device, dtype=dt).contiguous()

    return Domain(tuple(dom.shape), dom.fd_order, dom.h, t(dom.psi, cd), t(dom.v_loc, rd),
                  t(dom.proj, cd), t(dom.d, rd), t(dom.occ, rd))


def oracle_inputs(dom, precision):
    """The FP64 oracle consumes the same rounded inputs the GPU path sees."""
    return dom if precision == "fp64" else dom.rounded(np.float32)


def rel_fro(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


class Errors(NamedTuple):
    fro: float             # ||got - ref||_F / ||ref||_F over the whole array
    elem: float            # max |got - ref| / max |ref|
    orb: Optional[float]   # max over orbitals n of ||got_n - ref_n|| / ||ref_n|| (last axis)


def errors(got, ref, orbitals=True):
    """Three views of the error: the relative Frobenius norm (the bar's
    definition), the element-wise maximum relative to the largest reference
    value (a local error, e.g. one tile's halo, is not diluted by the rest of
    the array), and the worst orbital (the last axis) on its own norm."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    d = got - ref
    fro = float(np.linalg.norm(d) / np.linalg.norm(ref))
    elem = float(np.abs(d).max() / np.abs(ref).max())
    orb = None
    if orbitals and ref.ndim >= 2:
        ax = tuple(range(ref.ndim - 1))
        num = np.sqrt((np.abs(d) ** 2).sum(axis=ax))
        den = np.sqrt((np.abs(ref) ** 2).sum(axis=ax))
        orb = float((num / den).max())
    return Errors(fro, elem, orb)


def assert_close(got, ref, tol, orbitals=True, label=""):
    """All three error views of ``errors`` within ``tol`` (one number for all
    three, or an ``Errors`` of per-view bounds); the measured values are
    printed (``pytest -s`` shows them) and named in the failure."""
    e = errors(got, ref, orbitals)
    t = tol if isinstance(tol, Errors) else Errors(tol, tol, tol)
    test = os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0]
    orb = "-" if e.orb is None else f"{e.orb:.2e}"
    tol_s = f"{t.fro:.1e}/{t.elem:.1e}/{t.orb:.1e}" if isinstance(tol, Errors) else f"{tol:.1e}"
    msg = f"[parity] {test} {label} fro={e.fro:.2e} elem={e.elem:.2e} orb={orb} tol={tol_s}"
    print(msg)
    assert e.fro <= t.fro and e.elem <= t.elem and (e.orb is None or e.orb <= t.orb), msg
    return e


U32 = 2.0 ** -24      # unit roundoff of FP32


def magnitude_h(dom, A, u):
    """|H(A)| |u|: every term of H(A) u by magnitude (absolute FD weights,
    |A_d|, |v_loc + |A|^2/2|, |B| |D| h^3 |B|^T), summed.  An FP32 evaluation
    of H u from FP32 inputs errs by a few units of roundoff of this sum
    (the forward error of a sum of terms is bounded by the sum of their
    magnitudes times the roundoff of its accumulation chain)."""
    from oracle import fd
    from oracle import hamiltonian as H
    A = np.asarray(A, dtype=np.float64)
    au = np.abs(u)
    u4 = H.grid4(au, dom.shape)
    c, a, h = fd.second(dom.fd_order), fd.first(dom.fd_order), dom.h
    out = 0.5 * abs(3 * c[0]) / h ** 2 * u4
    for d in range(3):
        ax = H._AXIS[d]
        for m in range(1, len(c)):
            out = out + 0.5 * abs(c[m]) / h ** 2 * (np.roll(u4, -m, axis=ax) + np.roll(u4, m, axis=ax))
        if A[d] != 0.0:
            for m in range(1, len(a) + 1):
                out = out + abs(A[d] * a[m - 1]) / h * (np.roll(u4, -m, axis=ax) + np.roll(u4, m, axis=ax))
    out = out.reshape(u.shape) + np.abs(dom.v_loc + 0.5 * float(A @ A))[:, None] * au
    if dom.n_proj:
        out = out + np.abs(dom.proj) @ (np.abs(dom.d)[:, None] * (dom.h ** 3 * (np.abs(dom.proj).T @ au)))
    return out


def fp32_operator_tol(dom, A, u, ref, c=2.0, c_elem=4.0, occ_scale=True):
    """Bounds on the three error views of an FP32 H u against the exact H u
    (``ref``) of the same FP32 inputs: c U32 kappa per view, kappa the
    condition number of the sum (the magnitude sum |H||u| against |H u|, in
    the norm of that view).  The measured errors of the library's stencil
    and projector products sit at 0.5-0.6 U32 kappa in the norm views and
    1.1-1.5 U32 kappa in the element-wise view (the largest of ~1e5
    elements' rounding errors); c = 2 (norms) and c_elem = 4 leave room for a
    different accumulation order without admitting a wrong term (which errs
    by O(kappa) times more).  occ_scale: ``ref`` is f_n H u_n, so the
    magnitudes carry the same occupation factors."""
    M = magnitude_h(dom, A, u)
    if occ_scale:
        M = M * np.abs(dom.occ)[None, :]
    ax = tuple(range(ref.ndim - 1))
    k_fro = np.linalg.norm(M) / np.linalg.norm(ref)
    k_elem = np.abs(M).max() / np.abs(ref).max()
    k_orb = (np.sqrt((M ** 2).sum(axis=ax)) / np.sqrt((np.abs(ref) ** 2).sum(axis=ax))).max()
    return Errors(c * U32 * k_fro, c_elem * U32 * k_elem, c * U32 * k_orb)


def propagate_logged(dom, a_mid, dt, psi, label="", chunk=10):
    """The oracle's propagate() in chunks of ``chunk`` steps, printing one
    progress line per chunk (long oracle runs inside GPU tests stay visible)."""
    import sys
    from oracle import propagate as P
    for k in range(0, len(a_mid), chunk):
        psi, _ = P.propagate(dom, a_mid[k:k + chunk], dt, psi)
        print(f"[oracle] {label} step {min(k + chunk, len(a_mid))}/{len(a_mid)}", flush=True)
        sys.stdout.flush()
    return psi


def a_tensor(a_mid, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a_mid, dtype=np.float64)).to(device)
