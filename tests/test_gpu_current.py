"""Macroscopic current (local plus nonlocal commutator part) through
dcmesh_current, and steps coupled to the Maxwell update of the field through
dcmesh_step_maxwell, against the FP64 oracle on the same (rounded) inputs:

* two domains of different shapes in one call, complex orbitals, a field with
  all three components; with and without the position-weighted projectors;
* six coupled steps from a field kick under a pulse: orbitals, induced field
  and its rate, per-step currents and step fields;
* the uniform electron gas on the GPU against the exact discrete plasma
  oscillation;
* the 64^3 / 128-orbital / 512-projector domain: the FP32 current against the
  oracle evaluated on the same orbitals.

FP64 is held to rounding; FP32 to 1e-5 of the scale of the terms that are
summed (the projector products accumulate in FP32).
"""
import math

import numpy as np
import pytest

from helpers import oracle_inputs, assert_close, to_device
from oracle import current as CUR
from synth import Domain, config, make_domain, projector_moments

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 1e-5}


def _perturbed(dom, seed, scale=0.2):
    rng = np.random.default_rng(seed)
    psi = dom.psi + scale * np.abs(dom.psi).max() * (rng.standard_normal(dom.psi.shape)
                                                     + 1j * rng.standard_normal(dom.psi.shape))
    return Domain(dom.shape, dom.h, dom.fd_order, psi, dom.v_loc, dom.proj, dom.d, dom.occ, dom.atoms)


def _proj_r(od, precision):
    """Position-weighted projectors of the (rounded) domain, rounded like the
    other inputs; returns (device tensor, the FP64 values the oracle uses)."""
    import torch
    from paper_2509_00966_amd import complex_dtype
    pr = projector_moments(od)
    if precision != "fp64":
        pr = pr.astype(np.complex64).astype(np.complex128)
    return torch.from_numpy(pr).to("cuda", complex_dtype(precision)).contiguous(), pr


def _scale(od, A, psi, pr):
    """Magnitude of the summed terms: the local current and the projector sum."""
    loc = np.abs(CUR.local_current(od, A, psi)).max()
    nl = 0.0
    if pr is not None and od.n_proj:
        from oracle import hamiltonian as H
        p = H.project(od, psi)
        nl = 2 * np.sum(np.abs(od.occ[None, :] * od.d[:, None] * p) *
                        np.max([np.abs(od.h ** 3 * (psi.conj().T @ pr[d]).conj().T) for d in range(3)], axis=0))
    return (loc + nl) / (od.n_grid * od.h ** 3)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nonlocal_part", [True, False])
def test_current_matches_oracle(precision, nonlocal_part):
    import torch
    import paper_2509_00966_amd as api
    doms = [_perturbed(make_domain(110, (16, 17, 18), 9, 2, proj_per_atom=8, h=0.4, fd_order=6), 1),
            _perturbed(make_domain(111, (12, 13, 11), 5, 1, proj_per_atom=4, h=0.45, fd_order=4), 2)]
    A = np.array([[0.07, -0.04, 0.11], [-0.02, 0.05, 0.03]])
    g = [to_device(d, precision) for d in doms]
    ods = [oracle_inputs(d, precision) for d in doms]
    prs = [_proj_r(od, precision) for od in ods]
    ws = api.Workspace.for_domains(g, precision)
    a = torch.from_numpy(A).to("cuda")
    got = api.current(g, a, precision, ws, proj_r=[p[0] for p in prs] if nonlocal_part else None,
                      a_per_domain=True).cpu().numpy()
    for i, od in enumerate(ods):
        pr = prs[i][1] if nonlocal_part else None
        ref = CUR.macroscopic_current(od, A[i], od.psi, pr)
        scale = _scale(od, A[i], od.psi, pr)
        assert np.abs(got[i] - ref).max() <= TOL[precision] * scale, (i, got[i], ref)
        if nonlocal_part:
            assert np.abs(CUR.nonlocal_current(od, od.psi, pr)).max() > 1e-4   # the term is exercised


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_coupled_steps_match_oracle(precision):
    import torch
    import paper_2509_00966_amd as api
    dom = _perturbed(make_domain(112, (16, 15, 17), 8, 2, proj_per_atom=8, h=0.4, fd_order=6), 3, 0.1)
    n, dt = 6, 0.02
    t = np.arange(n + 1) * dt
    a_ext = np.zeros((n + 1, 3))
    a_ext[:, 2] = 0.3 * np.sin(2.0 * t)
    a_ext[:, 0] = 0.05
    field0 = np.array([0.01, 0.0, -0.02, 0.3, -0.1, 0.2])
    g = to_device(dom, precision)
    od = oracle_inputs(dom, precision)
    pr_dev, pr = _proj_r(od, precision)
    ws = api.Workspace.for_domains([g], precision)
    field = torch.from_numpy(field0[None, :].copy()).to("cuda")
    mids, cur = api.step_maxwell([g], torch.from_numpy(a_ext).to("cuda"), dt, n, precision, ws, field,
                                 proj_r=[pr_dev], want_current=True)
    torch.cuda.synchronize()
    psi, a_ind, b, cur_ref, mids_ref = CUR.maxwell_propagate(od, a_ext, dt, od.psi, pr, field0[:3], field0[3:])
    tol = TOL[precision]
    assert_close(g.psi.cpu().numpy(), psi, tol)
    f = field.cpu().numpy()[0]
    assert np.abs(f[:3] - a_ind).max() < tol * np.abs(a_ind).max()
    assert np.abs(f[3:] - b).max() < tol * np.abs(b).max()
    assert np.abs(mids.cpu().numpy()[0] - mids_ref).max() < tol * np.abs(mids_ref).max()
    scale = _scale(od, a_ext[0] + field0[:3], od.psi, pr)
    assert np.abs(cur.cpu().numpy()[0] - cur_ref).max() < 10 * tol * scale


def test_uniform_gas_plasma_oscillation_on_gpu():
    import torch
    import paper_2509_00966_amd as api
    shape, h = (6, 7, 8), 0.5
    n_g = int(np.prod(shape))
    vol = n_g * h ** 3
    psi = np.full((n_g, 1), 1.0 / math.sqrt(vol), dtype=np.complex128)
    dom = Domain(shape, h, 4, psi, np.zeros(n_g), np.zeros((n_g, 0), np.complex128), np.zeros(0), np.array([2.0]))
    n, dt = 60, 0.05
    g = to_device(dom, "fp64")
    ws = api.Workspace.for_domains([g], "fp64")
    field = torch.tensor([[0.0, 0.0, 0.0, 0.0, 0.0, 0.01]], dtype=torch.float64, device="cuda")
    mids, cur = api.step_maxwell([g], torch.zeros(n + 1, 3, dtype=torch.float64, device="cuda"), dt, n, "fp64",
                                 ws, field, want_current=True)
    w2 = 4 * math.pi * 2.0 / vol
    theta = math.acos(1 - w2 * dt ** 2 / 2)
    k = np.arange(n + 1)
    a = dt * 0.01 * np.sin(k * theta) / math.sin(theta)
    assert abs(field.cpu().numpy()[0, 2] - a[n]) < 1e-12
    assert np.abs(mids.cpu().numpy()[0, :, 2] - 0.5 * (a[:n] + a[1:])).max() < 1e-12
    assert np.abs(cur.cpu().numpy()[0, :, 2] - 2.0 / vol * a[:n]).max() < 1e-12


def test_full_size_current_fp32():
    import torch
    import paper_2509_00966_amd as api
    w = config(2)
    dom = _perturbed(w.domains[0], 4, 0.05)
    g = to_device(dom, "fp32")
    od = oracle_inputs(dom, "fp32")
    pr_dev, pr = _proj_r(od, "fp32")
    ws = api.Workspace.for_domains([g], "fp32")
    A = np.array([0.0, 0.0, 0.05])
    got = api.current([g], torch.from_numpy(A).to("cuda"), "fp32", ws, proj_r=[pr_dev]).cpu().numpy()[0]
    ref = CUR.macroscopic_current(od, A, od.psi, pr)
    assert np.abs(got - ref).max() <= 1e-5 * _scale(od, A, od.psi, pr)
