"""Occupations f_s of the reference orbitals and the excited-electron count
n_exc through dcmesh_occupations, against the FP64 oracle on the same inputs:

* three ragged domains in one call (5, 21 and 70 orbitals: one, two and three
  64-wide overlap tiles with tails), orbitals rotated partly out of the
  reference span, every precision mode; the optional overlap output on one;
* a domain propagated under a pulse through dcmesh_step (its orbitals are not
  eigenstates, so weight leaves the initial span): n_exc at the start and
  after the steps against the oracle on the same orbitals;
* the 64^3 / 128-orbital / 512-projector workload after FP32 steps, against
  the oracle on the same orbitals (a property that holds at any size).

The overlap accumulates exact FP64 products of the stored values, so every
mode is held to FP64 rounding of the sums.
"""
import numpy as np
import pytest

from helpers import a_tensor, oracle_inputs, to_device
from oracle import occupations as OC
from synth import Domain, config, make_domain, pulse_midpoints

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _rotated(dom, seed, scale):
    """Orbitals mixed inside the span and rotated partly out of it."""
    rng = np.random.default_rng(seed)
    n = dom.psi.shape[1]
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    leak = rng.standard_normal(dom.psi.shape) + 1j * rng.standard_normal(dom.psi.shape)
    psi = dom.psi @ q + scale * np.abs(dom.psi).max() * leak
    return Domain(dom.shape, dom.h, dom.fd_order, psi, dom.v_loc, dom.proj, dom.d, dom.occ)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "split_bf16", "split_fp16"])
def test_ragged_batch_matches_oracle(precision):
    import torch
    import paper_2509_00966_amd as api
    refs = [make_domain(60, (9, 10, 11), 5, 1, proj_per_atom=4, h=0.45, fd_order=4),
            make_domain(61, (14, 12, 13), 21, 2, proj_per_atom=8, h=0.4, fd_order=6),
            make_domain(62, (16, 15, 17), 70, 3, proj_per_atom=8, h=0.4, fd_order=6)]
    for i, d in enumerate(refs):
        d.occ = np.linspace(2.0, 0.5, d.psi.shape[1])
    now = [_rotated(d, 70 + i, 0.05 * (i + 1)) for i, d in enumerate(refs)]
    g = [to_device(d, precision) for d in now]
    g0 = [to_device(d, precision) for d in refs]
    ws = api.Workspace.for_domains(g, precision)
    s_out = torch.zeros(70, 70, 2, dtype=torch.float64, device="cuda")
    f, n_exc = api.occupations(g, [x.psi for x in g0], precision, ws, overlap=[None, None, s_out])
    torch.cuda.synchronize()
    for i, (r, d) in enumerate(zip(refs, now)):
        o0, o1 = oracle_inputs(r, precision), oracle_inputs(d, precision)
        f_ref, n_ref = OC.occupations(o1, o0.psi, o1.psi)
        tot = o1.occ.sum()
        assert np.abs(f[i].cpu().numpy() - f_ref).max() < TOL * tot, i
        assert abs(n_exc[i].item() - n_ref) < TOL * tot, i
        assert n_ref > 1e-3 * tot                    # the leak is visible
    s_ref = OC.cross_overlap(oracle_inputs(now[2], precision), oracle_inputs(refs[2], precision).psi,
                             oracle_inputs(now[2], precision).psi)
    got = s_out.cpu().numpy()
    assert np.abs(got[..., 0] + 1j * got[..., 1] - s_ref).max() < TOL


def test_propagation_moves_weight_out_of_the_span():
    import torch
    import paper_2509_00966_amd as api
    dom = make_domain(63, (20, 20, 20), 16, 4, proj_per_atom=8, h=0.4, fd_order=6)
    n, dt = 40, 0.02
    a_mid = pulse_midpoints(n, dt, n) * 40.0          # a strong pulse along z
    g = to_device(dom, "fp32")
    psi0 = g.psi.clone()
    ws = api.Workspace.for_domains([g], "fp32")
    _, e0 = api.occupations([g], [psi0], "fp32", ws)
    api.step([g], a_tensor(a_mid), dt, n, "fp32", ws)
    f, e1 = api.occupations([g], [psi0], "fp32", ws)
    torch.cuda.synchronize()
    od = oracle_inputs(dom, "fp32")
    cur = Domain(od.shape, od.h, od.fd_order, g.psi.cpu().numpy().astype(np.complex128), od.v_loc,
                 od.proj, od.d, od.occ)
    f_ref, n_ref = OC.occupations(cur, od.psi, cur.psi)
    _, n0_ref = OC.occupations(od, od.psi, od.psi)     # FP32-rounded orbitals are orthonormal to ~1e-7
    assert abs(e0.item() - n0_ref) < TOL * od.occ.sum()
    assert abs(n0_ref) < 1e-5 * od.occ.sum()
    assert n_ref > 1e-4 * od.occ.sum()
    assert abs(e1.item() - n_ref) < TOL * od.occ.sum()
    assert np.abs(f[0].cpu().numpy() - f_ref).max() < TOL * od.occ.sum()


def test_full_size_workload_matches_oracle_on_propagated_orbitals():
    import torch
    import paper_2509_00966_amd as api
    w = config(2)
    dom = w.domains[0]
    g = to_device(dom, "fp32")
    psi0 = g.psi.clone()
    ws = api.Workspace.for_domains([g], "fp32")
    api.step([g], a_tensor(w.a_mid[:5] * 20.0), w.dt, 5, "fp32", ws)
    f, n_exc = api.occupations([g], [psi0], "fp32", ws)
    torch.cuda.synchronize()
    od = oracle_inputs(dom, "fp32")
    psi_t = g.psi.cpu().numpy().astype(np.complex128)
    cur = Domain(od.shape, od.h, od.fd_order, psi_t, od.v_loc, od.proj, od.d, od.occ)
    f_ref, n_ref = OC.occupations(cur, od.psi, psi_t)
    tot = od.occ.sum()
    assert np.abs(f[0].cpu().numpy() - f_ref).max() < TOL * tot
    assert abs(n_exc[0].item() - n_ref) < TOL * tot
