"""GPU parity of the split-precision (BF16 / FP16 hi+lo) projector products.

Operator level: the library's H psi in split mode against the oracle's
split-form operator (same two-term rounding of every operand, products summed
exactly) -- the remaining difference is FP32 accumulation, bounded here by
2 U32 kappa in the norm views and 4 U32 kappa element-wise (kappa: the
condition number of the operator's sum of terms, helpers.fp32_operator_tol).  Propagation level: the split path against the FP64 oracle
after 20 steps, within 1e-4 (BF16) / 1e-5 (FP16) relative on psi.
"""
import numpy as np
import pytest

from helpers import a_tensor, assert_close, fp32_operator_tol, oracle_inputs, to_device
from oracle import hamiltonian as H
from oracle import propagate as P
from oracle import split as S
from synth import make_domain, pulse_midpoints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_2509_00966_amd as api
    return api


def _np(t):
    return t.detach().cpu().numpy()


def _dom(seed=51):
    return make_domain(seed, (19, 13, 21), 21, 3, proj_per_atom=8, h=0.4, fd_order=6)


@pytest.mark.parametrize("corr_variant", [-1, 0, 1, 2, 3, 4, 5, 7])
@pytest.mark.parametrize("precision,mode", [("split_bf16", "bf16"), ("split_fp16", "fp16")])
def test_split_hpsi_matches_split_reference(api, precision, mode, corr_variant):
    """Every correction tile variant (4 and 5: both tiles loaded into LDS
    directly, two-stage on four waves and three-stage on eight; 7: every
    orbital in one block); 21 orbitals and 24 projectors leave partial tiles
    in both dimensions."""
    import torch
    dom = _dom()
    A = np.array([0.05, -0.11, 0.23])
    g = to_device(dom, precision)
    ws = api.Workspace.for_domains([g], precision)
    hp = torch.empty_like(g.psi)
    try:
        api.set_tuning("correct", corr_variant)
        api.density([g], a_tensor(A[None]), precision, ws, [dict(hpsi_occ=hp)])
        torch.cuda.synchronize()
    finally:
        api.set_tuning("correct", -1)
    od = dom.rounded(np.float32)
    ref = (H.apply_hloc(od, A, od.psi) * od.occ[None, :]
           + S.apply_vnl_split(od, od.psi, mode, occ_scale=True))
    assert_close(_np(hp), ref, fp32_operator_tol(od, A, od.psi, ref))
    # and the split rounding is visible against the exact operator (the mode ran)
    exact = H.apply_h(od, A, od.psi) * od.occ[None, :]
    nl = np.linalg.norm(S.apply_vnl_split(od, od.psi, mode, occ_scale=True) - H.apply_vnl(od, od.psi) * od.occ)
    assert nl > 0
    assert_close(_np(hp), exact, (2e-4 if mode == "bf16" else 2e-5))


@pytest.mark.parametrize("corr_variant", [4, 5, 7])
@pytest.mark.parametrize("precision,mode", [("split_bf16", "bf16"), ("split_fp16", "fp16")])
def test_split_correction_stage_counts(api, precision, mode, corr_variant):
    """The correction kernels that load both tiles into LDS directly, over
    reductions of 9, 10 and 11 stages of 32 (136, 160 and 168 projectors):
    the three-stage ring ends on each of its three buffers; 70 orbitals give a
    ragged second column tile for the four-wave kernel."""
    import torch
    doms = [make_domain(53 + k, (12, 11, 13), 70, na, proj_per_atom=8, h=0.4, fd_order=4)
            for k, na in enumerate((17, 20, 21))]
    A = np.array([0.05, -0.11, 0.23])
    g = [to_device(d, precision) for d in doms]
    ws = api.Workspace.for_domains(g, precision)
    hp = [torch.empty_like(x.psi) for x in g]
    try:
        api.set_tuning("correct", corr_variant)
        api.density(g, a_tensor(A[None]), precision, ws, [dict(hpsi_occ=h) for h in hp])
        torch.cuda.synchronize()
    finally:
        api.set_tuning("correct", -1)
    for i, dom in enumerate(doms):
        od = dom.rounded(np.float32)
        ref = (H.apply_hloc(od, A, od.psi) * od.occ[None, :]
               + S.apply_vnl_split(od, od.psi, mode, occ_scale=True))
        assert_close(_np(hp[i]), ref, fp32_operator_tol(od, A, od.psi, ref), label=str(i))


@pytest.mark.parametrize("proj_variant", [0, 1, 2, 3, 4, 5, 6, 8])
@pytest.mark.parametrize("precision,mode", [("split_bf16", "bf16"), ("split_fp16", "fp16")])
def test_split_projection_variants_match_split_reference(api, precision, mode, proj_variant):
    """Every projection tile variant (4, 5 and 6: the projector planes loaded
    into LDS directly, two-stage 128 x 128, three-stage 128 x 256, two-stage
    64 x 64; 8: every orbital in one block, 64 projectors) on
    three domains: 24 projectors / 21 orbitals (one partial tile), 136
    projectors / 70 orbitals (a second tile in both dimensions with a ragged
    edge) and a 100-point grid (seven 16-point stages, fewer than one turn of
    the unrolled ring); the larger grids end in partial stages."""
    import torch
    doms = [_dom(), make_domain(52, (18, 17, 16), 70, 17, proj_per_atom=8, h=0.4, fd_order=4),
            make_domain(54, (5, 5, 4), 9, 2, proj_per_atom=8, h=0.5, fd_order=2)]
    A = np.array([0.05, -0.11, 0.23])
    g = [to_device(d, precision) for d in doms]
    ws = api.Workspace.for_domains(g, precision)
    hp = [torch.empty_like(x.psi) for x in g]
    try:
        api.set_tuning("project", proj_variant)
        api.density(g, a_tensor(np.stack([A, -A, A])), precision, ws, [dict(hpsi_occ=h) for h in hp],
                    a_per_domain=True)
        torch.cuda.synchronize()
    finally:
        api.set_tuning("project", -1)
    for i, dom in enumerate(doms):
        od = dom.rounded(np.float32)
        a = -A if i == 1 else A
        ref = (H.apply_hloc(od, a, od.psi) * od.occ[None, :]
               + S.apply_vnl_split(od, od.psi, mode, occ_scale=True))
        assert_close(_np(hp[i]), ref, fp32_operator_tol(od, a, od.psi, ref), label=str(i))


@pytest.mark.parametrize("precision,tol", [("split_bf16", 1e-4), ("split_fp16", 1e-5)])
def test_split_step_close_to_fp64_oracle(api, precision, tol):
    import torch
    dom = _dom(seed=52)
    n = 20
    a_mid = pulse_midpoints(n, 0.02, n) * 4.0
    g = to_device(dom, precision)
    ws = api.Workspace.for_domains([g], precision)
    e = torch.zeros(n, dtype=torch.float64, device="cuda")
    api.step([g], a_tensor(a_mid), 0.02, n, precision, ws, obs=[dict(energy=e)])
    torch.cuda.synchronize()
    od = oracle_inputs(dom, "fp32")
    ref, ro = P.propagate(od, a_mid, 0.02, od.psi, want_energy=True)
    assert_close(_np(g.psi), ref, tol)
    assert np.abs(_np(e) - ro["energy"]).max() < 10 * tol * np.abs(ro["energy"]).max()


def test_split_batched_equals_single(api):
    import torch
    doms = [make_domain(60 + i, shp, no, na, proj_per_atom=8, h=0.4, fd_order=6)
            for i, (shp, no, na) in enumerate([((20, 21, 22), 17, 4), ((22, 20, 20), 30, 7)])]
    a_mid = pulse_midpoints(2, 0.02, 2)
    for precision in ("split_bf16", "split_fp16"):
        gs = [to_device(d, precision) for d in doms]
        ws = api.Workspace.for_domains(gs, precision)
        api.step(gs, a_tensor(a_mid), 0.02, 2, precision, ws)
        for d, gb in zip(doms, gs):
            g1 = to_device(d, precision)
            ws1 = api.Workspace.for_domains([g1], precision)
            api.step([g1], a_tensor(a_mid), 0.02, 2, precision, ws1)
            torch.cuda.synchronize()
            if precision == "split_bf16":
                assert torch.equal(gb.psi, g1.psi)
            else:   # the FP16 scale is taken per domain: identical too
                assert torch.equal(gb.psi, g1.psi)


@pytest.mark.parametrize("batch", [False, True])
def test_fp16_multistep_call_equals_one_step_calls(api, batch):
    """FP16 scales: inside one call, each step's projection after the first
    takes max |u| from the correction that wrote u; a one-step call searches
    psi for it instead.  The two must give the same bits (the checkpoint
    recompute of the pulse gradient depends on it): five steps in one call
    against five one-step calls, on the ragged 19 x 13 x 21 domain and on a
    batch of three uneven domains."""
    import torch
    precision = "split_fp16"
    if batch:
        doms = [make_domain(80 + i, shp, no, na, proj_per_atom=8, h=0.4, fd_order=6)
                for i, (shp, no, na) in enumerate([((20, 21, 22), 17, 4), ((22, 20, 20), 30, 7),
                                                   ((21, 23, 19), 45, 11)])]
    else:
        doms = [_dom(seed=56)]
    n = 5
    at = a_tensor(pulse_midpoints(n, 0.02, n) * 4.0)
    multi = [to_device(d, precision) for d in doms]
    single = [to_device(d, precision) for d in doms]
    wsm = api.Workspace.for_domains(multi, precision)
    wss = api.Workspace.for_domains(single, precision)
    api.step(multi, at, 0.02, n, precision, wsm)
    for k in range(n):
        api.step(single, at[k:k + 1].contiguous(), 0.02, 1, precision, wss)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(multi, single)):
        assert torch.equal(a.psi, b.psi), i
