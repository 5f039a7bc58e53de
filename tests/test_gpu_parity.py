"""GPU parity: the HIP library against the FP64 oracle on the same seeded
inputs, at sizes that span several tiles of every kernel and leave ragged
tails (grid edges, orbital chunks, projector and orbital GEMM tiles).

Tolerances: FP64 path <= 1e-11 relative (rounding order only); FP32 path
<= 1e-5 relative on psi (the FP32 bar after 100 steps).  The FP32 H psi is
held to 2 U32 kappa in the norm views and 4 U32 kappa element-wise, kappa
the condition number of the operator's sum of terms
(helpers.fp32_operator_tol); the other FP32
operators (density, current, adjoint) to multiples of 2e-6.
"""
import numpy as np
import pytest

from helpers import a_tensor, assert_close, fp32_operator_tol, oracle_inputs, to_device
from oracle import adjoint as ADJ
from oracle import hamiltonian as H
from oracle import observables as O
from oracle import propagate as P
from synth import config, make_domain, pulse_midpoints

pytestmark = pytest.mark.gpu

TOL_OP = {"fp64": 1e-12, "fp32": 2e-6}
TOL_PSI = {"fp64": 1e-11, "fp32": 1e-5}


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def api():
    import paper_2509_00966_amd as api
    return api


def _ragged(seed=31, order=6):
    # 19 x 13 x 21 grid, 21 orbitals, 3 atoms x 8 projectors
    return make_domain(seed, (19, 13, 21), 21, 3, proj_per_atom=8, h=0.4, fd_order=order)


def _field(n=6, scale=4.0):
    a = pulse_midpoints(n, 0.02, n) * scale
    a[:, 0] = 0.07
    a[:, 1] = -0.04
    return a


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [2, 4, 6])
def test_hpsi_matches_oracle(api, precision, order):
    torch = _torch()
    dom = _ragged(order=order)
    A = np.array([0.05, -0.11, 0.23])
    g = to_device(dom, precision)
    ws = api.Workspace.for_domains([g], precision)
    hp = torch.empty_like(g.psi)
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    api.density([g], a_tensor(A[None]), precision, ws, [dict(hpsi_occ=hp, energy=e)])
    torch.cuda.synchronize()
    od = oracle_inputs(dom, precision)
    ref = O.occupied_h(od, A, od.psi)
    tol = TOL_OP["fp64"] if precision == "fp64" else fp32_operator_tol(od, A, od.psi, ref)
    assert_close(_np(hp), ref, tol)
    e_ref = O.energy(od, A, od.psi)
    assert abs(e.item() - e_ref) < TOL_OP[precision] * 10 * abs(e_ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_step_matches_oracle(api, precision):
    torch = _torch()
    dom = _ragged(seed=32)
    a_mid = _field(5)
    dt = 0.02
    g = to_device(dom, precision)
    ws = api.Workspace.for_domains([g], precision)
    api.step([g], a_tensor(a_mid), dt, len(a_mid), precision, ws)
    torch.cuda.synchronize()
    od = oracle_inputs(dom, precision)
    ref, _ = P.propagate(od, a_mid, dt, od.psi)
    assert_close(_np(g.psi), ref, TOL_PSI[precision])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_per_step_observables(api, precision):
    torch = _torch()
    dom = make_domain(33, (17, 18, 16), 10, 2, proj_per_atom=8, h=0.4, fd_order=4)
    a_mid = _field(3)
    dt = 0.02
    g = to_device(dom, precision)
    rd = api.real_dtype(precision)
    n = len(a_mid)
    obs = dict(rho=torch.zeros(n, dom.n_grid, dtype=rd, device="cuda"),
               j=torch.zeros(n, dom.n_grid, 3, dtype=rd, device="cuda"),
               energy=torch.zeros(n, dtype=torch.float64, device="cuda"))
    ws = api.Workspace.for_domains([g], precision)
    api.step([g], a_tensor(a_mid), dt, n, precision, ws, obs=[obs])
    torch.cuda.synchronize()
    od = oracle_inputs(dom, precision)
    ref, ro = P.propagate(od, a_mid, dt, od.psi, want_rho=True, want_j=True, want_energy=True)
    tol = TOL_OP[precision] * 5
    assert_close(_np(obs["rho"]), ro["rho"], tol, orbitals=False)
    assert_close(_np(obs["j"]), ro["j"], tol * 5, orbitals=False)
    assert np.abs(_np(obs["energy"]) - ro["energy"]).max() < tol * np.abs(ro["energy"]).max()
    assert_close(_np(g.psi), ref, TOL_PSI[precision])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_density_current_overlap(api, precision):
    torch = _torch()
    dom = _ragged(seed=34, order=4)
    A = np.array([0.0, 0.1, -0.2])
    g = to_device(dom, precision)
    rd = api.real_dtype(precision)
    out = dict(rho=torch.zeros(dom.n_grid, dtype=rd, device="cuda"),
               j=torch.zeros(dom.n_grid, 3, dtype=rd, device="cuda"),
               overlap=torch.zeros(dom.n_orb, dom.n_orb, 2, dtype=torch.float64, device="cuda"))
    ws = api.Workspace.for_domains([g], precision)
    api.density([g], a_tensor(A[None]), precision, ws, [out])
    torch.cuda.synchronize()
    od = oracle_inputs(dom, precision)
    assert_close(_np(out["rho"]), O.density(od, od.psi), TOL_OP[precision], orbitals=False)
    assert_close(_np(out["j"]), O.current(od, A, od.psi), TOL_OP[precision] * 10, orbitals=False)
    s = _np(out["overlap"])
    s = s[..., 0] + 1j * s[..., 1]
    # the overlap is accumulated in FP64 from the (rounded) inputs: tight in both modes
    assert np.abs(s - O.overlap(od, od.psi)).max() < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_step_matches_oracle(api, precision):
    torch = _torch()
    dom = make_domain(35, (17, 12, 14), 9, 2, proj_per_atom=8, h=0.4, fd_order=6)
    A = np.array([0.02, -0.03, 0.08])
    dt = 0.02
    rng = np.random.default_rng(3)
    lam = (rng.standard_normal(dom.psi.shape) + 1j * rng.standard_normal(dom.psi.shape)) * 0.05
    g = to_device(dom, precision)
    lam_d = torch.from_numpy(lam).to(device="cuda", dtype=api.complex_dtype(precision))
    grad = torch.zeros(3, dtype=torch.float64, device="cuda")
    ws = api.Workspace.for_domains([g], precision)
    api.adjoint_step([g], [lam_d], a_tensor(A[None]), dt, grad, precision, ws)
    torch.cuda.synchronize()
    od = oracle_inputs(dom, precision)
    lam_in = lam.astype(np.complex64).astype(np.complex128) if precision == "fp32" else lam
    lam_ref, g_ref = ADJ.adjoint_step(od, A, dt, od.psi, lam_in)
    assert_close(_np(lam_d), lam_ref, TOL_OP[precision] * 5)
    assert np.abs(_np(grad) - g_ref).max() < TOL_OP[precision] * 50 * np.abs(g_ref).max()


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("stencil", [-1, 9, 10, 11, 12, 2])
@pytest.mark.parametrize("order", [2, 4, 6])
def test_adjoint_gradient_from_sweep_and_from_separate_pass(api, precision, stencil, order):
    """The pulse gradient with its partials formed inside the ring sweeps
    (default and every ring-sweep tile, 9-12; the sweep applies (-i D1 + A) to
    mu and pairs it with u, the operator being Hermitian) and by the separate
    pass (variant 2, not a ring sweep), at each FD order: against the oracle,
    on a ragged domain with a field along every axis (so every gradient axis
    matters)."""
    torch = _torch()
    dom = make_domain(37, (19, 13, 21), 21, 3, proj_per_atom=8, h=0.4, fd_order=order)
    A = np.array([0.05, -0.04, 0.07])
    dt = 0.02
    rng = np.random.default_rng(38)
    lam = (rng.standard_normal(dom.psi.shape) + 1j * rng.standard_normal(dom.psi.shape)) * 0.05
    g = to_device(dom, precision)
    lam_d = torch.from_numpy(lam).to(device="cuda", dtype=api.complex_dtype(precision))
    grad = torch.zeros(3, dtype=torch.float64, device="cuda")
    ws = api.Workspace.for_domains([g], precision)
    try:
        api.set_tuning("stencil", stencil)
        api.adjoint_step([g], [lam_d], a_tensor(A[None]), dt, grad, precision, ws)
        torch.cuda.synchronize()
    finally:
        api.set_tuning("stencil", -1)
    od = oracle_inputs(dom, precision)
    lam_in = lam.astype(np.complex64).astype(np.complex128)
    lam_ref, g_ref = ADJ.adjoint_step(od, A, dt, od.psi, lam_in)
    # lambda: the operator bar (split: its BF16 hi+lo products); gradient: as
    # the existing adjoint test, 50 times the operator bar
    tol = {"fp32": TOL_OP["fp32"], "split_bf16": 2e-5}[precision]
    assert_close(_np(lam_d), lam_ref, tol * 5, label=f"lambda stencil={stencil}")
    err = np.abs(_np(grad) - g_ref).max() / np.abs(g_ref).max()
    print(f"[parity] gradient stencil={stencil} FD{order} {precision}: {err:.2e}")
    assert err < tol * 50


def test_config1_full_run_fp64(api):
    torch = _torch()
    w = config(1)
    dom = w.domains[0]
    g = to_device(dom, "fp64")
    n = w.n_steps
    obs = dict(energy=torch.zeros(n, dtype=torch.float64, device="cuda"))
    ws = api.Workspace.for_domains([g], "fp64")
    api.step([g], a_tensor(w.a_mid), w.dt, n, "fp64", ws, obs=[obs])
    torch.cuda.synchronize()
    ref, ro = P.propagate(dom, w.a_mid, w.dt, dom.psi, want_energy=True)
    assert_close(_np(g.psi), ref, 1e-12)
    assert np.abs(_np(obs["energy"]) - ro["energy"]).max() < 1e-12 * np.abs(ro["energy"]).max()


def test_no_projectors(api):
    torch = _torch()
    dom = _ragged(seed=36)
    dom.proj = np.zeros((dom.n_grid, 0), np.complex128)
    dom.d = np.zeros(0)
    a_mid = _field(3)
    g = to_device(dom, "fp64")
    ws = api.Workspace.for_domains([g], "fp64")
    api.step([g], a_tensor(a_mid), 0.02, 3, "fp64", ws)
    torch.cuda.synchronize()
    ref, _ = P.propagate(dom, a_mid, 0.02, dom.psi)
    assert_close(_np(g.psi), ref, 1e-11)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_equals_single_domains(api, precision):
    torch = _torch()
    doms = [make_domain(40 + i, shp, no, na, proj_per_atom=8, h=0.4, fd_order=fo)
            for i, (shp, no, na, fo) in enumerate([((20, 20, 20), 17, 4, 6), ((23, 21, 22), 33, 8, 6),
                                                   ((18, 19, 17), 5, 1, 4), ((21, 21, 21), 16, 4, 2)])]
    a_mid = _field(2)
    gs = [to_device(d, precision) for d in doms]
    ws = api.Workspace.for_domains(gs, precision)
    api.step(gs, a_tensor(a_mid), 0.02, 2, precision, ws)
    singles = []
    for d in doms:
        g1 = to_device(d, precision)
        ws1 = api.Workspace.for_domains([g1], precision)
        api.step([g1], a_tensor(a_mid), 0.02, 2, precision, ws1)
        singles.append(g1)
    torch.cuda.synchronize()
    for gb, g1, d in zip(gs, singles, doms):
        assert torch.equal(gb.psi, g1.psi)
        od = oracle_inputs(d, precision)
        ref, _ = P.propagate(od, a_mid, 0.02, od.psi)
        assert_close(_np(gb.psi), ref, TOL_PSI[precision])


def test_graph_replay_equals_eager_bitwise(api):
    torch = _torch()
    dom = _ragged(seed=37)
    a_mid = _field(4)
    ge = to_device(dom, "fp32")
    gg = to_device(dom, "fp32")
    wse = api.Workspace.for_domains([ge], "fp32")
    wsg = api.Workspace.for_domains([gg], "fp32")
    at = a_tensor(a_mid)
    graph = api.Graph([gg], at, 0.02, 2, "fp32", wsg)
    for rep in range(3):
        api.step([ge], at, 0.02, 2, "fp32", wse)
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(ge.psi, gg.psi), rep
    graph.close()


def test_repeat_is_bitwise_deterministic(api):
    torch = _torch()
    dom = _ragged(seed=38)
    a_mid = _field(3)
    outs = []
    for _ in range(2):
        g = to_device(dom, "fp32")
        ws = api.Workspace.for_domains([g], "fp32")
        e = torch.zeros(3, dtype=torch.float64, device="cuda")
        api.step([g], a_tensor(a_mid), 0.02, 3, "fp32", ws, obs=[dict(energy=e)])
        torch.cuda.synchronize()
        outs.append((g.psi.clone(), e.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_tile_variants_agree(api, variant):
    torch = _torch()
    dom = _ragged(seed=39)
    a_mid = _field(2)
    od = oracle_inputs(dom, "fp32")
    ref, _ = P.propagate(od, a_mid, 0.02, od.psi)
    try:
        for fam in ("stencil", "project", "correct"):
            api.set_tuning(fam, variant)
        g = to_device(dom, "fp32")
        ws = api.Workspace.for_domains([g], "fp32")
        api.step([g], a_tensor(a_mid), 0.02, 2, "fp32", ws)
        torch.cuda.synchronize()
    finally:
        for fam in ("stencil", "project", "correct"):
            api.set_tuning(fam, -1)
    assert_close(_np(g.psi), ref, TOL_PSI["fp32"])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("variant", list(range(13)))
def test_every_stencil_variant_matches_oracle(api, variant, order, precision):
    """Each stencil tile variant, at each FD order, on a ragged 19 x 13 x 21
    domain of 21 orbitals (partial x/y tiles and a partial orbital chunk);
    two steps with rho, j and E so every Horner stage and the fused density
    and energy partials run."""
    torch = _torch()
    n_var = api.tuning_options("stencil")
    if variant >= n_var:
        pytest.skip("variant not built")
    dom = _ragged(seed=41, order=order)
    a_mid = _field(2)
    od = oracle_inputs(dom, precision)
    ref, obs = P.propagate(od, a_mid, 0.02, od.psi, want_rho=True, want_j=True, want_energy=True)
    g = to_device(dom, precision)
    ws = api.Workspace.for_domains([g], precision)
    rd = torch.float64 if precision == "fp64" else torch.float32
    rho = torch.zeros(2, dom.n_grid, dtype=rd, device="cuda")
    j = torch.zeros(2, dom.n_grid, 3, dtype=rd, device="cuda")
    e = torch.zeros(2, dtype=torch.float64, device="cuda")
    try:
        api.set_tuning("stencil", variant)
        api.step([g], a_tensor(a_mid), 0.02, 2, precision, ws, obs=[dict(rho=rho, j=j, energy=e)])
        torch.cuda.synchronize()
    finally:
        api.set_tuning("stencil", -1)
    tol = TOL_PSI[precision]
    assert_close(_np(g.psi), ref, tol)
    assert_close(_np(rho), obs["rho"], tol, orbitals=False)
    assert_close(_np(j), obs["j"], tol * 10, orbitals=False)
    assert np.abs(_np(e) - obs["energy"]).max() < tol * np.abs(obs["energy"]).max()


@pytest.mark.parametrize("zseg", [1, 2, 3, 4])
def test_every_z_segment_choice_matches_oracle(api, zseg):
    """Fixed z segments of 8, 16, 32 planes and whole columns, on a 37-plane
    domain (ragged last segment), with the default and the sweep3 tiles."""
    torch = _torch()
    dom = make_domain(42, (12, 11, 37), 9, 2, proj_per_atom=8, h=0.4, fd_order=6)
    a_mid = _field(2)
    od = oracle_inputs(dom, "fp32")
    ref, _ = P.propagate(od, a_mid, 0.02, od.psi)
    for variant in (-1, 8):
        g = to_device(dom, "fp32")
        ws = api.Workspace.for_domains([g], "fp32")
        try:
            api.set_tuning("zseg", zseg)
            api.set_tuning("stencil", variant)
            api.step([g], a_tensor(a_mid), 0.02, 2, "fp32", ws)
            torch.cuda.synchronize()
        finally:
            api.set_tuning("zseg", -1)
            api.set_tuning("stencil", -1)
        assert_close(_np(g.psi), ref, TOL_PSI["fp32"], label=str(variant))


@pytest.mark.parametrize("shape,n_orb,n_atoms", [((19, 13, 21), 22, 3),     # N_g tail, 24 projectors
                                                ((16, 16, 16), 64, 8),      # whole stages, 64 projectors
                                                ((17, 15, 9), 21, 2),       # odd N_o
                                                ((12, 11, 10), 130, 3)])    # two orbital tiles
@pytest.mark.parametrize("family,variant", [("project", 4), ("project", 5), ("project", 7), ("project", 8),
                                            ("correct", 4), ("correct", 5), ("correct", 6), ("correct", 7)])
def test_direct_lds_products_match_oracle(api, family, variant, shape, n_orb, n_atoms):
    """The FP32 projection / correction with tiles loaded straight into LDS
    (tuning variant 4 of each family; variant 5: the projection on 64
    projectors, the correction on 64 complex columns; correction variant 6:
    as 5 with the output tile requested before the reduction; projection
    variant 7: the three-product kernel through registers on 64 x 32, with
    8-byte loads for odd orbital counts; projection variant 8 and correction
    variant 7: every orbital in one block, or the 64-column kernels past 96
    orbitals), two steps against the oracle."""
    torch = _torch()
    dom = make_domain(43, shape, n_orb, n_atoms, proj_per_atom=8, h=0.4, fd_order=6)
    a_mid = _field(2)
    od = oracle_inputs(dom, "fp32")
    ref, _ = P.propagate(od, a_mid, 0.02, od.psi)
    g = to_device(dom, "fp32")
    ws = api.Workspace.for_domains([g], "fp32")
    try:
        api.set_tuning(family, variant)
        api.step([g], a_tensor(a_mid), 0.02, 2, "fp32", ws)
        torch.cuda.synchronize()
    finally:
        api.set_tuning(family, -1)
    assert_close(_np(g.psi), ref, TOL_PSI["fp32"])


def test_check_finite_flags_nan(api):
    torch = _torch()
    from paper_2509_00966_amd._lib import DcmeshError
    dom = _ragged(seed=40)
    g = to_device(dom, "fp32")
    g.psi[5, 3] = complex(float("nan"), 0.0)
    ws = api.Workspace.for_domains([g], "fp32")
    with pytest.raises(DcmeshError) as ei:
        api.step([g], a_tensor(_field(1)), 0.02, 1, "fp32", ws, check_finite=True)
    assert ei.value.code == 5


@pytest.mark.parametrize("family,variant", [("project", 8), ("correct", 7)])
def test_narrow_products_every_width(api, family, variant):
    """The FP32 products with every orbital of a domain in one block, at each
    of their widths (16 NB orbitals, NB = 1..6: 9, 17, 40, 55, 70 and 96
    orbitals, odd and even, so both load widths run) in one batched call;
    24 and 72 projectors leave projection waves with no projectors (they
    skip their products); two steps against the oracle per domain."""
    torch = _torch()
    spec = [((11, 10, 9), 9, 3), ((12, 11, 10), 17, 3), ((10, 12, 11), 40, 9), ((9, 11, 12), 55, 3),
            ((11, 11, 11), 70, 9), ((10, 10, 12), 96, 12)]
    doms = [make_domain(120 + i, shp, no, na, proj_per_atom=8, h=0.4, fd_order=6)
            for i, (shp, no, na) in enumerate(spec)]
    a_mid = _field(2)
    gs = [to_device(d, "fp32") for d in doms]
    ws = api.Workspace.for_domains(gs, "fp32")
    try:
        api.set_tuning(family, variant)
        api.step(gs, a_tensor(a_mid), 0.02, 2, "fp32", ws)
        torch.cuda.synchronize()
    finally:
        api.set_tuning(family, -1)
    for d, g in zip(doms, gs):
        od = oracle_inputs(d, "fp32")
        ref, _ = P.propagate(od, a_mid, 0.02, od.psi)
        assert_close(_np(g.psi), ref, TOL_PSI["fp32"], label=f"N_o={d.n_orb} N_p={d.n_proj}")
