"""The batched divide-and-conquer workload: 16 seeded domains of the 512
(including the smallest and the largest), advanced together through a
captured 100-step HIP graph in FP32, split BF16 and split FP16, against the
FP64 oracle per domain on two orbitals (a seeded one and the last, which sits
at the ragged end of the orbital tiles; orbitals propagate independently, so
the oracle on those columns alone gives the same columns); graph replays equal
eager steps bitwise; the autotuner's choice runs and agrees."""
import numpy as np
import pytest

from helpers import a_tensor, assert_close, oracle_inputs, propagate_logged, to_device
from oracle import propagate as P
from synth import Domain, batched_domain, batched_subset, pulse_midpoints

pytestmark = pytest.mark.gpu

N_STEPS = 100


@pytest.fixture(scope="module")
def doms():
    return [batched_domain(i) for i in batched_subset()]


@pytest.fixture(scope="module")
def oracle_100(doms):
    """FP64 oracle after 100 steps (pulse with T = 100 dt) on two orbitals of
    every domain, from the FP32-rounded inputs the GPU path sees."""
    a_mid = pulse_midpoints(N_STEPS, 0.02, N_STEPS)
    rng = np.random.default_rng(405)
    refs = []
    for d in doms:
        od = oracle_inputs(d, "fp32")
        cols = np.array([int(rng.integers(d.n_orb - 1)), d.n_orb - 1])
        sub = Domain(od.shape, od.h, od.fd_order, np.ascontiguousarray(od.psi[:, cols]), od.v_loc, od.proj,
                     od.d, od.occ[cols])
        ref = propagate_logged(sub, a_mid, 0.02, sub.psi, label=f"{d.shape} N_o={d.n_orb}", chunk=50)
        refs.append((cols, ref))
    return a_mid, refs


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("split_bf16", 1e-4), ("split_fp16", 1e-5)])
def test_batched_subset_100_step_graph_matches_oracle(doms, oracle_100, precision, tol):
    import torch
    import paper_2509_00966_amd as api
    a_mid, refs = oracle_100
    gs = [to_device(d, precision) for d in doms]
    ws = api.Workspace.for_domains(gs, precision)
    graph = api.Graph(gs, a_tensor(a_mid), 0.02, N_STEPS, precision, ws)
    graph.launch()
    torch.cuda.synchronize()
    graph.close()
    for d, g, (cols, ref) in zip(doms, gs, refs):
        got = g.psi[:, torch.from_numpy(cols).to("cuda")].cpu().numpy()
        assert_close(got, ref, tol, label=f"{d.shape} N_o={d.n_orb} N_p={d.n_proj} orbitals {cols.tolist()}")


@pytest.mark.parametrize("precision", ["fp32", "split_bf16", "split_fp16"])
def test_batched_graph_equals_eager(doms, precision):
    import torch
    import paper_2509_00966_amd as api
    a_mid = pulse_midpoints(100, 0.02, 100)[:4]
    ge = [to_device(d, precision) for d in doms]
    gg = [to_device(d, precision) for d in doms]
    wse = api.Workspace.for_domains(ge, precision)
    wsg = api.Workspace.for_domains(gg, precision)
    at = a_tensor(a_mid)
    graph = api.Graph(gg, at, 0.02, 4, precision, wsg)
    for rep in range(2):
        api.step(ge, at, 0.02, 4, precision, wse)
        graph.launch()
        torch.cuda.synchronize()
        for a, b in zip(ge, gg):
            assert torch.equal(a.psi, b.psi), rep
    graph.close()


def test_autotuner_choice_runs_and_agrees(doms, tmp_path):
    import torch
    import paper_2509_00966_amd as api
    from paper_2509_00966_amd import autotune
    sub = doms[:4]
    a_mid = pulse_midpoints(100, 0.02, 100)[:2]
    gs = [to_device(d, "fp32") for d in sub]
    at = a_tensor(a_mid)
    best = autotune.tune(gs, at, 0.02, "fp32", cache_path=str(tmp_path / "tune.json"))
    assert set(best) == {"stencil", "project", "correct"}
    cached = autotune.tune(gs, at, 0.02, "fp32", cache_path=str(tmp_path / "tune.json"))
    assert cached == best
    try:
        autotune.apply(best)
        g2 = [to_device(d, "fp32") for d in sub]
        ws = api.Workspace.for_domains(g2, "fp32")
        api.step(g2, at, 0.02, 2, "fp32", ws)
        torch.cuda.synchronize()
    finally:
        autotune.reset()
    for d, g in zip(sub, g2):
        od = oracle_inputs(d, "fp32")
        ref, _ = P.propagate(od, a_mid, 0.02, od.psi)
        assert_close(g.psi.cpu().numpy(), ref, 1e-5)


@pytest.mark.parametrize("zseg", [-1, 2])
def test_stencil_work_orders_give_identical_results(doms, zseg):
    """Every stencil work order (each domain's orbital chunks dealt over the
    XCDs; each (domain, z segment) on one XCD, tiles before chunks or chunks
    before tiles) gives the same psi, rho, j and E bit for bit: the order moves
    work-groups, not arithmetic (the energy partials sit at the item's own slot
    in its domain).  zseg 2: 16-plane segments, so most domains have several."""
    import torch
    import paper_2509_00966_amd as api
    a_mid = pulse_midpoints(100, 0.02, 100)[:2]
    at = a_tensor(a_mid)
    runs = []
    try:
        api.set_tuning("zseg", zseg)
        for order in range(api.tuning_options("sorder")):
            api.set_tuning("sorder", order)
            gs = [to_device(d, "fp32") for d in doms]
            ws = api.Workspace.for_domains(gs, "fp32")
            obs = [{"rho": torch.empty(2, d.n_grid, device="cuda"), "j": torch.empty(2, d.n_grid, 3, device="cuda"),
                    "energy": torch.empty(2, dtype=torch.float64, device="cuda")} for d in gs]
            api.step(gs, at, 0.02, 2, "fp32", ws, obs=obs)
            torch.cuda.synchronize()
            runs.append((gs, obs))
    finally:
        api.set_tuning("sorder", -1)
        api.set_tuning("zseg", -1)
    g0, o0 = runs[0]
    for order, (gs, obs) in enumerate(runs[1:], 1):
        for i, (a, b) in enumerate(zip(g0, gs)):
            assert torch.equal(a.psi, b.psi), (order, i)
        for i, (a, b) in enumerate(zip(o0, obs)):
            for k in ("rho", "j", "energy"):
                assert torch.equal(a[k], b[k]), (order, i, k)
    # and the first order agrees with the oracle's energy on the first domain
    d = doms[0]
    od = oracle_inputs(d, "fp32")
    _, ob = P.propagate(od, a_mid, 0.02, od.psi, want_energy=True)
    e = o0[0]["energy"].cpu().numpy()
    assert np.abs(e - ob["energy"]).max() < 1e-5 * np.abs(ob["energy"]).max()


@pytest.mark.parametrize("a_per_domain", [False, True])
def test_batched_adjoint_gradient_matches_single_domains_and_oracle(doms, a_per_domain):
    """One adjoint step over 12 of the subset's domains at once (enough
    (domain, z segment) clusters for the per-XCD stencil order, gradient
    partials formed in the sweeps): lambda of every domain equals its
    single-domain call bitwise, the gradient (per domain, or summed over the
    batch) agrees with the single-domain gradients to FP64 rounding (a domain
    alone gets z segments to fill the GPU, so its block partials group the
    same terms differently), and the first domain's gradient agrees with the
    oracle's."""
    import torch
    import paper_2509_00966_amd as api
    from oracle import adjoint as ADJ
    sub = doms[:12]
    dt = 0.02
    A = np.array([0.03, -0.02, 0.06])
    rng = np.random.default_rng(406)
    lams = [(rng.standard_normal(d.psi.shape) + 1j * rng.standard_normal(d.psi.shape)) * 0.05 for d in sub]
    gs = [to_device(d, "fp32") for d in sub]
    lam_b = [torch.from_numpy(l).to("cuda", torch.complex64) for l in lams]
    n = len(sub)
    a = a_tensor(np.tile(A, (n, 1, 1)) if a_per_domain else A[None])
    grad_b = torch.zeros((n, 3) if a_per_domain else (3,), dtype=torch.float64, device="cuda")
    ws = api.Workspace.for_domains(gs, "fp32")
    api.adjoint_step(gs, lam_b, a.contiguous(), dt, grad_b, "fp32", ws, a_per_domain=a_per_domain)
    torch.cuda.synchronize()
    singles = []
    for d, g, l in zip(sub, gs, lams):
        lam_s = torch.from_numpy(l).to("cuda", torch.complex64)
        grad_s = torch.zeros(3, dtype=torch.float64, device="cuda")
        w1 = api.Workspace.for_domains([g], "fp32")
        api.adjoint_step([g], [lam_s], a_tensor(A[None]), dt, grad_s, "fp32", w1)
        torch.cuda.synchronize()
        singles.append((lam_s, grad_s.cpu().numpy()))
    for i, (lb, (ls, gsn)) in enumerate(zip(lam_b, singles)):
        assert torch.equal(lb, ls), i
        if a_per_domain:
            assert np.abs(grad_b[i].cpu().numpy() - gsn).max() <= 1e-12 * np.abs(gsn).max(), i
    if not a_per_domain:
        total = np.sum([g for _, g in singles], axis=0)
        assert np.abs(grad_b.cpu().numpy() - total).max() <= 1e-12 * np.abs(total).max()
    od = oracle_inputs(sub[0], "fp32")
    lam_in = lams[0].astype(np.complex64).astype(np.complex128)
    _, g_ref = ADJ.adjoint_step(od, A, dt, od.psi, lam_in)
    g0 = singles[0][1]
    assert np.abs(g0 - g_ref).max() < 1e-4 * np.abs(g_ref).max()
