"""The batched divide-and-conquer workload: 16 seeded domains of the 512
(including the smallest and the largest), advanced together in one call and
through a captured HIP graph, against the FP64 oracle per domain; graph
replays equal eager steps bitwise; the autotuner's choice runs and agrees."""
import numpy as np
import pytest

from helpers import a_tensor, oracle_inputs, rel_fro, to_device
from oracle import propagate as P
from synth import batched_domain, batched_domain_shapes, pulse_midpoints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def doms():
    shapes = batched_domain_shapes()
    size = np.array([n ** 3 * no * (8 * na) for n, no, na in shapes])
    pick = [int(size.argmin()), int(size.argmax())]
    rng = np.random.default_rng(404)
    for i in rng.permutation(len(shapes)):
        if len(pick) == 16:
            break
        if int(i) not in pick:
            pick.append(int(i))
    return [batched_domain(i) for i in pick]


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("split_bf16", 1e-4)])
def test_batched_subset_matches_oracle(doms, precision, tol):
    import torch
    import paper_2509_00966_amd as api
    n = 3
    a_mid = pulse_midpoints(100, 0.02, 100)[:n]
    gs = [to_device(d, precision) for d in doms]
    ws = api.Workspace.for_domains(gs, precision)
    api.step(gs, a_tensor(a_mid), 0.02, n, precision, ws)
    torch.cuda.synchronize()
    for d, g in zip(doms, gs):
        od = oracle_inputs(d, "fp32")
        ref, _ = P.propagate(od, a_mid, 0.02, od.psi)
        assert rel_fro(g.psi.cpu().numpy(), ref) < tol, (d.shape, d.n_orb, d.n_proj)


def test_batched_graph_equals_eager(doms):
    import torch
    import paper_2509_00966_amd as api
    a_mid = pulse_midpoints(100, 0.02, 100)[:4]
    ge = [to_device(d, "fp32") for d in doms]
    gg = [to_device(d, "fp32") for d in doms]
    wse = api.Workspace.for_domains(ge, "fp32")
    wsg = api.Workspace.for_domains(gg, "fp32")
    at = a_tensor(a_mid)
    graph = api.Graph(gg, at, 0.02, 4, "fp32", wsg)
    for rep in range(2):
        api.step(ge, at, 0.02, 4, "fp32", wse)
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
        assert rel_fro(g.psi.cpu().numpy(), ref) < 1e-5
