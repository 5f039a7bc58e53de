"""dcmesh_step_noalloc (the static device scratch, no allocation) against
dcmesh_step with a caller workspace: bitwise equal results on two calls in a
row, the second on a smaller input, in FP32 with the per-step observables
and in split FP16; a request larger than the scratch fails cleanly on the
host."""
import numpy as np
import pytest

from helpers import a_tensor, to_device
from synth import make_domain, pulse_midpoints

pytestmark = pytest.mark.gpu


def _run(api, doms, precision, n, noalloc):
    import torch
    gs = [to_device(d, precision) for d in doms]
    rd = api.real_dtype(precision)
    obs = [dict(rho=torch.zeros(n, d.n_grid, dtype=rd, device="cuda"),
                j=torch.zeros(n, d.n_grid, 3, dtype=rd, device="cuda"),
                energy=torch.zeros(n, dtype=torch.float64, device="cuda")) for d in doms]
    at = a_tensor(pulse_midpoints(n, 0.02, n) * 4.0)
    if noalloc:
        api.step_noalloc(gs, at, 0.02, n, precision, obs=obs)
    else:
        ws = api.Workspace.for_domains(gs, precision)
        api.step(gs, at, 0.02, n, precision, ws, obs=obs)
    torch.cuda.synchronize()
    return gs, obs


@pytest.mark.parametrize("precision", ["fp32", "split_fp16"])
def test_noalloc_step_equals_workspace_step(precision):
    import torch
    import paper_2509_00966_amd as api
    big = [make_domain(101, (19, 13, 21), 21, 3, proj_per_atom=8, h=0.4, fd_order=6),
           make_domain(102, (20, 18, 17), 33, 5, proj_per_atom=8, h=0.4, fd_order=4)]
    small = [make_domain(103, (12, 11, 10), 9, 2, proj_per_atom=8, h=0.4, fd_order=6)]
    for doms, n in ((big, 3), (small, 2)):
        ref, ref_obs = _run(api, doms, precision, n, noalloc=False)
        got, got_obs = _run(api, doms, precision, n, noalloc=True)
        for g, r, go, ro in zip(got, ref, got_obs, ref_obs):
            assert torch.equal(g.psi, r.psi)
            for k in ("rho", "j", "energy"):
                assert torch.equal(go[k], ro[k]), k


def test_noalloc_rejects_domains_beyond_the_scratch():
    import paper_2509_00966_amd as api
    from paper_2509_00966_amd._lib import DcmeshError
    dom = make_domain(104, (40, 40, 40), 64, 1, proj_per_atom=8, h=0.4, fd_order=6)
    g = to_device(dom, "fp32")
    with pytest.raises(DcmeshError) as ei:
        api.step_noalloc([g], a_tensor(np.zeros((1, 3))), 0.02, 1, "fp32")
    assert ei.value.code == 3
