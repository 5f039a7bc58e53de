"""Full-size parity: the 64^3 / 128-orbital / 512-projector workload for 100
steps with the laser pulse, against the FP64 oracle on 8 sampled orbitals
(seven seeded ones and the last, which sits at the ragged end of every
orbital tile).  The step acts on every orbital independently, so the oracle
run on those columns alone gives exactly the same columns.  Bars: FP32 path <= 1e-5
relative on psi after 100 steps; split BF16 <= 1e-4 and split FP16 <= 1e-5.
The per-step density, current and energy of the full run are checked on the
first step against the oracle with all orbitals."""
import numpy as np
import pytest

from helpers import a_tensor, assert_close, propagate_logged, to_device
from oracle import observables as O
from oracle import propagate as P
from synth import Domain, config

pytestmark = pytest.mark.gpu

N_STEPS = 100
SAMPLE = 8


@pytest.fixture(scope="module")
def workload():
    w = config(2)
    dom = w.domains[0]
    od = dom.rounded(np.float32)
    # seeded orbitals plus the last one (the ragged end of every orbital tile)
    cols = np.sort(np.append(np.random.default_rng(202).choice(dom.n_orb - 1, SAMPLE - 1, replace=False),
                             dom.n_orb - 1))
    sub = Domain(od.shape, od.h, od.fd_order, np.ascontiguousarray(od.psi[:, cols]), od.v_loc, od.proj, od.d,
                 od.occ[cols])
    ref = propagate_logged(sub, w.a_mid[:N_STEPS], w.dt, sub.psi, label="64^3, 8 orbitals")
    A0 = w.a_mid[0]
    obs_ref = (O.density(od, od.psi), O.current(od, A0, od.psi), O.energy(od, A0, od.psi))
    return w, dom, od, cols, ref, obs_ref


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("split_bf16", 1e-4), ("split_fp16", 1e-5)])
def test_full_size_100_steps(workload, precision, tol):
    import torch
    import paper_2509_00966_amd as api
    w, dom, od, cols, ref, (rho_ref, j_ref, e_ref) = workload
    g = to_device(dom, precision)
    ws = api.Workspace.for_domains([g], precision)
    rd = api.real_dtype(precision)
    obs = dict(rho=torch.zeros(1, dom.n_grid, dtype=rd, device="cuda"),
               j=torch.zeros(1, dom.n_grid, 3, dtype=rd, device="cuda"),
               energy=torch.zeros(1, dtype=torch.float64, device="cuda"))
    at = a_tensor(w.a_mid[:N_STEPS])
    api.step([g], at[:1].contiguous(), w.dt, 1, precision, ws, obs=[obs])
    api.step([g], at[1:].contiguous(), w.dt, N_STEPS - 1, precision, ws)
    torch.cuda.synchronize()
    got = g.psi[:, torch.from_numpy(cols).to("cuda")].cpu().numpy()
    assert_close(got, ref, tol, label=f"psi after {N_STEPS} steps, orbitals {cols.tolist()}")
    # first-step observables of the full orbital set
    assert_close(obs["rho"][0].cpu().numpy(), rho_ref, 1e-5, orbitals=False)
    assert_close(obs["j"][0].cpu().numpy(), j_ref, 1e-4, orbitals=False)
    assert abs(obs["energy"][0].item() - e_ref) < (1e-5 if precision == "fp32" else 1e-4) * abs(e_ref)
