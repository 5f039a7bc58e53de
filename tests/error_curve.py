"""Error of the FP32 and split-precision paths against the FP64 oracle at every
step of the 64^3 / 128-orbital / 512-projector workload with the laser pulse
(200 steps, the split-precision workload's length).

The library runs all 128 orbitals one step per call in FP32, split BF16 and
split FP16; the oracle runs 8 sampled orbitals (seven seeded ones and the
last) from the same FP32-rounded inputs.  Orbitals propagate independently,
so the oracle's columns are exactly the library's columns.  After every step
the three error views of each precision (relative Frobenius norm,
element-wise max over the largest value, worst orbital) are written as one
JSON line.

    python tests/error_curve.py [--steps 200] [--out error_curve.jsonl]

Not collected by pytest (it takes minutes of oracle time); it needs a GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--sample", type=int, default=8)
    ap.add_argument("--out", default="error_curve.jsonl")
    args = ap.parse_args()

    import torch
    import paper_2509_00966_amd as api
    from helpers import a_tensor, errors, to_device
    from oracle import propagate as P
    from synth import Domain, config

    w = config(3)
    dom = w.domains[0]
    od = dom.rounded(np.float32)
    n = min(args.steps, len(w.a_mid))
    cols = np.sort(np.append(np.random.default_rng(303).choice(dom.n_orb - 1, args.sample - 1, replace=False),
                             dom.n_orb - 1))
    sub = Domain(od.shape, od.h, od.fd_order, np.ascontiguousarray(od.psi[:, cols]), od.v_loc, od.proj, od.d,
                 od.occ[cols])
    precs = ("fp32", "split_bf16", "split_fp16")
    gs = {p: to_device(dom, p) for p in precs}
    ws = {p: api.Workspace.for_domains([gs[p]], p) for p in precs}
    at = a_tensor(w.a_mid[:n])
    ct = torch.from_numpy(cols).to("cuda")
    ref = sub.psi
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    t0 = time.perf_counter()
    with open(args.out, "w") as fh:
        fh.write(json.dumps({"workload": w.name, "steps": n, "orbitals": cols.tolist(), "dt": w.dt}) + "\n")
        for k in range(n):
            for p in precs:
                api.step([gs[p]], at[k:k + 1].contiguous(), w.dt, 1, p, ws[p])
            ref = P.taylor4_step(sub, w.a_mid[k], w.dt, ref)
            torch.cuda.synchronize()
            row = {"step": k + 1}
            for p in precs:
                e = errors(gs[p].psi[:, ct].cpu().numpy(), ref)
                row[p] = {"fro": e.fro, "elem": e.elem, "orb": e.orb}
            fh.write(json.dumps(row) + "\n")
            fh.flush()
            if (k + 1) % 10 == 0:
                print(f"step {k + 1}/{n} ({time.perf_counter() - t0:.0f} s): " +
                      ", ".join(f"{p} {row[p]['fro']:.2e}" for p in precs), flush=True)


if __name__ == "__main__":
    main()
