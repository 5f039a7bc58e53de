"""Benchmark of the real-time Kohn-Sham step on one MI355X.

Default workload: the batched divide-and-conquer step, 512 uneven periodic
domains (edge U{20..40}, orbitals U{16..96}, floor(N_o/4) atoms x 8 Gaussian
projectors, FD6, h = 0.4 bohr, complex64), the laser pulse A_z(t) =
0.05 sin(0.1 t) sin^2(pi t / 100 dt) at the step midpoints, dt = 0.02, all
domains advanced together and the K timed steps replayed from a captured HIP
graph.  The plain FP32 path gives ``value``; the same steps in split BF16
(hi+lo products, FP32 accumulation) are reported beside it.

A "step" is one Taylor-4 step: four applications of H (stencil + both
projector products).  The metric is orbital-gridpoint H.psi updates per
second = sum over domains of N_g N_o * 4 * steps / time.

    python bench.py [--steps K] [--warmup W] [--precision fp32|split_bf16|split_fp16|fp64]
                    [--workload batched|single|hpsi|eq2|adjoint]

Prints one JSON line.  Per-kernel times come from HIP events that the library
records around every launch on the call's stream (DCMESH_FLAG_PROFILE), over
the same K steps run eagerly right after the timed graph replays.
"""
import argparse
import hashlib
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "split_bf16": 2500.0, "split_fp16": 2500.0}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(dom, a_mid, dt, n_orb_sample=None, min_seconds=10.0, max_steps=8):
    """The FP64 oracle on the host: Taylor-4 steps of the same domain (all its
    orbitals unless ``n_orb_sample`` restricts them; orbitals propagate
    independently, so the per-orbital cost is that of the full step), repeated
    until ``min_seconds`` of work or ``max_steps`` steps."""
    from oracle import propagate as P
    from synth import Domain
    n_s = dom.n_orb if n_orb_sample is None else n_orb_sample
    sub = Domain(dom.shape, dom.h, dom.fd_order, np.ascontiguousarray(dom.psi[:, :n_s]),
                 dom.v_loc, dom.proj, dom.d, dom.occ[:n_s])
    psi = sub.psi
    steps, t = 0, 0.0
    while steps < max_steps and (steps == 0 or t < min_seconds):
        t0 = time.perf_counter()
        psi = P.taylor4_step(sub, a_mid[steps % len(a_mid)], dt, psi)
        t += time.perf_counter() - t0
        steps += 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    return {"value": dom.n_grid * n_s * 4 * steps / t, "unit": "orbital-gridpoint updates/s",
            "cores": int(threads), "kind": "oracle",
            "sample": f"{steps} Taylor-4 step(s) (4 H applications each) of the 64^3/512-projector domain "
                      f"on {n_s} of its {dom.n_orb} orbitals, FP64 numpy; {t:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "split_bf16", "split_fp16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="batched", choices=["batched", "single", "hpsi", "eq2", "adjoint"],
                    help="batched: 512 uneven domains, graph-replayed (default); single: the 64^3 / "
                         "128-orbital domain with rho, j, E every step; hpsi: the standalone H.psi of the "
                         "64^3 domain; eq2: Eq. 2 steps with the Eq. 5 nonlocal operator on the 64^3 "
                         "domain; adjoint: the pulse gradient on the 48^3 / 64-orbital domain")
    ap.add_argument("--no-split", action="store_true", help="batched: skip the split BF16 run beside FP32")
    ap.add_argument("--graph-steps", type=int, default=100,
                    help="batched: steps per captured graph when K is a multiple of it (else one K-step graph)")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--tuning", default="",
                    help="global tile choices before the run, e.g. stencil=9,project=8,correct=7")
    ap.add_argument("--stream-ceiling", action="store_true",
                    help="only measure what plain streams reach on this GPU (1 GiB operands: a read-only "
                         "sum, a copy, and a two-read one-write add) and print one JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy a 1 GiB buffer three times (reference dispatch "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.stream_ceiling:
        stream_ceiling()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: domains are independent, so a run over several GPUs "
              "would place whole domains (or orbital bands) on each and has no cross-GPU part to time.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2509_00966_amd as api
    from synth import config, pulse_midpoints

    for kv in filter(None, args.tuning.split(",")):
        fam, v = kv.split("=")
        api.set_tuning(fam.strip(), int(v))
        log(f"bench: tuning {fam.strip()} = {int(v)}")
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "adjoint":
        return run_adjoint(args)
    if args.workload == "hpsi":
        return run_hpsi(args)
    if args.workload == "eq2":
        return run_eq2(args)

    log("bench: generating the 64^3 / 128-orbital / 512-projector domain")
    w = config(2)
    dom = w.domains[0]
    K, W = args.steps, args.warmup
    a_mid = pulse_midpoints(max(200, K + W), w.dt, 200)
    prec = args.precision
    cd, rd = api.complex_dtype(prec), api.real_dtype(prec)
    dev = "cuda:0"
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x)).to(dev, dt)
    g = api.Domain(dom.shape, dom.fd_order, dom.h, t(dom.psi, cd), t(dom.v_loc, rd), t(dom.proj, cd),
                   t(dom.d, rd), t(dom.occ, rd))
    ws = api.Workspace.for_domains([g], prec)
    ng, no, npj = dom.n_grid, dom.n_orb, dom.n_proj
    a_dev = t(a_mid, torch.float64)
    obs = dict(rho=torch.zeros(K, ng, dtype=rd, device=dev), j=torch.zeros(K, ng, 3, dtype=rd, device=dev),
               energy=torch.zeros(K, dtype=torch.float64, device=dev))
    obs_w = dict(rho=torch.zeros(max(W, 1), ng, dtype=rd, device=dev),
                 j=torch.zeros(max(W, 1), ng, 3, dtype=rd, device=dev),
                 energy=torch.zeros(max(W, 1), dtype=torch.float64, device=dev))
    log(f"bench: warmup {W} steps")
    if W:
        api.step([g], a_dev[:W].contiguous(), w.dt, W, prec, ws, obs=[obs_w])
    torch.cuda.synchronize()
    api.profile_collect()
    log(f"bench: timing {K} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    api.step([g], a_dev[W:W + K].contiguous(), w.dt, K, prec, ws, obs=[obs], profile=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = api.profile_collect()
    log("bench: kernel times " + json.dumps({k: [round(v[0], 3), v[1]] for k, v in prof.items() if v[1]}))

    ms_step = elapsed * 1e3 / K
    updates = ng * no * 4 * K / elapsed
    flops_gemm = 8.0 * ng * no * npj              # per projection or correction launch
    # per launch, averaged over the four Horner stages: the first reads psi once
    # (it is both u and the base), the other three read u and psi; all write
    # out and read V
    bytes_stencil = ng * no * (16.0 + 3 * 24.0) / 4 + ng * 4.0
    bytes_gemm = ng * npj * 8.0 + ng * no * 8.0   # projectors once (FP32 or hi+lo 16-bit), orbitals once
    roofline, kernels = roofline_of(prof, flops_gemm, bytes_stencil, prec, bytes_gemm)
    if "stencil" in kernels and "achieved" in kernels["stencil"]:
        # the stencil reads two arrays and writes one: also report it against
        # what a plain two-read one-write stream reaches on this GPU
        st = stream_rates(cases=("2 reads + 1 write (add)",))["2 reads + 1 write (add)"]
        kernels["stencil"]["stream_2r1w_GBs"] = st["TB/s"] * 1e3
        kernels["stencil"]["frac_of_stream"] = kernels["stencil"]["achieved"] / (st["TB/s"] * 1e3)

    finite = bool(torch.isfinite(g.psi).all().item())
    if args.copy_calibration:
        copy_calibration()
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on a bounded sample")
        cpu = cpu_baseline(dom, a_mid, w.dt)
    out = {
        "metric": "orbital-gridpoint H.psi updates/s",
        "value": updates,
        "unit": "orbital-gridpoint updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "fp32", "fp64": "fp64", "split_bf16": "bf16x2+fp32", "split_fp16": "fp16x2+fp32"}[prec],
        "data": "synthetic",
        "config": {"workload": "single domain 64^3, h=0.4, 128 complex64 orbitals, 64 atoms x 8 projectors, "
                               "FD6, laser A_z(t), dt=0.02, Taylor-4, rho+j+E every step",
                   "precision": prec, "n_grid": ng, "n_orb": no, "n_proj": npj},
        "roofline": roofline,
        "kernels": kernels,
        "s_per_orbital_step": elapsed / K / no,
        "psi_finite": finite,
        "cpu_baseline": cpu,
    }
    out["kernel_source_hash"] = kernel_source_hash()
    print(json.dumps(out))


def copy_calibration():
    """Three copies of a 1 GiB buffer: the reference dispatch that scales the
    hardware byte counters (FETCH_SIZE, WRITE_SIZE) to bytes."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")     # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def c2_domain(api, prec, with_proj=True):
    """The 64^3 / 128-orbital / 512-projector domain (FD6, h = 0.4) on the GPU."""
    import torch
    from synth import config
    w = config(2)
    dom = w.domains[0]
    cd, rd = api.complex_dtype(prec), api.real_dtype(prec)
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", dt)
    proj = dom.proj if with_proj else np.zeros((dom.n_grid, 0), np.complex128)
    d = dom.d if with_proj else np.zeros(0)
    g = api.Domain(dom.shape, dom.fd_order, dom.h, t(dom.psi, cd), t(dom.v_loc, rd), t(proj, cd), t(d, rd),
                   t(dom.occ, rd))
    return w, dom, g


def run_hpsi(args):
    """The standalone local H.psi on the 64^3 / 128-orbital domain: out =
    f_n H_loc(A) psi_n (no projectors, no Taylor base), one stencil launch per
    call, K timed calls.  Algorithmic bytes per launch: read psi and write out
    (16 B per point-orbital) and V (4 B per point)."""
    import torch
    import paper_2509_00966_amd as api
    prec = args.precision if args.precision in ("fp32", "fp64") else "fp32"
    w, dom, g = c2_domain(api, prec, with_proj=False)
    ws = api.Workspace.for_domains([g], prec)
    out = torch.empty_like(g.psi)
    A = torch.tensor([[0.0, 0.0, 0.05]], dtype=torch.float64, device="cuda:0")
    for _ in range(max(1, args.warmup)):
        api.density([g], A, prec, ws, [dict(hpsi_occ=out)])
    torch.cuda.synchronize()
    api.profile_collect()
    K = args.steps
    t0 = time.perf_counter()
    for _ in range(K):
        api.density([g], A, prec, ws, [dict(hpsi_occ=out)], profile=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = api.profile_collect()
    ms, cnt = prof["stencil"]
    es = 8 if prec == "fp32" else 16
    nbytes = dom.n_grid * dom.n_orb * 2.0 * es + dom.n_grid * es / 2
    achieved = nbytes / (ms / cnt * 1e-3) / 1e9
    variants = None
    if args.autotune:
        # every stencil tile variant on the same call (the default is above)
        variants = {}
        for v in range(api.tuning_options("stencil")):
            api.set_tuning("stencil", v)
            try:
                api.density([g], A, prec, ws, [dict(hpsi_occ=out)])
                torch.cuda.synchronize()
                api.profile_collect()
                for _ in range(K):
                    api.density([g], A, prec, ws, [dict(hpsi_occ=out)], profile=True)
                pm, pc = api.profile_collect()["stencil"]
                variants[v] = round(nbytes / (pm / pc * 1e-3) / 1e9, 1)
            finally:
                api.set_tuning("stencil", -1)
        log("bench: stencil variants (GB/s) " + json.dumps(variants))
    st = stream_rates(cases=("2 reads + 1 write (add)", "copy"))
    out_line = {
        "metric": "standalone H.psi HBM bandwidth", "value": achieved, "unit": "GB/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms / cnt, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": "standalone local H.psi, 64^3 grid, h=0.4, 128 complex orbitals, FD6, A along z",
                   "precision": prec, "n_grid": dom.n_grid, "n_orb": dom.n_orb},
        "roofline": {"kernel": "stencil", "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None},
        "bytes_per_launch": nbytes, "wall_ms_per_call": elapsed * 1e3 / K,
        "orbital_gridpoint_hpsi_per_s": dom.n_grid * dom.n_orb / (ms / cnt * 1e-3),
        "stencil_variants_GBs": variants,
        "stream_copy_GBs": st["copy"]["TB/s"] * 1e3,
        "frac_of_copy_stream": achieved / (st["copy"]["TB/s"] * 1e3),
    }
    out_line["kernel_source_hash"] = kernel_source_hash()
    print(json.dumps(out_line))


def run_eq2(args):
    """Eq. 2 with the Eq. 5 nonlocal operator on the 64^3 domain: 128
    reference orbitals Psi(0) (N_p = N_o = 128), FP32, K steps after W
    warm-up steps, every launch bracketed by events.  Each step runs two
    normalised half-steps, each one overlap product h^3 Psi(0)^H Psi (the
    paper's CGEMM(1)) and one correction Psi -= delta Psi(0) S (CGEMM(2)),
    around the local Taylor-4 propagator."""
    import torch
    import paper_2509_00966_amd as api
    from synth import make_domain, pulse_midpoints
    prec = "fp32"
    w, dom, g0 = c2_domain(api, prec, with_proj=False)
    other = make_domain(92, dom.shape, dom.n_orb, 1, proj_per_atom=8, h=dom.h, fd_order=dom.fd_order)
    psi = torch.from_numpy(np.ascontiguousarray(other.psi)).to("cuda:0", torch.complex64)
    g = g0.with_psi(psi)
    psi0 = g0.psi
    ws = api.Workspace.for_domains([g], prec, eq2=True)
    K, W = args.steps, args.warmup
    a_dev = torch.from_numpy(pulse_midpoints(W + K, w.dt, 200)).to("cuda:0")
    if W:
        api.step_eq2([g], [psi0], 0.8, a_dev[:W].contiguous(), w.dt, W, prec, ws)
    torch.cuda.synchronize()
    api.profile_collect()
    t0 = time.perf_counter()
    api.step_eq2([g], [psi0], 0.8, a_dev[W:].contiguous(), w.dt, K, prec, ws, profile=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = api.profile_collect()
    ng, no = dom.n_grid, dom.n_orb
    flops = 8.0 * ng * no * no
    bytes_gemm = 2 * ng * no * 8.0
    bytes_stencil = ng * no * (16.0 + 3 * 24.0) / 4 + ng * 4.0
    roof, kernels = roofline_of(prof, flops, bytes_stencil, prec, bytes_gemm, workload="eq2")
    out = {
        "metric": "orbital-gridpoint H.psi updates/s", "value": ng * no * 4 * K / elapsed,
        "unit": "orbital-gridpoint updates/s (local Taylor-4 stages)", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": elapsed * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "Eq. 2 with the Eq. 5 nonlocal operator: 64^3 grid, h=0.4, 128 complex64 "
                               "orbitals, 128 reference orbitals, FD6, laser A_z(t), dt=0.02, v_nl=0.8",
                   "precision": prec, "n_grid": ng, "n_orb": no},
        "roofline": roof, "kernels": kernels,
        "cgemm_tflops": {"overlap_CGEMM1": kernels.get("project", {}).get("algorithmic_tflops"),
                         "correction_CGEMM2": kernels.get("correct", {}).get("algorithmic_tflops")},
        "psi_finite": bool(torch.isfinite(g.psi).all().item()),
    }
    out["kernel_source_hash"] = kernel_source_hash()
    print(json.dumps(out))


def roofline_of(prof, flops_gemm, bytes_stencil, prec, bytes_gemm=None, workload="single"):
    """Per-family achieved rate against its bound, on the algorithmic counts
    of one launch.  flops_gemm: 8 N_g N_o N_p of one projection or correction
    launch (the complex-product count); bytes_gemm: its compulsory bytes
    (projectors once, orbitals once).  A family is MFMA-bound when the
    algorithmic flops take longer at the dtype's peak than its bytes at the
    HBM peak; ``achieved`` is then the algorithmic flop rate.  The MFMA work
    actually executed differs: FP32 runs the three-real-product (Gauss) form,
    0.75 of the count, split modes three 16-bit products per real product, 3x;
    its fraction of the peak is reported as ``frac_executed_mfma``."""
    mfma_factor = {"fp32": 0.75, "fp64": 1.0, "split_bf16": 3.0, "split_fp16": 3.0}[prec]
    kernels = {}
    for fam, (ms, cnt) in prof.items():
        if not cnt:
            continue
        avg = ms / cnt
        entry = {"launches": cnt, "avg_ms": avg, "total_ms": ms}
        if fam in ("project", "correct"):
            exec_flops = flops_gemm * mfma_factor
            t_mfma = flops_gemm / (PEAK_TFLOPS[prec] * 1e12)
            t_hbm = (bytes_gemm or 0) / (PEAK_HBM_GBS * 1e9)
            entry["algorithmic_tflops"] = flops_gemm / (avg * 1e-3) / 1e12
            entry["frac_executed_mfma"] = exec_flops / (avg * 1e-3) / 1e12 / PEAK_TFLOPS[prec]
            if bytes_gemm:
                entry["hbm_GBs"] = bytes_gemm / (avg * 1e-3) / 1e9
            if t_hbm > t_mfma:
                entry.update(bound="hbm", achieved=bytes_gemm / (avg * 1e-3) / 1e9, unit="GB/s", peak=PEAK_HBM_GBS)
            else:
                entry.update(bound="mfma", achieved=flops_gemm / (avg * 1e-3) / 1e12, unit="TFLOP/s",
                             peak=PEAK_TFLOPS[prec])
        elif fam == "stencil":
            entry.update(bound="hbm", achieved=bytes_stencil / (avg * 1e-3) / 1e9, unit="GB/s", peak=PEAK_HBM_GBS)
        if "peak" in entry:
            entry["frac"] = entry["achieved"] / entry["peak"]
        kernels[fam] = entry
    dom_fam = max((f for f in kernels if "peak" in kernels[f]), key=lambda f: kernels[f]["total_ms"])
    dk = kernels[dom_fam]
    roof = {"kernel": dom_fam, "bound": dk["bound"], "achieved": dk["achieved"], "peak": dk["peak"],
            "unit": dk["unit"], "frac": dk["frac"], "traffic": measured_traffic(dom_fam, prec, workload)}
    if "frac_executed_mfma" in dk:
        roof["frac_executed_mfma"] = dk["frac_executed_mfma"]
    return roof, kernels


TRAFFIC_TABLES = {"single": os.path.join(ROOT, "profiles", "hbm_traffic_64cube_128orb_512proj.md"),
                  "batched": os.path.join(ROOT, "profiles", "hbm_traffic_batched_512dom.md")}
KERNEL_SOURCES = ("common.hpp", "stencil.hpp", "gemm.hpp", "gemm_split.hpp", "reduce.hpp", "dcmesh.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_00966_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stream_ceiling():
    """Print stream_rates() of every case as one JSON line."""
    print(json.dumps({"stream_ceiling": stream_rates(), "bytes_per_operand": 4 << 28}))


def stream_rates(cases=None):
    """Bandwidth that plain streams reach on this GPU, for reading the
    stencil's HBM fraction: torch's own kernels on 1 GiB float32 operands,
    best of five HIP-event-timed launches after a warm-up."""
    import torch
    dev = "cuda"
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.ones(n, dtype=torch.float32, device=dev)
    o = torch.empty(n, dtype=torch.float32, device=dev)
    s = torch.empty((), dtype=torch.float32, device=dev)
    all_cases = {"read (sum)": (lambda: torch.sum(a, dim=0, out=s), 1),
                 "copy": (lambda: o.copy_(a), 2),
                 "2 reads + 1 write (add)": (lambda: torch.add(a, b, out=o), 3)}
    res = {}
    for name, (fn, k) in all_cases.items():
        if cases is not None and name not in cases:
            continue
        fn()
        best = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        res[name] = {"ms": round(best, 4), "TB/s": round(k * 4.0 * n / best / 1e9, 3),
                     "frac_of_8TBs": round(k * 4.0 * n / best / 1e9 / 8.0, 3)}
    return res


def measured_traffic(family, prec, workload="single"):
    """HBM bytes per launch of a kernel family on a workload, from the
    FETCH_SIZE / WRITE_SIZE counter table in profiles/ (each counter scaled by
    what it reads for a copy of known size).  None when there is no table or
    it was taken from kernel sources other than the ones built here."""
    table = TRAFFIC_TABLES.get(workload)
    if table is None:
        return None
    try:
        with open(table) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"kernel source hash: `([0-9a-f]+)`", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    col = None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if "HBM bytes per launch" in cells:
            col = cells.index("HBM bytes per launch")
        elif col is not None and len(cells) > col and cells[0] == family and cells[1] == prec:
            try:
                return float(cells[col])
            except ValueError:
                return None
    return None


def run_adjoint(args):
    """Gradient of the absorbed energy with respect to 400 free A_z samples on
    the 48^3 / 64-orbital / 256-projector domain (FD6, dt 0.02): 400 steps
    forward with a checkpoint every 20, then the adjoint recursion backward with
    each segment recomputed from its checkpoint.  ``--steps`` counts pulse
    samples; one evaluation covers all 400, so the timed evaluations are
    max(1, steps // 400).  Prints one JSON line."""
    import torch
    import paper_2509_00966_amd as api
    from paper_2509_00966_amd.autograd import absorbed_energy
    from synth import config
    prec = args.precision
    w = config(5)
    dom = w.domains[0]
    cd, rd = api.complex_dtype(prec), api.real_dtype(prec)
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dt)
    g = api.Domain(dom.shape, dom.fd_order, dom.h, t(dom.psi, cd), t(dom.v_loc, rd), t(dom.proj, cd),
                   t(dom.d, rd), t(dom.occ, rd))
    ws = api.Workspace.for_domains([g], prec)
    n = w.n_steps
    az = w.a_mid[:, 2].copy()

    def evaluate():
        a = torch.from_numpy(az).to("cuda").requires_grad_(True)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        loss = absorbed_energy(a, g, w.dt, prec, 20, ws)
        e1.record()
        loss.backward()
        e2.record()
        e2.synchronize()
        return e0.elapsed_time(e1), e1.elapsed_time(e2), loss.item(), a.grad

    for _ in range(max(0, min(args.warmup, 1))):
        evaluate()
    reps = max(1, args.steps // n)
    fw, bw = [], []
    for _ in range(reps):
        f, b, loss, grad = evaluate()
        fw.append(f)
        bw.append(b)
    ms_eval = (sum(fw) + sum(bw)) / reps
    out = {
        "metric": "pulse-gradient orbital-gridpoint steps/s",
        "value": dom.n_grid * dom.n_orb * n / (ms_eval * 1e-3),
        "unit": "orbital-gridpoint steps/s (forward + adjoint per step)",
        "n_gpus": 1, "steps": n * reps, "warmup": min(args.warmup, 1) * n,
        "ms_per_step": ms_eval / n, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "fp32", "fp64": "f64", "split_bf16": "bf16x2+fp32", "split_fp16": "fp16x2+fp32"}[prec],
        "data": "synthetic",
        "config": {"workload": "48^3 grid, h=0.4, 64 complex64 orbitals, 32 atoms x 8 projectors, FD6, "
                               "400 free A_z samples, checkpoints every 20 steps, loss = absorbed energy",
                   "precision": prec, "n_grid": dom.n_grid, "n_orb": dom.n_orb, "n_proj": dom.n_proj},
        "forward_ms": sum(fw) / reps, "backward_ms": sum(bw) / reps,
        "loss": loss, "grad_norm": float(grad.norm().item()), "grad_finite": bool(torch.isfinite(grad).all().item()),
    }
    out["kernel_source_hash"] = kernel_source_hash()
    print(json.dumps(out))


def cpu_baseline_batched(subset, a_mid, dt, min_seconds=10.0, max_rounds=4):
    """The FP64 oracle on the host: one Taylor-4 step of each domain of the
    seeded 16-domain subset (smallest, largest and 14 seeded domains), all of
    their orbitals, repeated until ``min_seconds`` of work."""
    from oracle import propagate as P
    t, rounds, po = 0.0, 0, 0
    while rounds < max_rounds and (rounds == 0 or t < min_seconds):
        for d in subset:
            t0 = time.perf_counter()
            P.taylor4_step(d, a_mid[rounds % len(a_mid)], dt, d.psi)
            t += time.perf_counter() - t0
            po += d.n_grid * d.n_orb
        rounds += 1
    return {"value": po * 4 / t, "unit": "orbital-gridpoint updates/s", "cores": blas_threads(),
            "kind": "oracle",
            "sample": f"{rounds} Taylor-4 step(s) of each of 16 seeded domains of the 512 (the smallest, the "
                      f"largest and 14 more; all their orbitals, {po // rounds} point-orbitals per round), "
                      f"FP64 numpy; {t:.1f} s"}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] + [1]))
    except Exception:
        return os.cpu_count()


def batched_counts(doms):
    """Algorithmic counts of one launch of each family over all domains:
    the projector products 8 N_g N_o N_p flops (complex count), their
    compulsory bytes (B once + u once), and the stencil's bytes as fused
    into the Taylor stage (read u, read the base, write out: 24 B per
    point-orbital in three stages, 16 B in the first where u is the base;
    V 4 B per point)."""
    flops = sum(8.0 * d.n_grid * d.n_orb * d.n_proj for d in doms)
    bytes_gemm = sum(d.n_grid * d.n_proj * 8.0 + d.n_grid * d.n_orb * 8.0 for d in doms)
    bytes_stencil = sum(d.n_grid * d.n_orb * (16.0 + 3 * 24.0) / 4 + d.n_grid * 4.0 for d in doms)
    return flops, bytes_gemm, bytes_stencil


def run_batched(args):
    """512 uneven domains (edge U{20..40}, orbitals U{16..96}, floor(N_o/4) atoms x 8
    projectors, FD6, complex64), all advanced by one launch per kernel family
    and Taylor stage; W eager warm-up steps, then the K timed steps replayed
    from a captured HIP graph (one graph of K steps, or replays of a
    ``--graph-steps`` graph when K is a multiple of it), then the same K steps
    eagerly with per-launch events for the kernel breakdown.  FP32 gives
    ``value``; split BF16 runs the same steps from the same start."""
    import torch
    import paper_2509_00966_amd as api
    from synth import batched_domain, batched_domain_shapes, batched_subset, pulse_midpoints

    dev = "cuda:0"
    shapes = batched_domain_shapes()
    log(f"bench: generating {len(shapes)} domains")
    doms, t_gen = [], time.perf_counter()
    sub_idx = set(batched_subset())
    subset = []
    for i in range(len(shapes)):
        d = batched_domain(i)
        if i in sub_idx and not args.no_cpu_baseline:
            subset.append(d)
        t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x)).to(dev, dt)
        doms.append(api.Domain(d.shape, d.fd_order, d.h, t(d.psi, torch.complex64), t(d.v_loc, torch.float32),
                               t(d.proj, torch.complex64), t(d.d, torch.float32), t(d.occ, torch.float32)))
        if i % 64 == 63:
            log(f"bench: {i + 1} domains on the GPU ({time.perf_counter() - t_gen:.0f} s)")
    gen_s = time.perf_counter() - t_gen
    psi_start = [d.psi.clone() for d in doms]
    K, W = args.steps, args.warmup
    S = K if (K <= args.graph_steps or K % args.graph_steps) else args.graph_steps
    dt = 0.02
    a_mid = pulse_midpoints(W + K, dt, 100)
    a_dev = torch.from_numpy(a_mid).to(dev)
    po = sum(d.n_grid * d.n_orb for d in doms)
    flops, bytes_gemm, bytes_stencil = batched_counts(doms)
    precs = [args.precision]
    if args.precision == "fp32" and not args.no_split:
        precs.append("split_bf16")
    runs = {}
    for prec in precs:
        for d, p0 in zip(doms, psi_start):
            d.psi.copy_(p0)
        ws = api.Workspace.for_domains(doms, prec)
        log(f"bench: {prec}: workspace {ws.nbytes / 2**30:.1f} GiB; warmup {W} eager steps")
        if args.autotune:
            from paper_2509_00966_amd import autotune
            t_tune = time.perf_counter()
            table = autotune.tune_classes(doms, a_dev, dt, prec)
            autotune.apply_classes(doms, prec, table)
            log(f"bench: {prec}: tiles tuned per shape class in {time.perf_counter() - t_tune:.0f} s: "
                + json.dumps({str(k): v for k, v in sorted(table.items())}))
        if W:
            api.step(doms, a_dev[:W].contiguous(), dt, W, prec, ws)
        graph = api.Graph(doms, a_dev[W:W + S].contiguous(), dt, S, prec, ws)
        torch.cuda.synchronize()
        log(f"bench: {prec}: timing {K} steps ({K // S} replay(s) of a {S}-step graph)")
        t0 = time.perf_counter()
        for _ in range(K // S):
            graph.launch()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        graph.close()
        finite = bool(all(torch.isfinite(d.psi).all().item() for d in doms))
        log(f"bench: {prec}: {elapsed * 1e3 / K:.2f} ms per step; kernel breakdown over {K} eager steps")
        api.profile_collect()
        api.step(doms, a_dev[W:W + K].contiguous(), dt, K, prec, ws, profile=True)
        prof = api.profile_collect()
        log(f"bench: {prec}: kernel times " + json.dumps({k: [round(v[0], 3), v[1]] for k, v in prof.items() if v[1]}))
        roof, kernels = roofline_of(prof, flops, bytes_stencil, prec, bytes_gemm, workload="batched")
        runs[prec] = {"value": po * 4 * K / elapsed, "ms_per_step": elapsed * 1e3 / K, "roofline": roof,
                      "kernels": kernels, "psi_finite": finite,
                      "kernel_ms_per_step": sum(v[0] for v in prof.values()) / K}
        del ws
        torch.cuda.empty_cache()
        if args.autotune:
            from paper_2509_00966_amd import autotune
            autotune.reset_classes()
    if args.copy_calibration:
        copy_calibration()
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the 16-domain subset")
        cpu = cpu_baseline_batched(subset, a_mid, dt)
    main = runs[precs[0]]
    dtype = {"fp32": "fp32", "fp64": "fp64", "split_bf16": "bf16x2+fp32", "split_fp16": "fp16x2+fp32"}
    out = {
        "metric": "orbital-gridpoint H.psi updates/s",
        "value": main["value"],
        "unit": "orbital-gridpoint updates/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": main["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype[precs[0]],
        "data": "synthetic",
        "config": {"workload": "batched divide-and-conquer: 512 uneven periodic domains, edge U{20..40}, "
                               "orbitals U{16..96}, floor(N_o/4) atoms x 8 projectors, FD6, h=0.4, complex64, "
                               "laser A_z(t) (T = 100 dt), dt=0.02, Taylor-4; timed steps replayed from a "
                               f"{S}-step HIP graph", "precision": precs[0],
                   "domains": len(doms), "point_orbitals": po, "graph_steps": S},
        "roofline": main["roofline"],
        "kernels": main["kernels"],
        "kernel_ms_per_step": main["kernel_ms_per_step"],
        "s_per_orbital_step": main["ms_per_step"] * 1e-3 / sum(d.n_orb for d in doms),
        "psi_finite": main["psi_finite"],
        "cpu_baseline": cpu,
        "gen_seconds": gen_s,
    }
    for prec in precs[1:]:
        r = runs[prec]
        out[prec] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "dtype": dtype[prec],
                     "speedup_vs_" + precs[0]: r["value"] / main["value"], "roofline": r["roofline"],
                     "kernels": r["kernels"], "kernel_ms_per_step": r["kernel_ms_per_step"],
                     "psi_finite": r["psi_finite"]}
    out["kernel_source_hash"] = kernel_source_hash()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
