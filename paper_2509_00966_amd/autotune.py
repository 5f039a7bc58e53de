"""Tile autotuner for the step kernels.

For a set of domains and a precision, every tile variant of each kernel family
(stencil sweep, projection, correction) is timed with the library's own HIP
events (``DCMESH_FLAG_PROFILE``) over a few steps on a scratch copy of the
orbitals, and the fastest variant per family is kept.  Results are cached in
a JSON file keyed by the domain shapes, the precision and the GPU architecture,
so a later run reuses them without timing.

    from paper_2509_00966_amd import autotune
    best = autotune.tune(domains, a, dt, "fp32")      # {"stencil": v, "project": v, "correct": v}
    autotune.apply(best)
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Sequence

import torch

from . import api

FAMILIES = ("stencil", "project", "correct")
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dcmesh_autotune.json")


def _key(domains: Sequence[api.Domain], precision: str) -> str:
    arch = torch.cuda.get_device_properties(domains[0].psi.device).gcnArchName if torch.cuda.is_available() else "cpu"
    sig = sorted((d.shape, d.n_orb, d.n_proj, d.fd_order) for d in domains)
    h = hashlib.sha1(json.dumps([str(s) for s in sig]).encode()).hexdigest()[:16]
    return f"{arch}:{precision}:{len(domains)}:{h}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def apply(best: Dict[str, int]):
    for fam in FAMILIES:
        api.set_tuning(fam, int(best.get(fam, -1)))


def reset():
    for fam in FAMILIES:
        api.set_tuning(fam, -1)


def time_variants(domains, a, dt, precision, steps=2, work=None) -> Dict[str, Dict[int, float]]:
    """{family: {variant: average kernel ms per launch}} measured on scratch copies."""
    work = work or api.Workspace.for_domains(domains, precision)
    scratch = [d.with_psi(d.psi.clone()) for d in domains]
    out = {}
    try:
        for fam in FAMILIES:
            out[fam] = {}
            for v in range(api.tuning_options(fam)):
                reset()
                api.set_tuning(fam, v)
                api.step(scratch, a[:1].contiguous(), dt, 1, precision, work)      # warm
                torch.cuda.synchronize()
                api.profile_collect()
                api.step(scratch, a[:steps].contiguous(), dt, steps, precision, work, profile=True)
                prof = api.profile_collect()
                ms, cnt = prof[fam]
                out[fam][v] = ms / max(cnt, 1)
    finally:
        reset()
    return out


def tune(domains, a, dt, precision, cache_path: str = DEFAULT_CACHE, steps=2, force=False) -> Dict[str, int]:
    key = _key(domains, precision)
    cache = _load(cache_path)
    if key in cache and not force:
        return cache[key]["best"]
    times = time_variants(domains, a, dt, precision, steps)
    best = {fam: min(t, key=t.get) for fam, t in times.items()}
    cache[key] = {"best": best, "ms": {f: {str(k): v for k, v in t.items()} for f, t in times.items()}}
    os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
    with open(cache_path, "w") as f:
        json.dump(cache, f, indent=1)
    return best
