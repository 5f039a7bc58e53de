"""Tile autotuner for the step kernels.

For a set of domains and a precision, every tile variant of each kernel family
(stencil sweep, projection, correction) is timed with the library's own HIP
events (``DCMESH_FLAG_PROFILE``) over a few steps on a scratch copy of the
orbitals, and the fastest variant per family is kept.  Results are cached in
a JSON file keyed by the domain shapes, the precision and the GPU architecture,
so a later run reuses them without timing.

Two granularities:

* ``tune`` / ``apply``: one variant per family for the whole call (a global
  choice);
* ``tune_classes`` / ``apply_classes``: the domains are grouped into shape
  classes (grid edge and orbital count ranges), each class is timed on its
  own domains, and the winners go into the library's per-shape table
  (``dcmesh_set_tuning_shape``), so every domain runs the variant tuned for
  its class.

    from paper_2509_00966_amd import autotune
    best = autotune.tune(domains, a, dt, "fp32")      # {"stencil": v, "project": v, "correct": v}
    autotune.apply(best)
    table = autotune.tune_classes(domains, a, dt, "fp32")
    autotune.apply_classes(domains, "fp32", table)
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


EDGE_BINS = (20, 27, 34, 41)            # grid edges [20, 27), [27, 34), [34, 41)
ORB_BINS = (1, 17, 33, 49, 65, 81, 97)  # orbital counts in ranges of 16


def shape_class(d, edge_bins=EDGE_BINS, orb_bins=ORB_BINS):
    """(fd_order, edge range, orbital range) of a domain; shapes outside the
    ranges get their own open-ended class."""
    import bisect
    return (d.fd_order, bisect.bisect_right(edge_bins, max(d.shape)), bisect.bisect_right(orb_bins, d.n_orb))


def tune_classes(domains, a, dt, precision, cache_path: str = DEFAULT_CACHE, steps=2, force=False):
    """{class: {family: variant}}: each shape class's fastest variants, timed
    on that class's domains alone."""
    key = _key(domains, precision) + ":classes"
    cache = _load(cache_path)
    if key in cache and not force:
        return {tuple(json.loads(k)): v for k, v in cache[key]["table"].items()}
    groups = {}
    for i, d in enumerate(domains):
        groups.setdefault(shape_class(d), []).append(i)
    work = api.Workspace.for_domains(domains, precision)
    table, times = {}, {}
    for cls, idx in sorted(groups.items()):
        t = time_variants([domains[i] for i in idx], a, dt, precision, steps, work=work)
        table[cls] = {fam: min(tf, key=tf.get) for fam, tf in t.items()}
        times[cls] = t
    cache = _load(cache_path)
    cache[key] = {"table": {json.dumps(list(c)): v for c, v in table.items()},
                  "ms": {json.dumps(list(c)): {f: {str(k): x for k, x in tf.items()} for f, tf in t.items()}
                         for c, t in times.items()}}
    os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
    with open(cache_path, "w") as f:
        json.dump(cache, f, indent=1)
    return table


def apply_classes(domains, precision, table):
    """Fill the library's per-shape table: every domain's shape gets its
    class's variants."""
    for d in domains:
        best = table.get(shape_class(d))
        if best is None:
            continue
        for fam in FAMILIES:
            if fam in best:
                api.set_tuning_shape(fam, precision, tuple(d.shape), d.fd_order, d.n_orb, d.n_proj, int(best[fam]))


def reset_classes():
    api.clear_tuning_shapes()
