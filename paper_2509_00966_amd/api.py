"""Python binding over the C ABI: argument marshalling only.

Every array is a torch tensor on the GPU; the calls pass their data pointers
and the current HIP stream to the library, which queues all the work.  Nothing
here computes any part of the step.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import PRECISION, DcmeshDensityOut, DcmeshDomain, DcmeshObs, check, lib

_REAL = {"fp64": torch.float64, "fp32": torch.float32, "split_bf16": torch.float32,
         "split_fp16": torch.float32}
_CPLX = {"fp64": torch.complex128, "fp32": torch.complex64, "split_bf16": torch.complex64,
         "split_fp16": torch.complex64}


def real_dtype(precision: str):
    return _REAL[precision]


def complex_dtype(precision: str):
    return _CPLX[precision]


@dataclass
class Domain:
    """One periodic domain held in device tensors (layouts as in dcmesh.h)."""

    shape: tuple                  # (nx, ny, nz)
    fd_order: int
    h: float
    psi: torch.Tensor             # [N_g, N_o] complex
    v_loc: torch.Tensor           # [N_g] real
    proj: torch.Tensor            # [N_g, N_p] complex
    d: torch.Tensor               # [N_p] real
    occ: torch.Tensor             # [N_o] real

    @property
    def n_grid(self):
        return self.shape[0] * self.shape[1] * self.shape[2]

    @property
    def n_orb(self):
        return self.psi.shape[1]

    @property
    def n_proj(self):
        return self.proj.shape[1]

    def check(self, precision: str):
        cd, rd = _CPLX[precision], _REAL[precision]
        ng = self.n_grid
        for name, t, dt, shp in (("psi", self.psi, cd, (ng, self.n_orb)), ("v_loc", self.v_loc, rd, (ng,)),
                                 ("proj", self.proj, cd, (ng, self.n_proj)), ("d", self.d, rd, (self.n_proj,)),
                                 ("occ", self.occ, rd, (self.n_orb,))):
            if t.dtype != dt:
                raise TypeError(f"{name} must be {dt} for precision {precision}, got {t.dtype}")
            if tuple(t.shape) != shp:
                raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shp}")
            if not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
            if not t.is_cuda:
                raise ValueError(f"{name} must be a GPU tensor")

    def c_struct(self) -> DcmeshDomain:
        nx, ny, nz = self.shape
        ptr = lambda t: t.data_ptr() if t.numel() else None
        return DcmeshDomain(nx, ny, nz, self.fd_order, self.n_orb, self.n_proj, float(self.h),
                            self.psi.data_ptr(), self.v_loc.data_ptr(), ptr(self.proj), ptr(self.d),
                            self.occ.data_ptr())

    def with_psi(self, psi: torch.Tensor) -> "Domain":
        return Domain(self.shape, self.fd_order, self.h, psi, self.v_loc, self.proj, self.d, self.occ)


def _doms(domains: Sequence[Domain], precision: str):
    if precision not in PRECISION:
        raise ValueError(f"unknown precision {precision}")
    for d in domains:
        d.check(precision)
    arr = (DcmeshDomain * len(domains))(*[d.c_struct() for d in domains])
    return arr


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def workspace_bytes(domains: Sequence[Domain], precision: str, eq2: bool = False) -> int:
    arr = _doms(domains, precision)
    out = ctypes.c_size_t(0)
    flags = _lib.FLAG_EQ2 if eq2 else 0
    check(lib.dcmesh_workspace_bytes(arr, len(domains), PRECISION[precision], flags, ctypes.byref(out)))
    return out.value


class Workspace:
    """A 256-byte aligned device buffer of at least ``nbytes``."""

    def __init__(self, nbytes: int, device=None):
        self.raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
        off = (-self.raw.data_ptr()) % 256
        self.ptr = self.raw.data_ptr() + off
        self.nbytes = nbytes

    @classmethod
    def for_domains(cls, domains, precision, eq2=False):
        return cls(workspace_bytes(domains, precision, eq2), domains[0].psi.device)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def step(domains: Sequence[Domain], a: torch.Tensor, dt: float, n_steps: int, precision: str,
         work: Workspace, obs: Optional[List[dict]] = None, a_per_domain: bool = False,
         check_finite: bool = False, profile: bool = False, stream=None):
    """Advance every domain by n_steps Taylor-4 steps.  ``a``: float64 device
    tensor [n_steps, 3] (or [n_dom, n_steps, 3] with a_per_domain).  ``obs``:
    optional per-domain dict with 'rho' [n_steps, N_g], 'j' [n_steps, N_g, 3]
    real tensors and 'energy' [n_steps] float64."""
    arr = _doms(domains, precision)
    if a.dtype != torch.float64 or not a.is_contiguous() or not a.is_cuda:
        raise ValueError("a must be a contiguous float64 GPU tensor")
    stride = a.shape[-2]
    o = None
    if obs is not None:
        o = (DcmeshObs * len(domains))(*[DcmeshObs(_ptr(x.get("rho")), _ptr(x.get("j")), _ptr(x.get("energy")))
                                         for x in obs])
    flags = (_lib.FLAG_CHECK_FINITE if check_finite else 0) | (_lib.FLAG_PROFILE if profile else 0)
    check(lib.dcmesh_step(arr, len(domains), PRECISION[precision], a.data_ptr(), int(a_per_domain), stride,
                          float(dt), int(n_steps), o, work.ptr, work.nbytes, flags, _stream(stream)))


def step_noalloc(domains: Sequence[Domain], a: torch.Tensor, dt: float, n_steps: int, precision: str,
                 obs: Optional[List[dict]] = None, a_per_domain: bool = False, check_finite: bool = False,
                 stream=None):
    """``step`` without a workspace: the library's static device scratch
    (dcmesh_step_noalloc; 64 MiB, so small domains only)."""
    arr = _doms(domains, precision)
    if a.dtype != torch.float64 or not a.is_contiguous() or not a.is_cuda:
        raise ValueError("a must be a contiguous float64 GPU tensor")
    o = None
    if obs is not None:
        o = (DcmeshObs * len(domains))(*[DcmeshObs(_ptr(x.get("rho")), _ptr(x.get("j")), _ptr(x.get("energy")))
                                         for x in obs])
    flags = _lib.FLAG_CHECK_FINITE if check_finite else 0
    check(lib.dcmesh_step_noalloc(arr, len(domains), PRECISION[precision], a.data_ptr(), int(a_per_domain),
                                  a.shape[-2], float(dt), int(n_steps), o, flags, _stream(stream)))


def step_eq2(domains: Sequence[Domain], psi0: Sequence[torch.Tensor], v_nl: float, a: torch.Tensor, dt: float,
             n_steps: int, precision: str, work: Workspace, a_per_domain: bool = False, profile: bool = False,
             stream=None):
    """Eq. 2 steps with the reference-orbital nonlocal operator of Eq. 5 (see
    dcmesh_step_eq2); psi0: per-domain reference orbitals like psi."""
    arr = _doms(domains, precision)
    for p0, d in zip(psi0, domains):
        if p0.dtype != d.psi.dtype or tuple(p0.shape) != tuple(d.psi.shape) or not p0.is_contiguous():
            raise ValueError("psi0 must match psi in dtype, shape and be contiguous")
    pp = (ctypes.c_void_p * len(psi0))(*[p.data_ptr() for p in psi0])
    check(lib.dcmesh_step_eq2(arr, len(domains), PRECISION[precision], pp, float(v_nl), a.data_ptr(),
                              int(a_per_domain), a.shape[-2], float(dt), int(n_steps), work.ptr, work.nbytes,
                              _lib.FLAG_PROFILE if profile else 0, _stream(stream)))


def density(domains: Sequence[Domain], a: torch.Tensor, precision: str, work: Workspace,
            outs: List[dict], a_per_domain: bool = False, profile: bool = False, stream=None):
    """Observables of the current orbitals.  ``outs``: per-domain dict with any
    of 'rho', 'j', 'energy' (float64 [1]), 'hpsi_occ', 'overlap' (float64
    [N_o, N_o, 2])."""
    arr = _doms(domains, precision)
    o = (DcmeshDensityOut * len(domains))(*[
        DcmeshDensityOut(_ptr(x.get("rho")), _ptr(x.get("j")), _ptr(x.get("energy")), _ptr(x.get("hpsi_occ")),
                         _ptr(x.get("overlap"))) for x in outs])
    check(lib.dcmesh_density(arr, len(domains), PRECISION[precision], a.data_ptr(), int(a_per_domain), o,
                             work.ptr, work.nbytes,
                             _lib.FLAG_PROFILE if profile else 0, _stream(stream)))


def occupations(domains: Sequence[Domain], psi0: Sequence[torch.Tensor], precision: str, work: Workspace,
                overlap: Optional[Sequence[Optional[torch.Tensor]]] = None, stream=None):
    """Occupations f_s of the reference orbitals psi0 and the excited-electron
    count n_exc of every domain.  Returns (list of float64 [N_o] tensors,
    float64 [n_dom] tensor).  ``overlap``: optional per-domain float64
    [N_o, N_o, 2] outputs for S = h^3 Psi0^H Psi."""
    arr = _doms(domains, precision)
    cd = _CPLX[precision]
    for p0, d in zip(psi0, domains):
        if p0.dtype != cd or tuple(p0.shape) != tuple(d.psi.shape) or not p0.is_contiguous():
            raise ValueError("psi0 must match psi in dtype, shape and be contiguous")
    if len(psi0) != len(domains):
        raise ValueError("one psi0 per domain")
    dev = domains[0].psi.device
    f = [torch.empty(d.psi.shape[1], dtype=torch.float64, device=dev) for d in domains]
    n_exc = torch.empty(len(domains), dtype=torch.float64, device=dev)
    pp = (ctypes.c_void_p * len(domains))(*[x.data_ptr() for x in psi0])
    fp = (ctypes.c_void_p * len(domains))(*[x.data_ptr() for x in f])
    op = None
    if overlap is not None:
        for o, d in zip(overlap, domains):
            n = d.psi.shape[1]
            if o is not None and (o.dtype != torch.float64 or tuple(o.shape) != (n, n, 2) or not o.is_contiguous()):
                raise ValueError("overlap outputs are contiguous float64 [N_o, N_o, 2]")
        op = (ctypes.c_void_p * len(domains))(*[_ptr(o) for o in overlap])
    check(lib.dcmesh_occupations(arr, len(domains), PRECISION[precision], pp, op, fp, n_exc.data_ptr(),
                                 work.ptr, work.nbytes, 0, _stream(stream)))
    return f, n_exc


def _proj_r(proj_r, domains, precision):
    if proj_r is None:
        return None
    if len(proj_r) != len(domains):
        raise ValueError("one proj_r per domain")
    cd = _CPLX[precision]
    for b, d in zip(proj_r, domains):
        if b is None:
            continue
        if b.dtype != cd or tuple(b.shape) != (3,) + tuple(d.proj.shape) or not b.is_contiguous():
            raise ValueError("proj_r entries are contiguous [3, N_g, N_p] in the orbitals' complex dtype")
    return (ctypes.c_void_p * len(domains))(*[_ptr(b) for b in proj_r])


def current(domains: Sequence[Domain], a: torch.Tensor, precision: str, work: Workspace, proj_r=None,
            a_per_domain: bool = False, stream=None) -> torch.Tensor:
    """Macroscopic particle current density [n_dom, 3] (float64) of the current
    orbitals in the field ``a`` ([3] or [n_dom, 3], float64 device)."""
    arr = _doms(domains, precision)
    out = torch.empty(len(domains), 3, dtype=torch.float64, device=domains[0].psi.device)
    check(lib.dcmesh_current(arr, len(domains), PRECISION[precision], a.data_ptr(), int(a_per_domain),
                             _proj_r(proj_r, domains, precision), out.data_ptr(), work.ptr, work.nbytes, 0,
                             _stream(stream)))
    return out


def step_maxwell(domains: Sequence[Domain], a_ext: torch.Tensor, dt: float, n_steps: int, precision: str,
                 work: Workspace, field: torch.Tensor, proj_r=None, want_current: bool = False,
                 a_per_domain: bool = False, stream=None):
    """n_steps steps coupled to the Maxwell update of the field.  a_ext:
    float64 [n_steps + 1, 3] (or [n_dom, n_steps + 1, 3]) at the step times;
    field: float64 [n_dom, 6] (induced field, its rate), updated in place.
    Returns (step fields [n_dom, n_steps, 3], currents [n_dom, n_steps, 3] or None)."""
    arr = _doms(domains, precision)
    dev = domains[0].psi.device
    if field.dtype != torch.float64 or tuple(field.shape) != (len(domains), 6) or not field.is_contiguous():
        raise ValueError("field is contiguous float64 [n_dom, 6]")
    if a_ext.shape[-2] != n_steps + 1:
        raise ValueError("a_ext holds n_steps + 1 samples")
    a_mid = torch.empty(len(domains), max(n_steps, 1), 3, dtype=torch.float64, device=dev)
    cur = torch.empty_like(a_mid) if want_current else None
    check(lib.dcmesh_step_maxwell(arr, len(domains), PRECISION[precision], _proj_r(proj_r, domains, precision),
                                  a_ext.data_ptr(), int(a_per_domain), float(dt), int(n_steps), field.data_ptr(),
                                  a_mid.data_ptr(), _ptr(cur), work.ptr, work.nbytes, 0, _stream(stream)))
    return a_mid[:, :n_steps], (cur[:, :n_steps] if cur is not None else None)


def adjoint_step(domains: Sequence[Domain], lambdas: Sequence[torch.Tensor], a: torch.Tensor, dt: float,
                 grad: torch.Tensor, precision: str, work: Workspace, a_per_domain: bool = False, stream=None):
    """lambda <- U^H lambda in place; grad (float64 device, [3] or [n_dom, 3]) += dL/dA."""
    arr = _doms(domains, precision)
    cd = _CPLX[precision]
    for lam, d in zip(lambdas, domains):
        if lam.dtype != cd or tuple(lam.shape) != tuple(d.psi.shape) or not lam.is_contiguous():
            raise ValueError("lambda must match psi in dtype, shape and be contiguous")
    lp = (ctypes.c_void_p * len(lambdas))(*[l.data_ptr() for l in lambdas])
    check(lib.dcmesh_adjoint_step(arr, len(domains), PRECISION[precision], lp, a.data_ptr(), int(a_per_domain),
                                  float(dt), grad.data_ptr(), work.ptr, work.nbytes, 0, _stream(stream)))


class Graph:
    """n_steps of ``step`` captured once and replayed with ``launch``."""

    def __init__(self, domains, a, dt, n_steps, precision, work, obs=None, a_per_domain=False, stream=None):
        arr = _doms(domains, precision)
        o = None
        if obs is not None:
            o = (DcmeshObs * len(domains))(*[DcmeshObs(_ptr(x.get("rho")), _ptr(x.get("j")), _ptr(x.get("energy")))
                                             for x in obs])
        self._keep = (domains, a, work, obs)
        self.handle = ctypes.c_void_p(None)
        s = stream or torch.cuda.Stream()
        self.stream = s
        check(lib.dcmesh_graph_create(arr, len(domains), PRECISION[precision], a.data_ptr(), int(a_per_domain),
                                      a.shape[-2], float(dt), int(n_steps), o, work.ptr, work.nbytes, 0,
                                      ctypes.c_void_p(s.cuda_stream), ctypes.byref(self.handle)))

    def launch(self, stream=None):
        check(lib.dcmesh_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            check(lib.dcmesh_graph_destroy(self.handle))
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_collect() -> dict:
    """{family: (total kernel ms, launches)} for calls made with profile=True
    since the last collect (waits for their events)."""
    n = len(_lib.FAMILIES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    check(lib.dcmesh_profile_collect(ms, cnt, n))
    return {f: (ms[i], cnt[i]) for i, f in enumerate(_lib.FAMILIES)}


def set_tuning(kernel: str, variant: int):
    check(lib.dcmesh_set_tuning(_lib.KERNEL[kernel], int(variant)))


def set_tuning_shape(kernel: str, precision: str, shape: tuple, fd_order: int, n_orb: int, n_proj: int,
                     variant: int):
    """Variant of a kernel family for domains of exactly this shape ((nx, ny,
    nz), fd_order, n_orb, n_proj) in this precision; -1 removes the entry."""
    nx, ny, nz = shape
    d = DcmeshDomain(nx, ny, nz, fd_order, n_orb, n_proj, 0.0, None, None, None, None, None)
    check(lib.dcmesh_set_tuning_shape(_lib.KERNEL[kernel], PRECISION[precision], ctypes.byref(d), int(variant)))


def clear_tuning_shapes():
    check(lib.dcmesh_clear_tuning_shapes())


def tuning_options(kernel: str) -> int:
    n = ctypes.c_int32(0)
    check(lib.dcmesh_tuning_options(_lib.KERNEL[kernel], ctypes.byref(n)))
    return n.value
