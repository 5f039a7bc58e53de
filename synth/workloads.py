"""Seeded input generator for the per-domain Kohn-Sham propagation workloads.

The paper's production inputs (PbTiO3 pseudopotentials and atomic positions of a
skyrmion superlattice, Sec. VI.A) are not available, so every input here is a
synthetic stand-in with the shapes and value ranges of the five benchmark
workloads:

* orbitals: each a sum of 8 periodic Gaussians with random centres, widths and
  phases, then orthonormalised (Cholesky-QR) under <a|b> = h^3 sum conj(a) b;
* local potential: one attractive Gaussian well per atom;
* nonlocal projectors: per atom an s, p_x, p_y, p_z set of Gaussian-based
  functions (4 per atom), or that set at two radii (8 per atom), each column
  normalised to h^3 sum |beta|^2 = 1 and multiplied by a random unit phase;
* D: one real coupling constant per projector, U[-1, 1] Ha;
* occupations f_n = 2;
* A(t): the laser vector potential A0 sin(w t) sin^2(pi t / T) along z, sampled
  at the step midpoints t_k + dt/2 (the midpoint rule of Eq. 2).

Array layout (shared by every consumer): a grid point g = (z*ny + y)*nx + x sits
at r = h*(x, y, z); orbitals are stored [N_g][N_o] with the orbital index
fastest (the structure-of-arrays layout of Sec. V.B.2); projectors [N_g][N_p].

Draw order inside one domain (fixed, so a seed fixes every array): atom
positions, D, projector phases, well depths, well widths, orbital centres,
orbital widths, orbital phases.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Numbers shared by the five workloads.
H_SPACING = 0.4           # bohr
OCCUPATION = 2.0
GAUSS_PER_ORBITAL = 8
ORBITAL_WIDTH = (1.0, 2.0)
WELL_DEPTH = (0.5, 2.0)   # Ha
WELL_WIDTH = (0.8, 1.5)   # bohr
PROJ_RADII = (1.2, 0.8)   # bohr; 4 projectors/atom use the first, 8 use both
PULSE_A0 = 0.05
PULSE_OMEGA = 0.1


@dataclass
class Domain:
    """One periodic domain: grid, orbitals and the operators' data (FP64)."""

    shape: Tuple[int, int, int]          # (nx, ny, nz)
    h: float
    fd_order: int
    psi: np.ndarray                      # [N_g, N_o] complex128
    v_loc: np.ndarray                    # [N_g] float64
    proj: np.ndarray                     # [N_g, N_p] complex128
    d: np.ndarray                        # [N_p] float64
    occ: np.ndarray                      # [N_o] float64
    atoms: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))

    @property
    def n_grid(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    @property
    def n_orb(self) -> int:
        return self.psi.shape[1]

    @property
    def n_proj(self) -> int:
        return self.proj.shape[1]

    def astype(self, real_dtype) -> "Domain":
        """Copy with arrays rounded to ``real_dtype`` (float32 or float64)."""
        cdt = np.complex64 if np.dtype(real_dtype) == np.float32 else np.complex128
        return Domain(self.shape, self.h, self.fd_order,
                      np.ascontiguousarray(self.psi.astype(cdt)),
                      np.ascontiguousarray(self.v_loc.astype(real_dtype)),
                      np.ascontiguousarray(self.proj.astype(cdt)),
                      np.ascontiguousarray(self.d.astype(real_dtype)),
                      np.ascontiguousarray(self.occ.astype(real_dtype)),
                      self.atoms.copy())

    def rounded(self, real_dtype) -> "Domain":
        """Inputs rounded to ``real_dtype`` and widened back to FP64."""
        r = self.astype(real_dtype)
        return r.astype(np.float64)


@dataclass
class Workload:
    """A named workload: domains, time step, step count and A(t) samples."""

    name: str
    domains: List[Domain]
    dt: float
    n_steps: int
    a_mid: np.ndarray                    # [n_steps, 3] float64, A at t_k + dt/2
    precision: str                       # "fp64" | "fp32" | "split_bf16" | "split_fp16"
    notes: str = ""


# --------------------------------------------------------------------------
# periodic Gaussian factors (separable: the 27-image sum factorises per axis)
# --------------------------------------------------------------------------

def _axis_factor(n: int, h: float, c: float, s: float, linear: bool) -> np.ndarray:
    """Sum over the images m in {-1, 0, 1} of exp(-(x - c + mL)^2 / (2 s^2)),
    optionally weighted by the displacement (x - c + mL) (p-type factor)."""
    L = n * h
    x = h * np.arange(n)
    out = np.zeros(n)
    for m in (-1, 0, 1):
        dx = x - c + m * L
        g = np.exp(-dx * dx / (2.0 * s * s))
        out += dx * g if linear else g
    return out


def _outer3(fz: np.ndarray, fy: np.ndarray, fx: np.ndarray) -> np.ndarray:
    """Flattened outer product with x fastest: out[(z*ny + y)*nx + x]."""
    return (fz[:, None, None] * fy[None, :, None] * fx[None, None, :]).reshape(-1)


def _gauss3(shape, h, c, s) -> np.ndarray:
    nx, ny, nz = shape
    return _outer3(_axis_factor(nz, h, c[2], s, False),
                   _axis_factor(ny, h, c[1], s, False),
                   _axis_factor(nx, h, c[0], s, False))


def _orbitals(shape, h, centres, widths, phases) -> np.ndarray:
    """psi_n = sum_i exp(i phi_ni) G(r; c_ni, s_ni), assembled plane by plane:
    psi[z][(y, x), n] = sum_i (fy (x) fx)_ni[(y, x)] * exp(i phi_ni) fz_ni[z]."""
    nx, ny, nz = shape
    n_orb, n_g = centres.shape[0], centres.shape[1]
    fx = np.empty((n_orb, n_g, nx))
    fy = np.empty((n_orb, n_g, ny))
    fz = np.empty((n_orb, n_g, nz))
    for n in range(n_orb):
        for i in range(n_g):
            fx[n, i] = _axis_factor(nx, h, centres[n, i, 0], widths[n, i], False)
            fy[n, i] = _axis_factor(ny, h, centres[n, i, 1], widths[n, i], False)
            fz[n, i] = _axis_factor(nz, h, centres[n, i, 2], widths[n, i], False)
    yx = (fy[:, :, :, None] * fx[:, :, None, :]).reshape(n_orb, n_g, ny * nx)      # [N_o, 8, yx]
    wz = np.exp(1j * phases)[:, :, None] * fz                                       # [N_o, 8, nz]
    out = np.empty((nz, ny * nx, n_orb), dtype=np.complex128)
    for z in range(nz):
        out[z] = np.einsum("niy,ni->yn", yx, wz[:, :, z])
    return out.reshape(nz * ny * nx, n_orb)


def _orthonormalise(psi: np.ndarray, h: float) -> np.ndarray:
    """Cholesky-QR: Psi <- Psi R^-1 with R^H R = h^3 Psi^H Psi."""
    s = h ** 3 * (psi.conj().T @ psi)
    r = np.linalg.cholesky(s).conj().T          # upper, R^H R = S
    return psi @ np.linalg.inv(r)


def _projectors(shape, h, atoms, per_atom, phases) -> np.ndarray:
    """Columns s, p_x, p_y, p_z per atom and radius, assembled plane by plane
    from their separable factors, normalised and phased."""
    nx, ny, nz = shape
    radii = PROJ_RADII[:1] if per_atom == 4 else PROJ_RADII
    fxs, fys, fzs = [], [], []
    for c in atoms:
        for rc in radii:
            gx = _axis_factor(nx, h, c[0], rc, False)
            gy = _axis_factor(ny, h, c[1], rc, False)
            gz = _axis_factor(nz, h, c[2], rc, False)
            lx = _axis_factor(nx, h, c[0], rc, True)
            ly = _axis_factor(ny, h, c[1], rc, True)
            lz = _axis_factor(nz, h, c[2], rc, True)
            for fz, fy, fx in ((gz, gy, gx), (gz, gy, lx), (gz, ly, gx), (lz, gy, gx)):  # s, px, py, pz
                fxs.append(fx)
                fys.append(fy)
                fzs.append(fz)
    fx, fy, fz = np.array(fxs), np.array(fys), np.array(fzs)                      # [N_p, n]
    norms = np.sqrt(h ** 3 * np.sum(fx ** 2, 1) * np.sum(fy ** 2, 1) * np.sum(fz ** 2, 1))
    scale = np.exp(1j * np.asarray(phases)) / norms
    yx = np.ascontiguousarray((fy[:, :, None] * fx[:, None, :]).reshape(len(fx), ny * nx).T)   # [yx, N_p]
    out = np.empty((nz, ny * nx, len(fx)), dtype=np.complex128)
    for z in range(nz):
        np.multiply(yx, (fz[:, z] * scale)[None, :], out=out[z])
    return out.reshape(nz * ny * nx, len(fx))


def make_domain(seed, shape: Sequence[int], n_orb: int, n_atoms: int,
                proj_per_atom: int = 8, h: float = H_SPACING, fd_order: int = 6,
                rng: Optional[np.random.Generator] = None) -> Domain:
    """Build one seeded domain (all arrays FP64 / complex128)."""
    if proj_per_atom not in (4, 8):
        raise ValueError("proj_per_atom must be 4 or 8")
    shape = tuple(int(v) for v in shape)
    rng = np.random.default_rng(seed) if rng is None else rng
    L = np.array(shape, dtype=np.float64) * h
    n_proj = n_atoms * proj_per_atom
    atoms = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * L
    d = rng.uniform(-1.0, 1.0, size=n_proj)
    proj_phase = rng.uniform(0.0, 2 * np.pi, size=n_proj)
    depth = rng.uniform(*WELL_DEPTH, size=n_atoms)
    width = rng.uniform(*WELL_WIDTH, size=n_atoms)
    centres = rng.uniform(0.0, 1.0, size=(n_orb, GAUSS_PER_ORBITAL, 3)) * L
    widths = rng.uniform(*ORBITAL_WIDTH, size=(n_orb, GAUSS_PER_ORBITAL))
    phases = rng.uniform(0.0, 2 * np.pi, size=(n_orb, GAUSS_PER_ORBITAL))

    v = np.zeros(int(np.prod(shape)))
    for a in range(n_atoms):
        v -= depth[a] * _gauss3(shape, h, atoms[a], width[a])
    psi = _orthonormalise(_orbitals(shape, h, centres, widths, phases), h) if n_orb else \
        np.zeros((int(np.prod(shape)), 0), np.complex128)
    proj = _projectors(shape, h, atoms, proj_per_atom, proj_phase) if n_atoms else \
        np.zeros((int(np.prod(shape)), 0), np.complex128)
    occ = np.full(n_orb, OCCUPATION)
    return Domain(shape, h, fd_order, np.ascontiguousarray(psi), v, np.ascontiguousarray(proj),
                  d, occ, atoms)


def projector_moments(dom: Domain) -> np.ndarray:
    """Position-weighted projectors B_d[g, p] = (r_g - R_a)_d B[g, p], d = x, y, z,
    where r_g - R_a is the minimum-image displacement of grid point g from the
    atom a that projector column p belongs to (columns are atom-major, the same
    number per atom).  [3, N_g, N_p] complex128."""
    n_proj, n_atoms = dom.proj.shape[1], len(dom.atoms)
    out = np.zeros((3, dom.n_grid, n_proj), dtype=np.complex128)
    if n_proj == 0:
        return out
    per = n_proj // n_atoms
    nx, ny, nz = dom.shape
    L = np.array(dom.shape, dtype=np.float64) * dom.h
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = dom.h * np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    for a in range(n_atoms):
        disp = r - dom.atoms[a]
        disp -= L * np.round(disp / L)
        cols = slice(a * per, (a + 1) * per)
        for d in range(3):
            out[d][:, cols] = disp[:, d:d + 1] * dom.proj[:, cols]
    return out


def pulse_midpoints(n_steps: int, dt: float, period_steps: int,
                    a0: float = PULSE_A0, omega: float = PULSE_OMEGA) -> np.ndarray:
    """A(t_k + dt/2) for A_z(t) = a0 sin(omega t) sin^2(pi t / T), T = period_steps*dt."""
    t = (np.arange(n_steps) + 0.5) * dt
    T = period_steps * dt
    a = np.zeros((n_steps, 3))
    a[:, 2] = a0 * np.sin(omega * t) * np.sin(np.pi * t / T) ** 2
    return a


# --------------------------------------------------------------------------
# the batched divide-and-conquer workload
# --------------------------------------------------------------------------

def batched_domain_shapes(n_domains: int = 512, seed: int = 4):
    """(edge, n_orb, n_atoms) per domain: edge ~ U{20..40}, n_orb ~ U{16..96},
    n_atoms = floor(n_orb / 4); each domain draws from its own spawned stream."""
    seqs = np.random.SeedSequence(seed).spawn(n_domains)
    out = []
    for s in seqs:
        rng = np.random.default_rng(s)
        n = int(rng.integers(20, 41))
        n_orb = int(rng.integers(16, 97))
        out.append((n, n_orb, n_orb // 4))
    return out


def batched_domain(index: int, n_domains: int = 512, seed: int = 4) -> Domain:
    """Domain ``index`` of the batched workload (same stream as its shape draw)."""
    seqs = np.random.SeedSequence(seed).spawn(n_domains)
    rng = np.random.default_rng(seqs[index])
    n = int(rng.integers(20, 41))
    n_orb = int(rng.integers(16, 97))
    return make_domain(None, (n, n, n), n_orb, n_orb // 4, proj_per_atom=8,
                       fd_order=6, rng=rng)


def batched_subset(count: int = 16, seed: int = 404, n_domains: int = 512):
    """Indices of the seeded subset of the batched workload used for parity
    checks and the CPU baseline: the smallest and the largest domain (by
    N_g N_o N_p), then seeded picks until ``count``."""
    shapes = batched_domain_shapes(n_domains)
    size = np.array([n ** 3 * no * (8 * na) for n, no, na in shapes])
    pick = [int(size.argmin()), int(size.argmax())]
    rng = np.random.default_rng(seed)
    for i in rng.permutation(len(shapes)):
        if len(pick) == count:
            break
        if int(i) not in pick:
            pick.append(int(i))
    return pick


# --------------------------------------------------------------------------
# the five named workloads
# --------------------------------------------------------------------------

def config(i: int, domains: Optional[Sequence[int]] = None) -> Workload:
    """Workload ``i`` (1..5).  ``domains`` selects a subset for workload 4."""
    if i == 1:
        dom = make_domain(1, (24, 24, 24), 16, 8, proj_per_atom=4, fd_order=4)
        return Workload("single domain 24^3, 16 orbitals, 32 projectors, FD4, FP64", [dom],
                        0.02, 10, np.zeros((10, 3)), "fp64")
    if i in (2, 3):
        dom = make_domain(2, (64, 64, 64), 128, 64, proj_per_atom=8, fd_order=6)
        prec = "fp32" if i == 2 else "split_bf16"
        return Workload("single domain 64^3, 128 orbitals, 512 projectors, FD6, laser A_z(t)",
                        [dom], 0.02, 200, pulse_midpoints(200, 0.02, 200), prec)
    if i == 4:
        idx = range(512) if domains is None else domains
        doms = [batched_domain(k) for k in idx]
        return Workload("512 uneven domains, edge U{20..40}, orbitals U{16..96}, FD6",
                        doms, 0.02, 100, pulse_midpoints(100, 0.02, 100), "fp32")
    if i == 5:
        dom = make_domain(5, (48, 48, 48), 64, 32, proj_per_atom=8, fd_order=6)
        return Workload("48^3, 64 orbitals, 256 projectors, 400 free A_z samples",
                        [dom], 0.02, 400, pulse_midpoints(400, 0.02, 400), "fp32")
    raise ValueError(f"unknown workload {i}")


def fd_check_indices(n_steps: int = 400, count: int = 16, seed: int = 5) -> np.ndarray:
    """The sample indices of A used for the finite-difference gradient check."""
    return np.sort(np.random.default_rng(seed).choice(n_steps, count, replace=False))
