"""The C-ABI library loads, exports every entry point declared in
include/dcmesh.h, and rejects invalid arguments on the host (no GPU needed:
validation happens before any HIP call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2509_00966_amd import _lib
    return _lib


def test_exports_every_declared_symbol():
    L = _lib()
    header = open(os.path.join(ROOT, "include", "dcmesh.h")).read()
    declared = set(re.findall(r"\b(?:int|const char\*)\s+(dcmesh_\w+)\s*\(", header))
    assert declared == set(L.EXPORTS)
    for name in declared:
        assert hasattr(L.lib, name)


def _dom(L, **kw):
    fake = 0x10000
    d = dict(nx=10, ny=10, nz=10, fd_order=6, n_orb=4, n_proj=2, h=0.4, psi=fake, v_loc=fake,
             proj=fake, d=fake, occ=fake)
    d.update(kw)
    return (L.DcmeshDomain * 1)(L.DcmeshDomain(**d))


@pytest.mark.parametrize("kw,code", [
    (dict(fd_order=5), 1),
    (dict(nx=6), 1),                 # < fd_order + 1
    (dict(n_orb=0), 1),
    (dict(n_proj=-1), 1),
    (dict(h=0.0), 1),
    (dict(h=float("nan")), 1),
    (dict(psi=None), 1),
    (dict(proj=None), 1),
    (dict(proj=None, d=None, n_proj=0), 0),
])
def test_workspace_bytes_validation(kw, code):
    L = _lib()
    out = ctypes.c_size_t(0)
    rc = L.lib.dcmesh_workspace_bytes(_dom(L, **kw), 1, 1, 0, ctypes.byref(out))
    assert rc == code, L.lib.dcmesh_last_error()
    if code == 0:
        assert out.value > 10 * 10 * 10 * 4 * 8 * 2     # at least two psi-sized buffers


def test_bad_precision_and_counts():
    L = _lib()
    out = ctypes.c_size_t(0)
    assert L.lib.dcmesh_workspace_bytes(_dom(L), 1, 7, 0, ctypes.byref(out)) == 1
    assert L.lib.dcmesh_workspace_bytes(_dom(L), 0, 1, 0, ctypes.byref(out)) == 1
    assert L.lib.dcmesh_workspace_bytes(None, 1, 1, 0, ctypes.byref(out)) == 1
    assert L.lib.dcmesh_workspace_bytes(_dom(L), 1, 1, 0, None) == 1
    assert b"NULL" in L.lib.dcmesh_last_error()


def test_step_rejects_missing_or_small_workspace_before_touching_the_gpu():
    L = _lib()
    d = _dom(L)
    fake = ctypes.c_void_p(0x10000)
    rc = L.lib.dcmesh_step(d, 1, 1, fake, 0, 1, 0.02, 1, None, None, 0, 0, None)
    assert rc == L.DCMESH_ERR_WORKSPACE
    rc = L.lib.dcmesh_step(d, 1, 1, fake, 0, 1, 0.02, 1, None, ctypes.c_void_p(0x10000 + 8), 1 << 40, 0, None)
    assert rc == L.DCMESH_ERR_WORKSPACE                    # misaligned
    rc = L.lib.dcmesh_step(d, 1, 1, fake, 0, 1, 0.02, 1, None, ctypes.c_void_p(0x10000), 16, 0, None)
    assert rc == L.DCMESH_ERR_WORKSPACE                    # too small
    assert b"too small" in L.lib.dcmesh_last_error()
    rc = L.lib.dcmesh_step(d, 1, 1, None, 0, 1, 0.02, 1, None, ctypes.c_void_p(0x10000), 1 << 40, 0, None)
    assert rc == L.DCMESH_ERR_INVALID_ARGUMENT             # no A samples
    rc = L.lib.dcmesh_step(d, 1, 1, fake, 0, 0, 0.02, 1, None, ctypes.c_void_p(0x10000), 1 << 40, 0, None)
    assert rc == L.DCMESH_ERR_INVALID_ARGUMENT             # a_stride < n_steps
    rc = L.lib.dcmesh_step(d, 1, 1, fake, 0, 1, float("inf"), 1, None, ctypes.c_void_p(0x10000), 1 << 40, 0, None)
    assert rc == L.DCMESH_ERR_INVALID_ARGUMENT


def test_adjoint_and_density_argument_checks():
    L = _lib()
    d = _dom(L)
    fake = ctypes.c_void_p(0x10000)
    assert L.lib.dcmesh_adjoint_step(d, 1, 1, None, fake, 0, 0.02, fake, fake, 1 << 40, 0, None) == 1
    lam = (ctypes.c_void_p * 1)(None)
    assert L.lib.dcmesh_adjoint_step(d, 1, 1, lam, fake, 0, 0.02, fake, fake, 1 << 40, 0, None) == 1
    assert L.lib.dcmesh_density(d, 1, 1, fake, 0, None, fake, 1 << 40, 0, None) == 1
    g = ctypes.c_void_p(None)
    assert L.lib.dcmesh_graph_create(d, 1, 1, fake, 0, 1, 0.02, 1, None, fake, 1 << 40, 1, None,
                                     ctypes.byref(g)) == 1       # CHECK_FINITE cannot be captured
    assert L.lib.dcmesh_graph_launch(None, None) == 1
    assert L.lib.dcmesh_graph_destroy(None) == 1


def test_tuning_options():
    L = _lib()
    n = ctypes.c_int32(0)
    for k in (0, 1, 2, 3, 4):
        assert L.lib.dcmesh_tuning_options(k, ctypes.byref(n)) == 0 and n.value >= 2
        assert L.lib.dcmesh_set_tuning(k, n.value) == 1
        assert L.lib.dcmesh_set_tuning(k, -1) == 0
    assert L.lib.dcmesh_tuning_options(4, ctypes.byref(n)) == 0 and n.value == 3
    assert L.lib.dcmesh_tuning_options(9, ctypes.byref(n)) == 1
    # the z segment and the stencil order are process-wide only
    shape = _dom(L)
    for k in (3, 4):
        assert L.lib.dcmesh_set_tuning_shape(k, 1, shape, 0) == 1


def test_workspace_grows_with_problem():
    L = _lib()
    out1, out2 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.lib.dcmesh_workspace_bytes(_dom(L), 1, 1, 0, ctypes.byref(out1)) == 0
    assert L.lib.dcmesh_workspace_bytes(_dom(L, n_orb=8), 1, 1, 0, ctypes.byref(out2)) == 0
    assert out2.value > out1.value
    assert L.lib.dcmesh_workspace_bytes(_dom(L), 1, 0, 0, ctypes.byref(out2)) == 0   # FP64 is bigger
    assert out2.value > out1.value


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_workspace_size_does_not_depend_on_tuning(precision):
    """Every tile variant and z-segment choice fits the one workspace size
    (regression: the stencil's energy partials once followed the variant)."""
    L = _lib()
    shapes = [(20, 31, 40, 16, 32), (37, 22, 29, 70, 136), (64, 64, 64, 128, 512), (9, 10, 11, 5, 0)]
    doms = (L.DcmeshDomain * len(shapes))(*[
        L.DcmeshDomain(nx=a, ny=b, nz=c, fd_order=6, n_orb=o, n_proj=p, h=0.4, psi=0x10000,
                       v_loc=0x10000, proj=0x10000 if p else None, d=0x10000 if p else None,
                       occ=0x10000) for a, b, c, o, p in shapes])

    def size():
        out = ctypes.c_size_t(0)
        assert L.lib.dcmesh_workspace_bytes(doms, len(shapes), precision, 0, ctypes.byref(out)) == 0
        return out.value

    n = ctypes.c_int32(0)
    try:
        base = size()
        for k in range(5):
            assert L.lib.dcmesh_tuning_options(k, ctypes.byref(n)) == 0
            for v in range(n.value):
                assert L.lib.dcmesh_set_tuning(k, v) == 0
                assert size() == base, (k, v)
            assert L.lib.dcmesh_set_tuning(k, -1) == 0
        # every family at its smallest tiles at once
        for k, v in ((0, 3), (1, 1), (2, 2), (3, 1)):
            assert L.lib.dcmesh_set_tuning(k, v) == 0
        assert size() == base
    finally:
        for k in range(4):
            L.lib.dcmesh_set_tuning(k, -1)


def test_tuning_shape_table_validation():
    L = _lib()
    d = _dom(L)
    assert L.lib.dcmesh_set_tuning_shape(1, 1, None, 0) == 1
    assert L.lib.dcmesh_set_tuning_shape(1, 9, d, 0) == 1          # precision
    assert L.lib.dcmesh_set_tuning_shape(3, 1, d, 1) == 1          # the z segment is global only
    assert L.lib.dcmesh_set_tuning_shape(1, 1, d, 99) == 1         # variant out of range
    assert L.lib.dcmesh_set_tuning_shape(7, 1, d, 0) == 1          # unknown family
    assert L.lib.dcmesh_set_tuning_shape(1, 1, d, 2) == 0
    assert L.lib.dcmesh_set_tuning_shape(1, 1, d, -1) == 0         # removes the entry
    assert L.lib.dcmesh_clear_tuning_shapes() == 0


def test_noalloc_rejects_before_any_hip_call():
    L = _lib()
    # a 64^3 domain with 128 orbitals needs far more than the 64 MiB scratch
    big = _dom(L, nx=64, ny=64, nz=64, n_orb=128, n_proj=512)
    rc = L.lib.dcmesh_step_noalloc(big, 1, 1, 0x10000, 0, 1, 0.02, 1, None, 0, None)
    assert rc == 3, L.lib.dcmesh_last_error()
    assert b"static scratch" in L.lib.dcmesh_last_error()
    assert L.lib.dcmesh_step_noalloc(_dom(L, n_orb=0), 1, 1, 0x10000, 0, 1, 0.02, 1, None, 0, None) == 1
