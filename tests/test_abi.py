"""CPU checks of the C interface: the library loads, exports every symbol of
include/*.h, sizes workspaces, and rejects invalid input before touching the
device."""
import os
import re
from dataclasses import replace

import pytest

from paper_2110_12932_amd import tl
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for h in ("tl.h", "tl_ops.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(tl_[a-z_0-9]+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_exports_every_declared_symbol():
    lib = tl.load()
    declared = _declared_symbols()
    assert declared == set(tl.SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name


def test_workspace_bytes():
    wl = W.single_track_2mm()
    n = tl.tl_workspace_bytes(wl.mesh, wl.options)
    # 23 coarse + 10 fine FP64 arrays + 12 fine CG arrays, padded layouts
    pitch = lambda n: (n + 2 + 31) // 32 * 32   # n nodes + 2 ghosts, rounded to 32
    cpad = pitch(51) * (25 + 3) * (13 + 3)
    fpad = pitch(81) * (41 + 2) * (25 + 2)
    assert n >= (23 * cpad + 22 * fpad) * 8
    assert n < (23 * cpad + 22 * fpad) * 8 + 10 ** 6
    # mixed: the 12 fine CG arrays in FP32, and with the composite correction
    # 12 FP32 coarse CG arrays of its own
    mixed = tl.tl_workspace_bytes(wl.mesh, replace(wl.options, precision=W.MIXED))
    assert mixed >= (23 * cpad + 10 * fpad) * 8 + 12 * (fpad + cpad) * 4
    assert mixed < n
    assert tl.tl_workspace_bytes(replace(wl.mesh, refine=0), wl.options) == 0


class _FakeWorkspace:
    def __init__(self, n):
        self.n = n

    def data_ptr(self):
        return 256          # never dereferenced: validation fails first

    def numel(self):
        return self.n

    def element_size(self):
        return 1


@pytest.mark.parametrize("mutate, what", [
    (lambda wl: replace(wl, mesh=replace(wl.mesh, win_nx=wl.mesh.nx + 1)), "window"),
    (lambda wl: replace(wl, mesh=replace(wl.mesh, refine=0)), "refine"),
    (lambda wl: replace(wl, material=replace(wl.material, T_sol=1700.0)), "T_sol"),
    (lambda wl: replace(wl, material=replace(wl.material, rho=float("nan"))), "non-finite"),
    (lambda wl: replace(wl, material=replace(wl.material, pc_kind=1)), "pc_kind"),
    (lambda wl: replace(wl, material=replace(wl.material, h_conv=-1.0)), "surface"),
    (lambda wl: replace(wl, material=replace(wl.material, emissivity=1.5)), "surface"),
    (lambda wl: replace(wl, material=replace(wl.material, T_amb=0.0)), "surface"),
    (lambda wl: replace(wl, scan=W.ScanPath([])), "track"),
    (lambda wl: replace(wl, options=replace(wl.options, m_time=0)), "m_time"),
    (lambda wl: replace(wl, options=replace(wl.options, face_quad=7)), "face_quad"),
    (lambda wl: replace(wl, options=replace(wl.options, dt_coarse=-1.0)), "dt_coarse"),
    (lambda wl: replace(wl, options=replace(wl.options, coupling=5)), "coupling"),
    # sizes whose padded node counts would overflow a 32-bit int
    (lambda wl: replace(wl, mesh=replace(wl.mesh, nx=2**31 - 1, ny=2**31 - 1)), "too large"),
    (lambda wl: replace(wl, mesh=replace(wl.mesh, refine=2**30)), "too large"),
    (lambda wl: replace(wl, options=replace(wl.options, source=2)), "source"),
    # the volume model needs a depth and tracks along x or y
    (lambda wl: replace(wl, options=replace(wl.options, source=W.VOLUME)), "volume"),
    (lambda wl: replace(W.small_cases()["corner"],
                        scan=W.ScanPath([replace(t, depth=40e-6)
                                         for t in W.small_cases()["corner"].scan.tracks]),
                        options=replace(wl.options, source=W.VOLUME)), "volume"),
])
def test_create_rejects_invalid_input(mutate, what):
    wl = mutate(W.single_track_1mm())
    with pytest.raises(tl.TLError) as e:
        tl.tl_create(wl.mesh, wl.material, wl.scan, wl.options, _FakeWorkspace(1 << 30),
                     stream=0)
    assert e.value.status == tl.TL_EINVAL
    assert tl.tl_last_error() != ""


def test_create_rejects_small_workspace():
    wl = W.single_track_1mm()
    with pytest.raises(tl.TLError) as e:
        tl.tl_create(wl.mesh, wl.material, wl.scan, wl.options, _FakeWorkspace(1000), stream=0)
    assert e.value.status == tl.TL_ENOMEM


class _FakePool(_FakeWorkspace):
    def __init__(self, n, ptr=256):
        super().__init__(n)
        self.ptr = ptr

    def data_ptr(self):
        return self.ptr     # never dereferenced: validation fails first


@pytest.mark.parametrize("pool, slots, status", [
    (_FakePool(1 << 30, ptr=0), 8, tl.TL_EINVAL),      # null pool
    (_FakePool(1 << 30, ptr=264), 8, tl.TL_EINVAL),    # not 256-byte aligned
    (_FakePool(1 << 30), 0, tl.TL_EINVAL),             # no slots
    (_FakePool(1 << 30), 1025, tl.TL_EINVAL),          # too many slots
    (_FakePool(4096), 64, tl.TL_ENOMEM),               # smaller than its tables
])
def test_server_create_rejects_invalid_input(pool, slots, status):
    with pytest.raises(tl.TLError) as e:
        tl.tl_server_create(pool, 1 << 30, slots, stream=0)
    assert e.value.status == status
    assert tl.tl_last_error() != ""


def test_op_grid_too_large_is_rejected():
    for dims in ((2**31 - 1, 1, 1), (100000, 100000, 10)):
        grid = tl.to_grid(*dims, 1e-6, 1e-6, 1e-6)
        assert tl.tl_op_padded_size(grid) == 0


def test_create_static_rejects_before_the_device():
    """tl_create_static validates and sizes the problem before any HIP call:
    a problem larger than the static workspace is TL_ENOMEM with a message
    naming both sizes, an invalid mesh TL_EINVAL."""
    wl = W.raster_5mm(W.FP64)
    assert tl.tl_workspace_bytes(wl.mesh, wl.options) > tl.TL_STATIC_WORKSPACE_BYTES
    with pytest.raises(tl.TLError) as e:
        tl.tl_create_static(wl.mesh, wl.material, wl.scan, wl.options, stream=0)
    assert e.value.status == tl.TL_ENOMEM
    assert str(tl.TL_STATIC_WORKSPACE_BYTES) in str(e.value)
    bad = replace(wl.mesh, refine=0)
    with pytest.raises(tl.TLError) as e:
        tl.tl_create_static(bad, wl.material, wl.scan, wl.options, stream=0)
    assert e.value.status == tl.TL_EINVAL
    # the size limit in the header is the one the binding states
    src = open(os.path.join(ROOT, "include", "tl.h")).read()
    m = re.search(r"#define TL_STATIC_WORKSPACE_BYTES \((\d+)u \* (\d+)u \* (\d+)u\)", src)
    assert m and int(m.group(1)) * int(m.group(2)) * int(m.group(3)) == tl.TL_STATIC_WORKSPACE_BYTES


def test_sync_probe_rejects_before_the_device():
    """tl_op_sync_probe checks its arguments before any HIP call."""
    import ctypes as C
    lib = tl.load()
    us = C.c_double()
    assert lib.tl_op_sync_probe(256, 1, 0, None, 10, None, C.byref(us), None) == tl.TL_EINVAL
    fake = C.c_void_p(256)   # never dereferenced: the counts fail first
    assert lib.tl_op_sync_probe(256, 0, 0, fake, 10, fake, C.byref(us), None) == tl.TL_EINVAL
    assert lib.tl_op_sync_probe(0, 1, 0, fake, 10, fake, C.byref(us), None) == tl.TL_EINVAL
    assert lib.tl_op_sync_probe(256, 1, 0, fake, 0, fake, C.byref(us), None) == tl.TL_EINVAL


def test_op_apply_rejects_before_the_device():
    """tl_op_apply checks the kernel choice and the workgroup count before
    any HIP call."""
    import ctypes as C
    lib = tl.load()
    grid = tl.to_grid(8, 8, 8, 1e-5, 1e-5, 1e-5)
    fake = C.c_void_p(256)   # never dereferenced: the arguments fail first
    call = lambda prec, kern, blocks, rep=1: lib.tl_op_apply(
        C.byref(grid), prec, kern, blocks, fake, fake, fake, fake, rep, None)
    assert call(tl.TL_FP64, 3, 0) == tl.TL_EINVAL
    assert call(tl.TL_FP64, -1, 0) == tl.TL_EINVAL
    for blocks in (-8, 4, 12, 2**20 + 8):
        assert call(tl.TL_FP64, tl.OP_TILED, blocks) == tl.TL_EINVAL
    assert call(7, tl.OP_TILED, 0) == tl.TL_EINVAL
    assert call(tl.TL_MIXED, tl.OP_ZMARCH, 8, rep=0) == tl.TL_EINVAL
    assert lib.tl_op_apply(C.byref(grid), tl.TL_FP64, 0, 0, None, fake, fake, fake, 1,
                           None) == tl.TL_EINVAL
