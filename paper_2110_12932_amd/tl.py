"""Thin ctypes binding of the two-level thermal library (include/tl.h,
include/tl_ops.h).

Only argument marshalling lives here: every step of the solver runs in the
library's HIP kernels.  PyTorch provides device memory (a uint8 tensor as
the workspace) and the HIP stream.  Importing works without a GPU; any call
that needs the device fails loudly if libtl.so has not been built.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtl.so")

TL_OK, TL_EINVAL, TL_ENOMEM, TL_EDEVICE, TL_ENOCONV, TL_ESTATE, TL_EBUSY = 0, -1, -2, -3, -4, -5, -6
TL_STATIC_WORKSPACE_BYTES = 32 * 1024 * 1024   # as in include/tl.h
TL_FP64, TL_MIXED = 0, 1
STATUS_NAMES = {0: "TL_OK", -1: "TL_EINVAL", -2: "TL_ENOMEM", -3: "TL_EDEVICE",
                -4: "TL_ENOCONV", -5: "TL_ESTATE", -6: "TL_EBUSY"}


class TLError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class tl_mesh(C.Structure):
    _fields_ = [("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("refine", C.c_int),
                ("win_nx", C.c_int), ("win_ny", C.c_int), ("win_nz", C.c_int)]


class tl_material(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("rho", "T_lo", "T_hi", "c_lo", "c_hi", "k_lo", "k_hi",
                                          "latent", "T_sol", "T_liq", "sharpness")] + \
               [("pc_kind", C.c_int), ("T_init", C.c_double), ("T_bottom", C.c_double),
                ("h_conv", C.c_double), ("emissivity", C.c_double), ("T_amb", C.c_double),
                ("k_fict", C.c_double), ("rhoc_fict", C.c_double)]


class tl_track(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("x0", "y0", "x1", "y1", "speed", "power", "radius",
                                          "absorptivity", "depth")]


class tl_scan_path(C.Structure):
    _fields_ = [("n_tracks", C.c_int), ("tracks", C.POINTER(tl_track)), ("t_start", C.c_double)]


class tl_options(C.Structure):
    _fields_ = [("dt_coarse", C.c_double), ("m_time", C.c_int), ("precision", C.c_int),
                ("face_quad", C.c_int), ("newton_tol", C.c_double), ("cg_rtol", C.c_double),
                ("dn_tol", C.c_double), ("dn_theta", C.c_double), ("newton_max", C.c_int),
                ("cg_max", C.c_int), ("dn_max", C.c_int), ("coupling", C.c_int),
                ("source", C.c_int)]


class tl_ledger(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("stored", "stored0", "absorbed", "bottom", "remap",
                                          "surface")]


class tl_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("macro_steps", "micro_steps", "newton_fine",
                                         "newton_coarse", "cg_fine", "cg_coarse",
                                         "line_search_halvings", "dn_iters", "window_moves",
                                         "fine_solves", "coarse_solves")] + \
               [("fine_dof_steps", C.c_double), ("step_ms", C.c_double),
                ("fine_op_bytes", C.c_double), ("fine_op_applies", C.c_int64),
                ("fine_op_timed", C.c_int64), ("fine_op_timed_ms", C.c_double),
                ("fine_nodes", C.c_int * 3), ("coarse_nodes", C.c_int * 3),
                ("newton_corr", C.c_int64), ("cg_corr", C.c_int64),
                ("phase_ms", C.c_double * 4)]


class tl_request_info(C.Structure):
    _fields_ = [("submit_s", C.c_double), ("admit_s", C.c_double), ("done_s", C.c_double),
                ("state", C.c_int), ("pad", C.c_int), ("macro_steps", C.c_int64)]


class tl_grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double)]


# every symbol declared in include/tl.h and include/tl_ops.h
SYMBOLS = ["tl_workspace_bytes", "tl_create", "tl_create_static", "tl_step", "tl_get_temperature", "tl_get_ledger",
           "tl_get_stats", "tl_get_time", "tl_save", "tl_load", "tl_set_profiling", "tl_destroy",
           "tl_last_error",
           "tl_server_overhead_bytes", "tl_server_create", "tl_server_submit",
           "tl_server_tick", "tl_server_result", "tl_server_release", "tl_server_destroy",
           "tl_server_set_profiling", "tl_server_get_profile",
           "tl_op_padded_size", "tl_op_pack", "tl_op_unpack", "tl_op_apply",
           "tl_op_sync_probe"]

_lib = None


def load():
    """Load libtl.so (built by paper_2110_12932_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with "
                          "`python -m paper_2110_12932_amd.build` (there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    lib.tl_workspace_bytes.restype = sz
    lib.tl_workspace_bytes.argtypes = [C.POINTER(tl_mesh), C.POINTER(tl_options)]
    lib.tl_create.restype = C.c_int
    lib.tl_create.argtypes = [C.POINTER(tl_mesh), C.POINTER(tl_material), C.POINTER(tl_scan_path),
                              C.POINTER(tl_options), vp, sz, vp, C.POINTER(vp)]
    lib.tl_create_static.restype = C.c_int
    lib.tl_create_static.argtypes = [C.POINTER(tl_mesh), C.POINTER(tl_material),
                                     C.POINTER(tl_scan_path), C.POINTER(tl_options), vp,
                                     C.POINTER(vp)]
    lib.tl_step.restype = C.c_int
    lib.tl_step.argtypes = [vp, C.c_int]
    lib.tl_get_temperature.restype = C.c_int
    lib.tl_get_temperature.argtypes = [vp, C.c_int, C.POINTER(C.c_double), sz,
                                       C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.tl_get_ledger.restype = C.c_int
    lib.tl_get_ledger.argtypes = [vp, C.POINTER(tl_ledger)]
    lib.tl_get_stats.restype = C.c_int
    lib.tl_get_stats.argtypes = [vp, C.POINTER(tl_stats)]
    lib.tl_get_time.restype = C.c_int
    lib.tl_get_time.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.tl_save.restype = C.c_int
    lib.tl_save.argtypes = [vp, vp, sz, C.POINTER(sz)]
    lib.tl_load.restype = C.c_int
    lib.tl_load.argtypes = [vp, vp, sz]
    lib.tl_set_profiling.restype = C.c_int
    lib.tl_set_profiling.argtypes = [vp, C.c_int]
    lib.tl_destroy.restype = None
    lib.tl_destroy.argtypes = [vp]
    lib.tl_last_error.restype = C.c_char_p
    lib.tl_last_error.argtypes = []
    lib.tl_server_overhead_bytes.restype = sz
    lib.tl_server_overhead_bytes.argtypes = [C.c_int]
    lib.tl_server_create.restype = C.c_int
    lib.tl_server_create.argtypes = [vp, sz, sz, C.c_int, vp, C.POINTER(vp)]
    lib.tl_server_submit.restype = C.c_int
    lib.tl_server_submit.argtypes = [vp, C.POINTER(tl_mesh), C.POINTER(tl_material),
                                     C.POINTER(tl_scan_path), C.POINTER(tl_options), C.c_int,
                                     C.POINTER(C.c_uint64)]
    lib.tl_server_tick.restype = C.c_int
    lib.tl_server_tick.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                   C.POINTER(C.c_int)]
    lib.tl_server_result.restype = C.c_int
    lib.tl_server_result.argtypes = [vp, C.c_uint64, C.c_int, C.POINTER(C.c_double), sz,
                                     C.POINTER(C.c_int), C.POINTER(tl_stats),
                                     C.POINTER(tl_ledger), C.POINTER(tl_request_info)]
    lib.tl_server_release.restype = C.c_int
    lib.tl_server_release.argtypes = [vp, C.c_uint64]
    lib.tl_server_set_profiling.restype = C.c_int
    lib.tl_server_set_profiling.argtypes = [vp, C.c_int]
    lib.tl_server_get_profile.restype = C.c_int
    lib.tl_server_get_profile.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    lib.tl_server_destroy.restype = None
    lib.tl_server_destroy.argtypes = [vp]
    lib.tl_op_padded_size.restype = sz
    lib.tl_op_padded_size.argtypes = [C.POINTER(tl_grid)]
    for f in (lib.tl_op_pack, lib.tl_op_unpack):
        f.restype = C.c_int
        f.argtypes = [C.POINTER(tl_grid), C.c_int, C.c_int, vp, vp, vp]
    lib.tl_op_apply.restype = C.c_int
    lib.tl_op_apply.argtypes = [C.POINTER(tl_grid), C.c_int, C.c_int, C.c_int, vp, vp, vp, vp,
                                C.c_int, vp]
    lib.tl_op_sync_probe.restype = C.c_int
    lib.tl_op_sync_probe.argtypes = [C.c_int, C.c_int, C.c_int, vp, sz, vp,
                                     C.POINTER(C.c_double), vp]
    _lib = lib
    return lib


def _check(st):
    if st != TL_OK:
        raise TLError(st, load().tl_last_error().decode())


# ---- marshalling of the plain records in `workloads` -----------------------
def to_mesh(m):
    return tl_mesh(m.lx, m.ly, m.lz, m.nx, m.ny, m.nz, m.refine, m.win_nx, m.win_ny, m.win_nz)


def to_material(m):
    return tl_material(m.rho, m.T_lo, m.T_hi, m.c_lo, m.c_hi, m.k_lo, m.k_hi, m.latent,
                       m.T_sol, m.T_liq, m.sharpness, m.pc_kind, m.T_init, m.T_bottom,
                       m.h_conv, m.emissivity, m.T_amb, m.k_fict, m.rhoc_fict)


def to_scan(s):
    arr = (tl_track * max(1, len(s.tracks)))(*[
        tl_track(t.x0, t.y0, t.x1, t.y1, t.speed, t.power, t.radius, t.absorptivity,
                 t.depth)
        for t in s.tracks])
    sp = tl_scan_path(len(s.tracks), arr, s.t_start)
    sp._keep = arr
    return sp


def to_options(o):
    return tl_options(o.dt_coarse, o.m_time, o.precision, o.face_quad, o.newton_tol, o.cg_rtol,
                      o.dn_tol, o.dn_theta, o.newton_max, o.cg_max, o.dn_max,
                      o.coupling, o.source)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


# ---- tl.h -------------------------------------------------------------------
def tl_workspace_bytes(mesh, opts):
    return int(load().tl_workspace_bytes(C.byref(to_mesh(mesh)), C.byref(to_options(opts))))


def tl_create(mesh, material, scan, opts, workspace, stream=None):
    """workspace: a torch uint8 CUDA tensor of at least tl_workspace_bytes."""
    lib = load()
    h = C.c_void_p()
    sp = to_scan(scan)
    _check(lib.tl_create(C.byref(to_mesh(mesh)), C.byref(to_material(material)), C.byref(sp),
                         C.byref(to_options(opts)), C.c_void_p(workspace.data_ptr()),
                         workspace.numel() * workspace.element_size(),
                         C.c_void_p(_stream_ptr(stream)), C.byref(h)))
    return h


def tl_create_static(mesh, material, scan, opts, stream=None):
    """tl_create on the library's static device workspace (no allocation)."""
    lib = load()
    h = C.c_void_p()
    sp = to_scan(scan)
    _check(lib.tl_create_static(C.byref(to_mesh(mesh)), C.byref(to_material(material)),
                                C.byref(sp), C.byref(to_options(opts)),
                                C.c_void_p(_stream_ptr(stream)), C.byref(h)))
    return h


def tl_step(h, n_macro):
    _check(load().tl_step(h, int(n_macro)))


def tl_get_temperature(h, level):
    """Returns (T as float64 array of shape (nz, ny, nx), fine origin)."""
    lib = load()
    st = tl_get_stats(h)
    dims = st["fine_nodes"] if level == 1 else st["coarse_nodes"]
    buf = np.empty(dims[0] * dims[1] * dims[2], dtype=np.float64)
    d = (C.c_int * 3)()
    o = (C.c_int * 3)()
    _check(lib.tl_get_temperature(h, level, buf.ctypes.data_as(C.POINTER(C.c_double)),
                                  buf.size, d, o))
    return buf.reshape(d[2], d[1], d[0]), tuple(o)


def tl_get_ledger(h):
    led = tl_ledger()
    _check(load().tl_get_ledger(h, C.byref(led)))
    return {n: getattr(led, n) for n, _ in tl_ledger._fields_}


def tl_get_stats(h):
    st = tl_stats()
    _check(load().tl_get_stats(h, C.byref(st)))
    out = {}
    for n, _ in tl_stats._fields_:
        v = getattr(st, n)
        out[n] = tuple(v) if n.endswith("_nodes") or n == "phase_ms" else v
    return out


def tl_get_time(h):
    t = C.c_double()
    n = C.c_int64()
    _check(load().tl_get_time(h, C.byref(t), C.byref(n)))
    return t.value, n.value


def tl_save(h):
    lib = load()
    used = C.c_size_t()
    _check(lib.tl_save(h, None, 0, C.byref(used)))
    buf = C.create_string_buffer(used.value)
    _check(lib.tl_save(h, buf, used.value, C.byref(used)))
    return buf.raw[:used.value]


def tl_load(h, data):
    buf = C.create_string_buffer(bytes(data), len(data))
    _check(load().tl_load(h, buf, len(data)))


def tl_set_profiling(h, sample_every):
    _check(load().tl_set_profiling(h, int(sample_every)))


def tl_destroy(h):
    if h:
        load().tl_destroy(h)


def tl_last_error():
    return load().tl_last_error().decode()


# ---- tl_ops.h ----------------------------------------------------------------
def to_grid(nx, ny, nz, hx, hy, hz):
    return tl_grid(nx, ny, nz, hx, hy, hz)


def tl_op_padded_size(grid):
    return int(load().tl_op_padded_size(C.byref(grid)))


def tl_op_pack(grid, kind, plain, padded, stream=None):
    _check(load().tl_op_pack(C.byref(grid), kind, plain.element_size(),
                             C.c_void_p(plain.data_ptr()), C.c_void_p(padded.data_ptr()),
                             C.c_void_p(_stream_ptr(stream))))


def tl_op_unpack(grid, kind, padded, plain, stream=None):
    _check(load().tl_op_unpack(C.byref(grid), kind, plain.element_size(),
                               C.c_void_p(padded.data_ptr()), C.c_void_p(plain.data_ptr()),
                               C.c_void_p(_stream_ptr(stream))))


OP_AUTO, OP_TILED, OP_ZMARCH = 0, 1, 2


def tl_op_apply(grid, precision, d, kappa, v, y, repeat=1, stream=None, kernel=OP_AUTO,
                blocks=0):
    _check(load().tl_op_apply(C.byref(grid), precision, int(kernel), int(blocks),
                              C.c_void_p(d.data_ptr()),
                              C.c_void_p(kappa.data_ptr()), C.c_void_p(v.data_ptr()),
                              C.c_void_p(y.data_ptr()), int(repeat),
                              C.c_void_p(_stream_ptr(stream))))


# ---- convenience wrapper -------------------------------------------------------
class Sim:
    """One simulation on cuda:0 with a torch-allocated workspace, or with
    static=True on the library's static device workspace (tl_create_static)."""

    def __init__(self, workload, device="cuda", stream=None, static=False):
        self.wl = workload
        self.stream = stream
        self.workspace = None
        self.h = None
        if static:
            self.h = tl_create_static(workload.mesh, workload.material, workload.scan,
                                      workload.options, stream)
            return
        import torch
        nbytes = tl_workspace_bytes(workload.mesh, workload.options)
        if nbytes == 0:
            raise TLError(TL_EINVAL, "invalid mesh")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.h = tl_create(workload.mesh, workload.material, workload.scan, workload.options,
                           self.workspace, stream)

    def step(self, n=1):
        tl_step(self.h, n)

    def temperature(self, level):
        return tl_get_temperature(self.h, level)

    def ledger(self):
        return tl_get_ledger(self.h)

    def stats(self):
        return tl_get_stats(self.h)

    def close(self):
        if self.h:
            tl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving (tl.h, tl_server_*) ------------------------------------------------
def tl_server_overhead_bytes(max_slots):
    return int(load().tl_server_overhead_bytes(int(max_slots)))


def tl_server_create(pool, hbm_budget, max_slots, stream=None):
    """pool: a torch uint8 CUDA tensor holding the server's device memory."""
    h = C.c_void_p()
    _check(load().tl_server_create(C.c_void_p(pool.data_ptr()), pool.numel(), int(hbm_budget),
                                   int(max_slots), C.c_void_p(_stream_ptr(stream)), C.byref(h)))
    return h


def tl_server_submit(sv, mesh, material, scan, opts, n_macro):
    rid = C.c_uint64()
    sp = to_scan(scan)
    _check(load().tl_server_submit(sv, C.byref(to_mesh(mesh)), C.byref(to_material(material)),
                                   C.byref(sp), C.byref(to_options(opts)), int(n_macro),
                                   C.byref(rid)))
    return rid.value


def tl_server_tick(sv):
    a, q, f = C.c_int(), C.c_int(), C.c_int()
    _check(load().tl_server_tick(sv, C.byref(a), C.byref(q), C.byref(f)))
    return a.value, q.value, f.value


def _info_dict(info):
    return {n: getattr(info, n) for n, _ in tl_request_info._fields_ if n != "pad"}


def tl_server_info(sv, rid):
    """Timing/state record of a request (any state)."""
    info = tl_request_info()
    st = load().tl_server_result(sv, rid, 0, None, 0, None, None, None, C.byref(info))
    if st not in (TL_OK, TL_EBUSY, TL_ENOCONV):
        _check(st)
    return _info_dict(info)


def tl_server_result(sv, rid):
    """(coarse T, fine T, stats, ledger, info) of a finished request."""
    lib = load()
    out = []
    stats, led, info = tl_stats(), tl_ledger(), tl_request_info()
    for level in (0, 1):
        n = 1
        _check(lib.tl_server_result(sv, rid, level, None, 0, None, C.byref(stats), C.byref(led),
                                    C.byref(info)))
        dims = stats.fine_nodes if level == 1 else stats.coarse_nodes
        n = dims[0] * dims[1] * dims[2]
        buf = np.empty(n, dtype=np.float64)
        d = (C.c_int * 3)()
        _check(lib.tl_server_result(sv, rid, level, buf.ctypes.data_as(C.POINTER(C.c_double)),
                                    n, d, None, None, None))
        out.append(buf.reshape(d[2], d[1], d[0]))
    st = {n: (tuple(getattr(stats, n)) if n.endswith("_nodes") else getattr(stats, n))
          for n, _ in tl_stats._fields_}
    lg = {n: getattr(led, n) for n, _ in tl_ledger._fields_}
    return out[0], out[1], st, lg, _info_dict(info)


def tl_server_release(sv, rid):
    _check(load().tl_server_release(sv, rid))


def tl_server_set_profiling(sv, sample_every):
    _check(load().tl_server_set_profiling(sv, int(sample_every)))


def tl_server_get_profile(sv):
    n = C.c_int64()
    ms = C.c_double()
    _check(load().tl_server_get_profile(sv, C.byref(n), C.byref(ms)))
    return n.value, ms.value


def tl_server_destroy(sv):
    if sv:
        load().tl_server_destroy(sv)


class Server:
    """Serving loop on cuda:0 with a torch-allocated device pool."""

    def __init__(self, pool_bytes, hbm_budget=None, max_slots=64, device="cuda", stream=None):
        import torch
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
        budget = int(pool_bytes) if hbm_budget is None else int(hbm_budget)
        self.h = tl_server_create(self.pool, budget, max_slots, stream)

    def submit(self, workload, n_macro=None):
        return tl_server_submit(self.h, workload.mesh, workload.material, workload.scan,
                                workload.options,
                                workload.n_macro if n_macro is None else n_macro)

    def tick(self):
        return tl_server_tick(self.h)

    def result(self, rid):
        return tl_server_result(self.h, rid)

    def info(self, rid):
        return tl_server_info(self.h, rid)

    def close(self):
        if self.h:
            tl_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tl_op_sync_probe(blocks, rounds, barrier, data, ctl, stream=None):
    """data: torch float64 CUDA tensor; ctl: torch uint8 CUDA tensor of
    >= 1024 bytes.  Returns the elapsed microseconds."""
    us = C.c_double()
    _check(load().tl_op_sync_probe(int(blocks), int(rounds), int(barrier),
                                   C.c_void_p(data.data_ptr()), data.numel(),
                                   C.c_void_p(ctl.data_ptr()), C.byref(us),
                                   C.c_void_p(_stream_ptr(stream))))
    return us.value
