"""The five synthetic workloads (all sizes in SI units) and small variants.

Every random draw comes from numpy.random.default_rng with a stated seed and
a fixed draw order, so the oracle and the GPU path see identical inputs.
There is no public dataset behind the paper's experiments; these workloads
stand in for them with the paper's parameter ranges (Section 5.2-5.3:
powers of about 180 W, radii of tens of microns, speeds near 0.8 m/s,
alternating raster tracks).
"""
import math
from dataclasses import replace

import numpy as np

from .spec import (Mesh, Material, Track, ScanPath, Options, Workload,
                   FP64, MIXED, VOLUME, options_for)

UM = 1e-6
MM = 1e-3


def _laser(**kw):
    base = dict(speed=0.8, power=180.0, radius=50 * UM, absorptivity=0.4)
    base.update(kw)
    return base


def single_track_1mm(precision=FP64):
    """Plain FP64 two-level solve, one straight track: 1.0x0.5x0.25 mm,
    16x8x4 coarse cells, window 6x4x2 cells refined 2x, 4 micro steps per
    50 us macro step, 20 macro steps, track x = 0.1 -> 0.9 mm at y = 0.25 mm."""
    mesh = Mesh(1.0 * MM, 0.5 * MM, 0.25 * MM, 16, 8, 4, 2, 6, 4, 2)
    tr = Track(0.1 * MM, 0.25 * MM, 0.9 * MM, 0.25 * MM, **_laser())
    opts = options_for(precision, 50 * UM, 4)
    return Workload("single_track_1mm", mesh, Material(), ScanPath([tr]), opts, 20)


def single_track_2mm(precision=FP64):
    """Single track at paper-like resolution: 2x1x0.5 mm, 50x25x13 coarse
    cells (40 um in x,y), window 10x5x3 cells refined 8x (5 um), macro
    step 25 us with 8 micro steps, 100 macro steps, track x = 0 -> 2 mm at
    mid-width."""
    mesh = Mesh(2.0 * MM, 1.0 * MM, 0.5 * MM, 50, 25, 13, 8, 10, 5, 3)
    tr = Track(0.0, 0.5 * MM, 2.0 * MM, 0.5 * MM, **_laser())
    opts = options_for(precision, 25 * UM, 8)
    return Workload("single_track_2mm", mesh, Material(), ScanPath([tr]), opts, 100)


def raster_5mm(precision=MIXED, seed=0):
    """Raster of 10 alternating 4 mm tracks at 100 um hatch over a 5x5x1 mm
    plate, coarse h = 50 um, window 10x6x3 cells refined 8x (6.25 um),
    macro step 50 us, 8 micro steps, 1000 macro steps.  Track powers are
    drawn U(150, 250) W in track order from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    powers = rng.uniform(150.0, 250.0, size=10)
    tracks = []
    for k in range(10):
        y = 2.5 * MM + (k - 4.5) * 0.1 * MM
        xa, xb = (0.5 * MM, 4.5 * MM) if k % 2 == 0 else (4.5 * MM, 0.5 * MM)
        tracks.append(Track(xa, y, xb, y, **_laser(power=float(powers[k]))))
    mesh = Mesh(5.0 * MM, 5.0 * MM, 1.0 * MM, 100, 100, 20, 8, 10, 6, 3)
    opts = options_for(precision, 50 * UM, 8)
    return Workload("raster_5mm", mesh, Material(), ScanPath(tracks), opts, 1000)


def served_tracks(n=64, seed=0, mean_interarrival=1e-3, precision=MIXED):
    """Served stream: n single-track requests.  Per request, in this draw
    order: exponential inter-arrival [s], L_x ~ U(1,4) mm, coarse h in
    {40, 50} um, P ~ U(100,300) W, v ~ U(0.4,1.5) m/s, R ~ U(40,80) um.
    Width 1 mm, depth 0.5 mm, r = m = 8, window 10x6x3 coarse cells (the
    same 81x49x25 fine shape for every request), macro step half a coarse
    cell of travel, track x = 0 -> L_x at mid-width.  Returns a list of
    (arrival_time, Workload)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for q in range(n):
        t += float(rng.exponential(mean_interarrival))
        lx = float(rng.uniform(1.0, 4.0)) * MM
        h = (40 * UM, 50 * UM)[int(rng.integers(0, 2))]
        p = float(rng.uniform(100.0, 300.0))
        v = float(rng.uniform(0.4, 1.5))
        rad = float(rng.uniform(40.0, 80.0)) * UM
        nx = max(10, int(round(lx / h)))
        ny = int(round(1.0 * MM / h))
        nz = int(math.ceil(0.5 * MM / h - 1e-9))
        mesh = Mesh(lx, 1.0 * MM, 0.5 * MM, nx, ny, nz, 8, 10, 6, 3)
        dt = 0.5 * h / v
        tr = Track(0.0, 0.5 * MM, lx, 0.5 * MM, speed=v, power=p, radius=rad,
                   absorptivity=0.4)
        n_macro = int(math.ceil((lx / v) / dt - 1e-9))
        opts = options_for(precision, dt, 8)
        out.append((t, Workload(f"served_req{q}", mesh, Material(),
                                ScanPath([tr]), opts, n_macro)))
    return out


def raster_10mm(precision=MIXED):
    """Large multi-track build: 10x10x2 mm plate, 200x200x40 coarse cells
    (50 um), 20 alternating raster tracks x = 1 -> 9 mm at 100 um hatch,
    powers/speeds alternating (200 W, 0.8 m/s) and (280 W, 1.2 m/s), window
    12x8x3 cells refined 10x (5 um), macro step 25 us, 8 micro steps."""
    tracks = []
    for k in range(20):
        y = 5.0 * MM + (k - 9.5) * 0.1 * MM
        xa, xb = (1.0 * MM, 9.0 * MM) if k % 2 == 0 else (9.0 * MM, 1.0 * MM)
        p, v = (200.0, 0.8) if k % 2 == 0 else (280.0, 1.2)
        tracks.append(Track(xa, y, xb, y, **_laser(power=p, speed=v)))
    mesh = Mesh(10.0 * MM, 10.0 * MM, 2.0 * MM, 200, 200, 40, 10, 12, 8, 3)
    opts = options_for(precision, 25 * UM, 8)
    total = sum(8.0 * MM / t.speed for t in tracks)
    n_macro = int(math.ceil(total / opts.dt_coarse - 1e-9))
    return Workload("raster_10mm", mesh, Material(), ScanPath(tracks), opts,
                    n_macro)


def single_track_3d(precision=FP64):
    """The paper's three-dimensional single-track example (Section 5.2) with
    its volumetric local and smeared global sources and its parameters:
    P = 179.2 W, eta = 0.38, radius 85 um, depth 50 um, 0.8 m/s along x for
    2 mm on a plate 3 mm long and 1 mm deep (1.5 mm wide here; the width is
    not given); global h = 100 um, local window 1.2 x 0.5 x 0.1 mm at
    h = 20 um (refinement 5), local step 1e-4 s and a four times longer
    global step, 7 macro steps (the track takes 2.5 ms).  The material law is
    the linear law of this library (the paper's IN625 tables are only plotted)."""
    mesh = Mesh(3.0 * MM, 1.5 * MM, 1.0 * MM, 30, 15, 10, 5, 12, 5, 1)
    tr = Track(0.5 * MM, 0.75 * MM, 2.5 * MM, 0.75 * MM, speed=0.8, power=179.2,
               radius=85 * UM, absorptivity=0.38, depth=50 * UM)
    opts = replace(options_for(precision, 400 * UM, 4), source=VOLUME)
    return Workload("single_track_3d", mesh, Material(), ScanPath([tr]), opts, 7)


def by_name(name, **kw):
    return {"single_track_1mm": single_track_1mm, "single_track_2mm": single_track_2mm, "raster_5mm": raster_5mm,
            "raster_10mm": raster_10mm, "single_track_3d": single_track_3d}[name](**kw)


def small_cases():
    """Tiny two-level problems used by parity tests: variations of single_track_1mm
    that exercise clamped windows, window moves, m = 1, r = 1 and a
    window spanning the full depth."""
    base = single_track_1mm()
    cases = {}
    cases["c0"] = base
    w = replace(base, name="r1m1", n_macro=12,
                mesh=replace(base.mesh, refine=1),
                options=replace(base.options, m_time=1))
    cases["r1m1"] = w
    w = replace(base, name="r3m2", n_macro=10,
                mesh=replace(base.mesh, refine=3, win_nx=4, win_ny=3),
                options=replace(base.options, m_time=2))
    cases["r3m2"] = w
    w = replace(base, name="fulldepth", n_macro=8,
                mesh=replace(base.mesh, win_nz=4, win_nx=5, win_ny=3))
    cases["fulldepth"] = w
    tr = Track(0.05 * MM, 0.05 * MM, 0.95 * MM, 0.45 * MM, speed=1.2,
               power=220.0, radius=40 * UM, absorptivity=0.45)
    tr2 = Track(0.95 * MM, 0.45 * MM, 0.3 * MM, 0.05 * MM, speed=1.0,
                power=150.0, radius=60 * UM, absorptivity=0.35)
    w = replace(base, name="corner", n_macro=16,
                scan=ScanPath([tr, tr2], t_start=30 * UM),
                mesh=replace(base.mesh, win_nx=5, win_ny=3))
    cases["corner"] = w
    return cases


def k2_sweep_field(nx, ny, nz, lx, ly, lz, seed=0):
    """Nodal temperature field (K) for operator benchmarks: a hot spot of
    2500 K above ambient under the centre of the top face, widths 60 um in
    plane and 40 um in depth, plus N(0, 1 K) noise from default_rng(seed).
    Returned as a float64 array of shape (nz+1, ny+1, nx+1)."""
    rng = np.random.default_rng(seed)
    x = np.linspace(0.0, lx, nx + 1)[None, None, :]
    y = np.linspace(0.0, ly, ny + 1)[None, :, None]
    z = np.linspace(0.0, lz, nz + 1)[:, None, None]
    rho2 = (x - lx / 2) ** 2 + (y - ly / 2) ** 2
    f = 300.0 + 2500.0 * np.exp(-rho2 / (2 * (60 * UM) ** 2)
                                - (lz - z) ** 2 / (2 * (40 * UM) ** 2))
    return f + rng.normal(0.0, 1.0, size=f.shape)
