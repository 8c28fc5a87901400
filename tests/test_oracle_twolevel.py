"""Pins of the two-level method (Sections 3-4, Algorithm 1):
  * energy ledger identity per macro step (a discrete conservation law);
  * refinement 1 with equal macro and micro steps reproduces the
    single-level solve (the paper states this identity, Section 5.1);
  * a window covering the whole plate reproduces the single-level fine run;
  * trilinear prolongation is exact on trilinear fields, injection inverts it;
  * the window rule on hand-computed positions;
  * the multirate error grows with the number of micro steps per macro step
    (Section 5.1: error falls as the global step approaches the local one);
  * the two-level fixed point does not depend on the relaxation;
  * at refinement 2, against the brute-force single-level run on the whole
    plate refined twice: the difference grows with the macro step at fixed
    micro step and shows Section 5.1's sawtooth within each macro step."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from oracle import grid as G
from oracle import twolevel as TW
from workloads import single_track_1mm, small_cases, ScanPath, Track

UM = 1e-6


def _ledger_errors(sim):
    out = []
    for h in sim.history:
        lhs = h["E_end"] - h["E_start"]
        rhs = h["absorbed"] - h["bottom"] - h["surface"]
        out.append(abs(lhs - rhs) / h["absorbed"])
    return out


@pytest.mark.parametrize("name", ["c0", "corner", "fulldepth", "r3m2"])
def test_energy_ledger_identity(name):
    wl = small_cases()[name]
    sim = oracle.run(wl, min(wl.n_macro, 8))
    assert max(_ledger_errors(sim)) < 1e-9
    led = sim.ledger
    total = led["stored"] - led["stored0"]
    assert total == pytest.approx(led["absorbed"] - led["bottom"] - led["surface"] + led["remap"],
                                  rel=1e-9)


def test_full_single_track_1mm_runs_and_moves():
    sim = oracle.run(single_track_1mm())
    assert sim.stats["moves"] >= 5
    assert max(_ledger_errors(sim)) < 1e-9
    assert np.isfinite(sim.Tf).all() and sim.Tf.max() > 1623.0   # the track melts


def test_refinement1_single_macro_step_is_single_level():
    """r = 1, m = 1: two-level equals the single-level coarse solve to the
    iteration tolerances, including across window moves."""
    wl = small_cases()["r1m1"]
    n = 10
    sim = TW.TwoLevel(wl)
    c = sim.coarse
    ref = TW.single_level_run(c, wl.material, wl.scan, wl.options.dt_coarse, n, tol=1e-11)
    for s in range(n):
        sim.step()
        assert np.abs(sim.Tc - ref[s]).max() < 1e-7
    assert sim.stats["moves"] >= 2
    # the fine field on the window equals the coarse field there
    w = sim.win
    assert np.abs(sim.Tf[w.inject_f] - ref[-1][w.inject_c]).max() < 1e-7


def test_whole_plate_window_is_single_level_fine():
    wl = single_track_1mm()
    mesh = replace(wl.mesh, nx=6, ny=4, nz=3, lx=6 * 62.5 * UM, ly=4 * 62.5 * UM,
                   lz=3 * 62.5 * UM, win_nx=6, win_ny=4, win_nz=3)
    tr = Track(0.05e-3, 0.1e-3, 0.3e-3, 0.15e-3, 0.8, 150.0, 50 * UM, 0.4)
    wl = replace(wl, mesh=mesh, scan=ScanPath([tr]), n_macro=4)
    sim = TW.TwoLevel(wl)
    assert not sim.win.gamma_f.any()
    fine = sim.win.fine
    m = wl.options.m_time
    ref = TW.single_level_run(fine, wl.material, wl.scan, wl.options.dt_coarse / m,
                              4 * m, tol=1e-11)
    sim.run(4)
    assert np.abs(sim.Tf - ref[-1]).max() < 1e-7


def test_prolongation_exact_on_trilinear_and_injection():
    wl = small_cases()["r3m2"]
    sim = TW.TwoLevel(wl)
    c, w = sim.coarse, sim.win
    x, y, z = c.node_xyz()
    f = lambda x, y, z: 3.0 + 2.0 * x / 1e-3 - 1.5 * y / 1e-3 + 0.7 * z / 1e-3 + 4.0 * x * y * z / 1e-9
    fx, fy, fz = w.fine.node_xyz()
    assert np.allclose(w.P @ f(x, y, z), f(fx, fy, fz), rtol=0, atol=1e-12)
    assert np.allclose(w.P @ np.ones(c.n_nodes), 1.0, atol=1e-14)
    u = np.random.default_rng(3).normal(size=c.n_nodes)
    assert np.allclose((w.P @ u)[w.inject_f], u[w.inject_c], atol=1e-14)


def test_window_rule_hand_values():
    wl = single_track_1mm()
    c = TW.coarse_grid(wl.mesh)
    # t = 50 us: beam at x = 0.14 mm, y = 0.25 mm, moving +x; window 6x4 cells
    # of 62.5 um: x_lo = 0.14 - 0.25 < 0 -> clamp 0; y_lo = 0.125 mm -> J0 = 2
    assert TW.window_origin(wl.mesh, c, wl.scan, 50 * UM) == (0, 2)
    # t = 600 us: x = 0.58 mm, x_lo = 0.33 mm = 5.28 cells -> round 5
    assert TW.window_origin(wl.mesh, c, wl.scan, 600 * UM) == (5, 2)
    # t = 1 ms: x = 0.9 mm, x_lo = 0.65 mm = 10.4 cells -> 10 = nx - wx
    assert TW.window_origin(wl.mesh, c, wl.scan, 1000 * UM) == (10, 2)
    # beam off after the end keeps the current window
    assert TW.window_origin(wl.mesh, c, wl.scan, 2e-3, current=(7, 1)) == (7, 1)
    # moving -x: the beam sits one third of the length from the low edge
    back = ScanPath([Track(0.9e-3, 0.3e-3, 0.1e-3, 0.3e-3, 0.8, 180.0, 50 * UM, 0.4)])
    # t = 500 us: x = 0.5 mm, x_lo = 0.5 - 0.125 = 0.375 mm = 6 cells;
    # y_lo = 0.3 - 0.125 = 0.175 mm = 2.8 cells -> 3
    assert TW.window_origin(wl.mesh, c, back, 500 * UM) == (6, 3)


def test_multirate_error_grows_with_micro_steps():
    """Same micro step dt, refinement 1: m = 1 is the single-level solve,
    and the deviation grows with m (the paper's temporal study, Section 5.1,
    finds the error falling as the global step approaches the local one)."""
    base = small_cases()["r1m1"]
    dt = 25 * UM
    errs = {}
    n_fine = 8
    ref = TW.single_level_run(TW.coarse_grid(base.mesh), base.material, base.scan, dt, n_fine,
                              tol=1e-11)
    for m in (1, 2, 4):
        wl = replace(base, options=replace(base.options, m_time=m, dt_coarse=dt * m))
        sim = oracle.run(wl, n_fine // m)
        errs[m] = np.abs(sim.Tc - ref[-1]).max()
    assert errs[1] < 1e-7
    assert errs[1] < errs[2] < errs[4]
    assert errs[4] > 1e-3


def test_fixed_point_independent_of_relaxation():
    wl = small_cases()["c0"]
    a = oracle.run(wl, 3)
    b = oracle.run(replace(wl, options=replace(wl.options, dn_theta=0.75)), 3)
    assert np.abs(a.Tc - b.Tc).max() < 1e-7
    assert np.abs(a.Tf - b.Tf).max() < 1e-7


def test_two_level_against_full_fine_single_level():
    """Refinement 2 against brute force: the single-level run on the whole
    plate refined twice, with the micro step dt.  Section 5.1's temporal
    study fixes the expected shape: at fixed dt the two-level field moves
    towards the reference as the macro step Dt = m dt shrinks to dt, and
    within each macro step the difference grows over the micro steps (their
    Dirichlet data blend the coarse field with an uncorrected predictor) and
    falls back at the corrected step.  The window (10 x 6 x 2 coarse cells)
    holds the beam for all 16 micro steps, so it never moves."""
    base = single_track_1mm()
    r, dt, n_fine = 2, 12.5 * UM, 16
    mesh = replace(base.mesh, win_nx=10, win_ny=6, win_nz=2, refine=r)
    c = TW.coarse_grid(mesh)
    full = G.Grid(r * mesh.nx, r * mesh.ny, r * mesh.nz, c.hx / r, c.hy / r, c.hz / r)
    ref = TW.single_level_run(full, base.material, base.scan, dt, n_fine, tol=1e-10)
    err, multirate = {}, {}
    for m in (1, 2, 4):
        wl = replace(base, mesh=mesh, options=replace(base.options, m_time=m, dt_coarse=dt * m))
        sim = TW.TwoLevel(wl, newton_tol=1e-10, dn_tol=1e-10)
        sim.record = []
        sim.run(n_fine // m)
        assert sim.stats["moves"] == 0
        fi, fj, fk = sim.win.fine.node_ijk()
        oi, oj, ok = sim.fine_origin()
        on_full = full.node(fi + oi, fj + oj, fk + ok)
        assert [(n, j) for n, j, _ in sim.record] == [(q // m, q % m + 1) for q in range(n_fine)]
        fields = [T for _, _, T in sim.record]
        err[m] = [np.abs(T - ref[q][on_full]).max() for q, T in enumerate(fields)]
        multirate[m] = fields
    # the two-level field differs from the full-fine one (the plate outside
    # the window is coarse) ...
    assert err[1][-1] > 1.0
    # ... and at every common macro step the difference grows with m
    for q in range(3, n_fine, 4):
        assert err[1][q] < err[2][q] < err[4][q], (q, err[1][q], err[2][q], err[4][q])
    # sawtooth at m = 4: rising over micro steps 1..3, falling at the
    # correction, against the full-fine field and against the m = 1 run
    # (the same spatial discretisation: the multirate part alone)
    for n in range(n_fine // 4):
        e = err[4][4 * n:4 * n + 4]
        d = [np.abs(multirate[4][4 * n + j] - multirate[1][4 * n + j]).max() for j in range(4)]
        assert e[0] < e[1] < e[2] and e[3] < e[2], (n, e)
        assert d[0] < d[1] < d[2] and d[3] < d[2] / 5, (n, d)
