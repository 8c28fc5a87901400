"""Pins of the consistent global formulation of Section 3 (the global problem
on the whole plate, with constant coefficients of its own inside the window,
loaded there by the local solution):

  * equal levels (refinement 1, one micro step): the global field equals the
    single-level solution everywhere, inside the window too, and the local
    field equals it on the window, whatever the global coefficients inside
    -- the stronger consistency condition of Section 3, which the alternate
    formulation does not meet;
  * a linear material with global coefficients equal to the material's: the
    local equation turns the load from the local solution into the local
    laser load restricted to the coarse nodes, so the global field is the
    coarse single-level run with that load and does not depend on the local
    field at all (refinement 3, two micro steps);
  * the energy ledger, with the energy the global coefficients hold inside
    the window beyond the local field's, holds step by step through window
    moves."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from oracle import laser as L
from oracle import twolevel as TW
from oracle.level import implicit_step
from workloads import small_cases, single_track_1mm, CONSISTENT, ALTERNATE


def _consistent(wl, **mat):
    return replace(wl, options=replace(wl.options, coupling=CONSISTENT),
                   material=replace(wl.material, **mat))


@pytest.mark.parametrize("k_fict, rhoc_fict", [(0.0, 0.0), (50.0, 2.0e6)])
def test_equal_levels_reproduce_single_level_everywhere(k_fict, rhoc_fict):
    wl = _consistent(small_cases()["r1m1"], k_fict=k_fict, rhoc_fict=rhoc_fict)
    n = 6
    sim = TW.TwoLevel(wl, newton_tol=1e-11, dn_tol=1e-11)
    ref = TW.single_level_run(sim.coarse, wl.material, wl.scan, wl.options.dt_coarse, n,
                              tol=1e-11)
    for s in range(n):
        sim.step()
        assert np.abs(sim.Tc - ref[s]).max() < 1e-8, s
        w = sim.win
        assert np.abs(sim.Tf[w.inject_f] - sim.Tc[w.inject_c]).max() < 1e-8
    assert sim.stats["moves"] >= 1
    assert sim.Tc.max() > 1700.0          # the melt band was crossed


def test_alternate_misses_the_stronger_consistency():
    wl = replace(small_cases()["r1m1"], options=replace(small_cases()["r1m1"].options,
                                                        coupling=ALTERNATE))
    sim = TW.TwoLevel(wl, newton_tol=1e-11)
    ref = TW.single_level_run(sim.coarse, wl.material, wl.scan, wl.options.dt_coarse, 4,
                              tol=1e-11)
    sim.run(4)
    assert np.abs(sim.Tc - ref[-1]).max() > 1.0


def test_linear_material_with_matching_coefficients_decouples():
    base = small_cases()["r3m2"]
    lin = dict(k_lo=20.0, k_hi=20.0, c_lo=500.0, c_hi=500.0, latent=0.0)
    wl = _consistent(base, k_fict=20.0, rhoc_fict=base.material.rho * 500.0, **lin)
    sim = TW.TwoLevel(wl, newton_tol=1e-11, dn_tol=1e-11)
    c, mat, opts = sim.coarse, wl.material, wl.options
    m, Dt = opts.m_time, opts.dt_coarse
    bottom = sim.bottom_c
    T = sim.Tc.copy()
    for n in range(6):
        sim.step()
        w = sim.win
        spots = [L.laser_at(wl.scan, TW.micro_time(wl.scan, opts, n, j)) for j in range(1, m + 1)]
        Fout = sum(L.top_load(c, s, opts.face_quad, w.outside_face) for s in spots) / m
        Ffine = sum(L.top_load(w.fine, s, opts.face_quad) for s in spots) / m
        T, _, _ = implicit_step(c, mat, T, Dt, Fout + w.P.T @ Ffine, None, bottom,
                                np.full(c.n_nodes, mat.T_bottom), tol=1e-11)
        assert np.abs(sim.Tc - T).max() < 1e-8, n
    assert sim.stats["moves"] >= 1


@pytest.mark.parametrize("name", ["c0", "r3m2", "corner", "fulldepth"])
def test_energy_ledger(name):
    wl = _consistent(small_cases()[name], k_fict=50.0, rhoc_fict=2.0e6, h_conv=1e4)
    sim = oracle.run(wl, 5)
    for h in sim.history:
        lhs = h["E_end"] - h["E_start"]
        rhs = h["absorbed"] - h["bottom"] - h["surface"]
        assert abs(lhs - rhs) < 1e-10 * h["absorbed"]
    led = sim.ledger
    total = led["absorbed"] - led["bottom"] - led["surface"] + led["remap"]
    assert abs(led["stored"] - led["stored0"] - total) < 1e-10 * led["absorbed"]
    assert sim.stats["moves"] >= 1


def test_default_coefficients_are_the_law_at_the_initial_temperature():
    wl = _consistent(single_track_1mm())
    sim = TW.TwoLevel(wl)
    assert sim.k_fict == pytest.approx(10.0)
    assert sim.rhoc_fict == pytest.approx(8000.0 * 450.0)
