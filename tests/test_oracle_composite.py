"""Pins of the composite-grid form of the two-level correction: one Newton
solve on the coarse nodes outside the window interior together with the free
fine nodes, the fine interface values slaved to the coarse ones by P.

Its equations are the ones the Dirichlet-Neumann iteration of Section 3
satisfies at its fixed point, so both must give the same fields (to the
iteration tolerances) -- on windows that move, touch the plate's corner,
reach the plate bottom, and at r = 3, m = 2.  With r = 1 and m = 1 the
composite form also reduces to the single-level coarse solve (the identity
of Section 5.1), and the energy ledger holds as for the iteration."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from oracle import twolevel as TW
from workloads import small_cases


@pytest.mark.parametrize("name", ["c0", "corner", "fulldepth", "r3m2"])
def test_composite_equals_dirichlet_neumann(name):
    wl = small_cases()[name]
    n = min(wl.n_macro, 4)
    a = oracle.run(wl, n, newton_tol=1e-11, dn_tol=1e-11)
    b = oracle.run(wl, n, newton_tol=1e-11, dn_tol=1e-11, composite=True)
    assert a.win.I0 == b.win.I0 and a.win.J0 == b.win.J0
    assert np.abs(a.Tc - b.Tc).max() < 1e-9
    assert np.abs(a.Tf - b.Tf).max() < 1e-9
    for key in ("absorbed", "bottom", "surface", "remap"):
        assert b.ledger[key] == pytest.approx(a.ledger[key], rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("name", ["c0", "fulldepth"])
def test_composite_energy_ledger(name):
    wl = small_cases()[name]
    sim = oracle.run(wl, min(wl.n_macro, 6), composite=True)
    for h in sim.history:
        lhs = h["E_end"] - h["E_start"]
        rhs = h["absorbed"] - h["bottom"] - h["surface"]
        assert abs(lhs - rhs) < 1e-9 * h["absorbed"]


def test_composite_refinement1_is_single_level():
    wl = small_cases()["r1m1"]
    n = 6
    sim = TW.TwoLevel(wl, composite=True)
    ref = TW.single_level_run(sim.coarse, wl.material, wl.scan, wl.options.dt_coarse, n,
                              tol=1e-11)
    for s in range(n):
        sim.step()
        assert np.abs(sim.Tc - ref[s]).max() < 1e-7
    assert sim.stats["moves"] >= 1
    assert sim.stats["dn_iters"] == n     # one solve per macro step


def test_composite_with_surface_loss():
    wl = small_cases()["c0"]
    wl = replace(wl, material=replace(wl.material, h_conv=2e4, emissivity=0.8))
    a = oracle.run(wl, 3, newton_tol=1e-11, dn_tol=1e-11)
    b = oracle.run(wl, 3, newton_tol=1e-11, dn_tol=1e-11, composite=True)
    assert np.abs(a.Tc - b.Tc).max() < 1e-9
    assert np.abs(a.Tf - b.Tf).max() < 1e-9
    assert b.ledger["surface"] == pytest.approx(a.ledger["surface"], rel=1e-9)
