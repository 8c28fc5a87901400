"""Pins of the alternate global formulation of Section 3 (only the interface
jump term couples the global problem to the local one; it vanishes when both
levels share kappa(T), and the paper keeps latent heat in the local problem
only):

  * the global field is the single-level coarse solve with the global law
    (no latent heat) -- the local problem does not feed back;
  * with refinement 1, one micro step and a law without latent heat, the
    local field equals the global field on the window;
  * the global problem's energy ledger holds step by step."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from oracle import twolevel as TW
from workloads import small_cases, ALTERNATE


def _alternate(wl, **opts):
    return replace(wl, options=replace(wl.options, coupling=ALTERNATE, **opts))


def test_global_field_is_single_level_without_latent_heat():
    wl = _alternate(small_cases()["c0"], m_time=1)
    n = 6
    sim = TW.TwoLevel(wl, newton_tol=1e-11)
    ref = TW.single_level_run(sim.coarse, replace(wl.material, latent=0.0), wl.scan,
                              wl.options.dt_coarse, n, tol=1e-11)
    for s in range(n):
        sim.step()
        assert np.abs(sim.Tc - ref[s]).max() < 1e-7
    assert sim.stats["moves"] >= 1


def test_refinement1_local_equals_global():
    wl = small_cases()["r1m1"]
    wl = _alternate(replace(wl, material=replace(wl.material, latent=0.0)))
    sim = TW.TwoLevel(wl, newton_tol=1e-11)
    for _ in range(6):
        sim.step()
        w = sim.win
        assert np.abs(sim.Tf[w.inject_f] - sim.Tc[w.inject_c]).max() < 1e-7


@pytest.mark.parametrize("name", ["c0", "fulldepth"])
def test_global_energy_ledger(name):
    wl = small_cases()[name]
    wl = _alternate(replace(wl, material=replace(wl.material, h_conv=1e4)))
    sim = oracle.run(wl, 6)
    for h in sim.history:
        lhs = h["E_end"] - h["E_start"]
        rhs = h["absorbed"] - h["bottom"] - h["surface"]
        assert abs(lhs - rhs) < 1e-9 * h["absorbed"]
    assert sim.ledger["remap"] == 0.0
