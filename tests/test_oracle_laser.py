"""Pins of the laser load and scan path: the flux integrates to eta P, the
Q1 load reproduces the spot centroid (Q1 bases reproduce linear functions),
symmetry at a corner, and hand-computed scan-path positions."""
import numpy as np
import pytest

from oracle import grid as G
from oracle import laser as L
from workloads import Track, ScanPath

UM = 1e-6


def _spot(x, y, P=150.0, R=50 * UM, eta=0.4):
    return (x, y, P, R, eta, 0)


def test_total_power_and_centroid():
    R = 50 * UM
    g = G.Grid(40, 40, 2, 12.5 * UM, 12.5 * UM, 10 * UM)   # 0.5 x 0.5 mm top
    sp = _spot(0.2512e-3, 0.2437e-3)
    for nq, tol in ((3, 2e-6), (6, 1e-12)):
        F = L.top_load(g, sp, nq)
        assert F.sum() == pytest.approx(0.4 * 150.0, rel=tol)
        x, y, z = g.node_xyz()
        assert (F * x).sum() / F.sum() == pytest.approx(sp[0], rel=tol)
        assert (F * y).sum() / F.sum() == pytest.approx(sp[1], rel=tol)
        assert np.all(F[z < z.max()] == 0.0)


def test_corner_quarter_and_mask():
    g = G.Grid(20, 20, 1, 10 * UM, 10 * UM, 10 * UM)
    F = L.top_load(g, _spot(0.0, 0.0), 6)
    assert F.sum() == pytest.approx(0.25 * 0.4 * 150.0, rel=1e-10)
    mask = np.zeros(g.nx * g.ny, dtype=bool)
    mask[::7] = True
    Fa = L.top_load(g, _spot(0.0, 0.0), 3, mask)
    Fb = L.top_load(g, _spot(0.0, 0.0), 3, ~mask)
    assert np.allclose(Fa + Fb, L.top_load(g, _spot(0.0, 0.0), 3), rtol=1e-14, atol=0)


def test_uniform_flux_limit():
    # a very wide spot is almost uniform: each top node gets flux * its area share
    g = G.Grid(4, 3, 1, 10 * UM, 10 * UM, 10 * UM)
    R = 1.0
    sp = _spot(20 * UM, 15 * UM, R=R)
    F = L.top_load(g, sp, 3)
    q0 = 3 * 0.4 * 150.0 / (np.pi * R * R)
    i, j, k = g.node_ijk()
    share = np.where((i == 0) | (i == 4), 0.5, 1.0) * np.where((j == 0) | (j == 3), 0.5, 1.0)
    expect = np.where(k == 1, q0 * share * 100e-12, 0.0)
    assert np.allclose(F, expect, rtol=1e-7, atol=0)


def test_scan_path_positions():
    t1 = Track(0.0, 0.0, 1e-3, 0.0, 0.5, 100.0, 50 * UM, 0.4)       # 2 ms
    t2 = Track(1e-3, 0.0, 1e-3, 0.4e-3, 0.8, 200.0, 60 * UM, 0.3)    # 0.5 ms
    sc = ScanPath([t1, t2], t_start=1e-4)
    assert L.laser_at(sc, 0.5e-4) is None
    s = L.laser_at(sc, 1e-4)
    assert s[:2] == pytest.approx((0.0, 0.0)) and s[5] == 0
    s = L.laser_at(sc, 1e-4 + 1e-3)
    assert s[0] == pytest.approx(0.5e-3) and s[2] == 100.0
    s = L.laser_at(sc, 1e-4 + 2e-3 + 0.25e-3)
    assert s[:2] == pytest.approx((1e-3, 0.2e-3)) and s[5] == 1 and s[2] == 200.0
    assert L.laser_at(sc, 1e-4 + 2.5e-3 + 1e-9) is None
    starts, end = L.track_start_times(sc)
    assert starts == pytest.approx([1e-4, 2.1e-3]) and end == pytest.approx(2.6e-3)
