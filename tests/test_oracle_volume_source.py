"""Pins of the volume laser model (paper Section 5.2): the volumetric
Gaussian of the local level and the smeared box source of the global level.

  * the volumetric Gaussian, with its amplitude normalised over the
    half-space below the surface, deposits eta P (closed form) -- this pins
    the reading of the printed prefactor;
  * its load vector equals brute-force Gauss quadrature of Q- phi_i over
    every element (pins the erf closed forms of the 1D factors);
  * the box load integrates to q |box| and, element by element, equals
    Gauss quadrature over the clipped box (exact for trilinear integrands);
    a box on element boundaries gives q |e| / 8 per corner;
  * the swept boxes of a step follow the track (hand values), including a
    step that ends one track and starts the next;
  * the two-level run with the volume model keeps the energy ledger."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from oracle import grid as G
from oracle import laser as L
from workloads import ScanPath, Track, single_track_3d, single_track_1mm, VOLUME

UM = 1e-6


def _spot(xc, yc, P=179.2, R=85 * UM, eta=0.38):
    return (xc, yc, P, R, eta, 0)


def test_volume_gaussian_deposits_eta_P():
    R, d = 85 * UM, 50 * UM
    # grid over +-5R in x and y and 6d in depth, surface at the top
    g = G.Grid(50, 50, 30, 10 * R / 50, 10 * R / 50, 6 * d / 30, -5 * R, -5 * R, -6 * d)
    F = L.volume_load(g, _spot(0.0, 0.0, R=R), d, 0.0)
    assert F.sum() == pytest.approx(0.38 * 179.2, rel=1e-9)
    # the load is centred on the spot
    x, y, z = g.node_xyz()
    assert abs((F * x).sum() / F.sum()) < 1e-9 * R
    assert abs((F * y).sum() / F.sum()) < 1e-9 * R


def test_volume_load_matches_quadrature():
    R, d = 60 * UM, 30 * UM
    g = G.Grid(4, 3, 2, 40 * UM, 35 * UM, 25 * UM, 0.0, 0.0, 0.0)
    z_top = g.nz * g.hz
    spot = _spot(70 * UM, 50 * UM, R=R)
    F = L.volume_load(g, spot, d, z_top)
    # brute force: 16-point Gauss-Legendre per direction on every element
    p, w = np.polynomial.legendre.leggauss(16)
    p, w = 0.5 * (p + 1.0), 0.5 * w
    ref = np.zeros(g.n_nodes)
    ei, ej, ek = g.elem_ijk()
    corners = g.element_corners()
    vol = g.hx * g.hy * g.hz
    for a in range(16):
        for b in range(16):
            for c in range(16):
                x = g.x0 + (ei + p[a]) * g.hx
                y = g.y0 + (ej + p[b]) * g.hy
                z = g.z0 + (ek + p[c]) * g.hz
                q = L.volume_density(x, y, z, spot, d, z_top) * (w[a] * w[b] * w[c] * vol)
                for cc in range(8):
                    ca, cb, cg = cc & 1, (cc >> 1) & 1, cc >> 2
                    phi = ((p[a] if ca else 1 - p[a]) * (p[b] if cb else 1 - p[b])
                           * (p[c] if cg else 1 - p[c]))
                    np.add.at(ref, corners[:, cc], q * phi)
    assert np.abs(F - ref).max() <= 1e-10 * np.abs(ref).max()


def _box_load_by_quadrature(g, boxes, mask=None):
    """The same integral by 2-point Gauss quadrature on each clipped
    element box (exact for the trilinear basis)."""
    F = np.zeros(g.n_nodes)
    p = 0.5 + np.array([-0.5, 0.5]) / np.sqrt(3.0)
    ei, ej, ek = g.elem_ijk()
    corners = g.element_corners()
    for (x0, x1, y0, y1, z0, z1, q) in boxes:
        for e in range(g.n_elems):
            if mask is not None and not mask[e]:
                continue
            ex, ey, ez = g.x0 + ei[e] * g.hx, g.y0 + ej[e] * g.hy, g.z0 + ek[e] * g.hz
            lo = [max(x0, ex), max(y0, ey), max(z0, ez)]
            hi = [min(x1, ex + g.hx), min(y1, ey + g.hy), min(z1, ez + g.hz)]
            if any(h <= l for l, h in zip(lo, hi)):
                continue
            v = np.prod([h - l for l, h in zip(lo, hi)]) / 8.0
            for a in p:
                for b in p:
                    for c in p:
                        x = lo[0] + a * (hi[0] - lo[0])
                        y = lo[1] + b * (hi[1] - lo[1])
                        z = lo[2] + c * (hi[2] - lo[2])
                        u, s, t = (x - ex) / g.hx, (y - ey) / g.hy, (z - ez) / g.hz
                        for cc in range(8):
                            ca, cb, cg = cc & 1, (cc >> 1) & 1, cc >> 2
                            phi = ((u if ca else 1 - u) * (s if cb else 1 - s)
                                   * (t if cg else 1 - t))
                            F[corners[e, cc]] += q * v * phi
    return F


def test_box_load_exact():
    g = G.Grid(5, 4, 3, 100 * UM, 100 * UM, 100 * UM)
    box = (123 * UM, 377 * UM, 141 * UM, 226 * UM, 250 * UM, 300 * UM, 2.5e12)
    F = L.box_load(g, [box])
    vol = (377 - 123) * (226 - 141) * (300 - 250) * UM ** 3
    assert F.sum() == pytest.approx(2.5e12 * vol, rel=1e-12)
    ref = _box_load_by_quadrature(g, [box])
    assert np.abs(F - ref).max() <= 1e-12 * np.abs(ref).max()
    mask = np.arange(g.n_elems) % 3 != 0
    assert np.abs(L.box_load(g, [box], mask) - _box_load_by_quadrature(g, [box], mask)).max() \
        <= 1e-12 * np.abs(ref).max()
    # a box on element boundaries: q |e| / 8 at each corner of each element
    aligned = (100 * UM, 300 * UM, 100 * UM, 200 * UM, 200 * UM, 300 * UM, 1.0)
    F = L.box_load(g, [aligned])
    e8 = (100 * UM) ** 3 / 8.0
    assert F[g.node(1, 1, 3)] == pytest.approx(e8)          # one element's corner
    assert F[g.node(2, 1, 3)] == pytest.approx(2 * e8)      # shared by two


def test_swept_boxes_hand_values():
    R, d, v, P, eta = 80 * UM, 40 * UM, 0.5, 200.0, 0.4
    t1 = Track(0.1e-3, 0.5e-3, 0.3e-3, 0.5e-3, speed=v, power=P, radius=R,
               absorptivity=eta, depth=d)
    t2 = Track(0.3e-3, 0.5e-3, 0.3e-3, 0.9e-3, speed=v, power=P, radius=R,
               absorptivity=eta, depth=d)
    scan = ScanPath([t1, t2])
    z_top = 1e-3
    # inside track 1: one box from x0 + v t0 to x0 + v t1
    b = L.swept_boxes(scan, 100e-6, 300e-6, z_top)
    assert len(b) == 1
    x0, x1, y0, y1, z0, z1, q = b[0]
    assert (x0, x1) == pytest.approx((0.1e-3 + v * 100e-6, 0.1e-3 + v * 300e-6))
    assert (y0, y1) == pytest.approx((0.5e-3 - R / 2, 0.5e-3 + R / 2))
    assert (z0, z1) == pytest.approx((z_top - d, z_top))
    assert q == pytest.approx(eta * P / (R * d * v * 200e-6))
    # across the corner: track 1 ends at 400 us, track 2 runs along y
    b = L.swept_boxes(scan, 300e-6, 500e-6, z_top)
    assert len(b) == 2
    lens = [b[0][1] - b[0][0], b[1][3] - b[1][2]]
    assert lens == pytest.approx([v * 100e-6, v * 100e-6])
    assert b[1][0:2] == pytest.approx((0.3e-3 - R / 2, 0.3e-3 + R / 2))
    energy = sum((x1 - x0) * (y1 - y0) * (z1 - z0) * q for x0, x1, y0, y1, z0, z1, q in b)
    assert energy == pytest.approx(eta * P)     # power averaged over the step


def test_two_level_ledger_with_volume_sources():
    sim = oracle.run(single_track_3d(), 4)
    for h in sim.history:
        lhs = h["E_end"] - h["E_start"]
        rhs = h["absorbed"] - h["bottom"] - h["surface"]
        assert abs(lhs - rhs) < 1e-9 * h["absorbed"]
    # the beam's absorbed power over the run
    assert sim.ledger["absorbed"] == pytest.approx(0.38 * 179.2 * 4 * 400e-6, rel=1e-4)
    assert sim.stats["moves"] >= 2
