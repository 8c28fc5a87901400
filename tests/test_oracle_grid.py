"""Pins of the Q1 operator: hand-derived element values, brute-force
quadrature of the basis gradients, and the exact discrete eigenmodes of the
assembled operator on a box (Dirichlet bottom, insulated elsewhere)."""
import itertools

import numpy as np
import pytest

from oracle import grid as G
from oracle import level as LV
from workloads import Material


def test_isotropic_cube_values():
    h = 0.7
    Ke = G.element_stiffness(h, h, h)
    for a, b in itertools.product(range(8), range(8)):
        nd = bin(a ^ b).count("1")    # how many coordinates differ
        expect = {0: h / 3, 1: 0.0, 2: -h / 12, 3: -h / 12}[nd]
        assert Ke[a, b] == pytest.approx(expect, abs=1e-15)
    assert np.allclose(Ke.sum(axis=1), 0.0, atol=1e-15)


def _basis_grad(c, xi, h):
    """Gradient of the trilinear basis function of corner c at reference
    point xi in [0,1]^3 of a box with sides h."""
    bits = [(c >> d) & 1 for d in range(3)]
    vals = [xi[d] if bits[d] else 1.0 - xi[d] for d in range(3)]
    ders = [(1.0 if bits[d] else -1.0) / h[d] for d in range(3)]
    return np.array([ders[0] * vals[1] * vals[2], vals[0] * ders[1] * vals[2],
                     vals[0] * vals[1] * ders[2]])


def test_anisotropic_element_brute_force():
    h = (0.3, 1.1, 0.45)
    g = 0.5 * (1 + np.array([-1, 1]) / np.sqrt(3.0))
    Kq = np.zeros((8, 8))
    vol = h[0] * h[1] * h[2]
    for p in itertools.product(g, g, g):
        grads = [_basis_grad(c, p, h) for c in range(8)]
        for a in range(8):
            for b in range(8):
                Kq[a, b] += 0.125 * vol * grads[a] @ grads[b]
    assert np.allclose(G.element_stiffness(*h), Kq, rtol=1e-13, atol=1e-15)


def test_lumped_mass_and_assembly_invariants():
    g = G.Grid(5, 4, 3, 0.2, 0.3, 0.1)
    m = G.lumped_mass(g)
    assert m.sum() == pytest.approx(1.0 * 1.2 * 0.3)
    mask = np.zeros(g.n_elems)
    mask[::3] = 1.0
    assert G.lumped_mass(g, mask).sum() == pytest.approx(mask.sum() * g.volume())
    rng = np.random.default_rng(1)
    kap = rng.uniform(5, 30, g.n_elems)
    K = G.stiffness(g, kap)
    assert abs(K - K.T).max() < 1e-15
    assert np.abs(K @ np.ones(g.n_nodes)).max() < 1e-13
    v = rng.normal(size=g.n_nodes)
    assert v @ (K @ v) > 0


def _eigen_setup(nx=6, ny=5, nz=4, L=(1.0e-3, 0.8e-3, 0.5e-3), p=2, q=1, s=1):
    g = G.Grid(nx, ny, nz, L[0] / nx, L[1] / ny, L[2] / nz)
    x, y, z = g.node_xyz()
    phi = (np.cos(p * np.pi * x / L[0]) * np.cos(q * np.pi * y / L[1])
           * np.sin((2 * s + 1) * np.pi * z / (2 * L[2])))
    th = [p * np.pi * g.hx / L[0], q * np.pi * g.hy / L[1], (2 * s + 1) * np.pi * g.hz / (2 * L[2])]
    hh = [g.hx, g.hy, g.hz]
    lam = 0.0
    for a in range(3):
        term = 2.0 / hh[a] ** 2 * (1 - np.cos(th[a]))
        for b in range(3):
            if b != a:
                term *= (2 + np.cos(th[b])) / 3
        lam += term
    return g, phi, lam


def test_exact_discrete_eigenmode():
    g, phi, lam = _eigen_setup()
    K = G.stiffness(g, np.ones(g.n_elems))
    m = G.lumped_mass(g)
    _, _, k = g.node_ijk()
    free = k > 0
    lhs = (K @ phi)[free]
    rhs = lam * m[free] * phi[free]
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12 * np.abs(rhs).max())


def test_linear_backward_euler_decay():
    """Constant rho c and kappa, no latent heat, no laser: n backward-Euler
    steps multiply the eigenmode by (1 + alpha tau lambda_h)^-n."""
    mat = Material(c_lo=500.0, c_hi=500.0, k_lo=20.0, k_hi=20.0, latent=0.0)
    g, phi, lam = _eigen_setup()
    _, _, k = g.node_ijk()
    bottom = k == 0
    Tb, A, tau = 300.0, 50.0, 2e-3
    T = Tb + A * phi
    alpha = 20.0 / (mat.rho * 500.0)
    for n in range(1, 4):
        T, R, it = LV.implicit_step(g, mat, T, tau, np.zeros(g.n_nodes), None, bottom,
                                    np.full(g.n_nodes, Tb), tol=1e-12)
        expect = Tb + A * phi * (1 + alpha * tau * lam) ** (-n)
        assert np.abs(T - expect).max() < 1e-10
