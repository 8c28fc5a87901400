"""Structured Q1 hexahedral grids and the assembled heat operator.

The method uses uniform, structured meshes on both levels (the paper stresses
that two-level meshes can stay uniform, Sections 1 and 5.3).  Here a level
is a box of nx x ny x nz trilinear (Q1) cells of spacing (hx, hy, hz); the
element type replaces the paper's linear tetrahedra (Section 5.2) by
hexahedra, which fit the structured grid.

Node (i, j, k) has flat index i + (nx+1) * (j + (ny+1) * k); element
(i, j, k) spans nodes (i..i+1, j..j+1, k..k+1); local corner c = a + 2b + 4g
with (a, b, g) the offsets in x, y, z.
"""
import numpy as np
import scipy.sparse as sp

# 1D linear element on [0, 1]: stiffness and consistent mass (unit length).
K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
M1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])


class Grid:
    def __init__(self, nx, ny, nz, hx, hy, hz, x0=0.0, y0=0.0, z0=0.0):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.hx, self.hy, self.hz = float(hx), float(hy), float(hz)
        self.x0, self.y0, self.z0 = float(x0), float(y0), float(z0)
        self.shape = (self.nz + 1, self.ny + 1, self.nx + 1)  # (k, j, i)
        self.n_nodes = (self.nx + 1) * (self.ny + 1) * (self.nz + 1)
        self.n_elems = self.nx * self.ny * self.nz
        self._pattern = None

    def node(self, i, j, k):
        return i + (self.nx + 1) * (j + (self.ny + 1) * k)

    def node_ijk(self):
        """Integer (i, j, k) arrays of every node in flat order."""
        k, j, i = np.meshgrid(np.arange(self.nz + 1), np.arange(self.ny + 1),
                              np.arange(self.nx + 1), indexing="ij")
        return i.ravel(), j.ravel(), k.ravel()

    def node_xyz(self):
        i, j, k = self.node_ijk()
        return (self.x0 + i * self.hx, self.y0 + j * self.hy, self.z0 + k * self.hz)

    def elem_ijk(self):
        k, j, i = np.meshgrid(np.arange(self.nz), np.arange(self.ny),
                              np.arange(self.nx), indexing="ij")
        return i.ravel(), j.ravel(), k.ravel()

    def element_corners(self):
        """(n_elems, 8) node indices, corner c = a + 2b + 4g."""
        if getattr(self, "_corners", None) is not None:
            return self._corners
        i, j, k = self.elem_ijk()
        cols = []
        for g in (0, 1):
            for b in (0, 1):
                for a in (0, 1):
                    cols.append(self.node(i + a, j + b, k + g))
        self._corners = np.stack(cols, axis=1)
        return self._corners

    def volume(self):
        return self.hx * self.hy * self.hz


def element_stiffness(hx, hy, hz):
    """8x8 Q1 element matrix of int grad(phi_a).grad(phi_b) over an
    hx x hy x hz box: the tensor-product form
        (hy hz/hx) K1(x) M1(y) M1(z) + (hx hz/hy) M1 K1 M1 + (hx hy/hz) M1 M1 K1,
    which is what 2x2x2 Gauss quadrature gives exactly.  The x factor is the
    fastest-varying one, matching corner numbering a + 2b + 4g."""
    return ((hy * hz / hx) * np.kron(M1, np.kron(M1, K1))
            + (hx * hz / hy) * np.kron(M1, np.kron(K1, M1))
            + (hx * hy / hz) * np.kron(K1, np.kron(M1, M1)))


def lumped_mass(grid, elem_mask=None):
    """Row-sum lumped mass: m_i = sum over elements e (in the mask) that
    contain node i of |e| / 8."""
    corners = grid.element_corners()
    w = np.full(grid.n_elems, grid.volume() / 8.0)
    if elem_mask is not None:
        w = w * elem_mask
    m = np.zeros(grid.n_nodes)
    for c in range(8):
        np.add.at(m, corners[:, c], w)
    return m


def element_mean(grid, T):
    """Mean of the 8 nodal values of every element."""
    return T[grid.element_corners()].mean(axis=1)


def _pattern(grid):
    """Sparsity pattern of the assembled operator and, for every entry
    (e, a, b) of every element matrix, the CSR slot it is summed into."""
    if grid._pattern is None:
        corners = grid.element_corners()
        rows = np.repeat(corners[:, :, None], 8, axis=2).ravel()
        cols = np.repeat(corners[:, None, :], 8, axis=1).ravel()
        key = rows.astype(np.int64) * grid.n_nodes + cols
        ukey, slot = np.unique(key, return_inverse=True)
        urow = ukey // grid.n_nodes
        ucol = ukey % grid.n_nodes
        indptr = np.searchsorted(urow, np.arange(grid.n_nodes + 1))
        grid._pattern = (slot, ucol.astype(np.int32), indptr.astype(np.int32))
    return grid._pattern


def stiffness(grid, kappa_e):
    """Assembled K = sum_e kappa_e K_e as a CSR matrix (kappa_e = 0 removes
    an element)."""
    slot, indices, indptr = _pattern(grid)
    if getattr(grid, "_Ke", None) is None:
        grid._Ke = element_stiffness(grid.hx, grid.hy, grid.hz)
    Ke = grid._Ke
    vals = (np.asarray(kappa_e, dtype=np.float64)[:, None, None] * Ke[None, :, :]).ravel()
    data = np.bincount(slot, weights=vals, minlength=len(indices))
    return sp.csr_matrix((data, indices, indptr), shape=(grid.n_nodes, grid.n_nodes))
