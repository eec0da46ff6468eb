"""Dense Laplacian stiffness of one cell, and the interior-cell operator.  Test infrastructure only.

Definition (the cell term of the paper's weak form, §2.1, evaluated on the cells that the boundary does
not intersect as in §2.5, Algorithm 1):

    w_{K,i} = integral_K grad u_K . grad phi_i dx,   i.e.   [K_K]_{ab} = integral_K grad phi_a . grad phi_b dx

for the (k+1)^d continuous Q_k basis functions of a cell K on GLL nodes, numbered lexicographically over
the cell (x fastest).  Evaluated in physical coordinates: the 1D Lagrange polynomials of the cell are
expanded in x and differentiated directly; a tensor Gauss-Legendre rule with k+1 points per axis is
exact (the integrand has degree at most 2k per axis).  1D values in 60-digit mpmath rounded to
float64; the d-dimensional quadrature sum in float64.  The operator on the node lattice is

    y = sum over INSIDE cells K of R_K^T K_K R_K u.
"""

import mpmath
import numpy as np

from . import basis
from .mesh import INSIDE, linear_index


def cell_values(k, corner, h):
    """Gauss points on [corner, corner + h]: basis values V[q, i], derivatives D[q, i], weights W[q]."""
    pts, wts = basis.gauss_legendre(k + 1)
    polys = basis.physical_lagrange(k, corner, h)
    dpolys = [basis.poly_deriv(c) for c in polys]
    corner, h = mpmath.mpf(corner), mpmath.mpf(h)
    xs = [corner + h * x for x in pts]
    V = np.array([[float(basis.poly_eval(c, x)) for c in polys] for x in xs])
    D = np.array([[float(basis.poly_eval(c, x)) for c in dpolys] for x in xs])
    W = np.array([float(h * w) for w in wts])
    return V, D, W


def cell_stiffness(d, k, lo, h, cell):
    """Dense stiffness K_K ((k+1)^d x (k+1)^d, float64) of the cell with lower-corner index `cell`."""
    one = [cell_values(k, mpmath.mpf(lo[a]) + cell[a] * mpmath.mpf(h), h) for a in range(d)]
    K1 = k + 1
    loc = np.array([np.unravel_index(p, (K1,) * d, order="F") for p in range(K1 ** d)])
    qs = loc  # the quadrature grid has the same shape: multi-index per point, x fastest
    Wq = np.ones(len(qs))
    for a in range(d):
        Wq *= one[a][2][qs[:, a]]
    Kmat = np.zeros((K1 ** d, K1 ** d))
    for a in range(d):
        B = np.ones((len(qs), K1 ** d))  # B[q, p] = d/dx_a phi_p (x_q)
        for b in range(d):
            tab = one[b][1] if b == a else one[b][0]
            B *= tab[qs[:, b][:, None], loc[:, b][None, :]]
        Kmat += (B.T * Wq[None, :]) @ B
    return Kmat


def cell_dofs(cells, k, L):
    """Global lattice indices (nc, (k+1)^d) of the nodes of the given cells, x fastest."""
    d = cells.shape[1]
    loc = np.array([np.unravel_index(p, (k + 1,) * d, order="F") for p in range((k + 1) ** d)])
    return linear_index(k * cells[:, None, :] + loc[None, :, :], L)


class CellOracle:
    """The Laplacian on the inside cells of a classified mesh (classes as in oracle.mesh)."""

    def __init__(self, d, n, lo, h, k, cls, check_cells=4, seed=0):
        self.d, self.n, self.lo, self.h, self.k = d, tuple(n), tuple(lo), float(h), k
        self.L = tuple(k * m + 1 for m in self.n)
        self.n_lattice = int(np.prod(self.L))
        self.cells = np.argwhere(np.asarray(cls) == INSIDE).astype(np.int64)
        self.K = None
        if len(self.cells):
            # every cell of a Cartesian mesh has the same matrix: assemble one, compare a seeded sample
            self.K = cell_stiffness(d, k, lo, h, self.cells[0])
            rng = np.random.default_rng(seed)
            scale = np.max(np.abs(self.K))
            for i in rng.choice(len(self.cells), size=min(check_cells, len(self.cells)), replace=False):
                other = cell_stiffness(d, k, lo, h, self.cells[i])
                if np.max(np.abs(other - self.K)) / scale > 1e-13:
                    raise AssertionError("cell matrices differ between cells")

    def apply(self, u):
        y = np.zeros(self.n_lattice)
        if self.K is None:
            return y
        dofs = cell_dofs(self.cells, self.k, self.L)
        np.add.at(y, dofs, u[dofs] @ self.K.T)
        return y

    def apply_at(self, u, nodes):
        """Entries of the apply at the given lattice nodes, from the inside cells that contain them only."""
        nodes = np.asarray(nodes, dtype=np.int64)
        if self.K is None:
            return np.zeros(len(nodes))
        dofs = cell_dofs(self.cells, self.k, self.L)
        mark = np.zeros(self.n_lattice, dtype=bool)
        mark[nodes] = True
        sel = mark[dofs].any(axis=1)
        y = np.zeros(self.n_lattice)
        np.add.at(y, dofs[sel], u[dofs[sel]] @ self.K.T)
        return y[nodes]
