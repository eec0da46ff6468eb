"""Dense two-cell patch matrix of one ghost face, by Gauss quadrature.  Test infrastructure only.

Definition (§2.2, bilinear form g_F; §2.4, local matrix G_{F,k}):

    [G_F]_{ab} = sum_{j=1..k} gamma_j * integral_F [d^j_n phi_a] [d^j_n phi_b] ds

for the (2k+1)(k+1)^{d-1} continuous Q_k basis functions phi_a of the two
cells sharing F, numbered lexicographically over the patch with 2k+1 nodes
along the normal (Fig. 2).  gamma_j carries every scalar factor of g_F
(gamma_A * h^{2j-1} / (j!)^2 for the paper's choice); the order-0 term is
absent because the jump of a continuous function is zero.

Everything is evaluated in physical coordinates: the 1D Lagrange
polynomials of each cell are expanded in the physical coordinate and
differentiated directly (no reference-cell scaling), and the face integral is
a tensor Gauss-Legendre rule with k+1 points per tangential axis, exact for
the degree-2k integrand.  The 1D values are computed in 60-digit mpmath and
rounded to float64; the d-dimensional quadrature sum is float64 numpy.
"""

import functools

import mpmath
import numpy as np

from . import basis
from .mesh import patch_extent, patch_local_nodes


@functools.lru_cache(maxsize=None)
def _gll(k):
    return tuple(basis.gll_nodes(k))


@functools.lru_cache(maxsize=None)
def _gauss(n):
    p, w = basis.gauss_legendre(n)
    return tuple(p), tuple(w)


def _cell_polys(k, a, h):
    a, h = mpmath.mpf(a), mpmath.mpf(h)
    return basis.lagrange_polys([a + h * xi for xi in _gll(k)])


def normal_jumps(k, left_corner, h, orders):
    """Jumps [d^j phi_i] = phi_i(right side)^(j) - phi_i(left side)^(j) at the face, i = 0..2k.

    left_corner: physical coordinate (mpmath) of the lower cell's lower end along
    the normal; the face sits at left_corner + h.  Returns an mpmath matrix as a
    list of lists [j][i] for j in `orders`.
    """
    h = mpmath.mpf(h)
    left = _cell_polys(k, left_corner, h)
    right = _cell_polys(k, mpmath.mpf(left_corner) + h, h)
    xf = mpmath.mpf(left_corner) + h
    out = []
    for j in orders:
        row = []
        for i in range(2 * k + 1):
            val = mpmath.mpf(0)
            if i >= k:  # piece on the upper cell: its local node i-k
                val += basis.poly_eval(basis.poly_deriv(right[i - k], j), xf)
            if i <= k:  # piece on the lower cell: its local node i
                val -= basis.poly_eval(basis.poly_deriv(left[i], j), xf)
            row.append(val)
        out.append(row)
    return out


def tangential_values(k, corner, h):
    """Physical quadrature points/weights on [corner, corner+h] and basis values V[q, i]."""
    pts, wts = _gauss(k + 1)
    polys = _cell_polys(k, corner, h)
    corner, h = mpmath.mpf(corner), mpmath.mpf(h)
    V = np.array([[float(basis.poly_eval(c, corner + h * x)) for c in polys] for x in pts])
    W = np.array([float(h * w) for w in wts])
    return V, W


def patch_matrix(d, k, axis, lower_cell, lo, h, gamma):
    """Dense patch matrix G_F (n_p x n_p, float64) of the face normal to `axis` above `lower_cell`.

    gamma: sequence of k coefficients gamma_1..gamma_k.
    """
    if len(gamma) != k:
        raise ValueError("need k coefficients")
    hm = mpmath.mpf(h)
    corner = [mpmath.mpf(lo[a]) + lower_cell[a] * hm for a in range(d)]
    jumps = normal_jumps(k, corner[axis], hm, range(1, k + 1))
    J = np.array([[float(v) for v in row] for row in jumps])  # (k, 2k+1)
    tang = [a for a in range(d) if a != axis]
    Vt, Wt = {}, {}
    for a in tang:
        Vt[a], Wt[a] = tangential_values(k, corner[a], hm)

    ext = patch_extent(d, k, axis)
    n_p = int(np.prod(ext))
    # local multi-index of each patch node, x fastest
    loc = patch_local_nodes(d, k, axis)

    # face quadrature points: multi-index over tangential axes
    qgrid = list(np.ndindex(*[k + 1] * len(tang)))
    nq = len(qgrid)
    T = np.ones((nq, n_p))       # product of tangential basis values
    Wq = np.ones(nq)
    for qi, q in enumerate(qgrid):
        for t_pos, a in enumerate(tang):
            T[qi, :] *= Vt[a][q[t_pos], loc[:, a]]
            Wq[qi] *= Wt[a][q[t_pos]]

    G = np.zeros((n_p, n_p))
    for j in range(k):
        B = T * J[j, loc[:, axis]][None, :]          # B[q, p] = [d^j phi_p](x_q)
        G += gamma[j] * (B.T * Wq[None, :]) @ B
    return G


def jump_vectors_reference(k):
    """Jump vectors of the reference patch (h = 1, face at xi = 1), orders j = 0..k, as mpmath rows.

    Used by the pins on the 1D quantities; order 0 must vanish identically.
    """
    return normal_jumps(k, mpmath.mpf(0), mpmath.mpf(1), range(0, k + 1))


def mass_reference(k):
    """Exact 1D mass matrix on [0, 1]: M[a, b] = integral l_a l_b, by (k+1)-point Gauss (mpmath)."""
    pts, wts = _gauss(k + 1)
    polys = _cell_polys(k, 0, 1)
    M = [[mpmath.mpf(0)] * (k + 1) for _ in range(k + 1)]
    for x, w in zip(pts, wts):
        vals = [basis.poly_eval(c, x) for c in polys]
        for a in range(k + 1):
            for b in range(k + 1):
                M[a][b] += w * vals[a] * vals[b]
    return M
