"""Dense two-cell patch matrix of the macro-patch stabilisation.  Test infrastructure only.

Definition (§2.2, the alternative to the derivative-jump penalty: the difference between the function on
one cell and the extension of the function from the neighbouring cell, integrated; the paper states that
it has the same tensor-product structure but prints no formula, so the form below is a reading):

    [S_F]_{ab} = gamma_M h^{-2} integral_{omega_F} (E_1 phi_a - E_2 phi_a)(E_1 phi_b - E_2 phi_b) dx

* omega_F = K_1 u K_2 is the two-cell patch of the face F (lower cell K_1, upper cell K_2 along the
  normal).
* E_i phi is the polynomial extension of phi restricted to K_i: the cell's Q_k polynomial evaluated on
  the whole patch.
* The integral runs over the whole patch, which makes the form symmetric in the two cells.
* h^{-2} scales S_F like the derivative form with gamma_j = gamma_A h^{2j-1} / (j!)^2 (both ~ h^{d-2}).

Evaluation follows patch.patch_matrix. The 1D Lagrange polynomials of each cell are expanded in the
physical coordinate and simply evaluated outside their cell. The patch integral is a tensor
Gauss-Legendre rule with k+1 points per axis on each of the two cells, which is exact because the
integrand has degree 2k per axis. The 1D values are computed in 60-digit mpmath and rounded to float64;
the d-dimensional quadrature sum is in float64.
"""

import mpmath
import numpy as np

from .mesh import patch_extent, patch_local_nodes
from .patch import _cell_polys, _gauss, tangential_values
from . import basis


def extension_differences(k, left_corner, h, points):
    """D[q, i] = (E_1 psi_i - E_2 psi_i)(points[q]) for the 2k+1 continuous 1D patch functions psi_i.

    psi_i restricted to the lower cell is its Lagrange polynomial of local node i (zero for i > k); on
    the upper cell, that of local node i - k (zero for i < k).  Returns an mpmath list of lists.
    """
    h = mpmath.mpf(h)
    left = _cell_polys(k, left_corner, h)
    right = _cell_polys(k, mpmath.mpf(left_corner) + h, h)
    out = []
    for x in points:
        row = []
        for i in range(2 * k + 1):
            v = mpmath.mpf(0)
            if i <= k:
                v += basis.poly_eval(left[i], x)
            if i >= k:
                v -= basis.poly_eval(right[i - k], x)
            row.append(v)
        out.append(row)
    return out


def patch_points(k, left_corner, h):
    """Gauss points and weights of the 1D two-cell patch [c, c + 2h]: k+1 points on each cell (mpmath)."""
    pts, wts = _gauss(k + 1)
    c, h = mpmath.mpf(left_corner), mpmath.mpf(h)
    xs = [c + h * p for p in pts] + [c + h + h * p for p in pts]
    ws = [h * w for w in wts] * 2
    return xs, ws


def macro_matrix_1d(k, left_corner, h):
    """integral over [c, c + 2h] of (E_1 psi_a - E_2 psi_a)(E_1 psi_b - E_2 psi_b) dx, (2k+1)^2 float64.

    No gamma and no h^{-2}: the bare 1D integral, for the pins.
    """
    xs, ws = patch_points(k, left_corner, h)
    D = extension_differences(k, left_corner, h, xs)
    NN = 2 * k + 1
    S = [[mpmath.mpf(0)] * NN for _ in range(NN)]
    for row, w in zip(D, ws):
        for a in range(NN):
            for b in range(NN):
                S[a][b] += w * row[a] * row[b]
    return np.array([[float(v) for v in r] for r in S])


def macro_patch_matrix(d, k, axis, lower_cell, lo, h, gamma):
    """Dense macro-patch matrix S_F (n_p x n_p, float64) of the face normal to `axis` above `lower_cell`.

    gamma: sequence of one coefficient gamma_M.
    """
    if len(gamma) != 1:
        raise ValueError("the macro-patch form takes one coefficient")
    hm = mpmath.mpf(h)
    corner = [mpmath.mpf(lo[a]) + lower_cell[a] * hm for a in range(d)]
    xs, ws = patch_points(k, corner[axis], hm)
    Dn = np.array([[float(v) for v in r] for r in extension_differences(k, corner[axis], hm, xs)])
    Wn = np.array([float(w) for w in ws])
    tang = [a for a in range(d) if a != axis]
    Vt, Wt = {}, {}
    for a in tang:
        Vt[a], Wt[a] = tangential_values(k, corner[a], hm)

    n_p = int(np.prod(patch_extent(d, k, axis)))
    loc = patch_local_nodes(d, k, axis)
    # patch quadrature points: normal point index first, then the tangential multi-index
    qgrid = list(np.ndindex(len(xs), *[k + 1] * len(tang)))
    B = np.ones((len(qgrid), n_p))   # B[q, p] = (E_1 phi_p - E_2 phi_p)(x_q)
    Wq = np.ones(len(qgrid))
    for qi, q in enumerate(qgrid):
        B[qi, :] *= Dn[q[0], loc[:, axis]]
        Wq[qi] *= Wn[q[0]]
        for t_pos, a in enumerate(tang):
            B[qi, :] *= Vt[a][q[1 + t_pos], loc[:, a]]
            Wq[qi] *= Wt[a][q[1 + t_pos]]
    return (gamma[0] / (h * h)) * ((B.T * Wq[None, :]) @ B)
