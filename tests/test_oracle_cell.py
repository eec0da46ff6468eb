"""Pins of the oracle's interior-cell Laplacian (oracle/cell.py) against closed forms and invariants."""

import numpy as np
import pytest

from oracle import cell, mesh


def test_q1_square_element_matrix():
    """The bilinear element on a square has the textbook stiffness (1/6)[[4,-1,-1,-2], ...], whatever h."""
    ref = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    for h in (1.0, 0.25, 0.37):
        np.testing.assert_allclose(cell.cell_stiffness(2, 1, (0.3, -0.2), h, (2, 5)), ref, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("d,k", [(2, k) for k in range(1, 8)] + [(3, k) for k in (1, 2, 3, 5, 7)])
def test_cell_stiffness_invariants(d, k):
    """Symmetric, positive semi-definite with exactly the constants as null space; the energy of a
    linear function is the cell volume, that of x0*x1 its exact integral of x0^2 + x1^2."""
    lo, h, c = (-1.0,) * d, 0.125, (3, 4, 5)[:d]
    K = cell.cell_stiffness(d, k, lo, h, c)
    scale = np.max(np.abs(K))
    assert np.max(np.abs(K - K.T)) <= 1e-14 * scale
    ev = np.linalg.eigvalsh(K)
    assert ev[0] > -1e-12 * scale and ev[1] > 1e-6 * scale
    assert np.max(np.abs(K @ np.ones(len(K)))) <= 1e-12 * scale
    loc = np.array([np.unravel_index(p, (k + 1,) * d, order="F") for p in range((k + 1) ** d)])
    from oracle.basis import gll_nodes
    xi = np.array([float(x) for x in gll_nodes(k)])
    x = h * xi[loc]  # node coordinates relative to the cell's lower corner (K annihilates the shift)
    for axis in range(d):
        u = x[:, axis]
        assert abs(u @ K @ u - h ** d) <= 1e-12 * h ** d
    u = x[:, 0] * x[:, 1]
    exact = 2 * h ** (d + 2) / 3  # integral of x1^2 + x0^2 over [0, h]^d
    assert abs(u @ K @ u - exact) <= 1e-11 * abs(exact)


def test_interior_operator_energy_and_constants():
    """On a classified mesh: the operator annihilates constants, and a linear function's energy is the
    total volume of the inside cells."""
    n, lo, h, k = (10, 9, 8), (-1.0, -0.9, -0.8), 0.2, 3
    cls = mesh.classify_ball(n, lo, h, (0.011, 0.017, 0.023), 0.73)
    o = cell.CellOracle(3, n, lo, h, k, cls)
    assert len(o.cells) == int(np.sum(cls == mesh.INSIDE)) > 0
    L = o.L
    I = np.stack(np.unravel_index(np.arange(o.n_lattice), L, order="F"), -1)
    from oracle.basis import gll_nodes
    xi = np.array([float(v) for v in gll_nodes(k)])
    cidx = np.minimum(I // k, np.array(n) - 1)
    coords = np.array(lo) + h * (cidx + xi[I - k * cidx])
    assert np.max(np.abs(o.apply(np.ones(o.n_lattice)))) <= 1e-12
    for axis in range(3):
        u = coords[:, axis]
        assert abs(u @ o.apply(u) - len(o.cells) * h ** 3) <= 1e-11 * len(o.cells) * h ** 3


def test_apply_at_matches_apply():
    """apply_at sums the same cells as apply at the sampled nodes."""
    d, k, n = 3, 2, (9, 8, 7)
    lo, h = (-1.0,) * 3, 2.0 / 9
    cls = mesh.classify_ball(n, lo, h, (0.011, 0.017, 0.023), 0.73)
    co = cell.CellOracle(d, n, lo, h, k, cls)
    u = np.random.default_rng(3).uniform(-1, 1, co.n_lattice)
    y = co.apply(u)
    nodes = np.random.default_rng(4).choice(co.n_lattice, 300, replace=False)
    np.testing.assert_allclose(co.apply_at(u, nodes), y[nodes], rtol=0, atol=1e-14 * np.max(np.abs(y)))
