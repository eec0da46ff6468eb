"""Pins of the oracle's classification, face set, gradients, lumped mass and CG."""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import basis, mesh, patch
from oracle.operator import GhostOracle, cg_reference

BALLS = [
    ((32, 32), (-1.0, -1.0), 2 / 32, (0.013, 0.021), 0.71),
    ((12, 11, 10), (-1.0, -0.95, -0.9), 2 / 12, (0.011, 0.017, 0.023), 0.73),
    ((16, 16, 16), (-1.0, -1.0, -1.0), 2 / 16, (0.011, 0.017, 0.023), 0.73),
]


@pytest.mark.parametrize("n,lo,h,centre,radius", BALLS)
def test_classification_and_faces_brute_force(n, lo, h, centre, radius):
    cls = mesh.classify_ball(n, lo, h, centre, radius)
    np.testing.assert_array_equal(cls, mesh.classify_ball_loop(n, lo, h, centre, radius))
    fa, fb = mesh.ghost_faces(cls), mesh.ghost_faces_loop(cls)
    for a in range(len(n)):
        np.testing.assert_array_equal(fa[a], fb[a])
        # every face joins two active cells, at least one cut (Fig. 1)
        for c in fa[a]:
            nb = c.copy()
            nb[a] += 1
            p, q = cls[tuple(c)], cls[tuple(nb)]
            assert p != mesh.OUTSIDE and q != mesh.OUTSIDE and mesh.CUT in (p, q)


@pytest.mark.parametrize("n,lo,h,centre,radius", BALLS[:2])
def test_classification_by_sampling(n, lo, h, centre, radius):
    """Sample points in every cell: a point strictly inside the ball makes the cell active;
    a point strictly outside means the cell is not inside."""
    d = len(n)
    cls = mesh.classify_ball(n, lo, h, centre, radius)
    s = (np.arange(9) + 0.5) / 9
    grid = np.stack(np.meshgrid(*[s] * d, indexing="ij"), -1).reshape(-1, d)
    corners = np.stack(np.meshgrid(*[[0.0, 1.0]] * d, indexing="ij"), -1).reshape(-1, d)
    pts = np.concatenate([grid, corners])
    for c in np.ndindex(*n):
        x = np.array(lo) + (np.array(c) + pts) * h
        r = np.linalg.norm(x - np.array(centre), axis=1)
        if np.any(r < radius):
            assert cls[c] != mesh.OUTSIDE
        if np.any(r > radius):
            assert cls[c] != mesh.INSIDE
        if cls[c] == mesh.INSIDE:
            assert np.all(r <= radius)


UNIONS = [
    ((16, 16, 16), (-1.0,) * 3, 2 / 16, [(0.31, -0.22, 0.05, 0.37), (-0.4, 0.3, -0.35, 0.52), (0.1, 0.12, 0.3, 0.29)]),
    ((20, 18), (-1.0, -0.9), 2 / 20, [(0.213, 0.131, 0.0, 0.337), (-0.351, -0.207, 0.0, 0.419), (0.423, -0.509, 0.0, 0.271)]),
]


@pytest.mark.parametrize("n,lo,h,balls", UNIONS)
def test_union_of_balls_classification(n, lo, h, balls):
    """Union of balls: the same classes in any ball order; one ball alone reduces to classify_ball; by
    sampling, a point strictly inside some ball makes a cell active, and an inside cell lies in one
    ball as a whole (its corners, hence the cell, within that ball's radius)."""
    d = len(n)
    cls = mesh.classify_balls(n, lo, h, balls)
    np.testing.assert_array_equal(cls, mesh.classify_balls(n, lo, h, balls[::-1]))
    np.testing.assert_array_equal(mesh.classify_balls(n, lo, h, balls[:1]),
                                  mesh.classify_ball(n, lo, h, balls[0][:d], balls[0][3]))
    assert np.sum(cls == mesh.CUT) > 0 and np.sum(cls == mesh.INSIDE) > 0
    s = (np.arange(7) + 0.5) / 7
    grid = np.stack(np.meshgrid(*[s] * d, indexing="ij"), -1).reshape(-1, d)
    corners = np.stack(np.meshgrid(*[[0.0, 1.0]] * d, indexing="ij"), -1).reshape(-1, d)
    for c in np.ndindex(*n):
        x = np.array(lo) + (np.array(c) + grid) * h
        xc = np.array(lo) + (np.array(c) + corners) * h
        r = np.stack([np.linalg.norm(x - np.array(b[:d]), axis=1) for b in balls])
        rc = np.stack([np.linalg.norm(xc - np.array(b[:d]), axis=1) for b in balls])
        radii = np.array([b[3] for b in balls])[:, None]
        if np.any(r < radii):
            assert cls[c] != mesh.OUTSIDE
        if cls[c] == mesh.INSIDE:
            assert np.any(np.all(rc <= radii, axis=1))
        else:
            assert not np.any(np.all(rc <= radii, axis=1))


def test_union_cell_covered_only_jointly_is_cut():
    """The reading for unions: the cell [0,1]^2 lies in the union of two balls (every point of it is
    within 0.71 of one centre) but in neither ball alone, and is classified cut."""
    cls = mesh.classify_balls((1, 1), (0.0, 0.0), 1.0, [(0.0, 0.5, 0.0, 0.8), (1.0, 0.5, 0.0, 0.8)])
    assert cls[0, 0] == mesh.CUT


def _gamma(k, h):
    return [0.5 * h ** (2 * j - 1) / math.factorial(j) ** 2 for j in range(1, k + 1)]


def _small_op(k=2):
    n, lo, h, centre, radius = (8, 8, 8), (-1.0,) * 3, 0.25, (0.011, 0.017, 0.023), 0.73
    return GhostOracle(3, n, lo, h, k, _gamma(k, h), centre=centre, radius=radius, per_face=True)


def test_gradients_by_central_differences():
    """L = 0.5|G(gamma)u - t|^2 is quadratic in u and in gamma, so central differences are exact
    up to rounding; L(+)-L(-) is formed as sum (y+ - y-)(y+ + y- - 2t)/2 to avoid cancellation."""
    op = _small_op(2)
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, op.n_lattice)
    t = rng.uniform(-1, 1, op.n_lattice)
    _, du, dg = op.gradients(u, t)
    G = op.sparse()
    for _ in range(3):
        v = rng.uniform(-1, 1, op.n_lattice)
        eps = 1e-6
        yp, ym = G @ (u + eps * v), G @ (u - eps * v)
        fd = np.sum((yp - ym) * (yp + ym - 2 * t)) / 2 / (2 * eps)
        assert abs(fd - du @ v) <= 1e-6 * abs(du @ v)
    for j in range(op.k):
        step = 1e-6 * op.gamma[j]
        gp, gm = op.gamma.copy(), op.gamma.copy()
        gp[j] += step
        gm[j] -= step
        yp, ym = op.sparse(gamma=gp) @ u, op.sparse(gamma=gm) @ u
        fd = np.sum((yp - ym) * (yp + ym - 2 * t)) / 2 / (2 * step)
        assert abs(fd - dg[j]) <= 1e-6 * abs(dg[j])
    # the vjp form agrees with the gradient for w = G u - t
    du2, dg2 = op.vjp(u, G @ u - t)
    np.testing.assert_allclose(du2, du, rtol=0, atol=1e-14 * np.max(np.abs(du)))
    np.testing.assert_allclose(dg2, dg, rtol=1e-12)


def test_order_matrices_sum_to_operator():
    op = _small_op(3)
    G = op.sparse()
    S = sum(g * Gj for g, Gj in zip(op.gamma, op.order_matrices()))
    assert abs(G - S).max() <= 1e-13 * abs(G).max()


def test_lumped_mass():
    """Sum of the lumped mass = measure of the active cells (GLL weights sum to 1); an interior
    node of an active cell carries h^d prod w; inactive nodes carry 0."""
    op = _small_op(3)
    m = op.lumped_mass()
    n_active = int(np.sum(op.cls != mesh.OUTSIDE))
    assert abs(m.sum() - n_active * op.h ** 3) <= 1e-13 * m.sum()
    w = [float(x) for x in basis.gll_weights(3)]
    c = np.argwhere(op.cls != mesh.OUTSIDE)[0]
    I = 3 * c + 1
    L = op.L
    assert abs(m[I[0] + L[0] * I[1] + L[0] * L[1] * I[2]] - op.h ** 3 * w[1] ** 3) < 1e-16
    # support of the ghost penalty lies inside the active nodes
    sup = op.support()
    assert np.all(m[sup] > 0)


def test_cg_reference_solves_system():
    op = _small_op(2)
    A, active = op.system()
    b = np.random.default_rng(3).uniform(-1, 1, len(active))
    x, it, res = cg_reference(A, b, tol=1e-10)
    assert res <= 1e-10 and it > 0
    xs = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(b - A @ xs) / np.linalg.norm(b) <= 1e-10
    # A is symmetric positive definite on the active nodes
    Ad = A.toarray()
    assert np.max(np.abs(Ad - Ad.T)) <= 1e-15 * np.max(np.abs(Ad))
    assert np.linalg.eigvalsh(Ad).min() > 0


def test_planted_mistakes_are_caught(monkeypatch):
    """Mutation check of the pins: a sign error in one derivative order or a wrong tangential
    weight makes the closed-form energy of a single face wrong."""
    k, h = 3, 0.25
    gamma = _gamma(k, h)
    xi = np.array([float(x) for x in basis.gll_nodes(k)])
    xs = np.concatenate([xi, 1 + xi[1:]]) * h            # normal coordinates, face at h
    tq = np.polynomial.Polynomial([0.3, -0.2, 0.5, 0.1])
    ty = tq(xi * h)

    def energy(m):
        G = patch.patch_matrix(2, k, 0, [0, 0], [0.0, 0.0], h, gamma)
        u = np.outer(ty, np.maximum(xs - h, 0) ** m).ravel()  # x fastest
        q = (tq * tq).integ()
        return u @ G @ u, gamma[m - 1] * math.factorial(m) ** 2 * (q(h) - q(0))

    for m in range(1, k + 1):
        got, want = energy(m)
        assert abs(got - want) <= 1e-12 * abs(want)

    orig = patch.normal_jumps
    monkeypatch.setattr(patch, "normal_jumps",
                        lambda *a: [[-v for v in r] if i == 1 else r for i, r in enumerate(orig(*a))])
    got, want = energy(2)   # sign flip is invisible in g g^T ...
    assert abs(got - want) <= 1e-12 * abs(want)
    monkeypatch.setattr(patch, "normal_jumps",
                        lambda *a: [[2 * v for v in r] if i == 1 else r for i, r in enumerate(orig(*a))])
    got, want = energy(2)   # ... but a scale error is not
    assert abs(got - want) > 1e-3 * abs(want)
    monkeypatch.setattr(patch, "normal_jumps", orig)
    origt = patch.tangential_values
    monkeypatch.setattr(patch, "tangential_values", lambda *a: (origt(*a)[0], origt(*a)[1][::-1] * 1.01))
    got, want = energy(1)
    assert abs(got - want) > 1e-3 * abs(want)
