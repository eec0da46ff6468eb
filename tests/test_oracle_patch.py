"""Pins of the oracle's patch matrices and global operator.

* Kronecker form of §2.4 (G_{F,k} = M^h (x) M^h (x) G^h_k, with the penalty
  factor in the position of the normal axis) against the quadrature assembly.
* Symmetry, positive semi-definiteness, translation invariance, h-scaling.
* Closed-form energies: for u = (x_n - x_F)_+^m q(tangential), the only
  nonzero jump is the m-th normal derivative on the plane x_n = x_F, equal to
  m! q, so u^T G u = gamma_m (m!)^2 * sum over set faces on that plane of the
  face integral of q^2.
* Null space: G p = 0 for every p in Q_k (§2.2: the penalty glues the two
  cells into one polynomial).
"""

import math

import numpy as np
import pytest

from oracle import basis, mesh, patch
from oracle.operator import GhostOracle


def _ref_tables(k):
    J = patch.jump_vectors_reference(k)
    g = np.array([[float(v) for v in J[j]] for j in range(1, k + 1)])
    M = np.array([[float(v) for v in r] for r in patch.mass_reference(k)])
    return g, M


def _kron_form(d, k, axis, h, gamma):
    g, M = _ref_tables(k)
    total = 0
    for j in range(1, k + 1):
        P = np.outer(g[j - 1], g[j - 1])
        factors = [P if a == axis else M for a in reversed(range(d))]  # slowest axis leftmost
        K = factors[0]
        for f in factors[1:]:
            K = np.kron(K, f)
        total = total + gamma[j - 1] * h ** (d - 1 - 2 * j) * K
    return total


def _gamma(k, h):
    return [0.5 * h ** (2 * j - 1) / math.factorial(j) ** 2 for j in range(1, k + 1)]


def test_fig2_numbering():
    """2D, k=2, face normal to x: patch index = i_x + 5 i_y (Fig. 2)."""
    loc = mesh.patch_local_nodes(2, 2, 0)
    assert loc.shape == (15, 2)
    for p in range(15):
        assert tuple(loc[p]) == (p % 5, p // 5)
    # and its lattice indices for the face above cell (1, 2) on a 4x4 mesh (L = 9)
    idx = mesh.patch_dofs(np.array([[1, 2]]), 2, 0, (9, 9))[0]
    assert idx[0] == 2 + 9 * 4 and idx[4] == 6 + 9 * 4 and idx[5] == 2 + 9 * 5


@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (2, 3), (2, 5), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_kronecker_form(d, k):
    h = 0.125
    gamma = _gamma(k, h)
    for axis in range(d):
        cell = [3] * d
        G = patch.patch_matrix(d, k, axis, cell, [-1.0] * d, h, gamma)
        K = _kron_form(d, k, axis, h, gamma)
        assert np.max(np.abs(G - K)) <= 1e-13 * np.max(np.abs(K))


@pytest.mark.parametrize("d,k", [(2, 3), (3, 2), (3, 3)])
def test_symmetric_psd_and_translation_invariant(d, k):
    h = 2 / 24
    gamma = _gamma(k, h)
    for axis in range(d):
        G0 = patch.patch_matrix(d, k, axis, [0] * d, [-1.0] * d, h, gamma)
        G1 = patch.patch_matrix(d, k, axis, [17, 5, 11][:d], [-1.0] * d, h, gamma)
        s = np.max(np.abs(G0))
        assert np.max(np.abs(G0 - G0.T)) <= 1e-14 * s
        assert np.max(np.abs(G0 - G1)) <= 1e-13 * s
        ev = np.linalg.eigvalsh(G0)
        assert ev.min() >= -1e-13 * ev.max()
        assert np.sum(ev > 1e-10 * ev.max()) == k * (k + 1) ** (d - 1)


@pytest.mark.parametrize("d", [2, 3])
def test_h_scaling(d):
    """At fixed reference coefficients gamma_j h^{1-2j}, G_F scales as h^{d-2}."""
    k = 3
    ghat = [0.5 / math.factorial(j) ** 2 for j in range(1, k + 1)]
    mats = []
    for h in (1.0, 0.25):
        gamma = [gj * h ** (2 * j - 1) for j, gj in zip(range(1, k + 1), ghat)]
        mats.append(patch.patch_matrix(d, k, d - 1, [2] * d, [0.5] * d, h, gamma))
    ratio = 0.25 ** (d - 2)
    assert np.max(np.abs(mats[1] - ratio * mats[0])) <= 1e-12 * np.max(np.abs(mats[1]))


def _node_coords(n, lo, h, k):
    xi = np.array([float(x) for x in basis.gll_nodes(k)])
    out = []
    for a in range(len(n)):
        I = np.arange(k * n[a] + 1)
        c = np.minimum(I // k, n[a] - 1)
        i = I - k * c
        out.append(lo[a] + h * (c + xi[i]))
    return out


def _lattice_field(coords, factors):
    """Values of prod_a f_a(x_a) on the lattice, x fastest."""
    val = np.ones([len(c) for c in reversed(coords)])
    d = len(coords)
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = len(coords[a])
        val = val * factors[a](coords[a]).reshape(shape)
    return val.ravel()


CASES = [
    (2, 2, (12, 12), (-1.0, -1.0), 2 / 12, (0.013, 0.021), 0.71),
    (2, 3, (10, 9), (-1.0, -0.9), 0.2, (0.05, 0.02), 0.737),
    (3, 2, (6, 6, 6), (-1.0, -1.0, -1.0), 2 / 6, (0.011, 0.017, 0.023), 0.73),
]


@pytest.mark.parametrize("d,k,n,lo,h,centre,radius", CASES)
def test_closed_form_energy(d, k, n, lo, h, centre, radius):
    """Per face on the plane x_n = x_F: u_F^T G_F u_F = gamma_m (m!)^2 prod_t int q_t^2,
    u_F^T G_F v_F = 0 between orders, and G u vanishes away from that plane's patches."""
    gamma = _gamma(k, h)
    op = GhostOracle(d, n, lo, h, k, gamma, centre=centre, radius=radius, per_face=True)
    G = op.sparse()
    coords = _node_coords(n, lo, h, k)
    rng = np.random.default_rng(7)
    for axis in range(d):
        faces = op.faces[axis]
        assert len(faces) > 0
        plane = int(np.bincount(faces[:, axis]).argmax()) + 1  # busiest face plane
        xF = lo[axis] + plane * h
        sel = np.nonzero(faces[:, axis] == plane - 1)[0]
        idx = op.patch_dofs(axis)
        mats = op.face_matrices(axis)
        near = np.zeros(op.n_lattice, dtype=bool)
        near[idx[sel].ravel()] = True
        polys = {a: np.polynomial.Polynomial(rng.uniform(-1, 1, k + 1)) for a in range(d) if a != axis}
        fields = {}
        for m in range(1, k + 1):
            fac = {axis: (lambda x, m=m: np.maximum(x - xF, 0.0) ** m)}
            fac.update({a: (lambda x, p=p: p(x)) for a, p in polys.items()})
            fields[m] = _lattice_field(coords, [fac[a] for a in range(d)])
        for m in range(1, k + 1):
            u = fields[m]
            for i in sel:
                f, GF, uF = faces[i], mats[i], u[idx[i]]
                want = gamma[m - 1] * math.factorial(m) ** 2
                for a, p in polys.items():
                    q = (p * p).integ()
                    x0 = lo[a] + f[a] * h
                    want *= q(x0 + h) - q(x0)
                got = uF @ GF @ uF
                # rounding bound eps*|u|^T|G||u|; the pin sits far above it, so a
                # dropped or mis-scaled term cannot hide in the tolerance
                scale = np.abs(uF) @ np.abs(GF) @ np.abs(uF)
                assert abs(want) > 1e-6 * scale
                assert abs(got - want) <= 1e-13 * scale, (axis, m, got, want, scale)
                for m2 in range(1, m):
                    vF = fields[m2][idx[i]]
                    assert abs(vF @ GF @ uF) <= 1e-13 * (np.abs(vF) @ np.abs(GF) @ np.abs(uF))
            # globally, only the patches on the plane see a jump
            y = G @ u
            assert np.max(np.abs(y[~near])) <= 1e-12 * np.max(np.abs(G) @ np.abs(u))
            assert np.max(np.abs(y[near])) > 1e-6 * np.max(np.abs(G) @ np.abs(u))


@pytest.mark.parametrize("d,k,n,lo,h,centre,radius", CASES)
def test_global_null_space_symmetry_psd(d, k, n, lo, h, centre, radius):
    op = GhostOracle(d, n, lo, h, k, _gamma(k, h), centre=centre, radius=radius, per_face=True)
    G = op.sparse()
    coords = _node_coords(n, lo, h, k)
    rng = np.random.default_rng(3)
    polys = [np.polynomial.Polynomial(rng.uniform(-1, 1, k + 1)) for _ in range(d)]
    p = _lattice_field(coords, polys)
    r = rng.uniform(-1, 1, p.size) * np.max(np.abs(p))
    assert np.max(np.abs(G @ p)) <= 1e-12 * np.max(np.abs(G @ r))
    # oracle apply agrees with its own assembled matrix
    np.testing.assert_allclose(op.apply(r), G @ r, rtol=0, atol=1e-13 * np.max(np.abs(G @ r)))
    if p.size <= 3000:
        D = G.toarray()
        assert np.max(np.abs(D - D.T)) <= 1e-14 * np.max(np.abs(D))
        ev = np.linalg.eigvalsh(D)
        assert ev.min() >= -1e-12 * ev.max()


def test_per_axis_cache_matches_per_face():
    d, k, n, lo, h, centre, radius = CASES[2]
    a = GhostOracle(d, n, lo, h, k, _gamma(k, h), centre=centre, radius=radius, per_face=True)
    b = GhostOracle(d, n, lo, h, k, _gamma(k, h), centre=centre, radius=radius, per_face=False)
    u = np.random.default_rng(1).uniform(-1, 1, a.n_lattice)
    ya, yb = a.apply(u), b.apply(u)
    assert np.max(np.abs(ya - yb)) <= 1e-13 * np.max(np.abs(ya))
    sup = a.support()
    sel = sup[::7]
    np.testing.assert_allclose(b.apply_at(u, sel), ya[sel], rtol=0, atol=1e-13 * np.max(np.abs(ya)))
    off = np.setdiff1d(np.arange(a.n_lattice), sup)
    assert np.all(ya[off] == 0)
