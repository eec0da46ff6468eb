"""Pins of the oracle's macro-patch stabilisation (oracle.macro).

* 1D closed forms on the two-cell patch [x_F - h, x_F + h]:
  - a field that vanishes on the lower cell and equals -(x - x_F)^m on the upper cell (m = 1..k) has the
    extension difference (x - x_F)^m, so the 1D matrix's Gram values between two such fields are
    integral over [-h, h] of t^{m+m'} dt;
  - every polynomial of degree <= k on the whole patch is in the null space.
  These two sets span the 2k+1 patch functions, so together they fix every entry.
  Hand values: k = 1 gives (2h/3) v v^T with v = (-1, 2, -1); at k = 2 and h = 1, entry [0, 0] is
  34/15 (the lower-cell function of node 0 is 2(x - 1/2)(x - 1), whose square integrated over
  [0, 2] is 4 * (2/5 + 1/6)).
* The d-dimensional assembly equals the Kronecker form: the 1D patch matrix along the normal and the
  exact tangential mass h M on the other axes.  Symmetric, PSD, of rank k (k+1)^{d-1}, translation
  invariant, scaling as h^{d-2} at fixed gamma_M.
* At k = 1 it equals the derivative-jump form with gamma_1 = 2 gamma_M h / 3.  That is an independent
  assembly from another definition: one derivative order, whose jump fixes the linear extension
  difference.
* Global operator: G p = 0 for every p in Q_k; symmetric PSD; the gradient in gamma_M.
"""


import numpy as np
import pytest

from oracle import basis, patch
from oracle.macro import macro_matrix_1d, macro_patch_matrix
from oracle.operator import GhostOracle


def _patch_nodes_1d(k, c, h):
    xi = [float(x) for x in basis.gll_nodes(k)]
    return np.array([c + h * x for x in xi] + [c + h + h * x for x in xi[1:]])


@pytest.mark.parametrize("c,h", [(0.0, 1.0), (-0.7, 0.3)])
def test_k1_closed_form(c, h):
    v = np.array([-1.0, 2.0, -1.0])
    S = macro_matrix_1d(1, c, h)
    np.testing.assert_allclose(S, 2 * h / 3 * np.outer(v, v), rtol=0, atol=1e-15)


def test_k2_hand_entry():
    assert abs(macro_matrix_1d(2, 0.0, 1.0)[0, 0] - 34 / 15) <= 1e-15


@pytest.mark.parametrize("k", range(1, 8))
@pytest.mark.parametrize("c,h", [(0.0, 1.0), (-0.55, 0.125)])
def test_1d_gram_and_null_space(k, c, h):
    S = macro_matrix_1d(k, c, h)
    x = _patch_nodes_1d(k, c, h)
    xF = c + h
    t = x - xF
    scale = np.max(np.abs(S))
    # null space: polynomials of degree <= k on the whole patch
    for m in range(k + 1):
        assert np.max(np.abs(S @ t ** m)) <= 2e-13 * scale * max(1.0, h ** m) * len(x)
    # range: zero on the lower cell, -(x - x_F)^m on the upper one
    fields = [np.where(np.arange(2 * k + 1) <= k, 0.0, -t ** m) for m in range(1, k + 1)]
    for i, u in enumerate(fields, start=1):
        for j, w in enumerate(fields, start=1):
            p = i + j
            want = 0.0 if p % 2 else 2 * h ** (p + 1) / (p + 1)
            got = u @ S @ w
            bound = 1e-13 * (np.abs(u) @ np.abs(S) @ np.abs(w))
            assert abs(got - want) <= bound, (i, j, got, want)
            if p % 2 == 0:
                assert want > 1e3 * bound


def _ref_mass(k):
    return np.array([[float(v) for v in r] for r in patch.mass_reference(k)])


@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (2, 4), (3, 1), (3, 2), (3, 3)])
def test_kronecker_form(d, k):
    h, gm = 0.125, 0.8
    lo = [-1.0] * d
    for axis in range(d):
        cell = [3, 5, 2][:d]
        S = macro_patch_matrix(d, k, axis, cell, lo, h, [gm])
        c = lo[axis] + cell[axis] * h
        factors = [macro_matrix_1d(k, c, h) if a == axis else h * _ref_mass(k) for a in reversed(range(d))]
        K = factors[0]
        for f in factors[1:]:
            K = np.kron(K, f)
        K = gm / h ** 2 * K
        assert np.max(np.abs(S - K)) <= 1e-13 * np.max(np.abs(K))


@pytest.mark.parametrize("d,k", [(2, 3), (3, 2), (3, 4)])
def test_symmetric_psd_rank_translation(d, k):
    h = 2 / 24
    for axis in range(d):
        S0 = macro_patch_matrix(d, k, axis, [0] * d, [-1.0] * d, h, [1.0])
        S1 = macro_patch_matrix(d, k, axis, [17, 5, 11][:d], [-1.0] * d, h, [1.0])
        s = np.max(np.abs(S0))
        assert np.max(np.abs(S0 - S0.T)) <= 1e-14 * s
        assert np.max(np.abs(S0 - S1)) <= 1e-13 * s
        ev = np.linalg.eigvalsh(S0)
        assert ev.min() >= -1e-13 * ev.max()
        assert np.sum(ev > 1e-10 * ev.max()) == k * (k + 1) ** (d - 1)


@pytest.mark.parametrize("d", [2, 3])
def test_h_scaling(d):
    k = 3
    mats = [macro_patch_matrix(d, k, d - 1, [2] * d, [0.5] * d, h, [0.7]) for h in (1.0, 0.25)]
    assert np.max(np.abs(mats[1] - 0.25 ** (d - 2) * mats[0])) <= 1e-12 * np.max(np.abs(mats[1]))


@pytest.mark.parametrize("d", [2, 3])
def test_k1_equals_derivative_form(d):
    h, gm = 0.2, 1.3
    for axis in range(d):
        S = macro_patch_matrix(d, 1, axis, [1, 2, 3][:d], [-0.4] * d, h, [gm])
        G = patch.patch_matrix(d, 1, axis, [1, 2, 3][:d], [-0.4] * d, h, [2 * gm * h / 3])
        assert np.max(np.abs(S - G)) <= 1e-14 * np.max(np.abs(G))


def _lattice_poly(n, lo, h, k, polys):
    xi = np.array([float(x) for x in basis.gll_nodes(k)])
    val = np.ones([k * m + 1 for m in reversed(n)])
    d = len(n)
    for a in range(d):
        I = np.arange(k * n[a] + 1)
        c = np.minimum(I // k, n[a] - 1)
        x = lo[a] + h * (c + xi[I - k * c])
        shape = [1] * d
        shape[d - 1 - a] = len(x)
        val = val * polys[a](x).reshape(shape)
    return val.ravel()


@pytest.mark.parametrize("d,k,n,h", [(2, 3, (10, 9), 0.2), (3, 2, (6, 6, 6), 2 / 6)])
def test_global_null_space_symmetry_psd(d, k, n, h):
    lo = (-1.0,) * d
    centre = (0.05, 0.02, 0.03)[:d]
    op = GhostOracle(d, n, lo, h, k, [0.9], centre=centre, radius=0.71, per_face=True, penalty="macro")
    assert op.n_faces() > 0
    G = op.sparse()
    rng = np.random.default_rng(3)
    p = _lattice_poly(n, lo, h, k, [np.polynomial.Polynomial(rng.uniform(-1, 1, k + 1)) for _ in range(d)])
    r = rng.uniform(-1, 1, p.size) * np.max(np.abs(p))
    assert np.max(np.abs(G @ p)) <= 1e-12 * np.max(np.abs(G @ r))
    np.testing.assert_allclose(op.apply(r), G @ r, rtol=0, atol=1e-13 * np.max(np.abs(G @ r)))
    D = G.toarray()
    assert np.max(np.abs(D - D.T)) <= 1e-14 * np.max(np.abs(D))
    ev = np.linalg.eigvalsh(D)
    assert ev.min() >= -1e-12 * ev.max()


def test_gradient_in_gamma():
    d, k, n, h = 2, 2, (8, 8), 0.25
    args = dict(centre=(0.03, 0.01), radius=0.66, per_face=True, penalty="macro")
    op = GhostOracle(d, n, (-1.0, -1.0), h, k, [0.6], **args)
    rng = np.random.default_rng(5)
    u, t = rng.uniform(-1, 1, op.n_lattice), rng.uniform(-1, 1, op.n_lattice)
    L, du, dg = op.gradients(u, t)
    assert dg.shape == (1,)
    step = 1e-3
    Lp = GhostOracle(d, n, (-1.0, -1.0), h, k, [0.6 + step], **args).gradients(u, t)[0]
    Lm = GhostOracle(d, n, (-1.0, -1.0), h, k, [0.6 - step], **args).gradients(u, t)[0]
    # L is quadratic in gamma_M: the central difference is exact up to rounding
    assert abs((Lp - Lm) / (2 * step) - dg[0]) <= 1e-9 * abs(dg[0])


def test_bad_arguments():
    with pytest.raises(ValueError):
        macro_patch_matrix(2, 2, 0, [0, 0], [0.0, 0.0], 0.5, [1.0, 2.0])
    with pytest.raises(ValueError):
        GhostOracle(2, (4, 4), (-1.0, -1.0), 0.5, 2, [1.0, 1.0], centre=(0, 0), radius=0.6, penalty="macro")
    with pytest.raises(ValueError):
        GhostOracle(2, (4, 4), (-1.0, -1.0), 0.5, 2, [1.0], centre=(0, 0), radius=0.6, penalty="volume")
