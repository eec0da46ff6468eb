"""Pins of the oracle's 1D quantities against closed forms and exact identities."""

import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import basis, patch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def _ev(expr):
    return eval(expr, {"sqrt": math.sqrt})


@pytest.mark.parametrize("row", list(_rows("gll_nodes_weights.txt")))
def test_gll_closed_forms(row):
    k, nodes, weights = [s.strip() for s in row.split("|")]
    k = int(k)
    xs = [(_ev(e) + 1) / 2 for e in nodes.split(",")]
    ws = [_ev(e) / 2 for e in weights.split(",")]
    got_x = [float(x) for x in basis.gll_nodes(k)]
    got_w = [float(w) for w in basis.gll_weights(k)]
    np.testing.assert_allclose(got_x, xs, rtol=0, atol=1e-15)
    np.testing.assert_allclose(got_w, ws, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", range(1, 8))
def test_gll_rule_exactness(k):
    """The GLL rule integrates x^m exactly on [0, 1] for m <= 2k-1, and not for m = 2k."""
    xs, ws = basis.gll_nodes(k), basis.gll_weights(k)
    for m in range(2 * k):
        q = sum(w * x ** m for x, w in zip(xs, ws))
        assert abs(q - mpmath.mpf(1) / (m + 1)) < mpmath.mpf(10) ** -50
    q = sum(w * x ** (2 * k) for x, w in zip(xs, ws))
    assert abs(q - mpmath.mpf(1) / (2 * k + 1)) > 1e-30


@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_rule_exactness(n):
    xs, ws = basis.gauss_legendre(n)
    for m in range(2 * n):
        q = sum(w * x ** m for x, w in zip(xs, ws))
        assert abs(q - mpmath.mpf(1) / (m + 1)) < mpmath.mpf(10) ** -50
    np.testing.assert_allclose(sorted(float(x) for x in xs),
                               (np.polynomial.legendre.leggauss(n)[0] + 1) / 2, atol=1e-15)


@pytest.mark.parametrize("k", range(1, 8))
def test_lagrange_cardinal_and_partition(k):
    nodes = basis.gll_nodes(k)
    polys = basis.lagrange_polys(nodes)
    for i, c in enumerate(polys):
        for m, x in enumerate(nodes):
            assert abs(basis.poly_eval(c, x) - (1 if i == m else 0)) < 1e-50
    total = [sum(c[m] for c in polys) for m in range(k + 1)]
    assert abs(total[0] - 1) < 1e-45 and all(abs(t) < 1e-45 for t in total[1:])


def test_reference_jumps_golden():
    for row in _rows("reference_jumps.txt"):
        head, vals = row.split("|")
        k, j = map(int, head.split())
        want = [float(v) for v in vals.split()]
        got = [float(v) for v in patch.jump_vectors_reference(k)[j]]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-40)


@pytest.mark.parametrize("k", range(1, 8))
def test_reference_jumps_closed_form(k):
    """On the reference patch [0,2] with the face at 1:

    * order 0 vanishes (continuity);
    * every order annihilates a global polynomial of degree <= k;
    * order j applied to samples of (x-1)_+^m gives m! if j = m, else 0.
    """
    J = patch.jump_vectors_reference(k)
    nodes = basis.gll_nodes(k)
    xs = list(nodes) + [1 + x for x in nodes[1:]]  # 2k+1 patch node coordinates
    assert all(abs(v) < 1e-50 for v in J[0])
    for deg in range(k + 1):
        samples = [x ** deg for x in xs]
        for j in range(1, k + 1):
            assert abs(sum(a * b for a, b in zip(J[j], samples))) < 1e-40
    for m in range(1, k + 1):
        samples = [max(x - 1, 0) ** m for x in xs]
        for j in range(1, k + 1):
            want = math.factorial(m) if j == m else 0
            assert abs(sum(a * b for a, b in zip(J[j], samples)) - want) < 1e-40


def test_reference_mass_golden():
    for row in _rows("reference_mass.txt"):
        head, body = row.split("|")
        k, den = map(int, head.split())
        want = np.array([[float(v) for v in r.split()] for r in body.split(";")]) / den
        got = np.array([[float(v) for v in r] for r in patch.mass_reference(k)])
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-16)


@pytest.mark.parametrize("k", range(1, 8))
def test_reference_mass_integrates_products(k):
    """v^T M w equals the exact integral of p q over [0,1] for p, q of degree <= k (samples v, w)."""
    M = patch.mass_reference(k)
    nodes = basis.gll_nodes(k)
    for a in range(k + 1):
        for b in range(k + 1):
            v = [x ** a for x in nodes]
            w = [x ** b for x in nodes]
            q = sum(v[i] * M[i][j] * w[j] for i in range(k + 1) for j in range(k + 1))
            assert abs(q - Fraction(1, a + b + 1)) < 1e-45


def _penalty_1d(k):
    J = patch.jump_vectors_reference(k)
    g = np.array([[float(v) for v in J[j]] for j in range(1, k + 1)])
    gam = np.array([1.0 / math.factorial(j) ** 2 for j in range(1, k + 1)])
    return (g.T * gam) @ g


def test_penalty_eigenvalues_k2():
    """k=2: g_1 = [-1,4,-6,4,-1] and g_2 = [-4,8,0,-8,4] are orthogonal, so
    P = g_1 g_1^T + g_2 g_2^T / 4 has eigenvalues |g_1|^2 = 70 and |g_2|^2/4 = 40."""
    ev = np.sort(np.linalg.eigvalsh(_penalty_1d(2)))
    np.testing.assert_allclose(ev, [0, 0, 0, 40, 70], atol=1e-12)


@pytest.mark.parametrize("k", range(1, 8))
def test_penalty_rank_and_nullity(k):
    P = _penalty_1d(k)
    ev = np.linalg.eigvalsh(P)
    assert np.all(ev > -1e-9 * ev.max())
    assert np.sum(ev > 1e-9 * ev.max()) == k
