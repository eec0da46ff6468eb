"""1D building blocks of the Q_k basis, in 60-digit mpmath.  Test infrastructure only.

The paper uses Lagrange elements of order k on a Cartesian mesh (§2) with the
tensor-product basis of §2.4 (eq. tensor_product).  The node family is not
fixed by the paper; the workloads use Gauss-Lobatto-Legendre (GLL) nodes.

Polynomials are lists of mpmath numbers, coefficient of x^m at position m.
"""

from fractions import Fraction

import mpmath

mpmath.mp.dps = 60


def legendre_coeffs(n):
    """Monomial coefficients (exact rationals) of the Legendre polynomial P_n on [-1, 1].

    Bonnet recurrence (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}.
    """
    p_prev, p = [Fraction(1)], [Fraction(0), Fraction(1)]
    if n == 0:
        return p_prev
    for m in range(1, n):
        nxt = [Fraction(0)] * (m + 2)
        for i, c in enumerate(p):
            nxt[i + 1] += Fraction(2 * m + 1, m + 1) * c
        for i, c in enumerate(p_prev):
            nxt[i] -= Fraction(m, m + 1) * c
        p_prev, p = p, nxt
    return p


def poly_deriv(c, j=1):
    """Coefficients of the j-th derivative of the polynomial with coefficients c."""
    c = list(c)
    for _ in range(j):
        c = [m * c[m] for m in range(1, len(c))] or [mpmath.mpf(0)]
    return c


def poly_eval(c, x):
    """Horner evaluation of the polynomial c at x (mpmath)."""
    acc = mpmath.mpf(0)
    for coef in reversed(c):
        acc = acc * x + coef
    return acc


def poly_mul(a, b):
    out = [mpmath.mpf(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _real_roots(coeffs):
    """Real roots, ascending, of a polynomial given by low-to-high coefficients."""
    hi_to_lo = [mpmath.mpf(c.numerator) / c.denominator for c in reversed(coeffs)]
    roots = mpmath.polyroots(hi_to_lo, maxsteps=400, extraprec=400)
    return sorted(mpmath.re(r) for r in roots)


def gll_nodes(k):
    """GLL nodes on [0, 1] for degree k: the endpoints and the roots of P_k' mapped from [-1, 1]."""
    if k < 1:
        raise ValueError("k >= 1")
    interior = []
    if k >= 2:
        dp = [Fraction(m) * c for m, c in enumerate(legendre_coeffs(k))][1:]
        interior = _real_roots(dp)
    xs = [mpmath.mpf(-1)] + interior + [mpmath.mpf(1)]
    return [(x + 1) / 2 for x in xs]


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [0, 1]: (points, weights), exact for degree 2n-1."""
    pc = legendre_coeffs(n)
    roots = _real_roots(pc)
    dpc = [mpmath.mpf(m * c.numerator) / c.denominator for m, c in enumerate(pc)][1:]
    pts, wts = [], []
    for x in roots:
        dp = poly_eval(dpc, x)
        w = 2 / ((1 - x * x) * dp * dp)
        pts.append((x + 1) / 2)
        wts.append(w / 2)
    return pts, wts


def lagrange_polys(nodes):
    """Monomial coefficients of the Lagrange polynomials l_i with l_i(nodes[m]) = delta_im."""
    polys = []
    for i, xi in enumerate(nodes):
        c = [mpmath.mpf(1)]
        for m, xm in enumerate(nodes):
            if m == i:
                continue
            c = poly_mul(c, [-xm / (xi - xm), 1 / (xi - xm)])
        polys.append(c)
    return polys


def physical_lagrange(k, a, h):
    """Lagrange basis of one cell [a, a+h] in the physical coordinate x.

    The nodes are a + h * xi_m with xi_m the GLL nodes; the polynomials are expanded
    directly in x, so derivatives are taken in physical coordinates without any
    chain-rule factor.
    """
    a, h = mpmath.mpf(a), mpmath.mpf(h)
    return lagrange_polys([a + h * xi for xi in gll_nodes(k)])


def gll_weights(k):
    """Weights of the GLL quadrature on [0, 1]: w_i = integral over [0, 1] of l_i.

    This is the definition of an interpolatory rule on the GLL nodes.
    """
    out = []
    for c in lagrange_polys(gll_nodes(k)):
        out.append(sum(coef / (m + 1) for m, coef in enumerate(c)))
    return out
