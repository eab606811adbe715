"""Exact-rational 1D B-spline integrals -- TEST INFRASTRUCTURE ONLY.

Independent of the floating-point oracle and of any quadrature rule: every
basis function is built as an exact piecewise polynomial (coefficients are
``fractions.Fraction``) by running the Cox--de Boor recursion of Sec. 2.3,
eqs. (cox1)/(cox2) (0/0 := 0), symbolically in x on each knot span.
Derivatives are taken by differentiating those polynomials (not by the
B-spline derivative formula the floating-point oracle uses), and integrals
are taken from exact antiderivatives.

For a separable coefficient kappa(x, y, z) = rx(x) ry(y) rz(z) the global
mass and stiffness matrices of the tensor-product basis (eq. (basis_construction),
x-fastest global numbering) are Kronecker products of 1D matrices::

    M = Mz (x) My (x) Mx
    K = Mz (x) My (x) Ax + Mz (x) Ay (x) Mx + Az (x) My (x) Mx

with M_d[i][j] = int r_d N_i N_j and A_d[i][j] = int r_d N_i' N_j'.  The
tests use this to pin the oracle's element integration and assembly.
"""
from fractions import Fraction

# --- polynomials as coefficient lists, lowest degree first ----------------


def padd(a, b):
    n = max(len(a), len(b))
    return [(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)]


def pmul(a, b):
    if not a or not b:
        return []
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x == 0:
            continue
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def pscale(a, s):
    return [s * x for x in a]


def pderiv(a):
    return [i * a[i] for i in range(1, len(a))]


def pint(a, lo, hi):
    """Exact integral of polynomial a over [lo, hi]."""
    tot = Fraction(0)
    for i, c in enumerate(a):
        tot += c * (Fraction(hi) ** (i + 1) - Fraction(lo) ** (i + 1)) / (i + 1)
    return tot


def peval(a, x):
    return sum(c * Fraction(x) ** i for i, c in enumerate(a))


# --- knots and basis --------------------------------------------------------


def open_uniform_knots(K, p):
    """Open knot vector of eq. (knot_vector) on [0,1] with K uniform elements:
    p+1 zeros, interior knots k/K, p+1 ones (K+2p+1 knots)."""
    return [Fraction(0)] * (p + 1) + [Fraction(k, K) for k in range(1, K)] + [Fraction(1)] * (p + 1)


def basis_on_spans(t, p):
    """Piecewise polynomials of the K+p B-splines of degree p.

    Returns (spans, B) where spans is the list of non-empty spans (lo, hi)
    and B[i][s] is the polynomial of function i on span s."""
    t = [Fraction(x) for x in t]
    nk = len(t)
    spans = [(i, t[i], t[i + 1]) for i in range(nk - 1) if t[i] < t[i + 1]]
    out = []
    for (si, lo, hi) in spans:
        # degree 0: indicator of [t_i, t_{i+1}) on this span
        b = [[Fraction(1)] if i == si else [] for i in range(nk - 1)]
        for q in range(1, p + 1):
            nb = []
            for i in range(nk - 1 - q):
                term = []
                dl = t[i + q] - t[i]
                if dl != 0 and b[i]:
                    term = padd(term, pmul([-t[i] / dl, 1 / dl], b[i]))
                dr = t[i + q + 1] - t[i + 1]
                if dr != 0 and b[i + 1]:
                    term = padd(term, pmul([t[i + q + 1] / dr, -1 / dr], b[i + 1]))
                nb.append(term)
            b = nb
        out.append(b)
    nbasis = nk - p - 1
    B = [[out[s][i] for s in range(len(spans))] for i in range(nbasis)]
    return [(lo, hi) for (_, lo, hi) in spans], B


def matrices_1d(t, p, weight=(Fraction(1),)):
    """Exact 1D mass M[i][j] = int w N_i N_j and stiffness A[i][j] = int w N_i' N_j'
    over the whole knot range, for a polynomial weight w (coefficient list)."""
    spans, B = basis_on_spans(t, p)
    w = [Fraction(c) for c in weight]
    n = len(B)
    M = [[Fraction(0)] * n for _ in range(n)]
    A = [[Fraction(0)] * n for _ in range(n)]
    for s, (lo, hi) in enumerate(spans):
        for i in range(n):
            bi = B[i][s]
            if not bi:
                continue
            dbi = pderiv(bi)
            for j in range(n):
                bj = B[j][s]
                if not bj:
                    continue
                M[i][j] += pint(pmul(w, pmul(bi, bj)), lo, hi)
                A[i][j] += pint(pmul(w, pmul(dbi, pderiv(bj))), lo, hi)
    return M, A


def mixed_1d(t, p, weight=(Fraction(1),)):
    """Exact 1D B[i][j] = int w N_i' N_j (derivative on the first index only),
    the factor a cross term d/dx_c d/dx_d (c != d) of a mapped-geometry
    stiffness leaves in each of its two directions."""
    spans, B = basis_on_spans(t, p)
    w = [Fraction(c) for c in weight]
    n = len(B)
    out = [[Fraction(0)] * n for _ in range(n)]
    for s, (lo, hi) in enumerate(spans):
        for i in range(n):
            if not B[i][s]:
                continue
            dbi = pderiv(B[i][s])
            for j in range(n):
                if B[j][s]:
                    out[i][j] += pint(pmul(w, pmul(dbi, B[j][s])), lo, hi)
    return out


def basis_values(t, p, x):
    """Exact values and derivatives of all basis functions at x (x inside
    [t_0, t_end]; the right end uses the last non-empty span)."""
    spans, B = basis_on_spans(t, p)
    x = Fraction(x)
    s = None
    for k, (lo, hi) in enumerate(spans):
        if lo <= x < hi:
            s = k
            break
    if s is None:
        s = len(spans) - 1
    vals = [peval(B[i][s], x) if B[i][s] else Fraction(0) for i in range(len(B))]
    ders = [peval(pderiv(B[i][s]), x) if B[i][s] else Fraction(0) for i in range(len(B))]
    return vals, ders


def greville(t, p):
    """Greville abscissae xi*_i = (t_{i+1} + ... + t_{i+p}) / p."""
    t = [Fraction(x) for x in t]
    return [sum(t[i + 1:i + p + 1]) / p for i in range(len(t) - p - 1)]
