"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test states what it pins and why a plausible mistake in the oracle would
fail it.  No expected value here comes from the HIP path.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import exact

# ---------------------------------------------------------------- Gauss rule


def test_gauss_closed_forms(orc):
    """Textbook Gauss-Legendre nodes/weights (Abramowitz & Stegun 25.4) for q=1..5."""
    ref = {
        1: ([0.0], [2.0]),
        2: ([-1 / math.sqrt(3), 1 / math.sqrt(3)], [1.0, 1.0]),
        3: ([-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)], [5 / 9, 8 / 9, 5 / 9]),
    }
    a = math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5))
    b = math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))
    wa = (18 + math.sqrt(30)) / 36
    wb = (18 - math.sqrt(30)) / 36
    ref[4] = ([-b, -a, a, b], [wb, wa, wa, wb])
    c = math.sqrt(5 - 2 * math.sqrt(10 / 7)) / 3
    d = math.sqrt(5 + 2 * math.sqrt(10 / 7)) / 3
    wc = (322 + 13 * math.sqrt(70)) / 900
    wd = (322 - 13 * math.sqrt(70)) / 900
    ref[5] = ([-d, -c, 0.0, c, d], [wd, wc, 128 / 225, wc, wd])
    for q, (xr, wr) in ref.items():
        x, w = orc.gauss_legendre(q)
        np.testing.assert_allclose(x, xr, rtol=0, atol=4e-16)
        np.testing.assert_allclose(w, wr, rtol=0, atol=4e-16)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6, 7, 8, 10, 12])
def test_gauss_exactness(orc, q):
    """A q-point Gauss rule integrates x^m exactly on [-1,1] for m <= 2q-1,
    and not m = 2q (which tells a q-point rule from a (q+1)-point one)."""
    x, w = orc.gauss_legendre(q)
    assert np.all(np.diff(x) > 0)
    for m in range(2 * q):
        exact_val = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.dot(w, x ** m) - exact_val) < 1e-14
    assert abs(np.dot(w, x ** (2 * q)) - 2.0 / (2 * q + 1)) > 1e-10


# ---------------------------------------------------------------- Cox-de Boor


def _nonuniform_knots(K, p, seed):
    rng = np.random.default_rng(seed)
    inner = np.sort(rng.uniform(0.05, 0.95, K - 1))
    # keep them distinct and well separated
    inner = np.unique(np.round(inner, 3))
    assert len(inner) == K - 1
    return np.concatenate([[0.0] * (p + 1), inner, [1.0] * (p + 1)])


@pytest.mark.parametrize("K,p", [(1, 1), (1, 3), (4, 2), (5, 3), (7, 4), (3, 5)])
def test_partition_of_unity_and_derivative_sum(orc, K, p):
    """sum_i B_i(x) = 1 and sum_i B_i'(x) = 0 on [0,1]; B_i >= 0 (eqs. cox1/cox2)."""
    for t in (W.open_uniform_knots(K, p), _nonuniform_knots(K, p, 7) if K > 1 else None):
        if t is None:
            continue
        for x in np.linspace(0, 1, 37):
            B, dB = orc.basis_all(t, p, x)
            assert len(B) == K + p
            assert abs(B.sum() - 1) < 1e-14
            assert abs(dB.sum()) < 1e-11 * max(1.0, np.abs(dB).max())
            assert B.min() >= 0


def test_uniform_interior_segments(orc):
    """Uniform B-splines on an interior span equal the textbook cardinal pieces
    in local t in [0,1]:  p=2: (1-t)^2/2, (1+2t-2t^2)/2, t^2/2;
    p=3: (1-t)^3/6, (3t^3-6t^2+4)/6, (-3t^3+3t^2+3t+1)/6, t^3/6."""
    K = 8
    for p, pieces in [
        (2, [lambda t: (1 - t) ** 2 / 2, lambda t: (1 + 2 * t - 2 * t * t) / 2, lambda t: t * t / 2]),
        (3, [lambda t: (1 - t) ** 3 / 6, lambda t: (3 * t ** 3 - 6 * t ** 2 + 4) / 6,
             lambda t: (-3 * t ** 3 + 3 * t ** 2 + 3 * t + 1) / 6, lambda t: t ** 3 / 6]),
    ]:
        kn = W.open_uniform_knots(K, p)
        e = 4  # interior element [4/8, 5/8]: functions e..e+p
        for t in np.linspace(0, 0.999, 11):
            x = (e + t) / K
            B, _ = orc.basis_all(kn, p, x)
            for a in range(p + 1):
                assert abs(B[e + a] - pieces[a](t)) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_single_element_is_bernstein(orc, p):
    """K = 1: the basis is the Bernstein basis C(p,a) x^a (1-x)^(p-a); its
    derivative is p (b_{a-1,p-1} - b_{a,p-1})."""
    kn = W.open_uniform_knots(1, p)
    for x in np.linspace(0, 1, 13):
        B, dB = orc.basis_all(kn, p, x)
        for a in range(p + 1):
            assert abs(B[a] - math.comb(p, a) * x ** a * (1 - x) ** (p - a)) < 1e-14
            bm = lambda j: math.comb(p - 1, j) * x ** j * (1 - x) ** (p - 1 - j) if 0 <= j <= p - 1 else 0.0
            assert abs(dB[a] - p * (bm(a - 1) - bm(a))) < 1e-12


@pytest.mark.parametrize("K,p", [(4, 3), (5, 2), (3, 4)])
def test_greville_reproduction(orc, K, p):
    """sum_i xi*_i B_i(x) = x with Greville abscissae (linear precision)."""
    for t in (W.open_uniform_knots(K, p), _nonuniform_knots(K, p, 3)):
        g = np.array([float(v) for v in exact.greville(list(t), p)])
        for x in np.linspace(0, 1, 29):
            B, dB = orc.basis_all(t, p, x)
            assert abs(np.dot(g, B) - x) < 1e-14
            assert abs(np.dot(g, dB) - 1.0) < 1e-12


@pytest.mark.parametrize("K,p", [(1, 2), (3, 2), (4, 3), (2, 4)])
def test_basis_vs_exact_rational(orc, K, p):
    """Floating values and textbook-formula derivatives vs the exact piecewise
    polynomials of exact.py (derivatives there by polynomial differentiation)."""
    t = [Fraction(0)] * (p + 1) + [Fraction(k, K) for k in range(1, K)] + [Fraction(1)] * (p + 1)
    for x in [Fraction(0), Fraction(1, 7), Fraction(1, 3), Fraction(1, 2), Fraction(5, 6), Fraction(1)]:
        vals, ders = exact.basis_values(t, p, x)
        B, dB = orc.basis_all(np.array([float(v) for v in t]), p, float(x))
        np.testing.assert_allclose(B, [float(v) for v in vals], rtol=0, atol=2e-15)
        np.testing.assert_allclose(dB, [float(v) for v in ders], rtol=0, atol=1e-12 * K * p)


# ---------------------------------------------------------------- exact 1D matrices


def test_exact_1d_interior_rows_textbook():
    """Interior rows of the uniform 1D mass (/h) and stiffness (*h) matrices
    (exact integrals of cardinal B-spline products)."""
    mass = {2: ["11/20", "13/60", "1/120"],
            3: ["151/315", "397/1680", "1/42", "1/5040"],
            4: ["15619/36288", "44117/181440", "913/22680", "251/181440", "1/362880"]}
    stiff = {2: ["1", "-1/3", "-1/6"],
             3: ["2/3", "-1/8", "-1/5", "-1/120"],
             4: ["35/72", "-11/360", "-17/90", "-59/2520", "-1/5040"]}
    K = 16
    for p in (2, 3, 4):
        M, A = exact.matrices_1d(exact.open_uniform_knots(K, p), p)
        i = K // 2
        h = Fraction(1, K)
        assert [M[i][i + o] / h for o in range(p + 1)] == [Fraction(s) for s in mass[p]]
        assert [A[i][i + o] * h for o in range(p + 1)] == [Fraction(s) for s in stiff[p]]


def test_exact_1d_bernstein_mass():
    """K=1: int b_a b_b = C(p,a)C(p,b) / ((2p+1) C(2p,a+b))."""
    for p in (1, 2, 3, 4, 5):
        M, A = exact.matrices_1d(exact.open_uniform_knots(1, p), p)
        for a in range(p + 1):
            for b in range(p + 1):
                ref = Fraction(math.comb(p, a) * math.comb(p, b), (2 * p + 1) * math.comb(2 * p, a + b))
                assert M[a][b] == ref
            assert sum(A[a]) == 0


def test_golden_1d_K8_p2(orc):
    """Stored exact 1D matrices of the K=8, p=2 open uniform basis
    (tests/golden/bspline1d_K8_p2.txt, written by tests/golden/make_golden.py
    from oracle/exact.py)."""
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "bspline1d_K8_p2.txt")
    rows = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, i, vals = line.split(":")
        rows[(name, int(i))] = [Fraction(v) for v in vals.split()]
    M, A = exact.matrices_1d(exact.open_uniform_knots(8, 2), 2)
    for i in range(10):
        assert rows[("1920M", i)] == [1920 * v for v in M[i]]
        assert rows[("A", i)] == A[i]
    # printed structure: 1920*M first rows [48,28,4], [28,80,50,2], [4,50,132,52,2]
    assert rows[("1920M", 0)][:3] == [48, 28, 4]
    assert rows[("1920M", 1)][:4] == [28, 80, 50, 2]
    assert rows[("1920M", 2)][:5] == [4, 50, 132, 52, 2]
    assert sum(sum(r) for k, r in rows.items() if k[0] == "1920M") == 1920


# ---------------------------------------------------------------- element matrices


def _fkron(a, b, c):
    return np.kron(np.array(a, dtype=object), np.kron(np.array(b, dtype=object), np.array(c, dtype=object)))


def _patch(orc, K, p, knots=None):
    if knots is None:
        knots = [W.open_uniform_knots(k, p) for k in K]
    return orc.Patch(p, K, [p + 1] * 3, knots)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_single_element_kronecker(orc, p):
    """K = 1 in every direction, kappa = 1: element mass = Bernstein mass cubed
    (Kronecker, x fastest) times the cell volume; stiffness = sum of three
    Kronecker products with the exact 1D stiffness."""
    P = _patch(orc, (1, 1, 1), p)
    kap = W.kappa_constant(1, P.nq)
    Me, Ke = orc.element_matrices(P, kap)
    M1, A1 = exact.matrices_1d(exact.open_uniform_knots(1, p), p)
    Mr = _fkron(M1, M1, M1).astype(float)
    Kr = (_fkron(M1, M1, A1) + _fkron(M1, A1, M1) + _fkron(A1, M1, M1)).astype(float)
    np.testing.assert_allclose(Me[0], Mr, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Ke[0], Kr, rtol=0, atol=1e-13)


def test_element_invariants(orc):
    """For any positive kappa: element matrices symmetric, K_e 1 = 0 (gradient
    of a constant), sum of M_e entries = sum_q w_q kappa_q; for kappa=1 that
    sum is the cell volume."""
    P = _patch(orc, (3, 2, 4), 3)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=11)
    Me, Ke = orc.element_matrices(P, kap)
    xs = [orc.quad_nodes(P, d) for d in range(3)]
    for e in range(P.nelem):
        ex, ey, ez = e % 3, (e // 3) % 2, e // 6
        wq = np.einsum("k,j,i->kji", xs[2][1][ez], xs[1][1][ey], xs[0][1][ex]).reshape(-1)
        assert np.array_equal(Me[e], Me[e].T) or np.abs(Me[e] - Me[e].T).max() < 1e-17
        assert np.abs(Ke[e] - Ke[e].T).max() < 1e-14
        assert np.abs(Ke[e].sum(axis=1)).max() < 1e-13 * np.abs(Ke[e]).max()
        assert abs(Me[e].sum() - np.dot(wq, kap[e])) < 1e-15
    ones = W.kappa_constant(P.nelem, P.nq)
    Me1, _ = orc.element_matrices(P, ones, want_k=False)
    assert abs(Me1[0].sum() - (1 / 3) * (1 / 2) * (1 / 4)) < 1e-16


# ---------------------------------------------------------------- global matrices


def _structural_pattern(N, p):
    """(I,J) present iff |i_d - j_d| <= p for every direction; sorted columns."""
    Nx, Ny, Nz = N
    rp = [0]
    cols = []
    for k in range(Nz):
        for j in range(Ny):
            for i in range(Nx):
                for kk in range(max(0, k - p), min(Nz, k + p + 1)):
                    for jj in range(max(0, j - p), min(Ny, j + p + 1)):
                        for ii in range(max(0, i - p), min(Nx, i + p + 1)):
                            cols.append(ii + Nx * (jj + Ny * kk))
                rp.append(len(cols))
    return np.array(rp, dtype=np.int64), np.array(cols, dtype=np.int32)


def _csr_to_dense(rp, col, val, n):
    A = np.zeros((n, n))
    for r in range(n):
        A[r, col[rp[r]:rp[r + 1]]] = val[rp[r]:rp[r + 1]]
    return A


def test_global_w1_kronecker(orc):
    """8^3 elements, p=2, q=3, kappa=1: the assembled global mass equals
    M1 (x) M1 (x) M1 of the exact 1D mass matrix; nnz = 85 184 and the pattern
    is the structural one."""
    P = _patch(orc, (8, 8, 8), 2)
    kap = W.kappa_constant(P.nelem, P.nq)
    rp, col, Mv, Kv = orc.assemble(P, kap)
    assert rp[-1] == 85184
    rp_s, col_s = _structural_pattern(P.N, 2)
    assert np.array_equal(rp, rp_s) and np.array_equal(col, col_s)
    M1, A1 = exact.matrices_1d(exact.open_uniform_knots(8, 2), 2)
    Mref = _fkron(M1, M1, M1).astype(float)
    Kref = (_fkron(M1, M1, A1) + _fkron(M1, A1, M1) + _fkron(A1, M1, M1)).astype(float)
    Md = _csr_to_dense(rp, col, Mv, P.ndof)
    Kd = _csr_to_dense(rp, col, Kv, P.ndof)
    assert np.linalg.norm(Md - Mref) / np.linalg.norm(Mref) < 1e-14
    assert np.linalg.norm(Kd - Kref) / np.linalg.norm(Kref) < 1e-14
    assert abs(Mv.sum() - 1.0) < 1e-13


@pytest.mark.parametrize("p", [2, 3])
def test_global_separable_linear_kappa_exact(orc, p):
    """Anisotropic mesh K=(3,2,4), non-uniform knots, kappa = (1+x)(2+y)(3+z):
    (p+1)-point Gauss is exact for these integrands, so the assembled matrices
    equal the exact Kronecker forms with weighted 1D matrices.  Different
    weights per axis catch a transposed kappa layout or a swapped axis."""
    K = (3, 2, 4)
    knots = [W.open_uniform_knots(K[0], p), _nonuniform_knots(2, p, 5), _nonuniform_knots(4, p, 9)]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    xs = [orc.quad_nodes(P, d)[0] for d in range(3)]
    kap = W.kappa_separable(1 + xs[0], 2 + xs[1], 3 + xs[2])
    rp, col, Mv, Kv = orc.assemble(P, kap)
    tf = [[Fraction(float(v)) for v in k] for k in knots]
    Mx, Ax = exact.matrices_1d(tf[0], p, (1, 1))
    My, Ay = exact.matrices_1d(tf[1], p, (2, 1))
    Mz, Az = exact.matrices_1d(tf[2], p, (3, 1))
    Mref = _fkron(Mz, My, Mx).astype(float)
    Kref = (_fkron(Mz, My, Ax) + _fkron(Mz, Ay, Mx) + _fkron(Az, My, Mx)).astype(float)
    Md = _csr_to_dense(rp, col, Mv, P.ndof)
    Kd = _csr_to_dense(rp, col, Kv, P.ndof)
    assert np.linalg.norm(Md - Mref) / np.linalg.norm(Mref) < 1e-14
    assert np.linalg.norm(Kd - Kref) / np.linalg.norm(Kref) < 1e-13


def test_global_invariants_lognormal(orc):
    """Any kappa: sum of M = sum_q w_q kappa_q; K 1 = 0; symmetry; rows()
    equals the assembled rows."""
    P = _patch(orc, (4, 3, 5), 2)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=4)
    rp, col, Mv, Kv = orc.assemble(P, kap)
    xs = [orc.quad_nodes(P, d)[1] for d in range(3)]
    wq = W.kappa_separable(xs[0], xs[1], xs[2])
    assert abs(Mv.sum() - (wq * kap).sum()) < 1e-14
    Kd = _csr_to_dense(rp, col, Kv, P.ndof)
    Md = _csr_to_dense(rp, col, Mv, P.ndof)
    assert np.abs(Kd.sum(axis=1)).max() < 1e-13 * np.abs(Kd).sum(axis=1).max()
    assert np.abs(Kd - Kd.T).max() < 1e-15 and np.abs(Md - Md.T).max() < 1e-17
    dofs = np.array([0, 7, 33, P.ndof // 2, P.ndof - 1])
    for d, (c, m, k) in zip(dofs, orc.rows(P, kap, dofs)):
        assert np.array_equal(c, col[rp[d]:rp[d + 1]])
        np.testing.assert_allclose(m, Mv[rp[d]:rp[d + 1]], rtol=0, atol=1e-17)
        np.testing.assert_allclose(k, Kv[rp[d]:rp[d + 1]], rtol=0, atol=1e-14)


# ---------------------------------------------------------------- adjoint


def test_kappa_grad_closed_forms(orc):
    """dL/dkappa_q = w_q (u_h v_h + grad u_h . grad v_h)(x_q): with u = v = 1
    it is w_q; with u = v = Greville-x (u_h = x) it is w_q (x^2 + 1); with
    u = Greville-x, v = 1 it is w_q x (mass part only)."""
    p = 3
    K = (4, 3, 5)
    P = _patch(orc, K, p)
    xn = [orc.quad_nodes(P, d) for d in range(3)]
    wq = W.kappa_separable(xn[0][1], xn[1][1], xn[2][1])
    xq = W.kappa_separable(xn[0][0], np.ones_like(xn[1][0]), np.ones_like(xn[2][0]))
    ones = np.ones(P.ndof)
    g = orc.kappa_grad(P, ones, ones)
    np.testing.assert_allclose(g, wq, rtol=1e-14, atol=0)
    gx = np.array([float(v) for v in exact.greville(list(W.open_uniform_knots(K[0], p)), p)])
    ux = np.tile(gx, P.N[1] * P.N[2])
    g2 = orc.kappa_grad(P, ux, ux)
    np.testing.assert_allclose(g2, wq * (xq ** 2 + 1), rtol=1e-13, atol=0)
    g3 = orc.kappa_grad(P, ux, ones)
    np.testing.assert_allclose(g3, wq * xq, rtol=1e-13, atol=1e-18)


def test_kappa_grad_linearity(orc):
    """L(kappa) = u^T (K + M) v is linear in kappa, so L = sum_q kappa_q g_q
    exactly (Euler's identity); checked against the assembled CSR."""
    P = _patch(orc, (3, 4, 2), 2)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=2)
    u = W.normal_vector(P.ndof, 3)
    v = W.normal_vector(P.ndof, 4)
    rp, col, Mv, Kv = orc.assemble(P, kap)
    Av = np.zeros(P.ndof)
    for r in range(P.ndof):
        s = slice(rp[r], rp[r + 1])
        Av[r] = math.fsum((Mv[s] + Kv[s]) * v[col[s]])
    L = math.fsum(u * Av)
    g = orc.kappa_grad(P, u, v)
    assert abs(math.fsum((g * kap).reshape(-1)) - L) < 1e-12 * abs(L)


# ---------------------------------------------------------------- reduced continuity
# Repeated interior knots (the "more general B-spline basis functions" of
# Sec. 2.3): a knot of multiplicity m leaves the basis C^{p-m} there; a span
# of zero length is an element with zero Gauss weights.


def _bern_mass(p, a, b):
    """int_0^1 b_{a,p} b_{b,p} (Bernstein), 0 outside 0..p."""
    if not (0 <= a <= p and 0 <= b <= p):
        return Fraction(0)
    return Fraction(math.comb(p, a) * math.comb(p, b), (2 * p + 1) * math.comb(2 * p, a + b))


def _bern_blocks(p, breaks, mult):
    """1D mass and stiffness of a knot vector whose every interior breakpoint
    has multiplicity `mult` in {p, p+1}: the basis on each non-empty span is
    the Bernstein basis of that span, so the matrices are the Bernstein element
    matrices (mass h B, stiffness (p^2/h) D) placed at the span's functions,
    overlapping by one function for C^0 and not at all for C^-1."""
    pts = [Fraction(0)] + [Fraction(b) for b in breaks] + [Fraction(1)]
    nspan = len(pts) - 1
    step = p if mult == p else p + 1
    N = step * nspan + (1 if mult == p else 0)
    M = [[Fraction(0)] * N for _ in range(N)]
    A = [[Fraction(0)] * N for _ in range(N)]
    for s in range(nspan):
        h = pts[s + 1] - pts[s]
        o = s * step
        for a in range(p + 1):
            for b in range(p + 1):
                M[o + a][o + b] += h * _bern_mass(p, a, b)
                d = (_bern_mass(p - 1, a - 1, b - 1) - _bern_mass(p - 1, a - 1, b)
                     - _bern_mass(p - 1, a, b - 1) + _bern_mass(p - 1, a, b))
                A[o + a][o + b] += p * p * d / h
    return M, A


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("extra", [0, 1])
def test_exact_1d_broken_knots_are_bernstein_blocks(p, extra):
    """C^0 knots (multiplicity p) and C^-1 knots (multiplicity p+1): the exact
    piecewise-polynomial 1D matrices of exact.py equal the assembled Bernstein
    element matrices (closed forms), entry by entry as rationals."""
    breaks = [Fraction(1, 3), Fraction(1, 2)]
    t = ([Fraction(0)] * (p + 1) + [b for b in breaks for _ in range(p + extra)]
         + [Fraction(1)] * (p + 1))
    M, A = exact.matrices_1d(t, p)
    Mr, Ar = _bern_blocks(p, breaks, p + extra)
    assert len(M) == len(Mr) == len(t) - p - 1
    assert M == Mr and A == Ar


@pytest.mark.parametrize("p", [2, 3])
def test_repeated_knots_basis(orc, p):
    """Knots with every multiplicity 1..p+1: partition of unity, non-negativity,
    Greville reproduction (linear precision holds for any knot vector) and the
    exact piecewise polynomials of exact.py at seeded points."""
    fixed = W.repeated_knots([0.125, 0.25, 0.5, 0.75][:p + 1], list(range(1, p + 2)), p)
    seeded, _ = W.random_repeated_knots(5, p, seed=40 + p)
    rng = np.random.default_rng(7)
    for t, x in [(t, x) for t in (fixed, seeded) for x in np.concatenate([rng.uniform(0, 1, 25), [0.0, 1.0]])]:
        tf = [Fraction(float(v)) for v in t]
        g = np.array([float(v) for v in exact.greville(tf, p)])
        B, dB = orc.basis_all(t, p, x)
        assert abs(B.sum() - 1) < 1e-14 and B.min() >= 0
        assert abs(np.dot(g, B) - x) < 1e-14
        vals, ders = exact.basis_values(tf, p, Fraction(float(x)))
        np.testing.assert_allclose(B, [float(v) for v in vals], rtol=0, atol=2e-15)
        scale = max(1.0, max(abs(float(v)) for v in ders))
        np.testing.assert_allclose(dB, [float(v) for v in ders], rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("p", [2, 3])
def test_global_repeated_knots_exact(orc, p):
    """A C^0 breakpoint (x), seeded multiplicities 1..p+1 (y) and a C^-1
    breakpoint (z), kappa = (1+x)(2+y)(3+z): the assembled matrices equal the
    exact Kronecker forms; the elements on zero-length spans are exactly zero;
    the pattern is the structural one."""
    tx = W.repeated_knots([0.25, 0.6], [p, 1], p)
    ty, _ = W.random_repeated_knots(3, p, seed=60 + p)
    tz = W.repeated_knots([0.5], [p + 1], p)
    knots = [tx, ty, tz]
    K = tuple(len(t) - 2 * p - 1 for t in knots)
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    assert orc.validate(P)
    xs = [orc.quad_nodes(P, d)[0] for d in range(3)]
    kap = W.kappa_separable(1 + xs[0], 2 + xs[1], 3 + xs[2])
    rp, col, Mv, Kv = orc.assemble(P, kap)
    rp_s, col_s = _structural_pattern(P.N, p)
    assert np.array_equal(rp, rp_s) and np.array_equal(col, col_s)
    tf = [[Fraction(float(v)) for v in k] for k in knots]
    Mx, Ax = exact.matrices_1d(tf[0], p, (1, 1))
    My, Ay = exact.matrices_1d(tf[1], p, (2, 1))
    Mz, Az = exact.matrices_1d(tf[2], p, (3, 1))
    Mref = _fkron(Mz, My, Mx).astype(float)
    Kref = (_fkron(Mz, My, Ax) + _fkron(Mz, Ay, Mx) + _fkron(Az, My, Mx)).astype(float)
    Md = _csr_to_dense(rp, col, Mv, P.ndof)
    Kd = _csr_to_dense(rp, col, Kv, P.ndof)
    assert np.linalg.norm(Md - Mref) / np.linalg.norm(Mref) < 1e-14
    assert np.linalg.norm(Kd - Kref) / np.linalg.norm(Kref) < 1e-13
    Me, Ke = orc.element_matrices(P, kap)
    h = [np.diff(t)[p:p + k] for t, k in zip(knots, K)]
    for e in range(P.nelem):
        ex, ey, ez = e % K[0], (e // K[0]) % K[1], e // (K[0] * K[1])
        if h[0][ex] == 0 or h[1][ey] == 0 or h[2][ez] == 0:
            assert not Me[e].any() and not Ke[e].any()
        else:
            assert Me[e].any()
    assert min(min(x) for x in h) == 0.0    # the case has empty spans


def test_validate_repeated_knots(orc):
    """Multiplicity up to p+1 is accepted; p+2 (an identically zero function)
    is refused, at an end as well as inside."""
    p = 2
    ok = W.repeated_knots([0.5], [p + 1], p)
    bad = W.repeated_knots([0.5], [p + 2], p)
    bad_end = np.concatenate([[0.0] * (p + 2), [0.5], [1.0] * (p + 1)])
    for t, want in ((ok, True), (bad, False), (bad_end, False)):
        k = len(t) - 2 * p - 1
        P = orc.Patch(p, (k, 1, 1), [3] * 3, [t, W.open_uniform_knots(1, p), W.open_uniform_knots(1, p)])
        assert orc.validate(P) == want


# ---------------------------------------------------------------- mapped geometry
# x = F(xi): mass coefficient cm = kappa det J, stiffness tensor
# G = kappa det J J^-1 J^-T per point (workloads.mapped_geometry builds them).


def test_exact_mixed_1d_integration_by_parts():
    """int N_i' N_j + int N_i N_j' = [N_i N_j] at the ends, which on an open
    knot vector is e_last e_last^T - e_0 e_0^T; exact rationals."""
    for p, K in [(1, 3), (2, 4), (3, 2), (4, 3)]:
        for t in (exact.open_uniform_knots(K, p),
                  [Fraction(0)] * (p + 1) + [Fraction(1, 3)] * p + [Fraction(1)] * (p + 1)):
            B = exact.mixed_1d(t, p)
            n = len(B)
            for i in range(n):
                for j in range(n):
                    want = (1 if i == j == n - 1 else 0) - (1 if i == j == 0 else 0)
                    assert B[i][j] + B[j][i] == want


def _greville_dofs(knots, p):
    g = [np.array([float(v) for v in exact.greville([Fraction(float(x)) for x in t], p)]) for t in knots]
    N = [len(v) for v in g]
    i = np.arange(N[0] * N[1] * N[2])
    return np.stack([g[0][i % N[0]], g[1][(i // N[0]) % N[1]], g[2][i // (N[0] * N[1])]], axis=1)


def _points(orc, P):
    """Parametric node coordinates per direction and the per-point weight
    product, both in kappa layout [E][q^3]."""
    xs = [orc.quad_nodes(P, d) for d in range(3)]
    one = [np.ones_like(x[0]) for x in xs]
    X = W.kappa_separable(xs[0][0], one[1], one[2])
    Y = W.kappa_separable(one[0], xs[1][0], one[2])
    Z = W.kappa_separable(one[0], one[1], xs[2][0])
    wq = W.kappa_separable(xs[0][1], xs[1][1], xs[2][1])
    return xs, np.stack([X, Y, Z], axis=-1), wq


def test_geometry_scaling_equals_scaled_knots(orc):
    """F(xi) = diag(s) xi: integrating on the parameter cube with (cm, G) equals
    the identity-geometry oracle on knot vectors scaled to [0, s_d] (the same
    points, the same kappa values): element matrices and CSR values."""
    p, K, s = 2, (3, 2, 4), (2.0, 0.5, 3.0)
    knots = [_nonuniform_knots(k, p, 30 + d) for d, k in enumerate(K)]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    xs, _, _ = _points(orc, P)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=8)
    cm, G = W.mapped_geometry(xs[0][0], xs[1][0], xs[2][0], kap, A=np.diag(s))
    Ps = orc.Patch(p, K, [p + 1] * 3, [k * sd for k, sd in zip(knots, s)])
    Me, Ke = orc.element_matrices(P, cm, G=G)
    Me_s, Ke_s = orc.element_matrices(Ps, kap)
    assert np.linalg.norm(Me - Me_s) <= 1e-14 * np.linalg.norm(Me_s)
    assert np.linalg.norm(Ke - Ke_s) <= 1e-13 * np.linalg.norm(Ke_s)
    _, _, Mv, Kv = orc.assemble(P, cm, G=G)
    _, _, Mv_s, Kv_s = orc.assemble(Ps, kap)
    assert np.linalg.norm(Mv - Mv_s) <= 1e-14 * np.linalg.norm(Mv_s)
    assert np.linalg.norm(Kv - Kv_s) <= 1e-13 * np.linalg.norm(Kv_s)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_geometry_affine_kronecker(orc, p):
    """A general (non-symmetric) affine map and kappa = 1: the assembled
    stiffness equals sum_{c,d} G_cd T_cd with the exact 1D factors,
    T_cc = (A1 in direction c, M1 elsewhere) and, for c != d, B1 = int N' N in
    direction c, its transpose in direction d (x fastest Kronecker order);
    the mass equals det(A) M1 (x) M1 (x) M1."""
    K = (3, 2, 3)
    A = np.array([[1.5, 0.4, -0.2], [0.1, 0.8, 0.3], [-0.3, 0.2, 1.2]])
    knots = [W.open_uniform_knots(K[0], p), _nonuniform_knots(2, p, 3), _nonuniform_knots(3, p, 4)]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    xs, _, _ = _points(orc, P)
    cm, G = W.mapped_geometry(xs[0][0], xs[1][0], xs[2][0], W.kappa_constant(P.nelem, P.nq), A=A)
    rp, col, Mv, Kv = orc.assemble(P, cm, G=G)
    tf = [[Fraction(float(v)) for v in k] for k in knots]
    M1, A1, B1 = [], [], []
    for d in range(3):
        m, a = exact.matrices_1d(tf[d], p)
        M1.append(np.array(m, dtype=object))
        A1.append(np.array(a, dtype=object))
        B1.append(np.array(exact.mixed_1d(tf[d], p), dtype=object))
    Ai = np.linalg.inv(A)
    Gc = np.linalg.det(A) * Ai @ Ai.T

    def factor(d, c, e):
        """1D factor of direction d in the term d/dx_c (test) d/dx_e (trial)."""
        if d == c and d == e:
            return A1[d]
        if d == c:
            return B1[d]
        if d == e:
            return B1[d].T
        return M1[d]

    Kref = np.zeros((P.ndof, P.ndof))
    for c in range(3):
        for e in range(3):
            Kref += Gc[c, e] * _fkron(factor(2, c, e), factor(1, c, e), factor(0, c, e)).astype(float)
    Mref = np.linalg.det(A) * _fkron(M1[2], M1[1], M1[0]).astype(float)
    Kd = _csr_to_dense(rp, col, Kv, P.ndof)
    Md = _csr_to_dense(rp, col, Mv, P.ndof)
    assert np.linalg.norm(Kd - Kref) <= 1e-13 * np.linalg.norm(Kref)
    assert np.linalg.norm(Md - Mref) <= 1e-14 * np.linalg.norm(Mref)


def test_geometry_linear_patch_tests(orc):
    """(a) Affine map, log-normal kappa: physical linear functions are in the
    space (u_I = c.(A xi*_I + b) + d at the Greville points), so
    u^T K v = (c1.c2) sum_q w_q cm_q and u^T M v = sum_q w_q cm_q u(x_q) v(x_q)
    exactly (the quadrature sees the exact integrand).  (b) A curved map
    (amp = 0.1): parametric linear functions u = c.xi* give
    u^T K v = sum_q w_q c1^T G_q c2.  Both: K 1 = 0 and symmetry."""
    p, K = 3, (3, 4, 2)
    knots = [_nonuniform_knots(k, p, 50 + d) for d, k in enumerate(K)]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    xs, XI, wq = _points(orc, P)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=12)
    gr = _greville_dofs(knots, p)
    c1, c2 = np.array([0.7, -1.2, 0.4]), np.array([-0.3, 0.9, 1.6])
    A = np.array([[1.2, -0.3, 0.25], [0.15, 0.9, -0.2], [0.05, 0.4, 1.1]])
    b = np.array([0.3, -0.1, 0.2])
    # (a) affine
    cm, G = W.mapped_geometry(xs[0][0], xs[1][0], xs[2][0], kap, A=A, b=b)
    rp, col, Mv, Kv = orc.assemble(P, cm, G=G)
    Kd = _csr_to_dense(rp, col, Kv, P.ndof)
    Md = _csr_to_dense(rp, col, Mv, P.ndof)
    xg = gr @ A.T + b
    u, v = xg @ c1 + 0.5, xg @ c2 - 0.25
    vol = math.fsum((wq * cm).ravel().tolist())
    assert abs(u @ Kd @ v - np.dot(c1, c2) * vol) <= 1e-12 * abs(np.dot(c1, c2) * vol)
    xq = XI @ A.T + b
    mref = math.fsum((wq * cm * (xq @ c1 + 0.5) * (xq @ c2 - 0.25)).ravel().tolist())
    assert abs(u @ Md @ v - mref) <= 1e-12 * math.fsum(np.abs(wq * cm).ravel().tolist())
    # (b) curved
    cm2, G2 = W.mapped_geometry(xs[0][0], xs[1][0], xs[2][0], kap, amp=0.1)
    rp, col, Mv2, Kv2 = orc.assemble(P, cm2, G=G2)
    Kd2 = _csr_to_dense(rp, col, Kv2, P.ndof)
    Gq = np.zeros(G2.shape[:1] + G2.shape[2:] + (3, 3))
    for c, (r, t) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        Gq[..., r, t] = Gq[..., t, r] = G2[:, c, :]
    kref = math.fsum((wq * np.einsum("a,...ab,b->...", c1, Gq, c2)).ravel().tolist())
    assert abs((gr @ c1) @ Kd2 @ (gr @ c2) - kref) <= 1e-12 * abs(kref)
    for Kk in (Kd, Kd2):
        assert np.abs(Kk.sum(axis=1)).max() <= 1e-13 * np.abs(Kk).sum(axis=1).max()
        assert np.abs(Kk - Kk.T).max() <= 1e-14 * np.abs(Kk).max()


def test_geometry_kappa_grad(orc):
    """Gradient on a mapped geometry with cm = kappa cm0, G = kappa G0:
    (1) L is linear in kappa, so L(kappa) = <kappa, g> where L comes from the
        oracle's assembled matrices (element loops, not point values);
    (2) u = v = 1: g = alphaM w cm0 (constant functions have no gradient);
    (3) parametric linear u = c1.xi*, v = c2.xi* (Greville points):
        g = w (alphaM cm0 u v + alphaK c1^T G0 c2) at every point."""
    import scipy.sparse as sp

    p, K = 2, (3, 4, 3)
    knots = [_nonuniform_knots(k, p, 60 + d) for d, k in enumerate(K)]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    xs, XI, wq = _points(orc, P)
    cm0, G0 = W.mapped_geometry(xs[0][0], xs[1][0], xs[2][0], W.kappa_constant(P.nelem, P.nq), amp=0.1)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=14)
    u = W.normal_vector(P.ndof, 15)
    v = W.normal_vector(P.ndof, 16)
    aM, aK = 0.7, 1.3
    g = orc.kappa_grad(P, u, v, aM, aK, cm0=cm0, G0=G0)
    rp, col, Mv, Kv = orc.assemble(P, kap * cm0, G=kap[:, None, :] * G0)
    A = sp.csr_matrix((aM * Mv + aK * Kv, col, rp), shape=(P.ndof, P.ndof))
    L = math.fsum((u * (A @ v)).tolist())
    Lg = math.fsum((kap * g).ravel().tolist())
    assert abs(L - Lg) <= 1e-13 * abs(L)
    one = np.ones(P.ndof)
    g1 = orc.kappa_grad(P, one, one, aM, aK, cm0=cm0, G0=G0)
    np.testing.assert_allclose(g1, aM * wq * cm0, rtol=1e-13, atol=0)
    gr = _greville_dofs(knots, p)
    c1, c2 = np.array([0.4, -0.9, 1.2]), np.array([1.1, 0.3, -0.5])
    gl = orc.kappa_grad(P, gr @ c1, gr @ c2, aM, aK, cm0=cm0, G0=G0)
    Gq = np.zeros(G0.shape[:1] + G0.shape[2:] + (3, 3))
    for c, (r, t) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        Gq[..., r, t] = Gq[..., t, r] = G0[:, c, :]
    ref = wq * (aM * cm0 * (XI @ c1) * (XI @ c2) + aK * np.einsum("a,...ab,b->...", c1, Gq, c2))
    np.testing.assert_allclose(gl, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


# ---------------------------------------------------------------- weighted quadrature (f4)
# oracle/wq.py is pinned by what the method fixes: the point set's definition,
# exactness of every 1D rule for the trial products (against exact.py's
# rational integrals, not the oracle's own Gauss sums), the minimum-norm
# choice, exactness of the 3D matrices for kappa = 1 (exact Kronecker forms),
# the tensor structure for any kappa (a sum of separable kappas gives the
# sum of Kronecker products of 1D rule matrices, so by linearity every kappa
# on the point grid is covered), and convergence to the Galerkin integrals
# for a smooth kappa.


def test_wq_points_definition():
    from oracle import wq

    for p, K in ((1, 1), (2, 5), (3, 6), (5, 3)):
        t = W.open_uniform_knots(K, p)
        x, first = wq.points_1d(t, p)
        for e in range(K):
            R = p + 1 if e in (0, K - 1) else 2
            assert first[e + 1] - first[e] == R
            a, h = e / K, 1.0 / K
            want = [a + h * (r + 0.5) / R for r in range(R)]
            np.testing.assert_allclose(x[first[e]:first[e + 1]], want, rtol=0, atol=1e-15)
        assert np.all(np.diff(x) > 0)
    with pytest.raises(ValueError):
        wq.points_1d(W.repeated_knots([0.5], [2], 2), 2)


@pytest.mark.parametrize("p,K,nonuni", [(1, 4, False), (2, 6, True), (3, 7, False), (3, 5, True),
                                        (4, 5, False), (5, 6, True), (5, 1, False)])
def test_wq_rules_exact_against_rational_integrals(orc, p, K, nonuni):
    """sum_q w00[i][q] B_j(x_q) = int B_i B_j and sum_q w11[i][q] B_j'(x_q) =
    int B_i' B_j' for every overlapping pair, against exact.py's rational
    integrals (relative to the largest entry)."""
    from oracle import wq

    t = _nonuniform_knots(K, p, 70 + p) if nonuni else W.open_uniform_knots(K, p)
    R = wq.Rule1D(t, p)
    Mw, Aw = R.matrices()
    M1, A1 = exact.matrices_1d([Fraction(float(v)) for v in t], p)
    M1 = np.array(M1, dtype=object).astype(float)
    A1 = np.array(A1, dtype=object).astype(float)
    assert np.abs(Mw - M1).max() <= 1e-14 * np.abs(M1).max()
    assert np.abs(Aw - A1).max() <= 1e-13 * np.abs(A1).max()
    # and against the oracle's floating-point Gauss sums of its literal
    # Cox-de Boor values (independent of exact.py)
    Mg, Ag = wq._gram_1d(t, p)
    assert np.abs(Mw - Mg).max() <= 1e-13 * np.abs(Mg).max()
    assert np.abs(Aw - Ag).max() <= 1e-12 * np.abs(Ag).max()
    # entries beyond the band are structurally zero
    for i in range(R.N):
        for j in range(R.N):
            if abs(i - j) > p:
                assert Mw[i, j] == 0.0 and Aw[i, j] == 0.0


def test_wq_weights_are_minimum_norm(orc):
    """Each w00[i] solves its exactness system and lies in the row space of
    the system's matrix (the minimum-norm solution); the same for w11."""
    from oracle import wq

    p, K = 3, 6
    t = W.open_uniform_knots(K, p)
    R = wq.Rule1D(t, p)
    M1, A1 = exact.matrices_1d([Fraction(float(v)) for v in t], p)
    M1 = np.array(M1, dtype=object).astype(float)
    A1 = np.array(A1, dtype=object).astype(float)
    for i in range(R.N):
        lo, hi = R.lo[i], R.hi[i]
        j0, j1 = max(0, i - p), min(R.N - 1, i + p) + 1
        for w, T, G in ((R.w00[i], R.V, M1), (R.w11[i], R.D, A1)):
            A = T[lo:hi, j0:j1].T
            np.testing.assert_allclose(A @ w, G[i, j0:j1], rtol=0, atol=1e-13)
            y, *_ = np.linalg.lstsq(A.T, w, rcond=None)     # w = A^T y exactly?
            assert np.linalg.norm(A.T @ y - w) <= 1e-12 * np.linalg.norm(w)
        assert lo < hi and np.all(R.x[lo:hi] > t[i]) and np.all(R.x[lo:hi] < t[i + p + 1])


@pytest.mark.parametrize("p,K", [(1, (3, 2, 4)), (2, (3, 4, 2)), (3, (2, 3, 3))])
def test_wq_3d_constant_kappa_exact(orc, p, K):
    """kappa = 1: the weighted-quadrature matrices are the exact Galerkin
    matrices, M = Mz (x) My (x) Mx and K = Mz My Ax + Mz Ay Mx + Az My Mx
    (exact rationals); the pattern is the structural one."""
    from oracle import wq

    knots = [W.open_uniform_knots(k, p) for k in K]
    npts = [len(wq.points_1d(t, p)[0]) for t in knots]
    rp, col, Mv, Kv = wq.assemble(knots, p, np.ones((npts[2], npts[1], npts[0])))
    N = [k + p for k in K]
    rp_s, col_s = _structural_pattern(N, p)
    assert np.array_equal(rp, rp_s) and np.array_equal(col, col_s)
    ex = [exact.matrices_1d(exact.open_uniform_knots(k, p), p) for k in K]
    Mref = _fkron(ex[2][0], ex[1][0], ex[0][0]).astype(float)
    Kref = (_fkron(ex[2][0], ex[1][0], ex[0][1]) + _fkron(ex[2][0], ex[1][1], ex[0][0]) +
            _fkron(ex[2][1], ex[1][0], ex[0][0])).astype(float)
    n = N[0] * N[1] * N[2]
    assert np.linalg.norm(_csr_to_dense(rp, col, Mv, n) - Mref) / np.linalg.norm(Mref) < 1e-13
    assert np.linalg.norm(_csr_to_dense(rp, col, Kv, n) - Kref) / np.linalg.norm(Kref) < 1e-12


@pytest.mark.parametrize("p", [2, 3])
def test_wq_3d_sum_of_separable_kappas(orc, p):
    """kappa = sum_r f_r(x) g_r(y) h_r(z) (random positive factors on the
    point grid, three terms, different per axis): the 3D matrices equal
    sum_r of the Kronecker forms of the 1D rule matrices with weights f_r,
    g_r, h_r.  The 1D matrices are formed by a separate 1D loop, so a wrong
    index, axis or weight set in the 3D triple sum fails; by linearity in
    kappa this covers every kappa on the grid."""
    from oracle import wq

    K = (3, 2, 4)
    knots = [W.open_uniform_knots(K[0], p), _nonuniform_knots(2, p, 5), _nonuniform_knots(4, p, 9)]
    R = wq.rules(knots, p)
    rng = np.random.default_rng(7)
    kap = np.zeros((R[2].npts(), R[1].npts(), R[0].npts()))
    n = R[0].N * R[1].N * R[2].N
    Mref = np.zeros((n, n))
    Kref = np.zeros((n, n))
    for r in range(3):
        f = [rng.uniform(0.5, 2.0, R[d].npts()) for d in range(3)]
        kap += np.einsum("k,j,i->kji", f[2], f[1], f[0])
        m = [R[d].matrices(f[d]) for d in range(3)]
        Mref += np.kron(m[2][0], np.kron(m[1][0], m[0][0]))
        Kref += (np.kron(m[2][0], np.kron(m[1][0], m[0][1])) + np.kron(m[2][0], np.kron(m[1][1], m[0][0])) +
                 np.kron(m[2][1], np.kron(m[1][0], m[0][0])))
    rp, col, Mv, Kv = wq.assemble(knots, p, kap)
    assert np.linalg.norm(_csr_to_dense(rp, col, Mv, n) - Mref) / np.linalg.norm(Mref) < 1e-13
    assert np.linalg.norm(_csr_to_dense(rp, col, Kv, n) - Kref) / np.linalg.norm(Kref) < 1e-12
    # outside the structural band the Kronecker forms are zero too
    assert np.abs(Mref).sum() == pytest.approx(np.abs(Mv).sum(), rel=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_wq_converges_to_galerkin(orc, p):
    """For a smooth coefficient f(x) = exp(sin 3x) the 1D rule matrices
    approach the Galerkin integrals (a 12-point Gauss rule per element) as
    the mesh is refined: the relative Frobenius error at 64 elements is at
    most a quarter of that at 8."""
    from oracle import wq

    errs = []
    for K in (8, 64):
        t = W.open_uniform_knots(K, p)
        R = wq.Rule1D(t, p)
        Mw, Aw = R.matrices(np.exp(np.sin(3 * R.x)))
        xi, wi = np.polynomial.legendre.leggauss(12)
        N = K + p
        Mg = np.zeros((N, N))
        Ag = np.zeros((N, N))
        for e in range(K):
            a, b = t[e + p], t[e + p + 1]
            for k in range(12):
                x = a + 0.5 * (xi[k] + 1) * (b - a)
                B, dB = orc.basis_all(t, p, x)
                c = 0.5 * wi[k] * (b - a) * np.exp(np.sin(3 * x))
                Mg += c * np.outer(B, B)
                Ag += c * np.outer(dB, dB)
        errs.append((np.linalg.norm(Mw - Mg) / np.linalg.norm(Mg), np.linalg.norm(Aw - Ag) / np.linalg.norm(Ag)))
    assert errs[1][0] <= errs[0][0] / 4 and errs[1][1] <= errs[0][1] / 4, errs
