"""Weighted quadrature of the B-spline mass and stiffness matrices -- TEST
INFRASTRUCTURE (only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may use it).  Plain numpy, FP64, no sum factorisation.

The method is the one the paper names (Sec. 1, "Sum factorization") as the
variant that brings integration down to O(p^6): weighted quadrature, as
published by F. Calabro, G. Sangalli and M. Tani, "Fast formation of
isogeometric Galerkin matrices by weighted quadrature", Comput. Methods Appl.
Mech. Engrg. 316 (2017) 606-622.  The test function moves into the
quadrature weights: every 1D basis function B_i gets its own rule over a
fixed set of global points inside its support, exact for its products with
all trial functions,

    sum_q w00[i][q] B_j (x_q) = int B_i  B_j       (every j overlapping B_i)
    sum_q w11[i][q] B_j'(x_q) = int B_i' B_j'

and with kappa given at the tensor grid of those points the 3D matrices are

    M_IJ = sum_{q1,q2,q3} w00[i1][q1] w00[i2][q2] w00[i3][q3] kappa(q) B_j1(q1) B_j2(q2) B_j3(q3)
    K_IJ = sum_q kappa(q) [ w11 B_j1' . w00 B_j2 . w00 B_j3  (x derivative)
                          + w00 B_j1 . w11 B_j2' . w00 B_j3  (y)
                          + w00 B_j1 . w00 B_j2 . w11 B_j3' ](z)

Readings (the choices the method leaves open, fixed here):
  * points: two per element at its quarter points (a + h/4, a + 3h/4),
    except the first and the last element of each direction, which take
    p+1 points at a + h (r + 1/2)/(p+1), r = 0..p (a single element takes
    p+1); the points of direction d, in increasing order, form the grid on
    which kappa is given, kappa[q3][q2][q1] (x fastest);
  * knots: open, with simple interior knots (every element of positive
    length);
  * weights: the exactness conditions are fewer than the points in the
    support; the minimum-norm solution is taken (computed exactly, see
    Rule1D; the w11 system has one dependent condition, since the
    derivatives of the overlapping functions sum to zero on the support,
    and is consistent);
  * the integrals int B_i B_j, int B_i' B_j' are exact.
"""
from fractions import Fraction

import numpy as np

from . import basis_all, exact, gauss_legendre


def points_1d(t, p):
    """The weighted-quadrature points of one direction and, per element,
    the index of its first point: (x [npts], first [K+1])."""
    t = np.asarray(t, dtype=np.float64)
    K = len(t) - 2 * p - 1
    xs, first = [], [0]
    for e in range(K):
        a, b = t[e + p], t[e + p + 1]
        if not b > a:
            raise ValueError("weighted quadrature needs elements of positive length")
        R = p + 1 if (e == 0 or e == K - 1) else 2
        xs += [a + (b - a) * (r + 0.5) / R for r in range(R)]
        first.append(len(xs))
    return np.array(xs), np.array(first)


def _solve_exact(G, b):
    """Solve G y = b (G square, nonsingular; Fractions) by Gaussian
    elimination with exact arithmetic."""
    n = len(b)
    A = [list(G[r]) + [b[r]] for r in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        for r in range(c + 1, n):
            f = A[r][c] / A[c][c]
            if f:
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    y = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        y[r] = (A[r][n] - sum(A[r][k] * y[k] for k in range(r + 1, n))) / A[r][r]
    return y


def _min_norm_exact(A, b):
    """The minimum-norm solution w = A^T (A A^T)^-1 b of the full-row-rank
    system A w = b, in exact rational arithmetic."""
    m = len(A)
    G = [[sum(x * y for x, y in zip(A[r], A[c])) for c in range(m)] for r in range(m)]
    y = _solve_exact(G, b)
    return [sum(A[r][q] * y[r] for r in range(m)) for q in range(len(A[0]))]


def _gram_1d(t, p):
    """int B_i B_j and int B_i' B_j' (dense [N][N], floating point) by the
    (p+1)-point Gauss rule on every element, with the oracle's literal
    Cox-de Boor values (an independent check of the exact integrals)."""
    t = np.asarray(t, dtype=np.float64)
    K = len(t) - 2 * p - 1
    N = K + p
    xi, wi = gauss_legendre(p + 1)
    M = np.zeros((N, N))
    A = np.zeros((N, N))
    for e in range(K):
        a, b = t[e + p], t[e + p + 1]
        for k in range(p + 1):
            x = a + 0.5 * (xi[k] + 1.0) * (b - a)
            w = 0.5 * wi[k] * (b - a)
            B, dB = basis_all(t, p, x)
            M += w * np.outer(B, B)
            A += w * np.outer(dB, dB)
    return M, A


class Rule1D:
    """Weighted-quadrature rules of every basis function of one direction.

    x: points; first: first point of each element; lo[i], hi[i]: the points
    inside supp(B_i) are x[lo[i]:hi[i]]; w00[i], w11[i]: the weights on
    them; V, D: B_j(x_q), B_j'(x_q) for all points and functions.

    The knots (doubles, hence rationals) and the points are taken exactly;
    the basis polynomials and the integrals int B_i B_j, int B_i' B_j' come
    from exact.py, and every minimum-norm solve is done in rational
    arithmetic: the weights are the exact minimum-norm weights, rounded once
    to FP64 (the systems are ill-conditioned at high p, cond ~ 1e5 at p = 5,
    so a floating-point solve would carry errors of ~1e-12)."""

    def __init__(self, t, p):
        self.t = np.asarray(t, dtype=np.float64)
        self.p = p
        K = len(self.t) - 2 * p - 1
        N = K + p
        self.K, self.N = K, N
        self.x, self.first = points_1d(self.t, p)
        tf = [Fraction(float(v)) for v in self.t]
        spans, Bp = exact.basis_on_spans(tf, p)
        Mx, Ax = exact.matrices_1d(tf, p)
        # exact points: element e's r-th point a + h (2r + 1) / (2 R)
        xf, ef = [], []
        for e in range(K):
            a, b = tf[e + p], tf[e + p + 1]
            R = int(self.first[e + 1] - self.first[e])
            xf += [a + (b - a) * Fraction(2 * r + 1, 2 * R) for r in range(R)]
            ef += [e + p] * R   # the knot span holding the point
        sidx = {}
        for k, (lo, hi) in enumerate(spans):
            sidx.setdefault((lo, hi), k)
        Vf = [[Fraction(0)] * N for _ in xf]
        Df = [[Fraction(0)] * N for _ in xf]
        for q, (x, s) in enumerate(zip(xf, ef)):
            k = sidx[(tf[s], tf[s + 1])]
            for j in range(max(0, s - p), min(N - 1, s) + 1):
                if Bp[j][k]:
                    Vf[q][j] = exact.peval(Bp[j][k], x)
                    Df[q][j] = exact.peval(exact.pderiv(Bp[j][k]), x)
        self.V = np.array([[float(v) for v in row] for row in Vf])
        self.D = np.array([[float(v) for v in row] for row in Df])
        self.lo, self.hi, self.w00, self.w11 = [], [], [], []
        for i in range(N):
            lo, hi = self.first[max(0, i - p)], self.first[min(K - 1, i) + 1]
            j0, j1 = max(0, i - p), min(N - 1, i + p) + 1
            Av = [[Vf[q][j] for q in range(lo, hi)] for j in range(j0, j1)]
            Ad = [[Df[q][j] for q in range(lo, hi)] for j in range(j0, j1)]
            self.lo.append(lo)
            self.hi.append(hi)
            self.w00.append(np.array([float(v) for v in _min_norm_exact(Av, [Mx[i][j] for j in range(j0, j1)])]))
            # the derivatives of the overlapping functions sum to zero on the
            # support, so one condition is dependent: drop the last one (the
            # solution set, and so its minimum-norm element, is unchanged)
            self.w11.append(np.array([float(v) for v in
                                      _min_norm_exact(Ad[:-1], [Ax[i][j] for j in range(j0, j1 - 1)])]))

    def npts(self):
        return len(self.x)

    def matrices(self, f=None):
        """1D matrices of the rules with a weight f at the points (default 1):
        M[i][j] = sum_q w00[i][q] f(x_q) B_j(x_q), A[i][j] = sum_q w11[i][q]
        f(x_q) B_j'(x_q)  (dense [N][N])."""
        f = np.ones(self.npts()) if f is None else np.asarray(f, dtype=np.float64)
        M = np.zeros((self.N, self.N))
        A = np.zeros((self.N, self.N))
        for i in range(self.N):
            lo, hi = self.lo[i], self.hi[i]
            M[i] = (self.w00[i] * f[lo:hi]) @ self.V[lo:hi]
            A[i] = (self.w11[i] * f[lo:hi]) @ self.D[lo:hi]
        return M, A


def rules(knots, p):
    return [Rule1D(t, p) for t in knots]


def _row(R, kappa, I, p):
    """Row I = (i1, i2, i3): the structural columns (ascending) and their M
    and K values, each as the plain triple sum over the row's point box."""
    N = [r.N for r in R]
    i = [I % N[0], (I // N[0]) % N[1], I // (N[0] * N[1])]
    lo = [R[d].lo[i[d]] for d in range(3)]
    hi = [R[d].hi[i[d]] for d in range(3)]
    kb = kappa[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]          # [q3][q2][q1]
    js = [range(max(0, i[d] - p), min(N[d] - 1, i[d] + p) + 1) for d in range(3)]
    # per direction and column j: the weighted test values times the trial
    # values over the row's points
    a = [{j: R[d].w00[i[d]] * R[d].V[lo[d]:hi[d], j] for j in js[d]} for d in range(3)]
    g = [{j: R[d].w11[i[d]] * R[d].D[lo[d]:hi[d], j] for j in js[d]} for d in range(3)]
    cols, mv, kv = [], [], []
    for j3 in js[2]:
        for j2 in js[1]:
            for j1 in js[0]:
                wm = np.einsum("k,j,i->kji", a[2][j3], a[1][j2], a[0][j1])
                wk = (np.einsum("k,j,i->kji", a[2][j3], a[1][j2], g[0][j1]) +
                      np.einsum("k,j,i->kji", a[2][j3], g[1][j2], a[0][j1]) +
                      np.einsum("k,j,i->kji", g[2][j3], a[1][j2], a[0][j1]))
                cols.append(j1 + N[0] * (j2 + N[1] * j3))
                mv.append(float(np.sum(wm * kb)))
                kv.append(float(np.sum(wk * kb)))
    return np.array(cols, dtype=np.int32), np.array(mv), np.array(kv)


def assemble(knots, p, kappa):
    """CSR (row_ptr int64, col int32, Mval, Kval) of the weighted-quadrature
    matrices, structural pattern (|i_d - j_d| <= p), columns ascending.
    kappa: [npts_z][npts_y][npts_x] at the points of points_1d."""
    R = rules(knots, p)
    kappa = np.asarray(kappa, dtype=np.float64).reshape(R[2].npts(), R[1].npts(), R[0].npts())
    ndof = R[0].N * R[1].N * R[2].N
    rp = [0]
    cols, mv, kv = [], [], []
    for I in range(ndof):
        c, m, k = _row(R, kappa, I, p)
        cols.append(c)
        mv.append(m)
        kv.append(k)
        rp.append(rp[-1] + len(c))
    return (np.array(rp, dtype=np.int64), np.concatenate(cols), np.concatenate(mv), np.concatenate(kv))


def rows(knots, p, kappa, dofs):
    """The complete rows of the given global DOFs: list of (cols, M, K)."""
    R = rules(knots, p)
    kappa = np.asarray(kappa, dtype=np.float64).reshape(R[2].npts(), R[1].npts(), R[0].npts())
    return [_row(R, kappa, int(I), p) for I in dofs]
