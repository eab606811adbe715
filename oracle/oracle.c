/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of what the
 * B-spline element-integration path computes.  It exists to check the HIP
 * path; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header or table with the HIP path.
 *
 * What it follows (paper: "A study of efficient concurrent integration
 * methods of B-Spline basis functions in IGA-FEM", arXiv 2207.00280):
 *   - open knot vector, Sec. 2.3 eq. (knot_vector): p+1 repeated end knots;
 *     read as K+2p+1 knots indexed 0..K+2p.  Interior knots may repeat up
 *     to p+1 times (the "more general B-spline basis functions" the paper
 *     says the method extends to, Sec. 2.3): the recursion below is the
 *     literal definition and needs no change for them;
 *   - Cox-de Boor recursion, Sec. 2.3 eqs. (cox1)/(cox2), with 0/0 := 0,
 *     evaluated for ALL K+p functions of a direction (no local shortcut);
 *   - derivatives by the textbook B-spline derivative formula (the paper
 *     only integrates the Gram matrix; the stiffness comes from the weak
 *     form eq. (weak_space)), with every c/0 term := 0;
 *   - tensor Gauss-Legendre quadrature with per-direction orders, eq. (10);
 *     the rule is computed here by Newton iteration on P_q;
 *   - classical integration, Algorithm 1: per element, loops over test /
 *     trial functions in x, y, z, then over the quadrature points;
 *     the coefficient kappa sits in the J(x^n) slot of eq. (10) next to
 *     the Jacobian det = prod_d h_d/2 (identity geometry on the unit cube);
 *   - global matrix = sum of element contributions (Sec. 3.1), emitted as
 *     CSR with the structural pattern (union of element pairs), columns
 *     ascending, numerically-zero entries kept.
 *
 * Conventions fixed where the paper is silent: element e_d = 0..K_d-1 spans
 * [t[e_d+p], t[e_d+p+1]] and carries global functions e_d..e_d+p (a span of
 * zero length is still an element: its Gauss weights w*h/2 are zero, so it
 * adds nothing to any integral, but it keeps its place in every layout and
 * in the structural pattern); local index
 * I = a1 + n(a2 + n a3) (x fastest); global DOF g = i + Nx(j + Ny k);
 * kappa / gradient layout [E][qz][qy][qx], e = ex + Kx(ey + Ky ez).
 *
 * Every pin of this file lives in tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXQ 32

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1] (eq. (10) "proper exact quadrature").  */
/* Nodes ascending.  Newton iteration on the Legendre polynomial P_q,   */
/* starting from the Chebyshev-like guess cos(pi (i+3/4)/(q+1/2)).      */
/* ------------------------------------------------------------------ */
int orc_gauss_legendre(int q, double* x, double* w)
{
    if (q < 1 || q > ORC_MAXQ) return -1;
    for (int i = 0; i < q; ++i) {
        double z = cos(M_PI * (i + 0.75) / (q + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;               /* P_0, P_1 */
            for (int k = 2; k <= q; ++k) {         /* Bonnet recursion */
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pq = (q == 1) ? z : p1;
            double pqm1 = (q == 1) ? 1.0 : p0;
            dp = q * (z * pq - pqm1) / (z * z - 1.0);   /* P_q'(z) */
            double dz = pq / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        /* recompute P_q' at the converged node for the weight */
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pq = (q == 1) ? z : p1;
            double pqm1 = (q == 1) ? 1.0 : p0;
            dp = q * (z * pq - pqm1) / (z * z - 1.0);
        }
        x[q - 1 - i] = z;                      /* guesses run descending */
        w[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Cox-de Boor, eqs. (cox1)/(cox2): values of all nk-p-1 functions of   */
/* degree p at x, plus (optionally) their first derivatives.            */
/* The degree-0 indicator is half-open [t_i, t_{i+1}); at the right end */
/* of the parameter range (x == t[nk-1]) the last non-empty span is     */
/* taken as closed, so that the basis is defined on the whole [0,1].    */
/* ------------------------------------------------------------------ */
void orc_basis_all(const double* t, int nk, int p, double x, double* B, double* dB)
{
    int nb0 = nk - 1;                          /* number of degree-0 functions */
    double* b = (double*)malloc(sizeof(double) * (size_t)nb0);
    double* bm1 = (double*)malloc(sizeof(double) * (size_t)nb0);
    for (int i = 0; i < nb0; ++i)
        b[i] = (t[i] <= x && x < t[i + 1]) ? 1.0 : 0.0;
    if (x == t[nk - 1]) {                      /* closed right end */
        for (int i = nb0 - 1; i >= 0; --i)
            if (t[i] < t[i + 1]) { b[i] = 1.0; break; }
    }
    memcpy(bm1, b, sizeof(double) * (size_t)nb0);
    for (int q = 1; q <= p; ++q) {
        if (q == p) memcpy(bm1, b, sizeof(double) * (size_t)nb0);
        for (int i = 0; i + q + 1 < nk; ++i) {
            double dl = t[i + q] - t[i];
            double dr = t[i + q + 1] - t[i + 1];
            double left = (dl == 0.0) ? 0.0 : (x - t[i]) / dl * b[i];
            double right = (dr == 0.0) ? 0.0 : (t[i + q + 1] - x) / dr * b[i + 1];
            b[i] = left + right;               /* b[i+1] is still degree q-1 */
        }
    }
    int nb = nk - p - 1;
    for (int i = 0; i < nb; ++i) B[i] = b[i];
    if (dB) {
        /* textbook derivative: p/(t_{i+p}-t_i) B_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) B_{i+1,p-1} */
        for (int i = 0; i < nb; ++i) {
            double dl = t[i + p] - t[i];
            double dr = t[i + p + 1] - t[i + 1];
            double a = (dl == 0.0) ? 0.0 : p / dl * bm1[i];
            double c = (dr == 0.0) ? 0.0 : p / dr * bm1[i + 1];
            dB[i] = a - c;
        }
    }
    free(b);
    free(bm1);
}

/* ------------------------------------------------------------------ */
/* Patch description (the oracle's own; no header is shared).           */
/* ------------------------------------------------------------------ */
typedef struct {
    int p;
    int K[3];
    int q[3];
    const double* t[3];   /* knots, length K[d]+2p+1 */
} orc_patch;

static orc_patch make_patch(int p, const int* K, const int* q, const double* tx,
                            const double* ty, const double* tz)
{
    orc_patch P;
    P.p = p;
    for (int d = 0; d < 3; ++d) { P.K[d] = K[d]; P.q[d] = q[d]; }
    P.t[0] = tx;
    P.t[1] = ty;
    P.t[2] = tz;
    return P;
}

/* Returns 0 if the patch is acceptable: p >= 1, K_d >= 1, 1 <= q_d <= 32,
 * each knot vector of length K_d+2p+1, nondecreasing, open (first p+1 and
 * last p+1 knots equal), and no basis function identically zero: the
 * support [t_i, t_{i+p+1}] of every function is a non-empty interval. */
int orc_validate(int p, const int* K, const int* q, const double* tx, const double* ty,
                 const double* tz)
{
    if (p < 1) return -1;
    const double* ts[3] = {tx, ty, tz};
    for (int d = 0; d < 3; ++d) {
        if (K[d] < 1 || q[d] < 1 || q[d] > ORC_MAXQ || !ts[d]) return -1;
        const double* t = ts[d];
        int nk = K[d] + 2 * p + 1;
        for (int i = 0; i + 1 < nk; ++i)
            if (!(t[i] <= t[i + 1])) return -1;
        for (int i = 1; i <= p; ++i)
            if (t[i] != t[0] || t[nk - 1 - i] != t[nk - 1]) return -1;
        for (int i = 0; i + p + 1 < nk; ++i)
            if (!(t[i] < t[i + p + 1])) return -1;
    }
    return 0;
}

/* Per-direction, per-element 1D data: mapped nodes, weights w*h/2,
 * local basis values N[a][k] and derivatives dN[a][k], a=0..p. */
typedef struct {
    double x[ORC_MAXQ];
    double w[ORC_MAXQ];
    double N[ORC_MAXQ][ORC_MAXQ];  /* [a][k] */
    double dN[ORC_MAXQ][ORC_MAXQ];
} elem1d;

static void element_1d(const orc_patch* P, int d, int e, elem1d* out)
{
    int p = P->p, q = P->q[d];
    const double* t = P->t[d];
    int nk = P->K[d] + 2 * p + 1;
    int nb = nk - p - 1;
    double xi[ORC_MAXQ], wr[ORC_MAXQ];
    orc_gauss_legendre(q, xi, wr);
    double x0 = t[e + p], x1 = t[e + p + 1], h = x1 - x0;
    double* B = (double*)malloc(sizeof(double) * (size_t)nb);
    double* dB = (double*)malloc(sizeof(double) * (size_t)nb);
    for (int k = 0; k < q; ++k) {
        out->x[k] = x0 + (xi[k] + 1.0) * h / 2.0;
        out->w[k] = wr[k] * h / 2.0;
        orc_basis_all(t, nk, p, out->x[k], B, dB);
        for (int a = 0; a <= p; ++a) {
            out->N[a][k] = B[e + a];
            out->dN[a][k] = dB[e + a];
        }
    }
    free(B);
    free(dB);
}

/* Mapped quadrature nodes of direction d: x[e*q + k]. */
int orc_quad_nodes(int p, const int* K, const int* q, const double* tx, const double* ty,
                   const double* tz, int d, double* x, double* w)
{
    if (orc_validate(p, K, q, tx, ty, tz)) return -1;
    orc_patch P = make_patch(p, K, q, tx, ty, tz);
    for (int e = 0; e < K[d]; ++e) {
        elem1d E;
        element_1d(&P, d, e, &E);
        for (int k = 0; k < q[d]; ++k) {
            x[(size_t)e * q[d] + k] = E.x[k];
            if (w) w[(size_t)e * q[d] + k] = E.w[k];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Classical integration, Algorithm 1, for one element.                 */
/* Me/Ke: [n^3][n^3] row-major, may be NULL.  kap: the element's q^3   */
/* coefficient values, [qz][qy][qx].                                    */
/* ------------------------------------------------------------------ */
static void classical_element(const orc_patch* P, int ex, int ey, int ez, const double* kap,
                              double* Me, double* Ke)
{
    int p = P->p, n = p + 1, n3 = n * n * n;
    int qx = P->q[0], qy = P->q[1], qz = P->q[2];
    elem1d X, Y, Z;
    element_1d(P, 0, ex, &X);
    element_1d(P, 1, ey, &Y);
    element_1d(P, 2, ez, &Z);
    for (int i1 = 0; i1 < n; ++i1)              /* test x  */
    for (int j1 = 0; j1 < n; ++j1)              /* trial x */
    for (int i2 = 0; i2 < n; ++i2)              /* test y  */
    for (int j2 = 0; j2 < n; ++j2)              /* trial y */
    for (int i3 = 0; i3 < n; ++i3)              /* test z  */
    for (int j3 = 0; j3 < n; ++j3) {            /* trial z */
        double m = 0.0, k = 0.0;
        for (int k1 = 0; k1 < qx; ++k1)
        for (int k2 = 0; k2 < qy; ++k2)
        for (int k3 = 0; k3 < qz; ++k3) {
            double c = kap[k1 + qx * (k2 + qy * k3)] * X.w[k1] * Y.w[k2] * Z.w[k3];
            double nx = X.N[i1][k1] * X.N[j1][k1], dx = X.dN[i1][k1] * X.dN[j1][k1];
            double ny = Y.N[i2][k2] * Y.N[j2][k2], dy = Y.dN[i2][k2] * Y.dN[j2][k2];
            double nz = Z.N[i3][k3] * Z.N[j3][k3], dz = Z.dN[i3][k3] * Z.dN[j3][k3];
            m += nx * ny * nz * c;
            k += (dx * ny * nz + nx * dy * nz + nx * ny * dz) * c;
        }
        int I = i1 + n * (i2 + n * i3);
        int J = j1 + n * (j2 + n * j3);
        if (Me) Me[(size_t)I * n3 + J] = m;
        if (Ke) Ke[(size_t)I * n3 + J] = k;
    }
}

/* ------------------------------------------------------------------ */
/* Classical integration on a mapped geometry.  With x = F(xi) and      */
/* J = dF/dxi at a point, eq. (10)'s J(x^n) slot becomes, for the mass, */
/* the scalar cm = kappa det J and, for the stiffness, the symmetric   */
/* 3x3 tensor G = kappa det J J^-1 J^-T, since grad_x phi =            */
/* J^-T grad_xi phi (chain rule).  The stiffness integrand is then     */
/* grad_xi phi_I^T G grad_xi phi_J, every term of the 3x3 product kept. */
/* cm: the element's q^3 values [qz][qy][qx]; G: its 6 q^3 blocks in   */
/* the order xx, yy, zz, xy, xz, yz.                                    */
/* ------------------------------------------------------------------ */
static void classical_element_geo(const orc_patch* P, int ex, int ey, int ez, const double* cm,
                                  const double* G, double* Me, double* Ke)
{
    int p = P->p, n = p + 1, n3 = n * n * n;
    int qx = P->q[0], qy = P->q[1], qz = P->q[2];
    int nq = qx * qy * qz;
    elem1d X, Y, Z;
    element_1d(P, 0, ex, &X);
    element_1d(P, 1, ey, &Y);
    element_1d(P, 2, ez, &Z);
    for (int i1 = 0; i1 < n; ++i1)              /* test x  */
    for (int j1 = 0; j1 < n; ++j1)              /* trial x */
    for (int i2 = 0; i2 < n; ++i2)              /* test y  */
    for (int j2 = 0; j2 < n; ++j2)              /* trial y */
    for (int i3 = 0; i3 < n; ++i3)              /* test z  */
    for (int j3 = 0; j3 < n; ++j3) {            /* trial z */
        double m = 0.0, k = 0.0;
        for (int k1 = 0; k1 < qx; ++k1)
        for (int k2 = 0; k2 < qy; ++k2)
        for (int k3 = 0; k3 < qz; ++k3) {
            int kk = k1 + qx * (k2 + qy * k3);
            double w = X.w[k1] * Y.w[k2] * Z.w[k3];
            double fi = X.N[i1][k1] * Y.N[i2][k2] * Z.N[i3][k3];
            double fj = X.N[j1][k1] * Y.N[j2][k2] * Z.N[j3][k3];
            double gi[3] = {X.dN[i1][k1] * Y.N[i2][k2] * Z.N[i3][k3],
                            X.N[i1][k1] * Y.dN[i2][k2] * Z.N[i3][k3],
                            X.N[i1][k1] * Y.N[i2][k2] * Z.dN[i3][k3]};
            double gj[3] = {X.dN[j1][k1] * Y.N[j2][k2] * Z.N[j3][k3],
                            X.N[j1][k1] * Y.dN[j2][k2] * Z.N[j3][k3],
                            X.N[j1][k1] * Y.N[j2][k2] * Z.dN[j3][k3]};
            double Gm[3][3];
            Gm[0][0] = G[0 * nq + kk];
            Gm[1][1] = G[1 * nq + kk];
            Gm[2][2] = G[2 * nq + kk];
            Gm[0][1] = Gm[1][0] = G[3 * nq + kk];
            Gm[0][2] = Gm[2][0] = G[4 * nq + kk];
            Gm[1][2] = Gm[2][1] = G[5 * nq + kk];
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) s += gi[a] * Gm[a][b] * gj[b];
            m += w * cm[kk] * fi * fj;
            k += w * s;
        }
        int I = i1 + n * (i2 + n * i3);
        int J = j1 + n * (j2 + n * j3);
        if (Me) Me[(size_t)I * n3 + J] = m;
        if (Ke) Ke[(size_t)I * n3 + J] = k;
    }
}

/* One element by either integrand: G == NULL is the identity geometry with
 * kappa in the J(x^n) slot; otherwise (cm, G) as above. */
static void element_any(const orc_patch* P, int64_t e, const double* c, const double* G,
                        double* Me, double* Ke)
{
    int ex = (int)(e % P->K[0]);
    int ey = (int)((e / P->K[0]) % P->K[1]);
    int ez = (int)(e / ((int64_t)P->K[0] * P->K[1]));
    int64_t nq = (int64_t)P->q[0] * P->q[1] * P->q[2];
    if (G)
        classical_element_geo(P, ex, ey, ez, c + e * nq, G + e * 6 * nq, Me, Ke);
    else
        classical_element(P, ex, ey, ez, c + e * nq, Me, Ke);
}

/* Element matrices for elements [e0, e1) (flat index e = ex + Kx(ey + Ky ez)).
 * kappa is the FULL [E][q^3] array; Me/Ke receive (e1-e0) matrices. */
static int element_matrices_any(int p, const int* K, const int* q, const double* tx,
                                const double* ty, const double* tz, const double* c,
                                const double* G, int64_t e0, int64_t e1, double* Me, double* Ke)
{
    if (orc_validate(p, K, q, tx, ty, tz) || !c) return -1;
    orc_patch P = make_patch(p, K, q, tx, ty, tz);
    int64_t n3 = (int64_t)(p + 1) * (p + 1) * (p + 1);
    int64_t E = (int64_t)K[0] * K[1] * K[2];
    if (e0 < 0 || e1 > E || e0 > e1) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t e = e0; e < e1; ++e)
        element_any(&P, e, c, G, Me ? Me + (e - e0) * n3 * n3 : NULL,
                    Ke ? Ke + (e - e0) * n3 * n3 : NULL);
    return 0;
}

int orc_element_matrices(int p, const int* K, const int* q, const double* tx, const double* ty,
                         const double* tz, const double* kappa, int64_t e0, int64_t e1,
                         double* Me, double* Ke)
{
    return element_matrices_any(p, K, q, tx, ty, tz, kappa, NULL, e0, e1, Me, Ke);
}

/* The same on a mapped geometry: cm [E][q^3], G [E][6][q^3] (see
 * classical_element_geo). */
int orc_element_matrices_geo(int p, const int* K, const int* q, const double* tx,
                             const double* ty, const double* tz, const double* cm,
                             const double* G, int64_t e0, int64_t e1, double* Me, double* Ke)
{
    if (!G) return -1;
    return element_matrices_any(p, K, q, tx, ty, tz, cm, G, e0, e1, Me, Ke);
}

/* ------------------------------------------------------------------ */
/* Global assembly (Sec. 3.1: A = sum over elements of A^gamma).        */
/* Rows are built by inserting every (g(e,I), g(e,J)) pair of every    */
/* element, in element order, into a per-row sorted column list.        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t* col;
    double* m;
    double* k;
    int len, cap;
} orc_row;

static void row_add(orc_row* r, int32_t c, double m, double k)
{
    int lo = 0, hi = r->len;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (r->col[mid] < c) lo = mid + 1; else hi = mid;
    }
    if (lo < r->len && r->col[lo] == c) {
        r->m[lo] += m;
        r->k[lo] += k;
        return;
    }
    if (r->len == r->cap) {
        r->cap = r->cap ? 2 * r->cap : 16;
        r->col = (int32_t*)realloc(r->col, sizeof(int32_t) * (size_t)r->cap);
        r->m = (double*)realloc(r->m, sizeof(double) * (size_t)r->cap);
        r->k = (double*)realloc(r->k, sizeof(double) * (size_t)r->cap);
    }
    memmove(r->col + lo + 1, r->col + lo, sizeof(int32_t) * (size_t)(r->len - lo));
    memmove(r->m + lo + 1, r->m + lo, sizeof(double) * (size_t)(r->len - lo));
    memmove(r->k + lo + 1, r->k + lo, sizeof(double) * (size_t)(r->len - lo));
    r->col[lo] = c;
    r->m[lo] = m;
    r->k[lo] = k;
    r->len++;
}

/* Sizes of the global system: ndof and the number of structural nonzeros,
 * counted by brute force over element pairs (no closed form used). */
static int64_t ndof_of(const orc_patch* P)
{
    return (int64_t)(P->K[0] + P->p) * (P->K[1] + P->p) * (P->K[2] + P->p);
}

/* Assemble the global CSR matrices.  Two-call protocol: with col == NULL the
 * function only returns nnz through *nnz_out (and fills row_ptr[ndof+1]);
 * with buffers it fills col[nnz], Mval[nnz], Kval[nnz] (Mval/Kval nullable).
 * kappa: [E][q^3]. */
static int assemble_any(int p, const int* K, const int* q, const double* tx, const double* ty,
                        const double* tz, const double* kappa, const double* G, int64_t* row_ptr,
                        int32_t* col, double* Mval, double* Kval, int64_t* nnz_out)
{
    if (orc_validate(p, K, q, tx, ty, tz) || !kappa) return -1;
    orc_patch P = make_patch(p, K, q, tx, ty, tz);
    int n = p + 1, n3 = n * n * n;
    int64_t E = (int64_t)K[0] * K[1] * K[2];
    int64_t N = ndof_of(&P);
    int Nx = K[0] + p, Ny = K[1] + p;
    orc_row* rows = (orc_row*)calloc((size_t)N, sizeof(orc_row));
    double* Me = (double*)malloc(sizeof(double) * (size_t)n3 * n3);
    double* Ke = (double*)malloc(sizeof(double) * (size_t)n3 * n3);
    for (int64_t e = 0; e < E; ++e) {
        int ex = (int)(e % K[0]);
        int ey = (int)((e / K[0]) % K[1]);
        int ez = (int)(e / ((int64_t)K[0] * K[1]));
        element_any(&P, e, kappa, G, Me, Ke);
        for (int I = 0; I < n3; ++I) {
            int a1 = I % n, a2 = (I / n) % n, a3 = I / (n * n);
            int64_t gI = (ex + a1) + (int64_t)Nx * ((ey + a2) + (int64_t)Ny * (ez + a3));
            for (int J = 0; J < n3; ++J) {
                int b1 = J % n, b2 = (J / n) % n, b3 = J / (n * n);
                int64_t gJ = (ex + b1) + (int64_t)Nx * ((ey + b2) + (int64_t)Ny * (ez + b3));
                row_add(&rows[gI], (int32_t)gJ, Me[(size_t)I * n3 + J], Ke[(size_t)I * n3 + J]);
            }
        }
    }
    int64_t nnz = 0;
    for (int64_t r = 0; r < N; ++r) {
        if (row_ptr) row_ptr[r] = nnz;
        nnz += rows[r].len;
    }
    if (row_ptr) row_ptr[N] = nnz;
    if (nnz_out) *nnz_out = nnz;
    if (col) {
        for (int64_t r = 0; r < N; ++r) {
            int64_t o = row_ptr[r];
            for (int j = 0; j < rows[r].len; ++j) {
                col[o + j] = rows[r].col[j];
                if (Mval) Mval[o + j] = rows[r].m[j];
                if (Kval) Kval[o + j] = rows[r].k[j];
            }
        }
    }
    for (int64_t r = 0; r < N; ++r) {
        free(rows[r].col);
        free(rows[r].m);
        free(rows[r].k);
    }
    free(rows);
    free(Me);
    free(Ke);
    return 0;
}

int orc_assemble(int p, const int* K, const int* q, const double* tx, const double* ty,
                 const double* tz, const double* kappa, int64_t* row_ptr, int32_t* col,
                 double* Mval, double* Kval, int64_t* nnz_out)
{
    return assemble_any(p, K, q, tx, ty, tz, kappa, NULL, row_ptr, col, Mval, Kval, nnz_out);
}

/* The same on a mapped geometry: cm [E][q^3], G [E][6][q^3]. */
int orc_assemble_geo(int p, const int* K, const int* q, const double* tx, const double* ty,
                     const double* tz, const double* cm, const double* G, int64_t* row_ptr,
                     int32_t* col, double* Mval, double* Kval, int64_t* nnz_out)
{
    if (!G) return -1;
    return assemble_any(p, K, q, tx, ty, tz, cm, G, row_ptr, col, Mval, Kval, nnz_out);
}

/* Complete rows of the global matrices for selected DOFs, without building
 * the whole matrix: each row is the sum, over the elements that carry the
 * DOF (Remark "element-by-element pre-computations"), of that element's
 * matrix row.  Output per selected row: up to (2p+1)^3 entries, written at
 * out_col/out_m/out_k + r*stride, with out_len[r] entries (columns sorted). */
static int rows_any(int p, const int* K, const int* q, const double* tx, const double* ty,
                    const double* tz, const double* kappa, const double* G, const int64_t* dofs,
                    int64_t ndofs, int32_t* out_col, double* out_m, double* out_k,
                    int32_t* out_len, int64_t stride)
{
    if (orc_validate(p, K, q, tx, ty, tz) || !kappa) return -1;
    orc_patch P = make_patch(p, K, q, tx, ty, tz);
    int n = p + 1, n3 = n * n * n;
    int Nd[3] = {K[0] + p, K[1] + p, K[2] + p};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < ndofs; ++r) {
        int64_t g = dofs[r];
        int i[3] = {(int)(g % Nd[0]), (int)((g / Nd[0]) % Nd[1]), (int)(g / ((int64_t)Nd[0] * Nd[1]))};
        orc_row row = {0};
        double* Me = (double*)malloc(sizeof(double) * (size_t)n3 * n3);
        double* Ke = (double*)malloc(sizeof(double) * (size_t)n3 * n3);
        for (int ez = 0; ez < K[2]; ++ez)
        for (int ey = 0; ey < K[1]; ++ey)
        for (int ex = 0; ex < K[0]; ++ex) {
            int a1 = i[0] - ex, a2 = i[1] - ey, a3 = i[2] - ez;
            if (a1 < 0 || a1 > p || a2 < 0 || a2 > p || a3 < 0 || a3 > p) continue;
            int64_t e = ex + (int64_t)K[0] * (ey + (int64_t)K[1] * ez);
            element_any(&P, e, kappa, G, Me, Ke);
            int I = a1 + n * (a2 + n * a3);
            for (int J = 0; J < n3; ++J) {
                int b1 = J % n, b2 = (J / n) % n, b3 = J / (n * n);
                int64_t gJ = (ex + b1) + (int64_t)Nd[0] * ((ey + b2) + (int64_t)Nd[1] * (ez + b3));
                row_add(&row, (int32_t)gJ, Me[(size_t)I * n3 + J], Ke[(size_t)I * n3 + J]);
            }
        }
        out_len[r] = row.len;
        for (int j = 0; j < row.len && j < stride; ++j) {
            out_col[r * stride + j] = row.col[j];
            if (out_m) out_m[r * stride + j] = row.m[j];
            if (out_k) out_k[r * stride + j] = row.k[j];
        }
        free(row.col);
        free(row.m);
        free(row.k);
        free(Me);
        free(Ke);
    }
    return 0;
}

int orc_rows(int p, const int* K, const int* q, const double* tx, const double* ty,
             const double* tz, const double* kappa, const int64_t* dofs, int64_t ndofs,
             int32_t* out_col, double* out_m, double* out_k, int32_t* out_len, int64_t stride)
{
    return rows_any(p, K, q, tx, ty, tz, kappa, NULL, dofs, ndofs, out_col, out_m, out_k, out_len,
                    stride);
}

/* The same on a mapped geometry: cm [E][q^3], G [E][6][q^3]. */
int orc_rows_geo(int p, const int* K, const int* q, const double* tx, const double* ty,
                 const double* tz, const double* cm, const double* G, const int64_t* dofs,
                 int64_t ndofs, int32_t* out_col, double* out_m, double* out_k, int32_t* out_len,
                 int64_t stride)
{
    if (!G) return -1;
    return rows_any(p, K, q, tx, ty, tz, cm, G, dofs, ndofs, out_col, out_m, out_k, out_len, stride);
}

/* ------------------------------------------------------------------ */
/* Reference gradient of L(kappa) = alphaM u^T M(kappa) v               */
/*                                 + alphaK u^T K(kappa) v              */
/* with respect to the coefficient value at every quadrature point.     */
/* L is linear in kappa_q: dL/dkappa_q = w_q detJ (alphaM u_h v_h +     */
/* alphaK grad u_h . grad v_h)(x_q), where u_h = sum_I u_I phi_I is      */
/* evaluated here point by point from the plain basis values.           */
/* grad: [E][qz][qy][qx], scaled by `scale`.                            */
/* ------------------------------------------------------------------ */
static int kappa_grad_any(int p, const int* K, const int* q, const double* tx, const double* ty,
                          const double* tz, const double* cm0, const double* G0, const double* u,
                          const double* v, double alphaM, double alphaK, double scale, double* grad);

int orc_kappa_grad(int p, const int* K, const int* q, const double* tx, const double* ty,
                   const double* tz, const double* u, const double* v, double alphaM,
                   double alphaK, double scale, double* grad)
{
    return kappa_grad_any(p, K, q, tx, ty, tz, NULL, NULL, u, v, alphaM, alphaK, scale, grad);
}

/* The same on a mapped geometry with kappa entering both coefficients
 * linearly, cm = kappa cm0 and G = kappa G0 (cm0 = det J, G0 = det J J^-1 J^-T):
 *   dL/dkappa_q = w_q (alphaM cm0 u_h v_h + alphaK grad u_h^T G0 grad v_h)(x_q),
 * gradients with respect to the parameter coordinates.  cm0 [E][q^3],
 * G0 [E][6][q^3] (xx yy zz xy xz yz). */
int orc_kappa_grad_geo(int p, const int* K, const int* q, const double* tx, const double* ty,
                       const double* tz, const double* cm0, const double* G0, const double* u,
                       const double* v, double alphaM, double alphaK, double scale, double* grad)
{
    if (!cm0 || !G0) return -1;
    return kappa_grad_any(p, K, q, tx, ty, tz, cm0, G0, u, v, alphaM, alphaK, scale, grad);
}

static int kappa_grad_any(int p, const int* K, const int* q, const double* tx, const double* ty,
                          const double* tz, const double* cm0, const double* G0, const double* u,
                          const double* v, double alphaM, double alphaK, double scale, double* grad)
{
    if (orc_validate(p, K, q, tx, ty, tz)) return -1;
    orc_patch P = make_patch(p, K, q, tx, ty, tz);
    int n = p + 1;
    int Nx = K[0] + p, Ny = K[1] + p;
    int64_t E = (int64_t)K[0] * K[1] * K[2];
    int qx = q[0], qy = q[1], qz = q[2];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t e = 0; e < E; ++e) {
        int ex = (int)(e % K[0]);
        int ey = (int)((e / K[0]) % K[1]);
        int ez = (int)(e / ((int64_t)K[0] * K[1]));
        elem1d X, Y, Z;
        element_1d(&P, 0, ex, &X);
        element_1d(&P, 1, ey, &Y);
        element_1d(&P, 2, ez, &Z);
        for (int k3 = 0; k3 < qz; ++k3)
        for (int k2 = 0; k2 < qy; ++k2)
        for (int k1 = 0; k1 < qx; ++k1) {
            double uh = 0, vh = 0, ug[3] = {0, 0, 0}, vg[3] = {0, 0, 0};
            for (int a3 = 0; a3 < n; ++a3)
            for (int a2 = 0; a2 < n; ++a2)
            for (int a1 = 0; a1 < n; ++a1) {
                int64_t g = (ex + a1) + (int64_t)Nx * ((ey + a2) + (int64_t)Ny * (ez + a3));
                double f = X.N[a1][k1] * Y.N[a2][k2] * Z.N[a3][k3];
                double fx = X.dN[a1][k1] * Y.N[a2][k2] * Z.N[a3][k3];
                double fy = X.N[a1][k1] * Y.dN[a2][k2] * Z.N[a3][k3];
                double fz = X.N[a1][k1] * Y.N[a2][k2] * Z.dN[a3][k3];
                uh += u[g] * f;
                vh += v[g] * f;
                ug[0] += u[g] * fx; ug[1] += u[g] * fy; ug[2] += u[g] * fz;
                vg[0] += v[g] * fx; vg[1] += v[g] * fy; vg[2] += v[g] * fz;
            }
            double wq = X.w[k1] * Y.w[k2] * Z.w[k3];
            int64_t nq = (int64_t)qx * qy * qz, kk = k1 + qx * (k2 + qy * k3);
            double val;
            if (G0) {
                double Gm[3][3];
                const double* g0 = G0 + e * 6 * nq + kk;
                Gm[0][0] = g0[0];
                Gm[1][1] = g0[nq];
                Gm[2][2] = g0[2 * nq];
                Gm[0][1] = Gm[1][0] = g0[3 * nq];
                Gm[0][2] = Gm[2][0] = g0[4 * nq];
                Gm[1][2] = Gm[2][1] = g0[5 * nq];
                double s = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) s += ug[a] * Gm[a][b] * vg[b];
                val = alphaM * cm0[e * nq + kk] * uh * vh + alphaK * s;
            } else {
                val = alphaM * uh * vh + alphaK * (ug[0] * vg[0] + ug[1] * vg[1] + ug[2] * vg[2]);
            }
            grad[e * nq + kk] = scale * wq * val;
        }
    }
    return 0;
}
