// 1D basis tables (Cox-de Boor values and derivatives at the mapped Gauss
// nodes, Sec. 2.3 eqs. cox1/cox2) and the structural CSR pattern.
#include "common.h"
#include "launch.h"

namespace igaf {

// One thread per (element e, Gauss point k) of one direction.  The p+1
// functions that are non-zero on span s = e+p are built with the local
// triangular form of the Cox-de Boor recursion, the published scheme of
// Piegl and Tiller (The NURBS Book, 2nd ed., Algorithms A2.2 "BasisFuns" and
// A2.3 "DersBasisFuns": the ndu triangle holding the values of each degree
// above its diagonal and the knot differences below it, with the left/right
// distance arrays).  Every denominator is a knot difference that contains the
// span, so none is zero while the span is not empty; the first derivative
// uses the standard B-spline derivative formula (the same book, eq. 2.9) with
// the degree p-1 values of the same triangle.  A span of zero length (a
// repeated interior knot) has zero Gauss weights: all of its tables are zero,
// so the element adds nothing anywhere.  The elements of the run [r0, r1)
// (equal local knot windows) are all given the tables of element r0.
template <int P>
__global__ void k_basis_tables(const double* __restrict__ t, int K, const double* __restrict__ xi,
                               const double* __restrict__ wr, int Q, double* __restrict__ Wnn,
                               double* __restrict__ Wdd, double* __restrict__ Nv,
                               double* __restrict__ dN, double* __restrict__ wq, double* __restrict__ Wg,
                               int r0, int r1)
{
    constexpr int n = P + 1;
    constexpr int S = n * (n + 1) / 2;
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= K * Q) return;
    int e = gid / Q, k = gid % Q;
    int s = tab_elem(e, r0, r1) + P;   // the span whose values element e takes
    double x0 = t[s], x1 = t[s + 1], h = x1 - x0;
    double x = x0 + 0.5 * (xi[k] + 1.0) * h;
    double w = 0.5 * wr[k] * h;

    if (!(h > 0.0)) {
        for (int a = 0; a <= P; ++a) {
            Nv[((int64_t)e * n + a) * Q + k] = 0.0;
            dN[((int64_t)e * n + a) * Q + k] = 0.0;
        }
        wq[(int64_t)e * Q + k] = 0.0;
        for (int i = 0; i < 4 * n; ++i) Wg[((int64_t)e * 4 * n + i) * Q + k] = 0.0;
        for (int sp = 0; sp < S; ++sp) {
            Wnn[((int64_t)e * S + sp) * Q + k] = 0.0;
            Wdd[((int64_t)e * S + sp) * Q + k] = 0.0;
        }
        return;
    }
    double ndu[n][n];     // upper triangle: values per degree; lower: knot differences
    double left[n], right[n];
    ndu[0][0] = 1.0;
    for (int j = 1; j <= P; ++j) {
        left[j] = x - t[s + 1 - j];
        right[j] = t[s + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            ndu[j][r] = right[r + 1] + left[j - r];
            double tmp = ndu[r][j - 1] / ndu[j][r];
            ndu[r][j] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        ndu[j][j] = saved;
    }
    double N[n], D[n];
    for (int a = 0; a <= P; ++a) {
        N[a] = ndu[a][P];
        double lo = 0.0, hi = 0.0;
        if (a >= 1) lo = ndu[a - 1][P - 1] / (t[s + a] - t[s + a - P]);
        if (a <= P - 1) hi = ndu[a][P - 1] / (t[s + a + 1] - t[s + a + 1 - P]);
        D[a] = P * (lo - hi);
    }
    for (int a = 0; a <= P; ++a) {
        Nv[((int64_t)e * n + a) * Q + k] = N[a];
        dN[((int64_t)e * n + a) * Q + k] = D[a];
    }
    wq[(int64_t)e * Q + k] = w;
    for (int a = 0; a <= P; ++a) {
        Wg[(((int64_t)e * 4 + 0) * n + a) * Q + k] = w * N[a];
        Wg[(((int64_t)e * 4 + 1) * n + a) * Q + k] = w * D[a];
        Wg[(((int64_t)e * 4 + 2) * n + a) * Q + k] = N[a];
        Wg[(((int64_t)e * 4 + 3) * n + a) * Q + k] = D[a];
    }
    for (int b = 0; b <= P; ++b)
        for (int a = 0; a <= b; ++a) {
            int sp = pair_index(a, b);
            Wnn[((int64_t)e * S + sp) * Q + k] = w * N[a] * N[b];
            Wdd[((int64_t)e * S + sp) * Q + k] = w * D[a] * D[b];
        }
}

int launch_basis_tables(int p, const double* t, int K, const double* xi, const double* wr, int Q,
                        double* Wnn, double* Wdd, double* Nv, double* dN, double* wq, double* Wg,
                        int r0, int r1, hipStream_t st)
{
    int threads = 64;
    int blocks = (K * Q + threads - 1) / threads;
    switch (p) {
#define IGAF_CASE(PP)                                                                        \
    case PP:                                                                                 \
        hipLaunchKernelGGL(k_basis_tables<PP>, dim3(blocks), dim3(threads), 0, st, t, K, xi, \
                           wr, Q, Wnn, Wdd, Nv, dN, wq, Wg, r0, r1);                         \
        break;
        IGAF_CASE(1)
        IGAF_CASE(2)
        IGAF_CASE(3)
        IGAF_CASE(4)
        IGAF_CASE(5)
#undef IGAF_CASE
    default:
        return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// One thread per row (DOF): row_ptr from the closed form of RowMap and the
// ascending column list of the box |j_d - i_d| <= p (clipped to the patch).
__global__ void k_csr_pattern(RowMap rm, int64_t ndof, int64_t nnz, int64_t* __restrict__ row_ptr,
                              int32_t* __restrict__ col)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g > ndof) return;
    if (g == ndof) {
        row_ptr[ndof] = nnz;
        return;
    }
    int Nx = rm.N[0], Ny = rm.N[1], Nz = rm.N[2], p = rm.p;
    int ix = (int)(g % Nx);
    int iy = (int)((g / Nx) % Ny);
    int iz = (int)(g / ((int64_t)Nx * Ny));
    int64_t o = rm.row_start(ix, iy, iz);
    row_ptr[g] = o;
    for (int jz = band_lo(iz, p); jz <= band_hi(iz, p, Nz); ++jz)
        for (int jy = band_lo(iy, p); jy <= band_hi(iy, p, Ny); ++jy)
            for (int jx = band_lo(ix, p); jx <= band_hi(ix, p, Nx); ++jx)
                col[o++] = (int32_t)(jx + (int64_t)Nx * (jy + (int64_t)Ny * jz));
}

int launch_csr_pattern(const PatchDev& pd, int64_t* row_ptr, int32_t* col, hipStream_t st)
{
    RowMap rm = make_rowmap(pd);
    int threads = 256;
    int64_t blocks = (pd.ndof + 1 + threads - 1) / threads;
    hipLaunchKernelGGL(k_csr_pattern, dim3((unsigned)blocks), dim3(threads), 0, st, rm, pd.ndof,
                       pd.nnz, row_ptr, col);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace igaf
