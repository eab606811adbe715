// Shared device-side definitions of the HIP path (gfx950, FP64).
//
// Table layout of a patch, per direction d (built once per plan):
//   Wnn[e][s][k] = w_k (h_e/2) N_a(x_k) N_b(x_k)     s = pair index of a <= b
//   Wdd[e][s][k] = w_k (h_e/2) N'_a(x_k) N'_b(x_k)
//   Nv[e][a][k]  = N_{e+a}(x_k),  dN[e][a][k] = N'_{e+a}(x_k)
//   wq[e][k]     = w_k h_e/2
//   Wg[e][c][a][k] = w N_a, w N'_a, N_a, N'_a (c = 0..3): the ordered-pair
//                  factors of a mapped geometry, test side weighted
//   Lm[i][.]     = banded Cholesky factor and diagonal of the 1D mass matrix
//   pre[i]       = sum_{i' < i} L(i'),  L(i) = min(N-1, i+p) - max(0, i-p) + 1
// with x_k the Gauss nodes mapped to element e.  Pair products depend only on
// the unordered pair {a, b}, so S = (p+1)(p+2)/2 of them are stored.
//
// The values on an element depend only on its local knot window taken
// relative to the element (Sec. 2.3: the recursion reads the 2p knots around
// the span).  The elements [r0, r1) of a direction, a run whose windows agree
// up to the rounding of the knots (uniform spacing), all hold the tables
// computed for element r0, bit for bit; kernels that address the tables per
// element may read r0's copy for the whole run, which keeps the tables a
// workgroup touches in a few cache lines.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace igaf {

// Read-only table pointer in the constant address space: loads at
// wave-uniform addresses through it become scalar (SMEM) loads even where
// barriers or LDS traffic would stop the compiler from proving the global
// memory unclobbered.  Only for tables written before the kernel starts.
typedef const __attribute__((address_space(4))) double* ctab;
__host__ __device__ inline ctab as_ctab(const double* p) { return (ctab)(p); }

struct DirTables {
    const double* Wnn;
    const double* Wdd;
    const double* Nv;
    const double* dN;
    const double* wq;
    const double* Wg;     // [K][4][p+1][Q]
    const double* Lm;     // [N][p+2]: 1/L_ii, L_{i,i-1..i-p}, M_ii of the 1D mass (kappa = 1)
    const int64_t* pre;   // [N+1]
    int K, N, Q;
    int r0, r1;           // elements [r0, r1) hold the tables of element r0 (r0 = r1: none)
};

// the element whose copy of the tables element e may read
__host__ __device__ inline int tab_elem(int e, int r0, int r1) { return e >= r0 && e < r1 ? r0 : e; }

struct PatchDev {
    DirTables d[3];
    int p;
    int64_t E, ndof, nnz;
    int64_t T[3];   // number of (i, j) pairs with |i - j| <= p per direction
    int elem_grid;  // workgroups of the element kernels (grid-stride over elements)
};

// index of the unordered pair {a, b} among the (p+1)(p+2)/2 pairs
__host__ __device__ inline constexpr int pair_index(int a, int b)
{
    return a <= b ? b * (b + 1) / 2 + a : a * (a + 1) / 2 + b;
}

__host__ __device__ inline int band_lo(int i, int p) { return i - p < 0 ? 0 : i - p; }
__host__ __device__ inline int band_hi(int i, int p, int N) { return i + p > N - 1 ? N - 1 : i + p; }
__host__ __device__ inline int band_len(int i, int p, int N) { return band_hi(i, p, N) - band_lo(i, p) + 1; }

// Position in the CSR value arrays of entry (I, J), I = (ix,iy,iz), J = (jx,jy,jz),
// |i_d - j_d| <= p.  Rows are x-fastest; columns ascending.
struct RowMap {
    const int64_t* pre[3];
    int N[3];
    int p;
    int64_t T[3];   // T_d = pre_d[N_d]

    __device__ inline int64_t row_start(int ix, int iy, int iz) const
    {
        int64_t Lz = band_len(iz, p, N[2]);
        int64_t Ly = band_len(iy, p, N[1]);
        return pre[2][iz] * T[1] * T[0] + Lz * pre[1][iy] * T[0] + Lz * Ly * pre[0][ix];
    }
    __device__ inline int64_t pos(int ix, int iy, int iz, int jx, int jy, int jz) const
    {
        int Lx = band_len(ix, p, N[0]);
        int Ly = band_len(iy, p, N[1]);
        int off = ((jz - band_lo(iz, p)) * Ly + (jy - band_lo(iy, p))) * Lx + (jx - band_lo(ix, p));
        return row_start(ix, iy, iz) + off;
    }
};

inline RowMap make_rowmap(const PatchDev& pd)
{
    RowMap m;
    for (int d = 0; d < 3; ++d) {
        m.pre[d] = pd.d[d].pre;
        m.N[d] = pd.d[d].N;
    }
    m.p = pd.p;
    for (int d = 0; d < 3; ++d) m.T[d] = pd.T[d];
    return m;
}

// One patch of a batched launch, as the batched kernel reads it.
struct BatchPatch {
    PatchDev pd;
    RowMap rm;
    const double* kappa;
    double* Mv;
    double* Kv;
};

}  // namespace igaf
