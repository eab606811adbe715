// CSR values of the global mass and stiffness matrices, formed without
// atomics and without storing element matrices ("owner computes rows").
//
// The global matrix is the sum of the element matrices (Sec. 3.1).  Summing
// the sum-factorised element contractions over the elements that carry a
// pair of functions gives, for I = (ix,iy,iz), J = (jx,jy,jz):
//   M_IJ = sum_{gx,gy,gz} c[g] Bx(ix,jx)[gx] By(iy,jy)[gy] Bz(iz,jz)[gz]
// where g runs over the Gauss points of the elements in the common support
// and B(i,j)[g] = w N_i N_j is the pair table of the element holding g (the
// same tables the element kernels use).  The stiffness has the three
// derivative placements.  The contraction is done z -> y -> x as in
// Algorithm 2, but over global point sets, so every CSR value is summed in
// one thread and written once.
//
// Work decomposition (one workgroup = one pencil):
//   the pencil owns the rows iy in [Y0, Y0+RY), iz in [Z0, Z0+RZ), all ix;
//   it sweeps the x elements ex = 0..Kx-1 in order; for each x element it
//     phase 1 (stage z):  D[rz][oz][kx][gy]   for its y window of elements,
//     phase 2 (stage y):  C[ry][oy][rz][oz][kx] into a ring of p+1 slots,
//     phase 3 (stage x):  row ix = ex is now complete: every (ox, oy, oz)
//                         value of the owned rows with that ix is summed
//                         from the ring and stored (the p+1 last x rows after
//                         the sweep).
// o* in [0, 2p] are column offsets j = i + o - p.  Rows of one pencil are
// written as contiguous (2p+1)^3-entry CSR row segments.
#include "common.h"
#include "launch.h"

namespace igaf {

template <int P, int RY, int RZ>
struct RowsShape {
    static constexpr int n = P + 1;
    static constexpr int Q = P + 1;
    static constexpr int S = n * (n + 1) / 2;
    static constexpr int O = 2 * P + 1;
    static constexpr int Q3 = Q * Q * Q;
    static constexpr int WY = RY + P;              // y elements in the window
    static constexpr int WZ = RZ + P;
    static constexpr int GY = WY * Q;              // y Gauss points in the window
    static constexpr int NCOMBO = RY * O * RZ * O; // (ry, oy, rz, oz)
    static constexpr int DSZ = RZ * O * Q * GY;    // one D array
    static constexpr int CSZ = NCOMBO * Q;         // one C array (one ring slot)
};

template <int P, int RY, int RZ, int NT>
__global__ __launch_bounds__(NT) void k_rows(PatchDev pd, RowMap rm,
                                             const double* __restrict__ kappa,
                                             double* __restrict__ Mv, double* __restrict__ Kv)
{
    using Sh = RowsShape<P, RY, RZ>;
    constexpr int Q = Sh::Q, S = Sh::S, O = Sh::O, Q3 = Sh::Q3;
    constexpr int WY = Sh::WY, WZ = Sh::WZ, GY = Sh::GY;
    __shared__ double twy[2][WY][S * Q];
    __shared__ double twz[2][WZ][S * Q];
    __shared__ double twx[P + 2][2][S * Q];       // x tables, ring of p+2 x elements
    __shared__ double D[2][Sh::DSZ];
    __shared__ double C[P + 1][2][Sh::CSZ];       // ring of p+1 x elements

    const int tid = threadIdx.x;
    const int Kx = pd.d[0].K, Ky = pd.d[1].K, Kz = pd.d[2].K;
    const int Nx = pd.d[0].N, Ny = pd.d[1].N, Nz = pd.d[2].N;
    const int npy = (Ny + RY - 1) / RY;
    const int Y0 = (blockIdx.x % npy) * RY;
    const int Z0 = (blockIdx.x / npy) * RZ;
    const int ey0 = Y0 - P, ez0 = Z0 - P;         // first element of each window

    for (int i = tid; i < 2 * WY * S * Q; i += NT) {
        int w = i / (WY * S * Q), r = i % (WY * S * Q), ly = r / (S * Q), j = r % (S * Q);
        int ey = ey0 + ly;
        double v = 0.0;
        if (ey >= 0 && ey < Ky) v = (w ? pd.d[1].Wdd : pd.d[1].Wnn)[(int64_t)ey * S * Q + j];
        twy[w][ly][j] = v;
    }
    for (int i = tid; i < 2 * WZ * S * Q; i += NT) {
        int w = i / (WZ * S * Q), r = i % (WZ * S * Q), lz = r / (S * Q), j = r % (S * Q);
        int ez = ez0 + lz;
        double v = 0.0;
        if (ez >= 0 && ez < Kz) v = (w ? pd.d[2].Wdd : pd.d[2].Wnn)[(int64_t)ez * S * Q + j];
        twz[w][lz][j] = v;
    }

    // phase 3 for row ix: all owned (oy, oz) combos, all ox
    auto emit_row = [&](int ix) {
        for (int c = tid; c < Sh::NCOMBO; c += NT) {
            int oz = c % O, rz = (c / O) % RZ, oy = (c / (O * RZ)) % O, ry = c / (O * RZ * O);
            int iy = Y0 + ry, iz = Z0 + rz;
            int jy = iy + oy - P, jz = iz + oz - P;
            if (iy >= Ny || iz >= Nz || jy < 0 || jy >= Ny || jz < 0 || jz >= Nz) continue;
            int64_t rs = rm.row_start(ix, iy, iz);
            int Lx = band_len(ix, P, Nx), Ly = band_len(iy, P, Ny);
            int64_t base = rs + ((int64_t)(jz - band_lo(iz, P)) * Ly + (jy - band_lo(iy, P))) * Lx
                           - band_lo(ix, P);
            for (int ox = 0; ox < O; ++ox) {
                int jx = ix + ox - P;
                if (jx < 0 || jx >= Nx) continue;
                int lo = (ix > jx ? ix : jx) - P;
                int hi = ix < jx ? ix : jx;
                if (lo < 0) lo = 0;
                if (hi > Kx - 1) hi = Kx - 1;
                double m = 0.0, k = 0.0;
                for (int ex = lo; ex <= hi; ++ex) {
                    int sp = pair_index(ix - ex, jx - ex);
                    const double* wn = &twx[ex % (P + 2)][0][sp * Q];
                    const double* wd = &twx[ex % (P + 2)][1][sp * Q];
                    const double* ca = &C[ex % (P + 1)][0][c * Q];
                    const double* cb = &C[ex % (P + 1)][1][c * Q];
#pragma unroll
                    for (int kx = 0; kx < Q; ++kx) {
                        m += wn[kx] * ca[kx];
                        k += wd[kx] * ca[kx] + wn[kx] * cb[kx];
                    }
                }
                if (Mv) Mv[base + jx] = m;
                if (Kv) Kv[base + jx] = k;
            }
        }
    };

    for (int ex = 0; ex < Kx; ++ex) {
        for (int i = tid; i < 2 * S * Q; i += NT) {
            int w = i / (S * Q), j = i % (S * Q);
            twx[ex % (P + 2)][w][j] = (w ? pd.d[0].Wdd : pd.d[0].Wnn)[(int64_t)ex * S * Q + j];
        }
        __syncthreads();
        // phase 1, stage z: item (rz, gy, kx) -> D[.][rz][oz][kx][gy] for all oz
        for (int i = tid; i < RZ * GY * Q; i += NT) {
            int kx = i % Q, gy = (i / Q) % GY, rz = i / (Q * GY);
            int ly = gy / Q, ky = gy % Q;
            int ey = ey0 + ly;
            int iz = Z0 + rz;
            bool ok = ey >= 0 && ey < Ky && iz < Nz;
            // coefficient column of this (x, y) point over the z window
            double cz[WZ][Q];
#pragma unroll
            for (int lz = 0; lz < WZ; ++lz) {
                int ez = ez0 + lz;
                bool okz = ok && ez >= 0 && ez < Kz;
                const double* kp =
                    kappa + (ex + (int64_t)Kx * (ey + (int64_t)Ky * ez)) * Q3 + kx + Q * ky;
#pragma unroll
                for (int kz = 0; kz < Q; ++kz) cz[lz][kz] = okz ? kp[Q * Q * kz] : 0.0;
            }
#pragma unroll
            for (int oz = 0; oz < O; ++oz) {
                int jz = iz + oz - P;
                double d0 = 0.0, d1 = 0.0;
                if (ok && jz >= 0 && jz < Nz) {
                    int lo = (iz > jz ? iz : jz) - P, hi = iz < jz ? iz : jz;
                    if (lo < 0) lo = 0;
                    if (hi > Kz - 1) hi = Kz - 1;
#pragma unroll
                    for (int lz = 0; lz < WZ; ++lz) {
                        int ez = ez0 + lz;
                        if (ez < lo || ez > hi) continue;
                        int sp = pair_index(iz - ez, jz - ez);
#pragma unroll
                        for (int kz = 0; kz < Q; ++kz) {
                            d0 += twz[0][lz][sp * Q + kz] * cz[lz][kz];
                            d1 += twz[1][lz][sp * Q + kz] * cz[lz][kz];
                        }
                    }
                }
                int di = ((rz * O + oz) * Q + kx) * GY + gy;
                D[0][di] = d0;
                D[1][di] = d1;
            }
        }
        __syncthreads();
        // phase 2, stage y: item (ry, rz, oz, kx) -> C[slot][.][combo][kx] for all oy
        {
            const int slot = ex % (P + 1);
            for (int i = tid; i < RY * RZ * O * Q; i += NT) {
                int kx = i % Q, oz = (i / Q) % O, rz = (i / (Q * O)) % RZ, ry = i / (Q * O * RZ);
                int iy = Y0 + ry;
                const double* d0p = &D[0][((rz * O + oz) * Q + kx) * GY];
                const double* d1p = &D[1][((rz * O + oz) * Q + kx) * GY];
                for (int oy = 0; oy < O; ++oy) {
                    int jy = iy + oy - P;
                    double ca = 0.0, cb = 0.0;
                    if (iy < Ny && jy >= 0 && jy < Ny) {
                        int lo = (iy > jy ? iy : jy) - P, hi = iy < jy ? iy : jy;
                        if (lo < 0) lo = 0;
                        if (hi > Ky - 1) hi = Ky - 1;
                        for (int ey = lo; ey <= hi; ++ey) {
                            int ly = ey - ey0;
                            int sp = pair_index(iy - ey, jy - ey);
#pragma unroll
                            for (int ky = 0; ky < Q; ++ky) {
                                double wn = twy[0][ly][sp * Q + ky], wd = twy[1][ly][sp * Q + ky];
                                double a = d0p[ly * Q + ky], b = d1p[ly * Q + ky];
                                ca += wn * a;
                                cb += wd * a + wn * b;
                            }
                        }
                    }
                    int c = ((ry * O + oy) * RZ + rz) * O + oz;
                    C[slot][0][c * Q + kx] = ca;
                    C[slot][1][c * Q + kx] = cb;
                }
            }
        }
        __syncthreads();
        emit_row(ex);
    }
    for (int ix = Kx; ix < Nx; ++ix) emit_row(ix);
}

template <int P, int RY, int RZ, int NT>
static int launch_rows_t(const PatchDev& pd, const double* kappa, double* Mv, double* Kv,
                         hipStream_t st)
{
    RowMap rm = make_rowmap(pd);
    int npy = (pd.d[1].N + RY - 1) / RY;
    int npz = (pd.d[2].N + RZ - 1) / RZ;
    hipLaunchKernelGGL((k_rows<P, RY, RZ, NT>), dim3(npy * npz), dim3(NT), 0, st, pd, rm, kappa, Mv,
                       Kv);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_rows(const PatchDev& pd, const double* kappa, double* Mv, double* Kv, hipStream_t st)
{
    switch (pd.p) {
    case 1: return launch_rows_t<1, 4, 2, 256>(pd, kappa, Mv, Kv, st);
    case 2: return launch_rows_t<2, 2, 2, 256>(pd, kappa, Mv, Kv, st);
    case 3: return launch_rows_t<3, 2, 2, 256>(pd, kappa, Mv, Kv, st);
    case 4: return launch_rows_t<4, 2, 1, 256>(pd, kappa, Mv, Kv, st);
    case 5: return launch_rows_t<5, 1, 1, 256>(pd, kappa, Mv, Kv, st);
    default: return -4;
    }
}

}  // namespace igaf
