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

// ---------------------------------------------------------------------------
// Wavefront-per-pencil form (used for p <= 4).  One 64-lane wavefront owns
// the rows iy (one y row), iz in [Z0, Z0+RZ), all ix, and sweeps the x
// elements with no workgroup barrier.  In every phase the coefficient tables
// are read at wave-uniform addresses (scalar loads) and each lane keeps its
// data column in registers:
//   phase 1: lane (kx, gy) holds the kappa column over the z window and forms
//            D[zpair][kx][gy] for every owned z pair (rz, oz);
//   phase 2: lane (zpair, kx) holds the D column over gy and forms
//            C[ypair, zpair][kx] for every y pair oy, into an LDS ring of p+1
//            x elements;
//   phase 3: lane (oy, rz, oz) reads its ring column and forms all (2p+1)
//            x offsets of row ix, each value summed here and stored once.
// Pair supports are compile-time: for a row i and column offset o the element
// i-p+e contributes iff 0 <= o-e <= p, with local pair (p-e, o-e).

// A zero the compiler cannot see through, one per loop iteration: adding it
// to the y/z table pointers keeps their (loop-invariant) scalar loads inside
// the x sweep, where they hit the scalar cache, instead of hoisting hundreds
// of values out of the loop and spilling them.
__device__ inline int opaque_zero()
{
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int P, int RZ>
struct WaveShape {
    static constexpr int n = P + 1;
    static constexpr int Q = P + 1;
    static constexpr int S = n * (n + 1) / 2;
    static constexpr int O = 2 * P + 1;
    static constexpr int Q3 = Q * Q * Q;
    static constexpr int WZ = RZ + P;            // z elements in the window
    static constexpr int GY = (P + 1) * Q;       // y points in the window (one row)
    static constexpr int GYP = GY | 1;           // padded LDS stride
    static constexpr int NPR = RZ * O;           // owned z pairs
    static constexpr int NC = O * RZ * O;        // (oy, rz, oz) combos
    static constexpr int N1 = Q * GY;            // phase-1 items
    static constexpr int N2 = NPR * Q;           // phase-2 items
    static constexpr int DSZ = 2 * NPR * Q * GYP;
    static constexpr int CSZ = (P + 1) * 2 * Q * NC;
    static constexpr int WAVE_LDS = DSZ + CSZ;   // doubles per wavefront
};

template <int P, int RZ>
__device__ void rows_wave_pencil(const PatchDev& pd, const RowMap& rm,
                                 const double* __restrict__ kappa, double* __restrict__ Mv,
                                 double* __restrict__ Kv, int iy, int Z0, double* __restrict__ D,
                                 double* __restrict__ C, int lane)
{
    using Sh = WaveShape<P, RZ>;
    constexpr int Q = Sh::Q, S = Sh::S, O = Sh::O, Q3 = Sh::Q3, WZ = Sh::WZ, GY = Sh::GY;
    constexpr int GYP = Sh::GYP, NPR = Sh::NPR, NC = Sh::NC;
    constexpr int NP1 = (Sh::N1 + 63) / 64;        // phase-1 passes
    const int Kx = pd.d[0].K, Ky = pd.d[1].K, Kz = pd.d[2].K;
    const int Nx = pd.d[0].N, Ny = pd.d[1].N, Nz = pd.d[2].N;
    const ctab Wnx = as_ctab(pd.d[0].Wnn), Wdx = as_ctab(pd.d[0].Wdd);
    const ctab Wny = as_ctab(pd.d[1].Wnn), Wdy = as_ctab(pd.d[1].Wdd);
    const ctab Wnz = as_ctab(pd.d[2].Wnn), Wdz = as_ctab(pd.d[2].Wdd);
    const int ey0 = iy - P, ez0 = Z0 - P;
    auto clampi = [](int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); };

    // Elements outside the patch (or pairs with a column outside it) need no
    // branch: their kappa entries are loaded as zero, which makes every D, C
    // and row term they would feed exactly zero; table addresses are clamped
    // so that every load stays in bounds and can be issued early.

    // kappa column of phase-1 item `it` for x element ex: [lz][kz]
    auto load_col = [&](int ex, int it, double (&cz)[WZ][Q]) {
        const int kx = it % Q, gy = it / Q, ly = gy / Q, ky = gy % Q;
        const int ey = ey0 + ly;
        const bool oky = ey >= 0 && ey < Ky && it < Sh::N1;
#pragma unroll
        for (int lz = 0; lz < WZ; ++lz) {
            const int ez = ez0 + lz;
            const bool ok = oky && ez >= 0 && ez < Kz;
            const int64_t e = ex + (int64_t)Kx * (clampi(ey, Ky - 1) + (int64_t)Ky * clampi(ez, Kz - 1));
            const double* kp = kappa + e * Q3 + kx + Q * ky;
#pragma unroll
            for (int kz = 0; kz < Q; ++kz) {
                const double v = kp[Q * Q * kz];
                cz[lz][kz] = ok ? v : 0.0;
            }
        }
    };

    // phase 3 for row ix: values are staged in LDS (over the D buffer, dead
    // until the next phase 1) at their position inside the CSR row, then every
    // owned row is written as one contiguous, coalesced segment.
    static_assert(2 * RZ * O * O * O <= Sh::DSZ, "row staging must fit in D");
    auto emit_row = [&](int ix) {
        const int Lx = band_len(ix, P, Nx), Ly = band_len(iy, P, Ny);
        for (int c0 = 0; c0 < NC; c0 += 64) {
            const bool act = c0 + lane < NC;
            const int c = act ? c0 + lane : NC - 1;
            const int oz = c % O, rz = (c / O) % RZ, oy = c / (O * RZ);
            const int iz = Z0 + rz, jy = iy + oy - P, jz = iz + oz - P;
            double ca[P + 1][Q], cb[P + 1][Q];
#pragma unroll
            for (int e = 0; e <= P; ++e) {
                const int ex = ix - P + e;
                const bool ok = ex >= 0 && ex < Kx;
                const int slot = clampi(ex, Kx - 1) % (P + 1);
#pragma unroll
                for (int kx = 0; kx < Q; ++kx) {
                    const double a = C[((slot * 2 + 0) * Q + kx) * NC + c];
                    const double b = C[((slot * 2 + 1) * Q + kx) * NC + c];
                    ca[e][kx] = ok ? a : 0.0;
                    cb[e][kx] = ok ? b : 0.0;
                }
            }
            const bool okrow = act && iz < Nz && jy >= 0 && jy < Ny && jz >= 0 && jz < Nz;
            const int izc = iz < Nz ? iz : Nz - 1;
            // position of (jx = ix - p + ox) inside the CSR row: rowoff + ox
            const int rowoff = ((jz - band_lo(izc, P)) * Ly + (jy - band_lo(iy, P))) * Lx +
                               (ix - P - band_lo(ix, P));
            double* stM = D + (rz * 2 + 0) * (O * O * O);
            double* stK = D + (rz * 2 + 1) * (O * O * O);
#pragma unroll
            for (int ox = 0; ox < O; ++ox) {
                double m = 0.0, k = 0.0;
#pragma unroll
                for (int e = 0; e <= P; ++e) {
                    if (ox - e < 0 || ox - e > P) continue;          // compile time
                    const int exc = clampi(ix - P + e, Kx - 1);
                    const int sp = pair_index(P - e, ox - e);
                    const ctab wn = Wnx + ((int64_t)exc * S + sp) * Q;
                    const ctab wd = Wdx + ((int64_t)exc * S + sp) * Q;
#pragma unroll
                    for (int kx = 0; kx < Q; ++kx) {
                        m += wn[kx] * ca[e][kx];
                        k += wd[kx] * ca[e][kx] + wn[kx] * cb[e][kx];
                    }
                }
                const int jx = ix + ox - P;
                if (okrow && jx >= 0 && jx < Nx) {
                    stM[rowoff + ox] = m;
                    stK[rowoff + ox] = k;
                }
            }
        }
        wave_sync();
#pragma unroll
        for (int rz = 0; rz < RZ; ++rz) {
            const int iz = Z0 + rz;
            if (iz >= Nz) break;
            const int L = Lx * Ly * band_len(iz, P, Nz);
            const int64_t rs = rm.row_start(ix, iy, iz);
            const double* stM = D + (rz * 2 + 0) * (O * O * O);
            const double* stK = D + (rz * 2 + 1) * (O * O * O);
            for (int i = lane; i < L; i += 64) {
                if (Mv) Mv[rs + i] = stM[i];
                if (Kv) Kv[rs + i] = stK[i];
            }
        }
        wave_sync();
    };

    double czn[NP1][WZ][Q];                         // next slice's kappa columns
#pragma unroll
    for (int ps = 0; ps < NP1; ++ps) load_col(0, ps * 64 + lane, czn[ps]);

    for (int ex = 0; ex < Kx; ++ex) {
        const int z0 = opaque_zero();
        const ctab Wnzi = Wnz + z0, Wdzi = Wdz + z0, Wnyi = Wny + z0, Wdyi = Wdy + z0;
        // phase 1: stage z
#pragma unroll
        for (int ps = 0; ps < NP1; ++ps) {
            const int it = ps * 64 + lane;
            const bool act = it < Sh::N1;
            const int kx = it % Q, gy = it / Q;
            double cz[WZ][Q];
#pragma unroll
            for (int lz = 0; lz < WZ; ++lz)
#pragma unroll
                for (int kz = 0; kz < Q; ++kz) cz[lz][kz] = czn[ps][lz][kz];
#pragma unroll
            for (int rz = 0; rz < RZ; ++rz) {
#pragma unroll
                for (int oz = 0; oz < O; ++oz) {
                    double d0 = 0.0, d1 = 0.0;
#pragma unroll
                    for (int e = 0; e <= P; ++e) {
                        if (oz - e < 0 || oz - e > P) continue;      // compile time
                        const int ezc = clampi(Z0 + rz - P + e, Kz - 1);
                        const int sp = pair_index(P - e, oz - e);
                        const ctab wn = Wnzi + ((int64_t)ezc * S + sp) * Q;
                        const ctab wd = Wdzi + ((int64_t)ezc * S + sp) * Q;
#pragma unroll
                        for (int kz = 0; kz < Q; ++kz) {
                            d0 += wn[kz] * cz[rz + e][kz];
                            d1 += wd[kz] * cz[rz + e][kz];
                        }
                    }
                    const int pr = rz * O + oz;
                    if (act) {
                        D[((0 * NPR + pr) * Q + kx) * GYP + gy] = d0;
                        D[((1 * NPR + pr) * Q + kx) * GYP + gy] = d1;
                    }
                }
            }
        }
        // prefetch the next slice's kappa while phases 2 and 3 run
        if (ex + 1 < Kx) {
#pragma unroll
            for (int ps = 0; ps < NP1; ++ps) load_col(ex + 1, ps * 64 + lane, czn[ps]);
        }
        wave_sync();
        // phase 2: stage y into ring slot ex % (p+1)
        const int slot = ex % (P + 1);
        for (int it0 = 0; it0 < Sh::N2; it0 += 64) {
            const bool act = it0 + lane < Sh::N2;
            const int it = act ? it0 + lane : Sh::N2 - 1;
            const int kx = it % Q, pr = it / Q, rz = pr / O, oz = pr % O;
            double d0[GY], d1[GY];
#pragma unroll
            for (int g = 0; g < GY; ++g) {
                d0[g] = D[((0 * NPR + pr) * Q + kx) * GYP + g];
                d1[g] = D[((1 * NPR + pr) * Q + kx) * GYP + g];
            }
#pragma unroll
            for (int oy = 0; oy < O; ++oy) {
                double ca = 0.0, cb = 0.0;
#pragma unroll
                for (int e = 0; e <= P; ++e) {
                    if (oy - e < 0 || oy - e > P) continue;          // compile time
                    const int eyc = clampi(iy - P + e, Ky - 1);
                    const int sp = pair_index(P - e, oy - e);
                    const ctab wn = Wnyi + ((int64_t)eyc * S + sp) * Q;
                    const ctab wd = Wdyi + ((int64_t)eyc * S + sp) * Q;
#pragma unroll
                    for (int ky = 0; ky < Q; ++ky) {
                        ca += wn[ky] * d0[e * Q + ky];
                        cb += wd[ky] * d0[e * Q + ky] + wn[ky] * d1[e * Q + ky];
                    }
                }
                const int c = (oy * RZ + rz) * O + oz;
                if (act) {
                    C[((slot * 2 + 0) * Q + kx) * NC + c] = ca;
                    C[((slot * 2 + 1) * Q + kx) * NC + c] = cb;
                }
            }
        }
        wave_sync();
        emit_row(ex);
    }
    for (int ix = Kx; ix < Nx; ++ix) emit_row(ix);
    wave_sync();
}

// Logical block index with XCD-aware order: the hardware hands workgroup b to
// XCD b % 8, so XCD x receives the contiguous logical range [x*nb8, (x+1)*nb8)
// and neighbouring pencils (which share kappa and tables) share one L2.
__device__ inline int xcd_block(int b, int nb8) { return (b % 8) * nb8 + b / 8; }

template <int P, int RZ, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_rows_wave(PatchDev pd, RowMap rm,
                                                        const double* __restrict__ kappa,
                                                        double* __restrict__ Mv,
                                                        double* __restrict__ Kv, int npencil,
                                                        int nb8)
{
    using Sh = WaveShape<P, RZ>;
    __shared__ double lds[WPB][Sh::WAVE_LDS];
    // wave index made provably uniform, so that pencil-derived addresses are scalar
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
    const int pencil = xcd_block(blockIdx.x, nb8) * WPB + w;
    if (pencil >= npencil) return;
    const int Ny = pd.d[1].N;
    const int iy = pencil % Ny, Z0 = (pencil / Ny) * RZ;
    rows_wave_pencil<P, RZ>(pd, rm, kappa, Mv, Kv, iy, Z0, lds[w], lds[w] + Sh::DSZ, lane);
}

template <int P, int RZ, int WPB>
static int launch_rows_wave_t(const PatchDev& pd, const double* kappa, double* Mv, double* Kv,
                              hipStream_t st)
{
    RowMap rm = make_rowmap(pd);
    int npz = (pd.d[2].N + RZ - 1) / RZ;
    int npencil = pd.d[1].N * npz;
    int nb = (npencil + WPB - 1) / WPB;
    int nb8 = (nb + 7) / 8;
    hipLaunchKernelGGL((k_rows_wave<P, RZ, WPB>), dim3(nb8 * 8), dim3(64 * WPB), 0, st, pd, rm,
                       kappa, Mv, Kv, npencil, nb8);
    return hipGetLastError() == hipSuccess ? 0 : -3;
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
    case 1: return launch_rows_wave_t<1, 2, 4>(pd, kappa, Mv, Kv, st);
    case 2: return launch_rows_wave_t<2, 2, 4>(pd, kappa, Mv, Kv, st);
    case 3: return launch_rows_wave_t<3, 1, 4>(pd, kappa, Mv, Kv, st);
    case 4: return launch_rows_wave_t<4, 1, 1>(pd, kappa, Mv, Kv, st);
    case 5: return launch_rows_t<5, 1, 1, 256>(pd, kappa, Mv, Kv, st);
    default: return -4;
    }
}

}  // namespace igaf
