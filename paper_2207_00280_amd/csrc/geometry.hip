// Element matrices on a mapped geometry x = F(xi) of the parameter cube.
//
// Eq. (10) integrates with a per-point factor J(x^n); on a mapped geometry
// the pull-back to the parameter cube gives, per quadrature point,
//   mass:       cm = kappa det J                    (a scalar, as before)
//   stiffness:  G  = kappa det J J^-1 J^-T          (a symmetric 3x3 tensor)
// since grad_x phi = J^-T grad_xi phi.  The caller evaluates both at the
// points (its geometry is its own); this file integrates
//   M_e[I][J] = sum_q cm_q phi_I phi_J
//   K_e[I][J] = sum_q sum_{c,d} G_cd,q d_c phi_I d_d phi_J
// by sum factorisation (Algorithm 2 order, z -> y -> x).  A diagonal term
// G_cc keeps the symmetric per-direction factors N_aN_b and N'_aN'_b of the
// identity geometry; a cross term G_cd (c != d) puts N'_a N_b in direction c
// and N_a N'_b in direction d, which are not symmetric in (a, b), so every
// direction works with ordered pairs (n^2 per direction, n^6 values).
//
// Per direction and element the ordered-pair factors are
//   nn[a][b][k] = w N_a N_b,  dd = w N'_a N'_b,  dn = w N'_a N_b,  nd = w N_a N'_b
// and the stages, for one test-z index a3 at a time (z pairs (a3, b3)):
//   stage z  (9 sums over kz):  D0 = nn.cm  D1 = nn.Gxx  D2 = nn.Gyy  D3 = dd.Gzz
//                               D4 = nn.Gxy D5 = nd.Gxz  D6 = dn.Gxz  D7 = nd.Gyz  D8 = dn.Gyz
//   stage y  (5 sums over ky), grouped by the x factor they meet:
//     CM  = nn D0                                  (mass, x factor nn)
//     Cnn = dd D2 + nn D3 + dn D7 + nd D8          (Kyy, Kzz, Kyz; x factor nn)
//     Cdd = nn D1                                  (Kxx; x factor dd)
//     Cdn = nd D4 + nn D5                          (Kxy, Kxz; x factor dn)
//     Cnd = dn D4 + nn D6                          (Kxy, Kxz; x factor nd)
//   stage x  (sum over kx):  M = nn CM,  K = nn Cnn + dd Cdd + dn Cdn + nd Cnd.
// The rows of one a3 are contiguous in M_e / K_e (n^2 rows of n^3), so the
// stores of one stage x are one contiguous run per matrix.
//
// One 256-thread workgroup per element (grid-stride), the stages in LDS; the
// next element's point coefficients are fetched into registers while the
// current one is computed.
#include "common.h"
#include "launch.h"

namespace igaf {

constexpr int kGeoThreads = 256;

template <int P>
struct GeoShape {
    static constexpr int n = P + 1, Q = P + 1;
    static constexpr int n2 = n * n, n3 = n2 * n, n4 = n3 * n, n5 = n4 * n, n6 = n3 * n3;
    static constexpr int Q2 = Q * Q, Q3 = Q2 * Q;
    static constexpr int NF = 7;                 // cm, Gxx, Gyy, Gzz, Gxy, Gxz, Gyz
    static constexpr int TB = n * Q;             // one 1D table of one direction: [a][k]
    static constexpr int DSZ = n * Q2;           // stage z result per field: [b3][kx][ky]
    static constexpr int CSZ = n3 * Q;           // stage y result per kind: [a2][b2][b3][kx]
    static constexpr int NPF = (NF * Q3 + kGeoThreads - 1) / kGeoThreads;
};

// The ordered-pair factors are products of a weighted value of the test
// function and a plain value of the trial function, e.g. nn[a][b][k] =
// (w N_a)[k] N_b[k], dn = (w N'_a) N_b, nd = (w N_a) N'_b.  Each stage keeps
// its thread on a fixed set of trial indices, folds the trial values into its
// inputs once, and then loops over the test index, whose weighted values are
// the same for every lane (LDS broadcast reads).
template <int P>
__global__ __launch_bounds__(kGeoThreads) void k_element_geo(PatchDev pd, const double* __restrict__ cm,
                                                             const double* __restrict__ G,
                                                             double* __restrict__ Me,
                                                             double* __restrict__ Ke)
{
    using Sh = GeoShape<P>;
    constexpr int n = Sh::n, Q = Sh::Q, n3 = Sh::n3, Q3 = Sh::Q3, T = kGeoThreads;
    __shared__ double fld[Sh::NF][Q3];
    __shared__ double raw[3][2][Sh::TB];         // [dir][N, N'][a Q + k]
    __shared__ double wsc[3][2][Sh::TB];         // [dir][w N, w N'][a Q + k]
    __shared__ double D[9][Sh::DSZ];
    __shared__ double C[5][Sh::CSZ];

    const int tid = threadIdx.x;
    const int Kx = pd.d[0].K, Ky = pd.d[1].K;
    const bool want_m = Me, want_k = Ke;
    const int64_t E = pd.E;

    double pf[Sh::NPF];
    auto fetch = [&](int64_t e) {
#pragma unroll
        for (int r = 0; r < Sh::NPF; ++r) {
            const int i = tid + r * T;
            double v = 0.0;
            if (i < Q3) {
                if (want_m) v = cm[e * Q3 + i];
            } else if (i < Sh::NF * Q3) {
                if (want_k) v = G[(e * 6 + (i / Q3 - 1)) * Q3 + i % Q3];
            }
            pf[r] = v;
        }
    };
    if (blockIdx.x < E) fetch(blockIdx.x);

    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int ex = (int)(e % Kx);
        const int ey = (int)((e / Kx) % Ky);
        const int ez = (int)(e / ((int64_t)Kx * Ky));
#pragma unroll
        for (int r = 0; r < Sh::NPF; ++r)
            if (tid + r * T < Sh::NF * Q3) (&fld[0][0])[tid + r * T] = pf[r];
        for (int i = tid; i < 3 * Sh::TB; i += T) {
            const int d = i / Sh::TB, r = i % Sh::TB;
            const int ed = d == 0 ? ex : (d == 1 ? ey : ez);
            const DirTables& t = pd.d[d];
            const double w = t.wq[(int64_t)ed * Q + r % Q];
            const double Nv = t.Nv[(int64_t)ed * Sh::TB + r], dN = t.dN[(int64_t)ed * Sh::TB + r];
            raw[d][0][r] = Nv;
            raw[d][1][r] = dN;
            wsc[d][0][r] = w * Nv;
            wsc[d][1][r] = w * dN;
        }
        __syncthreads();
        if (e + gridDim.x < E) fetch(e + gridDim.x);

        for (int a3 = 0; a3 < n; ++a3) {
            // stage z: thread on (b3, kx, ky)
            for (int i = tid; i < Sh::DSZ; i += T) {
                const int b3 = i / Sh::Q2, kx = (i / Q) % Q, ky = i % Q;
                double d[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int kz = 0; kz < Q; ++kz) {
                    const int kk = kx + Q * (ky + Q * kz);
                    const double Nb = raw[2][0][b3 * Q + kz], Db = raw[2][1][b3 * Q + kz];
                    const double sN = wsc[2][0][a3 * Q + kz], sD = wsc[2][1][a3 * Q + kz];
                    const double nn = sN * Nb, dd = sD * Db, dn = sD * Nb, nd = sN * Db;
                    d[0] += nn * fld[0][kk];
                    d[1] += nn * fld[1][kk];
                    d[2] += nn * fld[2][kk];
                    d[3] += dd * fld[3][kk];
                    d[4] += nn * fld[4][kk];
                    d[5] += nd * fld[5][kk];
                    d[6] += dn * fld[5][kk];
                    d[7] += nd * fld[6][kk];
                    d[8] += dn * fld[6][kk];
                }
#pragma unroll
                for (int f = 0; f < 9; ++f) D[f][i] = d[f];
            }
            __syncthreads();
            // stage y: thread on (b2, b3, kx), loop over the test index a2
            for (int i = tid; i < Sh::n2 * Q; i += T) {
                const int b2 = i / (n * Q), b3 = (i / Q) % n, kx = i % Q;
                double p0[Q], p1[Q], pa[Q], pb[Q], pc[Q], pd4[Q], pe[Q];
#pragma unroll
                for (int ky = 0; ky < Q; ++ky) {
                    const int j = (b3 * Q + kx) * Q + ky;
                    const double Nb = raw[1][0][b2 * Q + ky], Db = raw[1][1][b2 * Q + ky];
                    p0[ky] = Nb * D[0][j];
                    p1[ky] = Nb * D[1][j];
                    pa[ky] = Nb * D[3][j];
                    pa[ky] += Db * D[8][j];
                    pb[ky] = Db * D[2][j];
                    pb[ky] += Nb * D[7][j];
                    pc[ky] = Db * D[4][j];
                    pc[ky] += Nb * D[5][j];
                    pd4[ky] = Nb * D[4][j];
                    pe[ky] = Nb * D[6][j];
                }
                for (int a2 = 0; a2 < n; ++a2) {
                    double cM = 0.0, cnn = 0.0, cdd = 0.0, cdn = 0.0, cnd = 0.0;
#pragma unroll
                    for (int ky = 0; ky < Q; ++ky) {
                        const double sN = wsc[1][0][a2 * Q + ky], sD = wsc[1][1][a2 * Q + ky];
                        cM += sN * p0[ky];
                        cnn += sN * pa[ky];
                        cnn += sD * pb[ky];
                        cdd += sN * p1[ky];
                        cdn += sN * pc[ky];
                        cnd += sD * pd4[ky];
                        cnd += sN * pe[ky];
                    }
                    const int o = ((a2 * n + b2) * n + b3) * Q + kx;
                    C[0][o] = cM;
                    C[1][o] = cnn;
                    C[2][o] = cdd;
                    C[3][o] = cdn;
                    C[4][o] = cnd;
                }
            }
            __syncthreads();
            // stage x + store: thread on (a2, J), loop over the test index a1;
            // lanes run along a row, so every store is a contiguous run
            const int64_t base = e * Sh::n6 + (int64_t)a3 * Sh::n5;
            if constexpr (n % 2 == 0) {
                // two neighbouring trial indices b1, b1+1 per thread: the C
                // values are shared and every store writes 16 bytes
                for (int i = tid; i < Sh::n4 / 2; i += T) {
                    const int a2 = i / (n3 / 2), J = 2 * (i % (n3 / 2));
                    const int b1 = J % n, b2 = (J / n) % n, b3 = J / (n * n);
                    const int ci = ((a2 * n + b2) * n + b3) * Q;
                    double u0[Q], v0[Q], w0[Q], u1[Q], v1[Q], w1[Q];
#pragma unroll
                    for (int kx = 0; kx < Q; ++kx) {
                        const double c0 = C[0][ci + kx], c1 = C[1][ci + kx], c2 = C[2][ci + kx];
                        const double c3 = C[3][ci + kx], c4 = C[4][ci + kx];
                        const double N0 = raw[0][0][b1 * Q + kx], D0 = raw[0][1][b1 * Q + kx];
                        const double N1 = raw[0][0][(b1 + 1) * Q + kx], D1 = raw[0][1][(b1 + 1) * Q + kx];
                        u0[kx] = N0 * c1;
                        u0[kx] += D0 * c4;
                        v0[kx] = D0 * c2;
                        v0[kx] += N0 * c3;
                        w0[kx] = N0 * c0;
                        u1[kx] = N1 * c1;
                        u1[kx] += D1 * c4;
                        v1[kx] = D1 * c2;
                        v1[kx] += N1 * c3;
                        w1[kx] = N1 * c0;
                    }
                    for (int a1 = 0; a1 < n; ++a1) {
                        double m0 = 0.0, k0 = 0.0, m1 = 0.0, k1 = 0.0;
#pragma unroll
                        for (int kx = 0; kx < Q; ++kx) {
                            const double sN = wsc[0][0][a1 * Q + kx], sD = wsc[0][1][a1 * Q + kx];
                            m0 += sN * w0[kx];
                            k0 += sN * u0[kx];
                            k0 += sD * v0[kx];
                            m1 += sN * w1[kx];
                            k1 += sN * u1[kx];
                            k1 += sD * v1[kx];
                        }
                        const int64_t at = base + (int64_t)(a2 * n + a1) * n3 + J;
                        if (Me) *reinterpret_cast<double2*>(Me + at) = make_double2(m0, m1);
                        if (Ke) *reinterpret_cast<double2*>(Ke + at) = make_double2(k0, k1);
                    }
                }
            } else {
                for (int i = tid; i < Sh::n4; i += T) {
                    const int a2 = i / n3, J = i % n3;
                    const int b1 = J % n, b2 = (J / n) % n, b3 = J / (n * n);
                    const int ci = ((a2 * n + b2) * n + b3) * Q;
                    double u[Q], v[Q], wm[Q];
#pragma unroll
                    for (int kx = 0; kx < Q; ++kx) {
                        const double Nb = raw[0][0][b1 * Q + kx], Db = raw[0][1][b1 * Q + kx];
                        u[kx] = Nb * C[1][ci + kx];
                        u[kx] += Db * C[4][ci + kx];
                        v[kx] = Db * C[2][ci + kx];
                        v[kx] += Nb * C[3][ci + kx];
                        wm[kx] = Nb * C[0][ci + kx];
                    }
                    for (int a1 = 0; a1 < n; ++a1) {
                        double m = 0.0, k = 0.0;
#pragma unroll
                        for (int kx = 0; kx < Q; ++kx) {
                            const double sN = wsc[0][0][a1 * Q + kx], sD = wsc[0][1][a1 * Q + kx];
                            m += sN * wm[kx];
                            k += sN * u[kx];
                            k += sD * v[kx];
                        }
                        const int64_t at = base + (int64_t)(a2 * n + a1) * n3 + J;
                        if (Me) Me[at] = m;
                        if (Ke) Ke[at] = k;
                    }
                }
            }
            __syncthreads();
        }
    }
}

template <int P>
static int launch_geo_t(const PatchDev& pd, const double* cm, const double* G, double* Me, double* Ke,
                        hipStream_t st)
{
    const int slots = device_slots((const void*)k_element_geo<P>, kGeoThreads);
    if (!slots) return -3;
    if (pd.E <= 0) return 0;
    const int64_t blocks = pd.E < slots ? pd.E : slots;
    hipLaunchKernelGGL(k_element_geo<P>, dim3((unsigned)blocks), dim3(kGeoThreads), 0, st, pd, cm, G, Me, Ke);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_element_geo(const PatchDev& pd, const double* cm, const double* G, double* Me, double* Ke, hipStream_t st)
{
    switch (pd.p) {
    case 1: return launch_geo_t<1>(pd, cm, G, Me, Ke, st);
    case 2: return launch_geo_t<2>(pd, cm, G, Me, Ke, st);
    case 3: return launch_geo_t<3>(pd, cm, G, Me, Ke, st);
    case 4: return launch_geo_t<4>(pd, cm, G, Me, Ke, st);
    case 5: return launch_geo_t<5>(pd, cm, G, Me, Ke, st);
    default: return -4;
    }
}

}  // namespace igaf
