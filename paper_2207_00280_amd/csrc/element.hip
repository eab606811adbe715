// Element matrices of eq. (88) integrated with the tensor Gauss rule of eq. (10):
//   M_e[I][J] = sum_q c_q  prod_d w N_{a_d} N_{b_d}
//   K_e[I][J] = sum_q c_q (N'N'.NN.NN + NN.N'N'.NN + NN.NN.N'N')     (x, y, z factors)
// with c_q = kappa_q (the weights w h/2 of each direction sit in the tables).
//
// Two algorithms, the same result up to rounding order:
//   classical (Algorithm 1): every distinct matrix value is a full q^3-point sum;
//   sum factorisation (Algorithm 2, eqs. finalsum / bufferC): contract the
//     quadrature axes one at a time, z -> y -> x:
//       D_nn[zp][kx][ky] = sum_kz Wnn_z[zp][kz] c[kx,ky,kz]      (D_dd with Wdd_z)
//       C_a [yp][zp][kx] = sum_ky Wnn_y[yp][ky] D_nn[zp][kx][ky]
//       C_bc[yp][zp][kx] = sum_ky Wdd_y[yp][ky] D_nn + Wnn_y[yp][ky] D_dd
//       M[xp][yp][zp]    = sum_kx Wnn_x[xp][kx] C_a
//       K[xp][yp][zp]    = sum_kx Wdd_x[xp][kx] C_a + Wnn_x[xp][kx] C_bc
// Every factor N_a N_b (or N'_a N'_b) is symmetric in (a, b), so only the S^3
// values over unordered per-direction pairs are computed; the dense n^3 x n^3
// matrices are their expansion (S = (p+1)(p+2)/2; 1000 of 4096 at p = 3).
//
// One 256-thread workgroup per element (grid-stride); the stages live in LDS,
// separated by barriers (the paper's Foata classes become barrier phases).
// For odd p with dense outputs (k_element_ws) half of the workgroup stores
// the previous element while the other half contracts the current one.
#include "common.h"
#include "launch.h"

namespace igaf {

constexpr int kElemThreads = 256;

template <int P>
struct ElemShape {
    static constexpr int n = P + 1;
    static constexpr int Q = P + 1;
    static constexpr int S = n * (n + 1) / 2;
    static constexpr int n3 = n * n * n;
    static constexpr int n6 = n3 * n3;
    static constexpr int Q3 = Q * Q * Q;
    static constexpr int S3 = S * S * S;
    // all S^3 values fit in LDS up to p = 4; p = 5 works one test-z index at a time
    static constexpr bool VFULL = P <= 4;
    static constexpr int VN = VFULL ? S3 : n * S * S;
};

// METHOD 0 = classical, 1 = sum factorisation.
template <int P, int METHOD, bool ATOMIC>
__global__ __launch_bounds__(kElemThreads) void k_element(PatchDev pd, RowMap rm,
                                                          const double* __restrict__ kappa,
                                                          double* __restrict__ Me,
                                                          double* __restrict__ Ke,
                                                          double* __restrict__ Mv,
                                                          double* __restrict__ Kv)
{
    using Sh = ElemShape<P>;
    constexpr int n = Sh::n, Q = Sh::Q, S = Sh::S, n3 = Sh::n3, Q3 = Sh::Q3;
    constexpr int T = kElemThreads;
    __shared__ double kap[Q3];
    __shared__ double tw[3][2][S * Q];                       // [dir][nn, dd][s*Q + k]
    __shared__ double D[2][METHOD ? S * Q * Q : 1];          // [nn, dd][(zp*Q + kx)*Q + ky]
    __shared__ double C[2][METHOD ? S * S * Q : 1];          // [a, bc][(yp*S + zp)*Q + kx]
    __shared__ double V[2][Sh::VN];                          // [M, K]

    const int tid = threadIdx.x;
    const int Kx = pd.d[0].K, Ky = pd.d[1].K;

    // value (xp, yp, zp) of M and K
    auto value = [&](int xp, int yp, int zp, double& m, double& k) {
        m = 0.0;
        k = 0.0;
        if (METHOD == 1) {
#pragma unroll
            for (int kx = 0; kx < Q; ++kx) {
                double ca = C[0][(yp * S + zp) * Q + kx];
                double cb = C[1][(yp * S + zp) * Q + kx];
                double wn = tw[0][0][xp * Q + kx], wd = tw[0][1][xp * Q + kx];
                m += wn * ca;
                k += wd * ca + wn * cb;
            }
        } else {
            // the integrand at each point, with the factors of the y and z
            // directions formed once per (ky, kz): c nx (ny nz) for M and
            // c (dx (ny nz) + nx (dy nz + ny dz)) for K
            for (int kz = 0; kz < Q; ++kz) {
                double nz = tw[2][0][zp * Q + kz], dz = tw[2][1][zp * Q + kz];
#pragma unroll
                for (int ky = 0; ky < Q; ++ky) {
                    double ny = tw[1][0][yp * Q + ky], dy = tw[1][1][yp * Q + ky];
                    const double nyz = ny * nz, dyz = dy * nz + ny * dz;
#pragma unroll
                    for (int kx = 0; kx < Q; ++kx) {
                        double c = kap[kx + Q * (ky + Q * kz)];
                        double nx = tw[0][0][xp * Q + kx], dx = tw[0][1][xp * Q + kx];
                        const double cn = c * nyz;
                        m += cn * nx;
                        k += cn * dx;
                        k += (c * dyz) * nx;
                    }
                }
            }
        }
    };

    auto emit = [&](int64_t e, int ex, int ey, int ez, int i, double m, double k) {
        if (Me) Me[e * Sh::n6 + i] = m;
        if (Ke) Ke[e * Sh::n6 + i] = k;
        if (ATOMIC) {
            int I = i / n3, J = i % n3;
            int a1 = I % n, a2 = (I / n) % n, a3 = I / (n * n);
            int b1 = J % n, b2 = (J / n) % n, b3 = J / (n * n);
            int64_t pos = rm.pos(ex + a1, ey + a2, ez + a3, ex + b1, ey + b2, ez + b3);
            if (Mv) unsafeAtomicAdd(Mv + pos, m);
            if (Kv) unsafeAtomicAdd(Kv + pos, k);
        }
    };

    // the next element's kappa and tables are fetched into registers while
    // the current element is computed and stored
    constexpr int NKP = (Q3 + T - 1) / T, NTW = (6 * S * Q + T - 1) / T;
    double pk[NKP], pt[NTW];
    auto fetch = [&](int64_t e) {
        const int ex = (int)(e % Kx);
        const int ey = (int)((e / Kx) % Ky);
        const int ez = (int)(e / ((int64_t)Kx * Ky));
#pragma unroll
        for (int r = 0; r < NKP; ++r) {
            const int i = tid + r * T;
            pk[r] = i < Q3 ? kappa[e * Q3 + i] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < NTW; ++r) {
            const int i = tid + r * T;
            double val = 0.0;
            if (i < 6 * S * Q) {
                const int d = i / (2 * S * Q), rr = i % (2 * S * Q);
                const int which = rr / (S * Q), j = rr % (S * Q);
                const int ed = d == 0 ? ex : (d == 1 ? ey : ez);
                const double* src = which ? pd.d[d].Wdd : pd.d[d].Wnn;
                val = src[(int64_t)ed * S * Q + j];
            }
            pt[r] = val;
        }
    };
    if (blockIdx.x < pd.E) fetch(blockIdx.x);

    for (int64_t e = blockIdx.x; e < pd.E; e += gridDim.x) {
        const int ex = (int)(e % Kx);
        const int ey = (int)((e / Kx) % Ky);
        const int ez = (int)(e / ((int64_t)Kx * Ky));
#pragma unroll
        for (int r = 0; r < NKP; ++r)
            if (tid + r * T < Q3) kap[tid + r * T] = pk[r];
#pragma unroll
        for (int r = 0; r < NTW; ++r)
            if (tid + r * T < 6 * S * Q) (&tw[0][0][0])[tid + r * T] = pt[r];
        __syncthreads();
        if (e + gridDim.x < pd.E) fetch(e + gridDim.x);
        if (METHOD == 1) {
            for (int i = tid; i < S * Q * Q; i += T) {       // stage z
                int zp = i / (Q * Q), kx = (i / Q) % Q, ky = i % Q;
                double d0 = 0.0, d1 = 0.0;
#pragma unroll
                for (int kz = 0; kz < Q; ++kz) {
                    double c = kap[kx + Q * (ky + Q * kz)];
                    d0 += tw[2][0][zp * Q + kz] * c;
                    d1 += tw[2][1][zp * Q + kz] * c;
                }
                D[0][i] = d0;
                D[1][i] = d1;
            }
            __syncthreads();
            for (int i = tid; i < S * S * Q; i += T) {       // stage y
                int yp = i / (S * Q), zp = (i / Q) % S, kx = i % Q;
                double ca = 0.0, cb = 0.0;
#pragma unroll
                for (int ky = 0; ky < Q; ++ky) {
                    double wn = tw[1][0][yp * Q + ky], wd = tw[1][1][yp * Q + ky];
                    double d0 = D[0][(zp * Q + kx) * Q + ky], d1 = D[1][(zp * Q + kx) * Q + ky];
                    ca += wn * d0;
                    cb += wd * d0 + wn * d1;
                }
                C[0][i] = ca;
                C[1][i] = cb;
            }
            __syncthreads();
        }
        if (Sh::VFULL) {
            for (int i = tid; i < Sh::S3; i += T) {          // stage x (or the full sums)
                int xp = i % S, yp = (i / S) % S, zp = i / (S * S);
                double m, k;
                value(xp, yp, zp, m, k);
                V[0][i] = m;
                V[1][i] = k;
            }
            __syncthreads();
            if (!ATOMIC && n3 % 2 == 0) {
                // expand + store two consecutive entries of a row per lane (16-byte stores)
                for (int i2 = tid; i2 < Sh::n6 / 2; i2 += T) {
                    const int i = 2 * i2, I = i / n3, J = i % n3;
                    const int a1 = I % n, a2 = (I / n) % n, a3 = I / (n * n);
                    const int b2 = (J / n) % n, b3 = J / (n * n), b1 = J % n;
                    const int vyz = S * (pair_index(a2, b2) + S * pair_index(a3, b3));
                    const int v0 = pair_index(a1, b1) + vyz, v1 = pair_index(a1, b1 + 1) + vyz;
                    if (Me)
                        *reinterpret_cast<double2*>(Me + e * Sh::n6 + i) = make_double2(V[0][v0], V[0][v1]);
                    if (Ke)
                        *reinterpret_cast<double2*>(Ke + e * Sh::n6 + i) = make_double2(V[1][v0], V[1][v1]);
                }
            } else {
                for (int i = tid; i < Sh::n6; i += T) {      // expand + store
                    int I = i / n3, J = i % n3;
                    int a1 = I % n, a2 = (I / n) % n, a3 = I / (n * n);
                    int b1 = J % n, b2 = (J / n) % n, b3 = J / (n * n);
                    int v = pair_index(a1, b1) + S * (pair_index(a2, b2) + S * pair_index(a3, b3));
                    emit(e, ex, ey, ez, i, V[0][v], V[1][v]);
                }
            }
        } else {
            for (int a3 = 0; a3 < n; ++a3) {                 // one test-z index at a time
                for (int i = tid; i < n * S * S; i += T) {
                    int xp = i % S, yp = (i / S) % S, b3 = i / (S * S);
                    double m, k;
                    value(xp, yp, pair_index(a3, b3), m, k);
                    V[0][i] = m;
                    V[1][i] = k;
                }
                __syncthreads();
                constexpr int rows = n * n;                  // rows with this a3 are contiguous
                for (int r = tid; r < rows * n3; r += T) {
                    int I = a3 * rows + r / n3, J = r % n3;
                    int a1 = I % n, a2 = (I / n) % n;
                    int b1 = J % n, b2 = (J / n) % n, b3 = J / (n * n);
                    int v = pair_index(a1, b1) + S * (pair_index(a2, b2) + S * b3);
                    emit(e, ex, ey, ez, I * n3 + J, V[0][v], V[1][v]);
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
}

// Sum factorisation with the dense store split off (odd p, dense outputs
// only): wavefronts 0-1 contract element t (stages z, y, x into V[t & 1])
// while wavefronts 2-3 expand and store element t-1 from V[(t-1) & 1], a
// quarter of it between each pair of the iteration's four barriers, so the
// store stream does not stop for the contractions.
template <int P>
__global__ __launch_bounds__(kElemThreads) void k_element_ws(PatchDev pd, const double* __restrict__ kappa,
                                                             double* __restrict__ Me,
                                                             double* __restrict__ Ke)
{
    using Sh = ElemShape<P>;
    constexpr int n = Sh::n, Q = Sh::Q, S = Sh::S, n3 = Sh::n3, Q3 = Sh::Q3;
    constexpr int TC = 128, TS = kElemThreads - TC;   // contracting / storing threads
    static_assert(Sh::VFULL && n3 % 2 == 0, "paired stores of the full value set");
    __shared__ double kap[Q3];
    __shared__ double tw[3][2][S * Q];                 // [dir][nn, dd][s*Q + k]
    __shared__ double D[2][S * Q * Q];                 // [nn, dd][(zp*Q + kx)*Q + ky]
    __shared__ double C[2][S * S * Q];                 // [a, bc][(yp*S + zp)*Q + kx]
    __shared__ double V[2][2][Sh::S3];                 // [buffer][M, K]

    const int tid = threadIdx.x;
    const int Kx = pd.d[0].K, Ky = pd.d[1].K;
    // elements e0, e0 + G, ... of this workgroup
    const int64_t G = gridDim.x, e0 = blockIdx.x;
    const int nt = e0 < pd.E ? (int)((pd.E - 1 - e0) / G + 1) : 0;
    auto elem = [&](int t) { return e0 + (int64_t)t * G; };

    if (tid < TC) {
        constexpr int NKP = (Q3 + TC - 1) / TC, NTW = (6 * S * Q + TC - 1) / TC;
        double pk[NKP], pt[NTW];
        auto fetch = [&](int64_t e) {
            const int ex = (int)(e % Kx);
            const int ey = (int)((e / Kx) % Ky);
            const int ez = (int)(e / ((int64_t)Kx * Ky));
#pragma unroll
            for (int r = 0; r < NKP; ++r) {
                const int i = tid + r * TC;
                pk[r] = i < Q3 ? kappa[e * Q3 + i] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < NTW; ++r) {
                const int i = tid + r * TC;
                double val = 0.0;
                if (i < 6 * S * Q) {
                    const int d = i / (2 * S * Q), rr = i % (2 * S * Q);
                    const int which = rr / (S * Q), j = rr % (S * Q);
                    const int ed = d == 0 ? ex : (d == 1 ? ey : ez);
                    const double* src = which ? pd.d[d].Wdd : pd.d[d].Wnn;
                    val = src[(int64_t)ed * S * Q + j];
                }
                pt[r] = val;
            }
        };
        if (nt > 0) fetch(elem(0));
        for (int t = 0; t <= nt; ++t) {
            const bool el = t < nt;
            if (el) {
#pragma unroll
                for (int r = 0; r < NKP; ++r)
                    if (tid + r * TC < Q3) kap[tid + r * TC] = pk[r];
#pragma unroll
                for (int r = 0; r < NTW; ++r)
                    if (tid + r * TC < 6 * S * Q) (&tw[0][0][0])[tid + r * TC] = pt[r];
            }
            __syncthreads();
            if (el) {
                if (t + 1 < nt) fetch(elem(t + 1));
                for (int i = tid; i < S * Q * Q; i += TC) {   // stage z
                    const int zp = i / (Q * Q), kx = (i / Q) % Q, ky = i % Q;
                    double d0 = 0.0, d1 = 0.0;
#pragma unroll
                    for (int kz = 0; kz < Q; ++kz) {
                        const double c = kap[kx + Q * (ky + Q * kz)];
                        d0 += tw[2][0][zp * Q + kz] * c;
                        d1 += tw[2][1][zp * Q + kz] * c;
                    }
                    D[0][i] = d0;
                    D[1][i] = d1;
                }
            }
            __syncthreads();
            if (el) {
                for (int i = tid; i < S * S * Q; i += TC) {   // stage y
                    const int yp = i / (S * Q), zp = (i / Q) % S, kx = i % Q;
                    double ca = 0.0, cb = 0.0;
#pragma unroll
                    for (int ky = 0; ky < Q; ++ky) {
                        const double wn = tw[1][0][yp * Q + ky], wd = tw[1][1][yp * Q + ky];
                        const double d0 = D[0][(zp * Q + kx) * Q + ky], d1 = D[1][(zp * Q + kx) * Q + ky];
                        ca += wn * d0;
                        cb += wd * d0 + wn * d1;
                    }
                    C[0][i] = ca;
                    C[1][i] = cb;
                }
            }
            __syncthreads();
            if (el) {
                double* const Vm = V[t & 1][0];
                double* const Vk = V[t & 1][1];
                for (int i = tid; i < Sh::S3; i += TC) {       // stage x
                    const int xp = i % S, yp = (i / S) % S, zp = i / (S * S);
                    double m = 0.0, k = 0.0;
#pragma unroll
                    for (int kx = 0; kx < Q; ++kx) {
                        const double ca = C[0][(yp * S + zp) * Q + kx];
                        const double cb = C[1][(yp * S + zp) * Q + kx];
                        const double wn = tw[0][0][xp * Q + kx], wd = tw[0][1][xp * Q + kx];
                        m += wn * ca;
                        k += wd * ca + wn * cb;
                    }
                    Vm[i] = m;
                    Vk[i] = k;
                }
            }
            __syncthreads();
        }
    } else {
        constexpr int NI2 = Sh::n6 / 2;                      // two consecutive row entries per item
        constexpr int PER = (NI2 + 4 * TS - 1) / (4 * TS);   // items per thread between two barriers
        const int ts = tid - TC;
        for (int t = 0; t <= nt; ++t) {
            const bool st = t >= 1;
            const int64_t e = elem(t - 1);
            const double* const Vm = V[(t - 1) & 1][0];
            const double* const Vk = V[(t - 1) & 1][1];
#pragma unroll 1
            for (int ph = 0; ph < 4; ++ph) {
                if (st) {
#pragma unroll
                    for (int r = 0; r < PER; ++r) {
                        const int i2 = ts + (ph * PER + r) * TS;
                        if (i2 < NI2) {
                            const int i = 2 * i2, I = i / n3, J = i % n3;
                            const int a1 = I % n, a2 = (I / n) % n, a3 = I / (n * n);
                            const int b2 = (J / n) % n, b3 = J / (n * n), b1 = J % n;
                            const int vyz = S * (pair_index(a2, b2) + S * pair_index(a3, b3));
                            const int v0 = pair_index(a1, b1) + vyz, v1 = pair_index(a1, b1 + 1) + vyz;
                            if (Me)
                                *reinterpret_cast<double2*>(Me + e * Sh::n6 + i) = make_double2(Vm[v0], Vm[v1]);
                            if (Ke)
                                *reinterpret_cast<double2*>(Ke + e * Sh::n6 + i) = make_double2(Vk[v0], Vk[v1]);
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
}

template <int P, int METHOD, bool ATOMIC>
static int launch_element_t(const PatchDev& pd, const double* kappa, double* Me, double* Ke,
                            double* Mv, double* Kv, hipStream_t st)
{
    RowMap rm = make_rowmap(pd);
    int64_t blocks = pd.E < pd.elem_grid ? pd.E : pd.elem_grid;
    if constexpr (METHOD == 1 && !ATOMIC && ElemShape<P>::VFULL && ElemShape<P>::n3 % 2 == 0)
        hipLaunchKernelGGL(k_element_ws<P>, dim3((unsigned)blocks), dim3(kElemThreads), 0, st, pd, kappa, Me,
                           Ke);
    else
        hipLaunchKernelGGL((k_element<P, METHOD, ATOMIC>), dim3((unsigned)blocks), dim3(kElemThreads), 0,
                           st, pd, rm, kappa, Me, Ke, Mv, Kv);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_element(const PatchDev& pd, int method, const double* kappa, double* Me, double* Ke,
                   double* Mv, double* Kv, hipStream_t st)
{
    bool atomic = Mv || Kv;
#define IGAF_EL(PP)                                                                            \
    case PP:                                                                                   \
        if (method == 1)                                                                       \
            return atomic ? launch_element_t<PP, 1, true>(pd, kappa, Me, Ke, Mv, Kv, st)       \
                          : launch_element_t<PP, 1, false>(pd, kappa, Me, Ke, Mv, Kv, st);     \
        return atomic ? launch_element_t<PP, 0, true>(pd, kappa, Me, Ke, Mv, Kv, st)           \
                      : launch_element_t<PP, 0, false>(pd, kappa, Me, Ke, Mv, Kv, st);
    switch (pd.p) {
        IGAF_EL(1)
        IGAF_EL(2)
        IGAF_EL(3)
        IGAF_EL(4)
        IGAF_EL(5)
    default:
        return -4;
    }
#undef IGAF_EL
}

}  // namespace igaf
