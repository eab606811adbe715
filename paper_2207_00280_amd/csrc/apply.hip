// Matrix-free operator apply: y = alphaM M(kappa) u + alphaK K(kappa) u.
//
// The global matrices are sums of element matrices (Sec. 3.1), so
//   y_I = sum_e sum_q c_q [alphaM phi_I u_h + alphaK grad phi_I . grad u_h](x_q)
// with c_q = kappa_q w_q (eq. (10), the coefficient in the J(x^n) slot).  Per
// element the n^3 coefficients of u are interpolated to the q^3 points by sum
// factorisation (x -> y -> z, value and derivative tables, as Algorithm 2
// contracts), weighted point by point, and contracted back against the test
// functions in the transposed order (z -> y -> x); no element or global
// matrix is formed.  The n^3 element results are added into y with FP64
// atomics (y is zeroed first), so the order of the additions, and the last
// bits of y, vary between runs.
//
// Work layout as in the adjoint: one 64-lane wavefront per x-run of elements
// (fixed ey, ez), elements in groups of G = 64 / n^2:
//   stage x:   lane (kx, a2, a3), one element at a time: sliding window of u
//              along x contracted with the x value / derivative tables;
//   stage y:   lane (g, kx, a3), every ky;
//   stage z:   lane (g, kx, ky), every kz: u_h and grad u_h at the points,
//              weighted there by kappa w (alphaM, alphaK folded in), then
//              contracted back over kz (transposed stage z);
//   stage y^T: lane (g, kx, a3), every a2;
//   stage x^T: lane (a1, a2, a3), one element at a time, every kx.  At
//              p <= 3 (one pass) the lanes of one DOF row along x pass their
//              partial sums down as the run advances, so each DOF takes one
//              atomic add per run instead of one per element (p+1 fewer).
#include "common.h"
#include "launch.h"

namespace igaf {

namespace {

constexpr int pmax(int a, int b) { return a > b ? a : b; }
constexpr int pmin(int a, int b) { return a < b ? a : b; }
constexpr int ppad16(int x, int r) { return x + (((r - x) % 16) + 16) % 16; }

// A zero the compiler cannot see through: table pointers rebased on it in
// every stage keep their scalar loads inside the stage instead of hoisting
// them for the whole run into scalar registers.
__device__ inline int ap_opaque_zero()
{
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}

__device__ inline void ap_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace

constexpr int kApplyRun = 32;   // elements per x-run of one wavefront

template <int P>
struct ApplyShape {
    static constexpr int n = P + 1, Q = P + 1, Q2 = Q * Q, Q3 = Q2 * Q;
    static constexpr int G = pmax(1, pmin(64 / (n * n), 8));    // elements per group
    static constexpr int NXI = n * n * Q, NXP = (NXI + 63) / 64;  // stage-x (and x^T) items per element
    static constexpr int NYI = G * Q * n;                         // stage-y (and y^T) items per group
    static constexpr int NZI = G * Q2;                            // stage-z items per group
    static_assert(NYI <= 64 && NZI <= 64, "one pass per group in stages y and z");
    // X[g][f2][a3][a2][kx] and Y[g][f3][a3][ky][kx] share one buffer
    static constexpr int XA3 = ppad16(n * Q, Q), XF = n * XA3, XG = 2 * XF;
    static constexpr int YA3 = ppad16(Q2, Q), YF = n * YA3, YG = 3 * YF;
    static constexpr int WS = pmax(G * XG, G * YG);               // doubles per wavefront
    static constexpr int RUN = kApplyRun;                         // elements per x-run
    // p <= 3: the run's finished DOF values, [a2 + n a3][ex - ex0], added to
    // y in one pass at the end of the run
    static constexpr int RB = NXP == 1 ? RUN * n * n : 0;
    // the x value / derivative tables of one group ([g][a][k], G n Q <= 64
    // values each), staged in LDS: one load per lane and table per group,
    // issued a group ahead
    static constexpr int TBN = G * n * Q;
    static_assert(TBN <= 64, "one table value per lane");
};

// GEO: a mapped geometry; `kappa` is the mass coefficient cm and Gt
// ([E][6][q^3]) the stiffness tensor, applied to the parametric gradient.
// MASS (alphaK = 0, the conjugate-gradient products of the Euler step): the
// gradient fields are neither interpolated nor contracted back.
template <int P, bool GEO, bool MASS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P <= 3 ? 4 : 2))) void k_apply(
    PatchDev pd, const double* __restrict__ kappa, const double* __restrict__ u, double alphaM,
    double alphaK, double* __restrict__ y, const double* __restrict__ Gt)
{
    using A = ApplyShape<P>;
    constexpr int n = A::n, Q = A::Q, Q2 = A::Q2, Q3 = A::Q3, G = A::G, NXP = A::NXP;
    __shared__ double lds[4][A::WS + A::RB + 128];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
    double* const B = lds[w];
    double* const RB = lds[w] + A::WS;
    double* const TB = lds[w] + A::WS + A::RB;   // [Nv | dN] of the group's elements
    const int Kx = pd.d[0].K, Ky = pd.d[1].K, Kz = pd.d[2].K;
    const int Nx = pd.d[0].N, Ny = pd.d[1].N;
    const double* __restrict__ Nvx = pd.d[0].Nv;
    const double* __restrict__ dNx = pd.d[0].dN;
    const double* __restrict__ wqx = pd.d[0].wq;
    const int nchunk = (Kx + A::RUN - 1) / A::RUN;
    const int nruns = nchunk * Ky * Kz;

    // fixed lane roles
    int xkx[NXP], xa2[NXP], xa3[NXP];   // stage x: item i = kx + Q (a2 + n a3)
    int ta1[NXP], ta2[NXP], ta3[NXP];   // stage x^T: item i = a1 + n (a2 + n a3)
#pragma unroll
    for (int ps = 0; ps < NXP; ++ps) {
        const int i = min(ps * 64 + lane, A::NXI - 1);
        xkx[ps] = i % Q;
        xa2[ps] = (i / Q) % n;
        xa3[ps] = i / (n * Q);
        ta1[ps] = i % n;
        ta2[ps] = (i / n) % n;
        ta3[ps] = i / (n * n);
    }
    const bool yact = lane < A::NYI;    // stages y, y^T: lane = kx + Q (a3 + n g)
    const int yl = yact ? lane : A::NYI - 1;
    const int ykx = yl % Q, ya3 = (yl / Q) % n, yg = yl / (Q * n);
    const bool zact = lane < A::NZI;    // stage z: lane = kx + Q (ky + Q g)
    const int zl = zact ? lane : A::NZI - 1;
    const int zkx = zl % Q, zky = (zl / Q) % Q, zg = zl / Q2;

    for (int run = blockIdx.x * 4 + w; run < nruns; run += gridDim.x * 4) {
        const int ch = run % nchunk, ey = (run / nchunk) % Ky, ez = run / (nchunk * Ky);
        const int ex0 = ch * A::RUN, ex1 = min(Kx, ex0 + A::RUN);
        const ctab Ny0 = as_ctab(pd.d[1].Nv) + (int64_t)ey * n * Q;
        const ctab Dy0 = as_ctab(pd.d[1].dN) + (int64_t)ey * n * Q;
        const ctab Nz0 = as_ctab(pd.d[2].Nv) + (int64_t)ez * n * Q;
        const ctab Dz0 = as_ctab(pd.d[2].dN) + (int64_t)ez * n * Q;
        const ctab wz0 = as_ctab(pd.d[2].wq) + (int64_t)ez * Q;
        const double wyl = pd.d[1].wq[(int64_t)ey * Q + zky];   // this lane's y weight
        // stage x^T with one pass (p <= 3): lane (a1, a2, a3) holds the partial
        // sum of DOF (ex + a1, ey + a2, ez + a3) over the run's elements so far
        double racc = 0.0;
        // sliding window of u along x at (a2, a3) of every stage-x item
        double uw[NXP][n];
        int64_t g0[NXP];
#pragma unroll
        for (int ps = 0; ps < NXP; ++ps) {
            g0[ps] = (int64_t)Nx * ((ey + xa2[ps]) + (int64_t)Ny * (ez + xa3[ps]));
#pragma unroll
            for (int a1 = 0; a1 < n; ++a1) uw[ps][a1] = u[g0[ps] + ex0 + a1];
        }
        // x tables of the group starting at element exg, this lane's value
        const int64_t tlast = (int64_t)Kx * n * Q - 1;
        double tnv = Nvx[min((int64_t)ex0 * n * Q + lane, tlast)];
        double tdn = MASS ? 0.0 : dNx[min((int64_t)ex0 * n * Q + lane, tlast)];
        // the u values a group shifts into the window (x = exg + n + g), also
        // loaded a group ahead
        double unx[NXP][G];
#pragma unroll
        for (int ps = 0; ps < NXP; ++ps)
#pragma unroll
            for (int g = 0; g < G; ++g) unx[ps][g] = u[g0[ps] + min(ex0 + n + g, Nx - 1)];
        const int64_t krow = (int64_t)Kx * (ey + (int64_t)Ky * ez);
        for (int exg = ex0; exg < ex1; exg += G) {
            const int ng = min(G, ex1 - exg);   // elements in this group
            // this lane's kappa (every kz) and x weight for stage z, loaded at
            // the group's start (a group ahead cost more in registers than it
            // hid)
            const int exz = exg + min(zg, ng - 1);
            double kc[Q];
            {
                const double* kp = kappa + (exz + krow) * Q3 + zky * Q + zkx;
#pragma unroll
                for (int kz = 0; kz < Q; ++kz) kc[kz] = kp[kz * Q2];
            }
            const double wxc = wqx[(int64_t)exz * Q + zkx];
            double ucur[NXP][G];
#pragma unroll
            for (int ps = 0; ps < NXP; ++ps)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    ucur[ps][g] = unx[ps][g];
                    unx[ps][g] = u[g0[ps] + min(exg + G + n + g, Nx - 1)];
                }
            TB[lane] = tnv;
            TB[64 + lane] = tdn;
            ap_wave_sync();
            if (exg + G < ex1) {   // the next group's tables, a group ahead
                tnv = Nvx[min((int64_t)(exg + G) * n * Q + lane, tlast)];
                if constexpr (!MASS) tdn = dNx[min((int64_t)(exg + G) * n * Q + lane, tlast)];
            }
            // ---- stage x, one element of the group at a time
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (g >= ng) break;   // wave-uniform
#pragma unroll
                for (int ps = 0; ps < NXP; ++ps) {
                    const bool act = ps * 64 + lane < A::NXI;
                    double s0 = 0.0, s1 = 0.0;
#pragma unroll
                    for (int a1 = 0; a1 < n; ++a1) {
                        const int t = (g * n + a1) * Q + xkx[ps];
                        s0 += uw[ps][a1] * TB[t];
                        if constexpr (!MASS) s1 += uw[ps][a1] * TB[64 + t];
                    }
                    if (act) {
                        double* xp = B + g * A::XG + xa3[ps] * A::XA3 + xa2[ps] * Q + xkx[ps];
                        xp[0] = s0;
                        if constexpr (!MASS) xp[A::XF] = s1;
                    }
#pragma unroll
                    for (int a1 = 0; a1 + 1 < n; ++a1) uw[ps][a1] = uw[ps][a1 + 1];
                    uw[ps][n - 1] = ucur[ps][g];
                }
            }
            ap_wave_sync();
            // ---- stage y: lane (g, kx, a3), every ky
            {
                const int z0 = ap_opaque_zero();
                const ctab Ny_ = Ny0 + z0, Dy_ = Dy0 + z0;
                double x0[n], x1[n];
                const double* xp = B + yg * A::XG + ya3 * A::XA3 + ykx;
#pragma unroll
                for (int a2 = 0; a2 < n; ++a2) {
                    x0[a2] = xp[a2 * Q];
                    x1[a2] = MASS ? 0.0 : xp[A::XF + a2 * Q];
                }
                ap_wave_sync();   // every read of X before the writes of Y over it
                double* yp = B + yg * A::YG + ya3 * A::YA3 + ykx;
#pragma unroll
                for (int ky = 0; ky < Q; ++ky) {
                    double o0 = 0.0, o1 = 0.0, o2 = 0.0;
#pragma unroll
                    for (int a2 = 0; a2 < n; ++a2) {
                        const double ny = Ny_[a2 * Q + ky];
                        o0 += ny * x0[a2];
                        if constexpr (!MASS) {
                            o1 += Dy_[a2 * Q + ky] * x0[a2];
                            o2 += ny * x1[a2];
                        }
                    }
                    if (yact && yg < ng) {
                        yp[ky * Q] = o0;
                        if constexpr (!MASS) {
                            yp[A::YF + ky * Q] = o1;
                            yp[2 * A::YF + ky * Q] = o2;
                        }
                    }
                }
            }
            ap_wave_sync();
            // ---- stage z: lane (g, kx, ky): the point values, weighted, and
            // straight back over kz (transposed stage z)
            {
                const int z0 = ap_opaque_zero();
                const ctab Nz_ = Nz0 + z0, Dz_ = Dz0 + z0, wz_ = wz0 + z0;
                double y0[n], y1[n], y2[n];
                const double* yp = B + zg * A::YG + zky * Q + zkx;
#pragma unroll
                for (int a3 = 0; a3 < n; ++a3) {
                    y0[a3] = yp[a3 * A::YA3];
                    y1[a3] = MASS ? 0.0 : yp[A::YF + a3 * A::YA3];
                    y2[a3] = MASS ? 0.0 : yp[2 * A::YF + a3 * A::YA3];
                }
                const double wxy = wxc * wyl;
                double s0[n], s1[n], s2[n];   // transposed stage z: [a3]
#pragma unroll
                for (int a3 = 0; a3 < n; ++a3) s0[a3] = s1[a3] = s2[a3] = 0.0;
#pragma unroll
                for (int kz = 0; kz < Q; ++kz) {
                    double h = 0.0, dz = 0.0, dy = 0.0, dx = 0.0;
#pragma unroll
                    for (int a3 = 0; a3 < n; ++a3) {
                        const double nz = Nz_[a3 * Q + kz];
                        h += nz * y0[a3];
                        if constexpr (!MASS) {
                            dz += Dz_[a3 * Q + kz] * y0[a3];
                            dy += nz * y1[a3];
                            dx += nz * y2[a3];
                        }
                    }
                    double t0, t1, t2, t3;
                    if constexpr (MASS) {
                        // the same products, in the same order, as the full forms below
                        if constexpr (GEO) t0 = alphaM * kc[kz] * (wxy * wz_[kz]) * h;
                        else t0 = alphaM * (kc[kz] * wxy * wz_[kz]) * h;
                        t1 = t2 = t3 = 0.0;
                    } else if constexpr (GEO) {
                        const double wk = wxy * wz_[kz];
                        const double* g = Gt + (exz + (int64_t)Kx * (ey + (int64_t)Ky * ez)) * 6 * Q3 + kz * Q2 +
                                          zky * Q + zkx;
                        const double gxx = g[0], gyy = g[Q3], gzz = g[2 * Q3];
                        const double gxy = g[3 * Q3], gxz = g[4 * Q3], gyz = g[5 * Q3];
                        t0 = alphaM * kc[kz] * wk * h;
                        t1 = alphaK * wk * (gxx * dx + gxy * dy + gxz * dz);
                        t2 = alphaK * wk * (gxy * dx + gyy * dy + gyz * dz);
                        t3 = alphaK * wk * (gxz * dx + gyz * dy + gzz * dz);
                    } else {
                        const double c = kc[kz] * wxy * wz_[kz];
                        t0 = alphaM * c * h;
                        t1 = alphaK * c * dx;
                        t2 = alphaK * c * dy;
                        t3 = alphaK * c * dz;
                    }
#pragma unroll
                    for (int a3 = 0; a3 < n; ++a3) {
                        const double nz = Nz_[a3 * Q + kz];
                        s0[a3] += nz * t0;
                        if constexpr (!MASS) {
                            s0[a3] += Dz_[a3 * Q + kz] * t3;
                            s1[a3] += nz * t1;
                            s2[a3] += nz * t2;
                        }
                    }
                }
                ap_wave_sync();   // every read of Y before the writes of S over it
                // S[g][f3][a3][ky][kx] in the Y layout
                double* sp = B + zg * A::YG + zky * Q + zkx;
                if (zact && zg < ng) {
#pragma unroll
                    for (int a3 = 0; a3 < n; ++a3) {
                        sp[a3 * A::YA3] = s0[a3];
                        if constexpr (!MASS) {
                            sp[A::YF + a3 * A::YA3] = s1[a3];
                            sp[2 * A::YF + a3 * A::YA3] = s2[a3];
                        }
                    }
                }
            }
            ap_wave_sync();
            // ---- stage y^T: lane (g, kx, a3), every a2
            {
                const int z0 = ap_opaque_zero();
                const ctab Ny_ = Ny0 + z0, Dy_ = Dy0 + z0;
                double v0[Q], v1[Q], v2[Q];
                const double* sp = B + yg * A::YG + ya3 * A::YA3 + ykx;
#pragma unroll
                for (int ky = 0; ky < Q; ++ky) {
                    v0[ky] = sp[ky * Q];
                    v1[ky] = MASS ? 0.0 : sp[A::YF + ky * Q];
                    v2[ky] = MASS ? 0.0 : sp[2 * A::YF + ky * Q];
                }
                ap_wave_sync();   // every read of S before the writes of R over it
                // R[g][f2][a3][a2][kx] in the X layout
                double* rp = B + yg * A::XG + ya3 * A::XA3 + ykx;
#pragma unroll
                for (int a2 = 0; a2 < n; ++a2) {
                    double r0 = 0.0, r1 = 0.0;
#pragma unroll
                    for (int ky = 0; ky < Q; ++ky) {
                        const double ny = Ny_[a2 * Q + ky];
                        r0 += ny * v0[ky];
                        if constexpr (!MASS) {
                            r0 += Dy_[a2 * Q + ky] * v2[ky];
                            r1 += ny * v1[ky];
                        }
                    }
                    if (yact && yg < ng) {
                        rp[a2 * Q] = r0;
                        if constexpr (!MASS) rp[A::XF + a2 * Q] = r1;
                    }
                }
            }
            ap_wave_sync();
            // ---- stage x^T, one element at a time: lane (a1, a2, a3), every
            // kx, and the element's contribution added into y
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (g >= ng) break;   // wave-uniform
                const int ex = exg + g;
#pragma unroll
                for (int ps = 0; ps < NXP; ++ps) {
                    const bool act = ps * 64 + lane < A::NXI;
                    const double* rp = B + g * A::XG + ta3[ps] * A::XA3 + ta2[ps] * Q;
                    double acc = 0.0;
#pragma unroll
                    for (int kx = 0; kx < Q; ++kx) {
                        const int t = (g * n + ta1[ps]) * Q + kx;
                        acc += TB[t] * rp[kx];
                        if constexpr (!MASS) acc += TB[64 + t] * rp[A::XF + kx];
                    }
                    const int64_t I = (ex + ta1[ps]) + (int64_t)Nx * ((ey + ta2[ps]) + (int64_t)Ny * (ez + ta3[ps]));
                    if constexpr (NXP == 1) {
                        // DOF ex (a1 = 0) has all its contributions of the run
                        // now (later elements touch DOFs beyond ex): keep it for
                        // the run's adds to y, then move every partial sum down
                        // one lane, so that lane a1 holds DOF ex + 1 + a1 for
                        // the next element.  (An atomic here would make every
                        // later table load of the run wait for it: loads and
                        // stores share one in-order counter.)
                        racc += acc;
                        if (act && ta1[0] == 0) RB[(ta2[0] + n * ta3[0]) * A::RUN + (ex - ex0)] = racc;
                        const double nxt = __shfl(racc, lane + 1);
                        racc = ta1[0] + 1 < n ? nxt : 0.0;
                    } else if (act) {
                        atomicAdd(&y[I], acc);
                    }
                }
            }
            ap_wave_sync();   // every read of R before the next group's stage x writes
        }
        if constexpr (NXP == 1) {
            // DOFs ex1 .. ex1 + p - 1 also take contributions from the next run
            const bool act = lane < A::NXI;
            const int64_t I = (ex1 - 1 + ta1[0] + 1) + (int64_t)Nx * ((ey + ta2[0]) + (int64_t)Ny * (ez + ta3[0]));
            if (act && ta1[0] + 1 < n) atomicAdd(&y[I], racc);
            racc = 0.0;
            // the run's finished DOFs: lanes along x, so each add instruction
            // covers runs of consecutive y entries
            const int len = ex1 - ex0;
            for (int i = lane; i < n * n * A::RUN; i += 64) {
                const int r = i / A::RUN, e = i % A::RUN;
                if (e < len)
                    atomicAdd(&y[(ex0 + e) + (int64_t)Nx * ((ey + r % n) + (int64_t)Ny * (ez + r / n))], RB[i]);
            }
        }
    }
}

int launch_apply(const PatchDev& pd, const double* kappa, const double* u, double alphaM,
                 double alphaK, double* y, hipStream_t st, const double* G)
{
    const int64_t runs = (int64_t)((pd.d[0].K + kApplyRun - 1) / kApplyRun) * pd.d[1].K * pd.d[2].K;
    int64_t blocks = (runs + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    const bool geo = G != nullptr, mass = alphaK == 0.0;
    switch (pd.p) {
#define IGAF_AP1(PP, GG, MM)                                                                          \
    hipLaunchKernelGGL((k_apply<PP, GG, MM>), dim3((unsigned)blocks), dim3(256), 0, st, pd, kappa, u, alphaM, \
                       alphaK, y, G)
#define IGAF_AP(PP)                                                                                   \
    case PP:                                                                                          \
        if (geo) {                                                                                    \
            if (mass) IGAF_AP1(PP, true, true);                                                       \
            else IGAF_AP1(PP, true, false);                                                           \
        } else {                                                                                      \
            if (mass) IGAF_AP1(PP, false, true);                                                      \
            else IGAF_AP1(PP, false, false);                                                          \
        }                                                                                             \
        break;
        IGAF_AP(1)
        IGAF_AP(2)
        IGAF_AP(3)
        IGAF_AP(4)
        IGAF_AP(5)
#undef IGAF_AP
#undef IGAF_AP1
    default:
        return -4;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace igaf
