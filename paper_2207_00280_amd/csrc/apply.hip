// Matrix-free operator apply: y = alphaM M(kappa) u + alphaK K(kappa) u.
//
// The global matrices are sums of element matrices (Sec. 3.1), so
//   y_I = sum_e sum_q c_q [alphaM phi_I u_h + alphaK grad phi_I . grad u_h](x_q)
// with c_q = kappa_q w_q (eq. (10), the coefficient in the J(x^n) slot).  Per
// element the n^3 coefficients of u are interpolated to the q^3 points by sum
// factorisation (x -> y -> z, value and derivative tables, as Algorithm 2
// contracts), weighted point by point, and contracted back against the test
// functions in the transposed order (z -> y -> x); no element or global
// matrix is formed.
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
//   stage x^T: lane (a1, a2, a3), one element at a time, every kx.
// The run's results are summed per DOF in LDS, in element order: at p <= 3
// (one pass of 64 lanes per element) the lanes of one DOF row along x pass
// their partial sums down as the run advances and a DOF is written once it
// is complete; at p = 4, 5 each element's values are added into the run's
// LDS rows.  A run touches the n^2 DOF rows (ey + a2, ez + a3) over x in
// [ex0, ex1 + p); at its end those values go to the run's slot of a
// workspace with plain coalesced stores.  A second kernel then forms each
// y_I from the slots of the (at most (p+1)^2, or 2 (p+1)^2 where x-runs
// meet) runs that touch it, in a fixed order: no atomics, so repeated calls
// give the same bits.
//
// The diagonal mode computes d_I = sum_q c_q phi_I(x_q)^2 = diag(M(kappa))
// with the same transposed stages, squared tables and no u (the Euler step's
// preconditioner scaling).
#include <mutex>
#include <vector>

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
    // the run's DOF values [a2 + n a3][x - ex0], x - ex0 < RUN + p
    static constexpr int RL = RUN + P;
    static constexpr int RB = n * n * RL;
    // the x value / derivative tables of one group ([g][a][k], G n Q <= 64
    // values each), staged in LDS: one load per lane and table per group,
    // issued a group ahead
    static constexpr int TBN = G * n * Q;
    static_assert(TBN <= 64, "one table value per lane");
};

enum { AP_FULL = 0, AP_MASS = 1, AP_DIAG = 2 };

// GEO: a mapped geometry; `kappa` is the mass coefficient cm and Gt
// ([E][6][q^3]) the stiffness tensor, applied to the parametric gradient.
// MODE AP_MASS (alphaK = 0, the conjugate-gradient products of the Euler
// step): the gradient fields are neither interpolated nor contracted back.
// MODE AP_DIAG: alphaM diag(M(kappa)), u unused.
// W: the runs' slots, RB doubles per run (run = ch + nchunk (ey + Ky ez)).
template <int P, bool GEO, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P <= 3 ? 4 : 2))) void k_apply(
    PatchDev pd, const double* __restrict__ kappa, const double* __restrict__ u, double alphaM,
    double alphaK, double* __restrict__ W, const double* __restrict__ Gt)
{
    constexpr bool MASS = MODE != AP_FULL;   // no gradient fields
    constexpr bool DIAG = MODE == AP_DIAG;   // no u: point values kappa w, squared tables
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
        const int len = ex1 - ex0;
        // stage x^T with one pass (p <= 3): lane (a1, a2, a3) holds the partial
        // sum of DOF (ex + a1, ey + a2, ez + a3) over the run's elements so far
        double racc = 0.0;
        if constexpr (NXP > 1) {   // several passes: the run's rows accumulate in LDS
            for (int i = lane; i < A::RB; i += 64) RB[i] = 0.0;
        }
        // sliding window of u along x at (a2, a3) of every stage-x item
        double uw[NXP][n];
        int64_t g0[NXP];
#pragma unroll
        for (int ps = 0; ps < NXP; ++ps) {
            g0[ps] = (int64_t)Nx * ((ey + xa2[ps]) + (int64_t)Ny * (ez + xa3[ps]));
#pragma unroll
            for (int a1 = 0; a1 < n; ++a1) uw[ps][a1] = DIAG ? 0.0 : u[g0[ps] + ex0 + a1];
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
            for (int g = 0; g < G; ++g) unx[ps][g] = DIAG ? 0.0 : u[g0[ps] + min(ex0 + n + g, Nx - 1)];
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
                    if constexpr (!DIAG) unx[ps][g] = u[g0[ps] + min(exg + G + n + g, Nx - 1)];
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
                if (DIAG || g >= ng) break;   // wave-uniform
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
            if constexpr (!DIAG) {
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
                    y0[a3] = DIAG ? 0.0 : yp[a3 * A::YA3];
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
                    if constexpr (DIAG) {
                        t0 = alphaM * (kc[kz] * wxy * wz_[kz]);
                        t1 = t2 = t3 = 0.0;
                    } else if constexpr (MASS) {
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
                        s0[a3] += (DIAG ? nz * nz : nz) * t0;
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
                        r0 += (DIAG ? ny * ny : ny) * v0[ky];
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
            // kx, and the element's contribution added into the run's rows
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
                        const double nx = TB[t];
                        acc += (DIAG ? nx * nx : nx) * rp[kx];
                        if constexpr (!MASS) acc += TB[64 + t] * rp[A::XF + kx];
                    }
                    if constexpr (NXP == 1) {
                        // DOF ex (a1 = 0) has all its contributions of the run
                        // now (later elements touch DOFs beyond ex): keep it in
                        // the run's rows, then move every partial sum down one
                        // lane, so that lane a1 holds DOF ex + 1 + a1 for the
                        // next element
                        racc += acc;
                        if (act && ta1[0] == 0) RB[(ta2[0] + n * ta3[0]) * A::RL + (ex - ex0)] = racc;
                        const double nxt = __shfl(racc, lane + 1);
                        racc = ta1[0] + 1 < n ? nxt : 0.0;
                    } else if (act) {
                        RB[(ta2[ps] + n * ta3[ps]) * A::RL + (ex - ex0 + ta1[ps])] += acc;
                    }
                }
                // the next element's adds read what other lanes wrote
                if constexpr (NXP > 1) ap_wave_sync();
            }
            ap_wave_sync();   // every read of R before the next group's stage x writes
        }
        // DOFs ex1 .. ex1 + p - 1 (x - ex0 = len + a1) take the rest of their
        // contributions from the next run
        if constexpr (NXP == 1) {
            if (lane < A::NXI && ta1[0] + 1 < n) RB[(ta2[0] + n * ta3[0]) * A::RL + len + ta1[0]] = racc;
            racc = 0.0;
        }
        ap_wave_sync();
        // the run's slot: rows of RL values, the first len + p of each written
        double* __restrict__ wr = W + (int64_t)run * A::RB;
        for (int i = lane; i < A::RB; i += 64)
            if (i % A::RL < len + P) wr[i] = RB[i];
        ap_wave_sync();   // every read of the rows before the next run rewrites them
    }
}

// y_I = the sum of the slots of the runs touching DOF I = (ix, iy, iz): runs
// (chunk c, ey = iy - a2, ez = iz - a3) for a3, a2 = 0..p in that order, and
// where ix is one of the first p DOFs of chunk c > 0 the slot of chunk c - 1
// (at x - ex0 = ix - (c - 1) RUN >= RUN) before chunk c's.  One thread per DOF,
// consecutive DOFs along x in consecutive lanes.
template <int P>
__global__ __launch_bounds__(256) void k_apply_sum(const double* __restrict__ W, double* __restrict__ y, int Kx,
                                                   int Ky, int Kz, int64_t ndof)
{
    using A = ApplyShape<P>;
    constexpr int n = A::n, RUN = A::RUN, RL = A::RL, RB = A::RB;
    const int Nx = Kx + P, Ny = Ky + P;
    const int nchunk = (Kx + RUN - 1) / RUN;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ndof; i += (int64_t)gridDim.x * 256) {
        const int ix = (int)(i % Nx), iy = (int)((i / Nx) % Ny), iz = (int)(i / ((int64_t)Nx * Ny));
        const int c = min(ix / RUN, nchunk - 1), xl = ix - c * RUN;
        const bool prev = c > 0 && xl < P;
        double s = 0.0;
#pragma unroll
        for (int a3 = 0; a3 < n; ++a3) {
            const int ez = iz - a3;
            if (ez < 0 || ez >= Kz) continue;
#pragma unroll
            for (int a2 = 0; a2 < n; ++a2) {
                const int ey = iy - a2;
                if (ey < 0 || ey >= Ky) continue;
                const double* w =
                    W + ((int64_t)c + (int64_t)nchunk * (ey + (int64_t)Ky * ez)) * RB + (a2 + n * a3) * RL;
                if (prev) s += w[xl + RUN - RB];
                s += w[xl];
            }
        }
        y[i] = s;
    }
}

// ---------------------------------------------------------------------------
// The allocation-free apply (igaf_apply_static): the runs' slots in a
// file-scope device array of fixed size instead of a caller workspace.  Every
// device the library runs on holds its own copy until the process ends; its
// address is looked up once per device (apply_scratch_init, called when a
// plan is created) and only that address is handed to the kernels.
constexpr int64_t kApplyScratchDoubles = int64_t(8) << 20;   // 64 MiB
static __device__ __align__(256) double scratch[kApplyScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // per device id
}  // namespace

int apply_scratch_init()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return -3;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)dev < g_scratch_ptr.size() && g_scratch_ptr[dev]) return 0;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return -3;
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
    return 0;
}

double* apply_scratch(int64_t* capacity)
{
    *capacity = kApplyScratchDoubles;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (size_t)dev < g_scratch_ptr.size() ? g_scratch_ptr[dev] : nullptr;
}

int64_t apply_workspace_doubles(const PatchDev& pd)
{
    const int64_t n = pd.p + 1;
    const int64_t runs = (int64_t)((pd.d[0].K + kApplyRun - 1) / kApplyRun) * pd.d[1].K * pd.d[2].K;
    return runs * n * n * (kApplyRun + pd.p);
}

template <int P, bool GEO, int MODE>
static int launch_apply_t(const PatchDev& pd, const double* kappa, const double* u, double alphaM, double alphaK,
                          double* y, double* W, hipStream_t st, const double* G)
{
    const int64_t runs = (int64_t)((pd.d[0].K + kApplyRun - 1) / kApplyRun) * pd.d[1].K * pd.d[2].K;
    int64_t blocks = (runs + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((k_apply<P, GEO, MODE>), dim3((unsigned)blocks), dim3(256), 0, st, pd, kappa, u, alphaM,
                       alphaK, W, G);
    int64_t sb = (pd.ndof + 255) / 256;
    if (sb > 8192) sb = 8192;
    hipLaunchKernelGGL(k_apply_sum<P>, dim3((unsigned)sb), dim3(256), 0, st, W, y, pd.d[0].K, pd.d[1].K,
                       pd.d[2].K, pd.ndof);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int P>
static int launch_apply_p(const PatchDev& pd, const double* kappa, const double* u, double alphaM, double alphaK,
                          double* y, double* W, hipStream_t st, const double* G, bool diag)
{
    if (diag) return launch_apply_t<P, false, AP_DIAG>(pd, kappa, u, alphaM, alphaK, y, W, st, nullptr);
    if (G) {
        if (alphaK == 0.0) return launch_apply_t<P, true, AP_MASS>(pd, kappa, u, alphaM, alphaK, y, W, st, G);
        return launch_apply_t<P, true, AP_FULL>(pd, kappa, u, alphaM, alphaK, y, W, st, G);
    }
    if (alphaK == 0.0) return launch_apply_t<P, false, AP_MASS>(pd, kappa, u, alphaM, alphaK, y, W, st, nullptr);
    return launch_apply_t<P, false, AP_FULL>(pd, kappa, u, alphaM, alphaK, y, W, st, nullptr);
}

int launch_apply(const PatchDev& pd, const double* kappa, const double* u, double alphaM, double alphaK,
                 double* y, double* W, hipStream_t st, const double* G, bool diag)
{
    switch (pd.p) {
    case 1: return launch_apply_p<1>(pd, kappa, u, alphaM, alphaK, y, W, st, G, diag);
    case 2: return launch_apply_p<2>(pd, kappa, u, alphaM, alphaK, y, W, st, G, diag);
    case 3: return launch_apply_p<3>(pd, kappa, u, alphaM, alphaK, y, W, st, G, diag);
    case 4: return launch_apply_p<4>(pd, kappa, u, alphaM, alphaK, y, W, st, G, diag);
    case 5: return launch_apply_p<5>(pd, kappa, u, alphaM, alphaK, y, W, st, G, diag);
    default: return -4;
    }
}

}  // namespace igaf
