// Adjoint of L(kappa) = alphaM u^T M(kappa) v + alphaK u^T K(kappa) v.
//
// kappa_q enters eq. (10) linearly in the J(x^n) slot, so
//   dL/dkappa_q = w_q (alphaM u_h v_h + alphaK grad u_h . grad v_h)(x_q),
// with u_h = sum_I u_I phi_I.  Per element the n^3 coefficients of u and v are
// gathered and interpolated to the q^3 points by sum factorisation
// (contract a1 -> x points, a2 -> y points, a3 -> z points, each with the
// value and the derivative table), so no element matrix is ever formed.
//
// One 64-lane wavefront per x-run of elements (fixed ey, ez; grid-stride over
// runs, four independent wavefronts per workgroup, synchronised only within
// the wavefront).  The run's y and z tables are wave-uniform (scalar loads).
// Elements go in groups of G = 64 / n^2, and each field (u, then v) passes
// through three stages per group:
//   stage x: lane (kx, a2, a3), one element at a time, contracts a1 from a
//            sliding window of the p+1 coefficients along x (one new value
//            per element): value and x-derivative, into LDS;
//   stage y: lane (g, kx, a3) contracts a2 for every ky: value, y-derivative
//            and the x-derivative carried along;
//   stage z: lane (g, kx, ky) contracts a3 for every kz: value and the three
//            derivatives at the quadrature points; the u results wait in
//            registers, the v pass combines them and writes the point's
//            gradient entry.
// Each LDS value is written once and read once; stage y's output reuses the
// buffer of stage x's.
#include "common.h"
#include "launch.h"

namespace igaf {

namespace {

constexpr int amax(int a, int b) { return a > b ? a : b; }
constexpr int amin(int a, int b) { return a < b ? a : b; }
// smallest y >= x with y = r (mod 16): LDS strides that spread lanes over banks
constexpr int apad16(int x, int r) { return x + (((r - x) % 16) + 16) % 16; }

// A zero the compiler cannot see through: adding it to the run's table
// pointers in every stage keeps their scalar loads inside the stage
// (scalar-cache hits) instead of hoisting 4 n q values per run into scalar
// registers and spilling them.
__device__ inline int adj_opaque_zero()
{
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}

__device__ inline void adj_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace

template <int P>
struct AdjShape {
    static constexpr int n = P + 1, Q = P + 1, Q2 = Q * Q, Q3 = Q2 * Q;
    static constexpr int G = amax(1, amin(64 / (n * n), 8));   // elements per group
    static constexpr int NXI = n * n * Q, NXP = (NXI + 63) / 64;  // stage-x items per element
    static constexpr int NYI = G * Q * n;                         // stage-y items per group
    static constexpr int NZI = G * Q2;                            // stage-z items per group
    static_assert(NYI <= 64 && NZI <= 64, "one pass per group in stages y and z");
    // X[g][f2][a3][a2][kx] and Y[g][f3][a3][ky][kx] share one buffer
    static constexpr int XA3 = apad16(n * Q, Q), XF = n * XA3, XG = 2 * XF;
    static constexpr int YA3 = apad16(Q2, Q), YF = n * YA3, YG = 3 * YF;
    static constexpr int WS = amax(G * XG, G * YG);               // doubles per wavefront
    static constexpr int RUN = 32;                                // elements per x-run
    // the x value / derivative tables of one group ([g][a][k], G n Q <= 64
    // values each), staged in LDS: one load per lane and table per group,
    // issued a group ahead
    static constexpr int TBN = G * n * Q;
    static_assert(TBN <= 64, "one table value per lane");
};

// GEO: a mapped geometry; the point value takes the geometry factors cm0
// (det J) and G0 (det J J^-1 J^-T, [E][6][q^3]) that kappa scales.
// scale_dev (nullable): a device scalar the gradient is also multiplied by.
// LOSS: no gradient is stored; each wavefront sums kappa_q g_q over its
// points (in its own fixed order), reduces the sum over its lanes in a fixed
// butterfly and writes it to part[wavefront] (the value of L, Euler's
// identity for a function linear in kappa).
template <int P, bool GEO, bool LOSS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P <= 3 ? 4 : 2))) void k_kappa_grad(
    PatchDev pd, const double* __restrict__ u, const double* __restrict__ v, double alphaM, double alphaK,
    double scale, const double* __restrict__ scale_dev, double* __restrict__ grad,
    const double* __restrict__ cm0, const double* __restrict__ G0, const double* __restrict__ kappa,
    double* __restrict__ part)
{
    using A = AdjShape<P>;
    constexpr int n = A::n, Q = A::Q, Q2 = A::Q2, Q3 = A::Q3, G = A::G, NXP = A::NXP;
    __shared__ double lds[4][A::WS + 128];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
    double* const B = lds[w];
    double* const TB = lds[w] + A::WS;   // [Nv | dN] of the group's elements
    const int Kx = pd.d[0].K, Ky = pd.d[1].K, Kz = pd.d[2].K;
    const int Nx = pd.d[0].N, Ny = pd.d[1].N;
    const double* __restrict__ Nvx = pd.d[0].Nv;
    const double* __restrict__ dNx = pd.d[0].dN;
    const double* __restrict__ wqx = pd.d[0].wq;
    const int nchunk = (Kx + A::RUN - 1) / A::RUN;
    const int nruns = nchunk * Ky * Kz;
    if (!LOSS && scale_dev) scale *= scale_dev[0];
    double lacc = 0.0;   // LOSS: this lane's sum of kappa_q g_q

    // fixed lane roles
    int xkx[NXP], xa2[NXP], xa3[NXP];   // stage x: item i = kx + Q (a2 + n a3)
#pragma unroll
    for (int ps = 0; ps < NXP; ++ps) {
        const int i = min(ps * 64 + lane, A::NXI - 1);
        xkx[ps] = i % Q;
        xa2[ps] = (i / Q) % n;
        xa3[ps] = i / (n * Q);
    }
    const bool yact = lane < A::NYI;      // stage y: lane = kx + Q (a3 + n g)
    const int yl = yact ? lane : A::NYI - 1;
    const int ykx = yl % Q, ya3 = (yl / Q) % n, yg = yl / (Q * n);
    const bool zact = lane < A::NZI;      // stage z: lane = kx + Q (ky + Q g)
    const int zl = zact ? lane : A::NZI - 1;
    const int zkx = zl % Q, zky = (zl / Q) % Q, zg = zl / Q2;

    for (int run = blockIdx.x * 4 + w; run < nruns; run += gridDim.x * 4) {
        const int ch = run % nchunk, ey = (run / nchunk) % Ky, ez = run / (nchunk * Ky);
        const int ex0 = ch * A::RUN, ex1 = min(Kx, ex0 + A::RUN);
        // the run's y and z tables: wave-uniform
        const ctab Ny0 = as_ctab(pd.d[1].Nv) + (int64_t)ey * n * Q;
        const ctab Dy0 = as_ctab(pd.d[1].dN) + (int64_t)ey * n * Q;
        const ctab Nz0 = as_ctab(pd.d[2].Nv) + (int64_t)ez * n * Q;
        const ctab Dz0 = as_ctab(pd.d[2].dN) + (int64_t)ez * n * Q;
        const ctab wz0 = as_ctab(pd.d[2].wq) + (int64_t)ez * Q;
        const double wyl = pd.d[1].wq[(int64_t)ey * Q + zky];   // this lane's y weight
        // sliding windows of u and v along x at (a2, a3) of every stage-x item
        double uw[NXP][n], vw[NXP][n];
        int64_t g0[NXP];
#pragma unroll
        for (int ps = 0; ps < NXP; ++ps) {
            g0[ps] = (int64_t)Nx * ((ey + xa2[ps]) + (int64_t)Ny * (ez + xa3[ps]));
#pragma unroll
            for (int a1 = 0; a1 < n; ++a1) {
                uw[ps][a1] = u[g0[ps] + ex0 + a1];
                vw[ps][a1] = v[g0[ps] + ex0 + a1];
            }
        }
        // x tables of the group starting at element exg, this lane's value
        const int64_t tlast = (int64_t)Kx * n * Q - 1;
        double tnv = Nvx[min((int64_t)ex0 * n * Q + lane, tlast)];
        double tdn = dNx[min((int64_t)ex0 * n * Q + lane, tlast)];
        for (int exg = ex0; exg < ex1; exg += G) {
            const int ng = min(G, ex1 - exg);   // elements in this group
            TB[lane] = tnv;
            TB[64 + lane] = tdn;
            adj_wave_sync();
            if (exg + G < ex1) {   // the next group's tables, a group ahead
                tnv = Nvx[min((int64_t)(exg + G) * n * Q + lane, tlast)];
                tdn = dNx[min((int64_t)(exg + G) * n * Q + lane, tlast)];
            }

            double ur[4][Q];                    // u, du/dx, du/dy, du/dz at this lane's points
            // field f = 0: u, f = 1: v
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const int z0 = adj_opaque_zero();
                const ctab Ny_ = Ny0 + z0, Dy_ = Dy0 + z0;
                // ---- stage x, one element of the group at a time (unrolled,
                // so that the loads of later elements are issued early)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    if (g >= ng) break;   // wave-uniform
                    const int ex = exg + g;
#pragma unroll
                    for (int ps = 0; ps < NXP; ++ps) {
                        const bool act = ps * 64 + lane < A::NXI;
                        double s0 = 0.0, s1 = 0.0;
#pragma unroll
                        for (int a1 = 0; a1 < n; ++a1) {
                            const double c = f == 0 ? uw[ps][a1] : vw[ps][a1];
                            const int t = (g * n + a1) * Q + xkx[ps];
                            s0 += c * TB[t];
                            s1 += c * TB[64 + t];
                        }
                        if (act) {
                            double* xp = B + g * A::XG + xa3[ps] * A::XA3 + xa2[ps] * Q + xkx[ps];
                            xp[0] = s0;
                            xp[A::XF] = s1;
                        }
                        // slide this field's window by one element
                        const int64_t gi = g0[ps] + min(ex + n, Nx - 1);
#pragma unroll
                        for (int a1 = 0; a1 + 1 < n; ++a1) {
                            if (f == 0) uw[ps][a1] = uw[ps][a1 + 1];
                            else vw[ps][a1] = vw[ps][a1 + 1];
                        }
                        if (f == 0) uw[ps][n - 1] = u[gi];
                        else vw[ps][n - 1] = v[gi];
                    }
                }
                adj_wave_sync();
                // ---- stage y: lane (g, kx, a3), every ky
                {
                    double x0[n], x1[n];
                    const double* xp = B + yg * A::XG + ya3 * A::XA3 + ykx;
#pragma unroll
                    for (int a2 = 0; a2 < n; ++a2) {
                        x0[a2] = xp[a2 * Q];
                        x1[a2] = xp[A::XF + a2 * Q];
                    }
                    adj_wave_sync();   // every read of X before the writes of Y over it
                    double* yp = B + yg * A::YG + ya3 * A::YA3 + ykx;
#pragma unroll
                    for (int ky = 0; ky < Q; ++ky) {
                        double o0 = 0.0, o1 = 0.0, o2 = 0.0;
#pragma unroll
                        for (int a2 = 0; a2 < n; ++a2) {
                            const double ny = Ny_[a2 * Q + ky], dy = Dy_[a2 * Q + ky];
                            o0 += ny * x0[a2];
                            o1 += dy * x0[a2];
                            o2 += ny * x1[a2];
                        }
                        if (yact && yg < ng) {
                            yp[ky * Q] = o0;
                            yp[A::YF + ky * Q] = o1;
                            yp[2 * A::YF + ky * Q] = o2;
                        }
                    }
                }
                adj_wave_sync();
                // ---- stage z: lane (g, kx, ky), every kz
                {
                    const int z1 = adj_opaque_zero();
                    const ctab Nz_ = Nz0 + z1, Dz_ = Dz0 + z1, wz_ = wz0 + z1;
                    double y0[n], y1[n], y2[n];
                    const double* yp = B + zg * A::YG + zky * Q + zkx;
#pragma unroll
                    for (int a3 = 0; a3 < n; ++a3) {
                        y0[a3] = yp[a3 * A::YA3];
                        y1[a3] = yp[A::YF + a3 * A::YA3];
                        y2[a3] = yp[2 * A::YF + a3 * A::YA3];
                    }
                    adj_wave_sync();   // every read of Y before the next stage x writes
                    const int exz = exg + min(zg, ng - 1);
                    const double wxl = wqx[(int64_t)exz * Q + zkx];
                    const int64_t e = exz + (int64_t)Kx * (ey + (int64_t)Ky * ez);
#pragma unroll
                    for (int kz = 0; kz < Q; ++kz) {
                        double h = 0.0, dz = 0.0, dy = 0.0, dx = 0.0;
#pragma unroll
                        for (int a3 = 0; a3 < n; ++a3) {
                            const double nz = Nz_[a3 * Q + kz], dzt = Dz_[a3 * Q + kz];
                            h += nz * y0[a3];
                            dz += dzt * y0[a3];
                            dy += nz * y1[a3];
                            dx += nz * y2[a3];
                        }
                        if (f == 0) {
                            ur[0][kz] = h;
                            ur[1][kz] = dx;
                            ur[2][kz] = dy;
                            ur[3][kz] = dz;
                        } else {
                            const int64_t pt = e * Q3 + kz * Q2 + zky * Q + zkx;
                            double r;
                            if constexpr (GEO) {
                                const double* g0 = G0 + e * 6 * Q3 + kz * Q2 + zky * Q + zkx;
                                const double gxx = g0[0], gyy = g0[Q3], gzz = g0[2 * Q3];
                                const double gxy = g0[3 * Q3], gxz = g0[4 * Q3], gyz = g0[5 * Q3];
                                const double vx = gxx * dx + gxy * dy + gxz * dz;
                                const double vy = gxy * dx + gyy * dy + gyz * dz;
                                const double vz = gxz * dx + gyz * dy + gzz * dz;
                                r = alphaM * cm0[pt] * ur[0][kz] * h +
                                    alphaK * (ur[1][kz] * vx + ur[2][kz] * vy + ur[3][kz] * vz);
                            } else {
                                r = alphaM * ur[0][kz] * h +
                                    alphaK * (ur[1][kz] * dx + ur[2][kz] * dy + ur[3][kz] * dz);
                            }
                            if (zact && zg < ng) {
                                if constexpr (LOSS) lacc += kappa[pt] * ((wxl * wyl * wz_[kz]) * r);
                                else grad[pt] = scale * (wxl * wyl * wz_[kz]) * r;
                            }
                        }
                    }
                }
            }
        }
    }
    if constexpr (LOSS) {
#pragma unroll
        for (int off = 32; off > 0; off /= 2) lacc += __shfl_xor(lacc, off);
        if (lane == 0) part[blockIdx.x * 4 + w] = lacc;
    }
}

// L = scale * (the sum of part[0..nparts)), in a fixed order
__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part, int nparts, double scale,
                                                    double* __restrict__ L)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h /= 2) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) L[0] = scale * red[0];
}

int launch_kappa_grad(const PatchDev& pd, const double* u, const double* v, double alphaM,
                      double alphaK, double scale, const double* scale_dev, double* grad, hipStream_t st,
                      const double* cm0, const double* G0)
{
    const int64_t runs = (int64_t)((pd.d[0].K + 31) / 32) * pd.d[1].K * pd.d[2].K;   // runs of 32 x elements
    int64_t blocks = (runs + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    const bool geo = G0 != nullptr;
    switch (pd.p) {
#define IGAF_A(PP)                                                                                    \
    case PP:                                                                                          \
        if (geo)                                                                                      \
            hipLaunchKernelGGL((k_kappa_grad<PP, true, false>), dim3((unsigned)blocks), dim3(256), 0, st, pd, \
                               u, v, alphaM, alphaK, scale, scale_dev, grad, cm0, G0, nullptr, nullptr); \
        else                                                                                          \
            hipLaunchKernelGGL((k_kappa_grad<PP, false, false>), dim3((unsigned)blocks), dim3(256), 0, st, pd, \
                               u, v, alphaM, alphaK, scale, scale_dev, grad, nullptr, nullptr, nullptr,   \
                               nullptr);                                                              \
        break;
        IGAF_A(1)
        IGAF_A(2)
        IGAF_A(3)
        IGAF_A(4)
        IGAF_A(5)
#undef IGAF_A
    default:
        return -4;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_bilinear(const PatchDev& pd, const double* kappa, const double* u, const double* v, double alphaM,
                    double alphaK, double* L, double* part, hipStream_t st)
{
    const int64_t runs = (int64_t)((pd.d[0].K + 31) / 32) * pd.d[1].K * pd.d[2].K;
    int64_t blocks = (runs + 3) / 4;
    if (blocks > kLossParts / 4) blocks = kLossParts / 4;
    switch (pd.p) {
#define IGAF_L(PP)                                                                                    \
    case PP:                                                                                          \
        hipLaunchKernelGGL((k_kappa_grad<PP, false, true>), dim3((unsigned)blocks), dim3(256), 0, st, pd, u, \
                           v, alphaM, alphaK, 1.0, nullptr, nullptr, nullptr, nullptr, kappa, part);  \
        break;
        IGAF_L(1)
        IGAF_L(2)
        IGAF_L(3)
        IGAF_L(4)
        IGAF_L(5)
#undef IGAF_L
    default:
        return -4;
    }
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, part, (int)(blocks * 4), 1.0, L);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace igaf
