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
// Work decomposition (one 64-lane wavefront = one work item, no workgroup
// barrier): a work item owns the rows iy (one y row), iz in [Z0, Z0+RZ) and
// all ix, restricted to the z column offsets oz in [OZ0, OZ0+OZC) (a row's
// oz offsets may be split over several items; they never share a CSR value).
// It sweeps the x elements ex = 0..Kx-1 in order; for each x element
//   phase 1 (stage z):  D[zpair][kx][gy] for its y window of elements,
//   phase 2 (stage y):  C[(oy, zpair)][kx] into an LDS ring of p+1 slots,
//   phase 3 (stage x):  row ix = ex is now complete: every (ox, oy, oz)
//                       value it owns is summed from the ring, staged in LDS
//                       at its place in the CSR row and written as one
//                       contiguous segment (the p last x rows after the sweep).
// o* in [0, 2p] are column offsets j = i + o - p.
#include "common.h"
#include "launch.h"

namespace igaf {


__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

template <int P, int RZ, int OZC>
struct WaveShape {
    static constexpr int n = P + 1;
    static constexpr int Q = P + 1;
    static constexpr int S = n * (n + 1) / 2;
    static constexpr int O = 2 * P + 1;
    static constexpr int Q3 = Q * Q * Q;
    static constexpr int WZ = RZ + P;            // z elements in the window
    static constexpr int GY = (P + 1) * Q;       // y points in the window (one row)
    static constexpr int GYP = GY | 1;           // padded LDS stride
    static constexpr int NPR = RZ * OZC;         // owned z pairs
    static constexpr int NC = O * RZ * OZC;      // (oy, rz, ozl) combos
    static constexpr int N1 = Q * GY;            // phase-1 items
    static constexpr int N2 = NPR * Q;           // phase-2 items
    static constexpr int NP1 = (N1 + 63) / 64;   // phase-1 passes
    static constexpr int NSPLIT = (O + OZC - 1) / OZC;
    static constexpr int DSZ = 2 * NPR * Q * GYP;
    static constexpr int CSZ = (P + 1) * 2 * Q * NC;
    static constexpr int WAVE_LDS = DSZ + CSZ;   // doubles per wavefront
    static_assert(2 * RZ * OZC * O * O <= DSZ, "row staging must fit in D");
};

template <int P, int RZ, int OZC, int SPLIT>
__device__ __forceinline__ void rows_wave_pencil(const PatchDev& pd, const RowMap& rm,
                                 const double* __restrict__ kappa, double* __restrict__ Mv,
                                 double* __restrict__ Kv, int iy, int Z0, double* __restrict__ D,
                                 double* __restrict__ C, int lane)
{
    using Sh = WaveShape<P, RZ, OZC>;
    constexpr int Q = Sh::Q, S = Sh::S, O = Sh::O, Q3 = Sh::Q3, WZ = Sh::WZ, GY = Sh::GY;
    constexpr int GYP = Sh::GYP, NPR = Sh::NPR, NC = Sh::NC, NP1 = Sh::NP1;
    constexpr int OZ0 = SPLIT * OZC;
    constexpr bool PREFETCH = NP1 <= 2;
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
            const double* kp = kappa + e * Q3 + (it < Sh::N1 ? kx + Q * ky : 0);
#pragma unroll
            for (int kz = 0; kz < Q; ++kz) {
                const double v = kp[Q * Q * kz];
                cz[lz][kz] = ok ? v : 0.0;
            }
        }
    };

    // phase 3 for row ix: values are staged in LDS (over the D buffer, dead
    // until the next phase 1) at their place in this item's contiguous part
    // of the CSR row, then written back with coalesced stores.
    auto emit_row = [&](int ix) {
        const int Lx = band_len(ix, P, Nx), Ly = band_len(iy, P, Ny);
        for (int c0 = 0; c0 < NC; c0 += 64) {
            const bool act0 = c0 + lane < NC;
            const int c = act0 ? c0 + lane : NC - 1;
            const int ozl = c % OZC, rz = (c / OZC) % RZ, oy = c / (OZC * RZ);
            const int oz = OZ0 + ozl;
            const int iz = Z0 + rz, jy = iy + oy - P, jz = iz + oz - P;
            const bool okrow = act0 && oz < O && iz < Nz && jy >= 0 && jy < Ny && jz >= 0 && jz < Nz;
            const int izc = iz < Nz ? iz : Nz - 1;
            const int jza = max(band_lo(izc, P), izc + OZ0 - P);   // first column z of this item
            const int sub = ((jz - jza) * Ly + (jy - band_lo(iy, P))) * Lx + (ix - P - band_lo(ix, P));
            // ring slots of elements outside [0, Kx) hold zeros
            double ca[P + 1][Q], cb[P + 1][Q];
#pragma unroll
            for (int e = 0; e <= P; ++e) {
                const int slot = (ix + 1 + e) % (P + 1);   // (ix - P + e) mod (P + 1)
#pragma unroll
                for (int kx = 0; kx < Q; ++kx) {
                    ca[e][kx] = C[((slot * 2 + 0) * Q + kx) * NC + c];
                    cb[e][kx] = C[((slot * 2 + 1) * Q + kx) * NC + c];
                }
            }
            double* stM = D + (rz * 2 + 0) * (OZC * O * O);
            double* stK = D + (rz * 2 + 1) * (OZC * O * O);
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
                        k += wd[kx] * ca[e][kx];
                        k += wn[kx] * cb[e][kx];
                    }
                }
                const int jx = ix + ox - P;
                if (okrow && jx >= 0 && jx < Nx) {
                    stM[sub + ox] = m;
                    stK[sub + ox] = k;
                }
            }
        }
        wave_sync();
#pragma unroll
        for (int rz = 0; rz < RZ; ++rz) {
            const int iz = Z0 + rz;
            if (iz >= Nz) break;
            const int jza = max(band_lo(iz, P), iz + OZ0 - P);
            const int jzb = min(band_hi(iz, P, Nz), iz + OZ0 + OZC - 1 - P);
            if (jzb < jza) continue;
            const int L = (jzb - jza + 1) * Ly * Lx;
            const int64_t rs = rm.row_start(ix, iy, iz) + (int64_t)(jza - band_lo(iz, P)) * Ly * Lx;
            const double* stM = D + (rz * 2 + 0) * (OZC * O * O);
            const double* stK = D + (rz * 2 + 1) * (OZC * O * O);
            for (int i = lane; i < L; i += 64) {
                if (Mv) Mv[rs + i] = stM[i];
                if (Kv) Kv[rs + i] = stK[i];
            }
        }
        wave_sync();
    };

    // the C ring starts zeroed: rows ix < P read the slots of elements
    // ix - P .. -1, which stay zero until elements 1 .. P overwrite them
    auto zero_slots = [&](int s0, int ns) {
        for (int i = lane; i < ns * 2 * Q * NC; i += 64) C[s0 * 2 * Q * NC + i] = 0.0;
    };
    zero_slots(0, P + 1);
    double czn[PREFETCH ? NP1 : 1][WZ][Q];          // next slice's kappa columns
    if (PREFETCH) {
#pragma unroll
        for (int ps = 0; ps < NP1; ++ps) load_col(0, ps * 64 + lane, czn[PREFETCH ? ps : 0]);
    }

    for (int ex = 0; ex < Kx; ++ex) {
        const int z0 = opaque_zero();
        const ctab Wnzi = Wnz + z0, Wdzi = Wdz + z0, Wnyi = Wny + z0, Wdyi = Wdy + z0;
        // phase 1: stage z
        auto phase1_pass = [&](int ps, double (&cz)[WZ][Q]) {
            const int it = ps * 64 + lane;
            const bool act = it < Sh::N1;
            const int kx = it % Q, gy = it / Q;
#pragma unroll
            for (int rz = 0; rz < RZ; ++rz) {
#pragma unroll
                for (int ozl = 0; ozl < OZC; ++ozl) {
                    const int oz = OZ0 + ozl;
                    double d0 = 0.0, d1 = 0.0;
#pragma unroll
                    for (int e = 0; e <= P; ++e) {
                        if (oz >= O || oz - e < 0 || oz - e > P) continue;   // compile time
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
                    const int pr = rz * OZC + ozl;
                    if (act) {
                        D[((0 * NPR + pr) * Q + kx) * GYP + gy] = d0;
                        D[((1 * NPR + pr) * Q + kx) * GYP + gy] = d1;
                    }
                }
            }
        };
        if constexpr (PREFETCH) {
#pragma unroll
            for (int ps = 0; ps < NP1; ++ps) phase1_pass(ps, czn[PREFETCH ? ps : 0]);
        } else {
#pragma unroll 1
            for (int ps = 0; ps < NP1; ++ps) {
                double cz[WZ][Q];
                load_col(ex, ps * 64 + lane, cz);
                phase1_pass(ps, cz);
            }
        }
        // prefetch the next slice's kappa while phases 2 and 3 run
        if (PREFETCH && ex + 1 < Kx) {
#pragma unroll
            for (int ps = 0; ps < NP1; ++ps) load_col(ex + 1, ps * 64 + lane, czn[PREFETCH ? ps : 0]);
        }
        wave_sync();
        // phase 2: stage y into ring slot ex % (p+1)
        const int slot = ex % (P + 1);
        for (int it0 = 0; it0 < Sh::N2; it0 += 64) {
            const bool act = it0 + lane < Sh::N2;
            const int it = act ? it0 + lane : Sh::N2 - 1;
            const int kx = it % Q, pr = it / Q, rz = pr / OZC, ozl = pr % OZC;
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
                        cb += wd[ky] * d0[e * Q + ky];
                        cb += wn[ky] * d1[e * Q + ky];
                    }
                }
                const int c = (oy * RZ + rz) * OZC + ozl;
                if (act) {
                    C[((slot * 2 + 0) * Q + kx) * NC + c] = ca;
                    C[((slot * 2 + 1) * Q + kx) * NC + c] = cb;
                }
            }
        }
        wave_sync();
        emit_row(ex);
    }
    for (int ix = Kx; ix < Nx; ++ix) {
        zero_slots(ix % (P + 1), 1);   // element ix is past the end
        wave_sync();
        emit_row(ix);
    }
    wave_sync();
}

// Per-degree work-item shapes.  Family 0 keeps every z offset of a row in one
// item at p <= 3; family 1 splits them more finely (less LDS per wavefront,
// more items).  The batched launch's autotuner picks the family.
template <int P, int FAM> struct RowsCfg;
template <int FAM> struct RowsCfg<1, FAM> { static constexpr int RZ = 2, OZC = 3; };
template <int FAM> struct RowsCfg<2, FAM> { static constexpr int RZ = 2, OZC = 5; };
template <> struct RowsCfg<3, 0> { static constexpr int RZ = 1, OZC = 7; };
template <> struct RowsCfg<3, 1> { static constexpr int RZ = 1, OZC = 4; };
template <> struct RowsCfg<4, 0> { static constexpr int RZ = 1, OZC = 5; };
template <> struct RowsCfg<4, 1> { static constexpr int RZ = 1, OZC = 3; };
template <> struct RowsCfg<5, 0> { static constexpr int RZ = 1, OZC = 4; };
template <> struct RowsCfg<5, 1> { static constexpr int RZ = 1, OZC = 2; };

template <int P, int FAM>
using CfgShape = WaveShape<P, RowsCfg<P, FAM>::RZ, RowsCfg<P, FAM>::OZC>;

template <int FAM>
struct FamilyLds {
    static constexpr int a = CfgShape<1, FAM>::WAVE_LDS, b = CfgShape<2, FAM>::WAVE_LDS;
    static constexpr int c = CfgShape<3, FAM>::WAVE_LDS, d = CfgShape<4, FAM>::WAVE_LDS;
    static constexpr int e = CfgShape<5, FAM>::WAVE_LDS;
    static constexpr int ab = a > b ? a : b, cd = c > d ? c : d, abcd = ab > cd ? ab : cd;
    static constexpr int MAX = abcd > e ? abcd : e;
};

// Number of work items of a patch of degree P in family FAM.
template <int P, int FAM>
__host__ __device__ inline int rows_items(int Ny, int Nz)
{
    constexpr int RZ = RowsCfg<P, FAM>::RZ;
    return Ny * ((Nz + RZ - 1) / RZ) * CfgShape<P, FAM>::NSPLIT;
}

// Run work item `item` of a degree-P patch: item = (split, z block, iy) with iy fastest.
template <int P, int FAM>
__device__ __forceinline__ void rows_item(const PatchDev& pd, const RowMap& rm, const double* kappa, double* Mv,
                          double* Kv, int item, double* lds, int lane)
{
    constexpr int RZ = RowsCfg<P, FAM>::RZ, OZC = RowsCfg<P, FAM>::OZC;
    using Sh = WaveShape<P, RZ, OZC>;
    const int Ny = pd.d[1].N, Nz = pd.d[2].N;
    const int nzb = (Nz + RZ - 1) / RZ;
    const int iy = item % Ny;
    const int zb = (item / Ny) % nzb;
    const int split = item / (Ny * nzb);
    double* D = lds;
    double* C = lds + Sh::DSZ;
    switch (split) {
#define IGAF_SPLIT(SP)                                                                       \
    case SP:                                                                                 \
        if constexpr (SP < Sh::NSPLIT)                                                       \
            rows_wave_pencil<P, RZ, OZC, SP>(pd, rm, kappa, Mv, Kv, iy, zb * RZ, D, C, lane); \
        break;
        IGAF_SPLIT(0)
        IGAF_SPLIT(1)
        IGAF_SPLIT(2)
        IGAF_SPLIT(3)
        IGAF_SPLIT(4)
        IGAF_SPLIT(5)
#undef IGAF_SPLIT
    default:
        break;
    }
}


int launch_rows(const PatchDev& pd, const double* kappa, double* Mv, double* Kv, hipStream_t st)
{
    // one patch: tiles of pencils per workgroup (stage z shared by a tile)
    return launch_rows_tile(pd, kappa, Mv, Kv, st);
}

int rows_item_count(int p, int fam, int Ny, int Nz)
{
#define IGAF_IC(PP)                                                                    \
    case PP:                                                                           \
        return fam ? rows_items<PP, 1>(Ny, Nz) : rows_items<PP, 0>(Ny, Nz);
    switch (p) {
        IGAF_IC(1)
        IGAF_IC(2)
        IGAF_IC(3)
        IGAF_IC(4)
        IGAF_IC(5)
    default:
        return 0;
    }
#undef IGAF_IC
}

// ---------------------------------------------------------------------------
// Batched persistent launch: every wavefront repeatedly takes the next work
// item (patch, item) from a cost-sorted list through an atomic counter and
// runs it with the kernel shape of the patch's degree.  The counters are
// reset by the last wavefront to leave, so the launch can be replayed (HIP
// graph) without any host-side reset.  Every wavefront exits once the list
// is exhausted.
template <class T>
__device__ inline T uniform_ptr(T p)
{
    uint64_t v = reinterpret_cast<uint64_t>(p);
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T>(((uint64_t)hi << 32) | lo);
}

__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline void uniform_patch(const BatchPatch& src, PatchDev& pd, RowMap& rm,
                                     const double*& kappa, double*& Mv, double*& Kv)
{
    pd = src.pd;
    rm = src.rm;
    for (int d = 0; d < 3; ++d) {
        pd.d[d].Wnn = uniform_ptr(pd.d[d].Wnn);
        pd.d[d].Wdd = uniform_ptr(pd.d[d].Wdd);
        pd.d[d].Nv = uniform_ptr(pd.d[d].Nv);
        pd.d[d].dN = uniform_ptr(pd.d[d].dN);
        pd.d[d].wq = uniform_ptr(pd.d[d].wq);
        pd.d[d].pre = uniform_ptr(pd.d[d].pre);
        pd.d[d].K = uniform_int(pd.d[d].K);
        pd.d[d].N = uniform_int(pd.d[d].N);
        pd.d[d].Q = uniform_int(pd.d[d].Q);
        rm.pre[d] = uniform_ptr(rm.pre[d]);
        rm.N[d] = uniform_int(rm.N[d]);
    }
    pd.p = uniform_int(pd.p);
    rm.p = uniform_int(rm.p);
    kappa = uniform_ptr(src.kappa);
    Mv = uniform_ptr(src.Mv);
    Kv = uniform_ptr(src.Kv);
}

template <int FAM>
__global__ __launch_bounds__(64) void k_rows_batch(const BatchPatch* __restrict__ patches,
                                                   const int2* __restrict__ items, int nitems,
                                                   int* __restrict__ ctr)
{
    __shared__ double lds[FamilyLds<FAM>::MAX];
    const int lane = threadIdx.x;
    for (;;) {
        int it = 0;
        if (lane == 0) it = atomicAdd(&ctr[0], 1);
        it = uniform_int(__shfl(it, 0));
        if (it >= nitems) break;
        const int2 w = items[it];
        const int pid = uniform_int(w.x), loc = uniform_int(w.y);
        PatchDev pd;
        RowMap rm;
        const double* kappa;
        double *Mv, *Kv;
        uniform_patch(patches[pid], pd, rm, kappa, Mv, Kv);
        switch (pd.p) {
        case 1: rows_item<1, FAM>(pd, rm, kappa, Mv, Kv, loc, lds, lane); break;
        case 2: rows_item<2, FAM>(pd, rm, kappa, Mv, Kv, loc, lds, lane); break;
        case 3: rows_item<3, FAM>(pd, rm, kappa, Mv, Kv, loc, lds, lane); break;
        case 4: rows_item<4, FAM>(pd, rm, kappa, Mv, Kv, loc, lds, lane); break;
        case 5: rows_item<5, FAM>(pd, rm, kappa, Mv, Kv, loc, lds, lane); break;
        default: break;
        }
    }
    if (lane == 0) {
        __threadfence();
        if (atomicAdd(&ctr[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&ctr[0], 0);
            atomicExch(&ctr[1], 0);
            __threadfence();
        }
    }
}

int launch_rows_batch(int fam, int grid, const BatchPatch* patches, const int2* items, int nitems,
                      int* ctr, hipStream_t st)
{
    if (fam == 0)
        hipLaunchKernelGGL(k_rows_batch<0>, dim3(grid), dim3(64), 0, st, patches, items, nitems, ctr);
    else
        hipLaunchKernelGGL(k_rows_batch<1>, dim3(grid), dim3(64), 0, st, patches, items, nitems, ctr);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int rows_batch_lds_bytes(int fam)
{
    return (int)sizeof(double) * (fam ? FamilyLds<1>::MAX : FamilyLds<0>::MAX);
}

}  // namespace igaf

namespace igaf {

// Approximate FMA count of one work item of degree p (family fam): used by the
// batch's cost model to order work items longest-first.
template <int P, int FAM>
static double item_cost_t(int Kx)
{
    using Sh = CfgShape<P, FAM>;
    constexpr int RZ = RowsCfg<P, FAM>::RZ, OZC = RowsCfg<P, FAM>::OZC;
    const double pairs = (double)(P + 1) * (P + 1) * Sh::Q;
    const double per_slice = pairs * (2.0 * Sh::N1 * RZ * OZC / Sh::O + 3.0 * Sh::N2 + 3.0 * Sh::NC);
    return per_slice * (Kx + P);
}

double rows_item_cost(int p, int fam, int Kx)
{
#define IGAF_C(PP) \
    case PP: return fam ? item_cost_t<PP, 1>(Kx) : item_cost_t<PP, 0>(Kx);
    switch (p) {
        IGAF_C(1)
        IGAF_C(2)
        IGAF_C(3)
        IGAF_C(4)
        IGAF_C(5)
    default:
        return 0.0;
    }
#undef IGAF_C
}

}  // namespace igaf
