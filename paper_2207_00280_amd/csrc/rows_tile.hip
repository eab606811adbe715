// CSR values of the global mass and stiffness matrices by owner-computes rows,
// one workgroup per tile of row pencils.
//
// The global matrix is the sum of the element matrices (Sec. 3.1).  Summing
// the sum-factorised element contractions over the elements that carry a pair
// of functions gives, for rows I = (ix,iy,iz) and columns J = I + o - p,
//   M_IJ = sum_{gx,gy,gz} c[g] Bx(ix,jx)[gx] By(iy,jy)[gy] Bz(iz,jz)[gz]
// where g runs over the Gauss points of the elements in the common support and
// B(i,j)[g] = w N_i N_j is the pair table of the element holding g (the tables
// the element kernels use).  The stiffness has the three derivative
// placements.  The contraction runs z -> y -> x as in Algorithm 2, but over
// global point sets, so every CSR value is summed in one thread and written
// once, without atomics.
//
// A workgroup owns the row pencils (iy, iz), iy in [iy0, iy0+TY), iz in
// [iz0, iz0+TZ), for the rows ix of one x segment.  It sweeps the x elements
// in order; for element ex:
//   stage z  (one wavefront group per z row iz, shared by the TY pencils):
//            D[iz][t][oz][ey][ky][kx] = sum_{ez,kz} Wz[t] kappa   for the
//            TY+p y elements of the tile's window (t: N N or N'N' pair table)
//   stage y  (one wavefront group per y row iy):
//            C[pen][0|1][kx][oy][oz] = sum_{ey,ky} Wy D  (the three products
//            of Algorithm 2's y stage folded into two: NN.NN and N'N.NN+NN.N'N')
//   stage x  (one thread per (pencil, oy, oz)): the thread keeps C of the last
//            p+1 x elements in registers (a ring), and row ix = ex is then
//            complete: its values for every ox are summed and staged in LDS
//            at their place in the CSR row,
//   stores   the staged rows go out as contiguous segments.
// Two schedules run these stages.  Sequential: every wavefront takes part in
// each stage in turn, four workgroup barriers per element.  Pipelined: stage-z/y
// wavefronts compute element ex (kappa of ex+1 already in their registers)
// while stage-x wavefronts finish and store row ex-1, with one C buffer
// (stage y rewrites it only after the barrier that ends stage x's reads of
// it) and two barriers per element; the two roles run separate loops, so the
// register ring and the kappa prefetch never share a wavefront's registers.
// Stages z and y use wave-uniform tables (scalar loads); stage x's tables
// depend on ix only.  o* in [0, 2p] are column offsets j = i + o - p.
#include "common.h"
#include "launch.h"
#include "rows_common.h"

namespace igaf {

namespace {

__device__ inline int opaque_zero_t()
{
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}

}  // namespace

template <int P_, int TY_, int TZ_, int WPE_, bool PREF_, bool PIPE_, int XS_ = 0>
struct Tile {
    static constexpr int P = P_, TY = TY_, TZ = TZ_;
    static constexpr int WPE = WPE_;                    // wavefronts per SIMD aimed at
    static constexpr bool PREF = PREF_;                 // sequential: kappa of the next element in registers
    static constexpr bool PIPE = PIPE_;                 // pipelined schedule
    // pipelined, stage-x wavefronts storing alone: XS > 0 sums the row's first
    // XS ring elements before the iteration's first barrier and the rest
    // after it, with two staged-row buffers, so that a row goes out in the
    // first phase of the next iteration (the stores and the stage-x sums
    // then fill both phases instead of the second only)
    static constexpr int XS = XS_;
    static constexpr int Q = P + 1, O = 2 * P + 1, S = (P + 1) * (P + 2) / 2;
    static constexpr int Q2 = Q * Q, Q3 = Q2 * Q;
    static constexpr int NLY = TY + P;                  // y elements in the window
    static constexpr int NPEN = TY * TZ;                // pencils per tile
    static constexpr int NZI = NLY * Q2, WZI = (NZI + 63) / 64;     // stage z, per z row
    static constexpr int NYI = TZ * O * Q, WYI = (NYI + 63) / 64;   // stage y, per y row
    static constexpr int NXI = NPEN * O * O, WX = (NXI + 63) / 64;  // stage x
    static constexpr int NWZ = TZ * WZI, NWY = TY * WYI, NWZY = cmax(NWZ, NWY);
    static constexpr int NW = PIPE ? NWZY + WX : cmax(NWZY, WX);
    static constexpr int NT = 64 * NW;
    static constexpr int XW0 = PIPE ? NWZY : 0;         // first stage-x wavefront
    // pipelined: the stage-z wavefronts without stage-y work (HW0..NWZY-1)
    // store rows beside the stage-x wavefronts
    static constexpr int HW0 = PIPE && NWY < NWZY ? NWY : NWZY;
    static constexpr int NTS = PIPE ? 64 * (WX + NWZY - HW0) : NT;   // threads that store rows
    // D[zr][t][oz][ly][ky][kx]
    static constexpr int DOZ = pad16(NZI, Q);
    static constexpr int DT = O * DOZ;
    static constexpr int DZR = pad16(2 * DT, Q * O);
    static constexpr int DSZ = TZ * DZR;
    // C[pen][t][kx][oy][oz]
    static constexpr int CKX = O * O;
    static constexpr int CT = Q * CKX;
    static constexpr int CPEN = pad16(2 * CT, O * O);
    static constexpr int CSZ = NPEN * CPEN;
    // staged rows [pen][t][row position | junk slot]; columns outside the
    // patch are written to the junk slot
    static constexpr int SROW = O * O * O + 1;
    static constexpr int SSZ = NPEN * 2 * SROW;
    static constexpr int SIT = (O * O * O + NTS - 1) / NTS;   // store passes per row
    static constexpr int SGP = PIPE && !XS ? NPEN : 1;  // pencils whose LDS reads go out together
    // LDS (doubles).  Sequential: [D | staged rows] [C]; the rows reuse D,
    // dead after stage y.  Pipelined: [D] [C] [staged rows]; one C suffices:
    // stage y writes it after the barrier that follows the stage-x reads.
    static constexpr int OFF_C = PIPE ? DSZ : cmax(DSZ, SSZ);
    static constexpr int OFF_S = PIPE ? DSZ + CSZ : 0;
    static constexpr int NSTG = XS ? 2 : 1;             // staged-row buffers
    static constexpr int LDS = PIPE ? DSZ + CSZ + NSTG * SSZ : cmax(DSZ, SSZ) + CSZ;
    static_assert(NW <= 16, "workgroup too large");
    static_assert(XS == 0 || (PIPE && HW0 == NWZY && XS <= P), "split stage x: pipelined, x wavefronts store");
};

// Tile shapes per degree (measured on MI355X): TY pencils share stage z; TZ
// rows fill the lanes of stage y; the register budget (WPE wavefronts per
// SIMD) and the LDS size let one to four workgroups share a CU.  At p = 5 the
// stage-x wavefronts carry the critical path (their sums and the row stores
// one after the other), hence the split stage x there.
template <int P> struct TileCfg;
template <> struct TileCfg<1> { using T = Tile<1, 4, 4, 4, true, false>; };
template <> struct TileCfg<2> { using T = Tile<2, 4, 2, 4, true, true>; };
template <> struct TileCfg<3> { using T = Tile<3, 5, 2, 2, false, true>; };
template <> struct TileCfg<4> { using T = Tile<4, 5, 1, 2, true, true>; };
template <> struct TileCfg<5> { using T = Tile<5, 2, 1, 2, false, true, 3>; };

// A second shape per degree for the batched launches, the batch autotuner
// choosing between the two per degree: for p <= 4 a smaller one (fewer
// pencils: less LDS, more workgroups per CU, less work lost at the borders of
// small patches), for p = 5 three pencils sharing stage z without the split.
template <int P> struct TileAlt;
template <> struct TileAlt<1> { using T = Tile<1, 2, 2, 4, true, false>; };
template <> struct TileAlt<2> { using T = Tile<2, 2, 2, 4, true, true>; };
template <> struct TileAlt<3> { using T = Tile<3, 2, 1, 4, false, true>; };
template <> struct TileAlt<4> { using T = Tile<4, 2, 1, 2, true, true>; };
template <> struct TileAlt<5> { using T = Tile<5, 3, 1, 2, false, true>; };

// ---- stage z: thread of wavefront w (< NWZ) holds item (kx, ky, ly) of z row zr
template <class T>
struct ZThread {
    int zr, item, off, key;
    __device__ ZThread(const TileCtx& c, int w, int lane)
    {
        zr = w / T::WZI;
        item = (w % T::WZI) * 64 + lane;
        const int it = item < T::NZI ? item : T::NZI - 1;
        off = it % T::Q + T::Q * ((it / T::Q) % T::Q);
        key = clampi_t(c.iy0 - T::P + it / T::Q2, c.Ky - 1);   // y elements outside are never read
    }
};

// kappa of the thread's z window for element ex: kw[e][kz], e = 0..P
template <class T>
__device__ __forceinline__ void z_load(const TileCtx& c, const ZThread<T>& zt, int ex,
                                       double (&kw)[T::P + 1][T::Q])
{
    constexpr int P = T::P, Q = T::Q, Q2 = T::Q2, Q3 = T::Q3;
    const double* kcol = c.kappa + ((int64_t)ex + (int64_t)c.Kx * zt.key) * Q3 + zt.off;
#pragma unroll
    for (int e = 0; e <= P; ++e) {
        const int ezc = clampi_t(c.iz0 + zt.zr - P + e, c.Kz - 1);
        const double* kp = kcol + (int64_t)c.Kx * c.Ky * Q3 * ezc;
#pragma unroll
        for (int k = 0; k < Q; ++k) kw[e][k] = kp[Q2 * k];
    }
}

// D for element ex.  FROM_REGS: kappa from kw; otherwise loaded here, one z
// element at a time (keeps the register budget of the sequential schedule).
template <class T, bool FROM_REGS>
__device__ __forceinline__ void z_stage(const TileCtx& c, const ZThread<T>& zt, int ex,
                                        const double (&kw)[T::P + 1][T::Q], double* D, int z0)
{
    constexpr int P = T::P, Q = T::Q, O = T::O, S = T::S, Q2 = T::Q2, Q3 = T::Q3;
    const int iz = c.iz0 + zt.zr + z0;   // z0 opaque (sequential): table bases recomputed per element
    const double* kcol = c.kappa + ((int64_t)ex + (int64_t)c.Kx * zt.key) * Q3 + zt.off;
    double d0[O], d1[O];
#pragma unroll
    for (int o = 0; o < O; ++o) d0[o] = d1[o] = 0.0;
    const ctab wnz = c.Wnz + z0, wdz = c.Wdz + z0;
#pragma unroll
    for (int e = 0; e <= P; ++e) {
        const int ez = iz - P + e;
        if (ez < 0 || ez >= c.Kz) continue;   // wave-uniform
        double kz[Q];
        if constexpr (FROM_REGS) {
#pragma unroll
            for (int k = 0; k < Q; ++k) kz[k] = kw[e][k];
        } else {
            const double* kp = kcol + (int64_t)c.Kx * c.Ky * Q3 * ez;
#pragma unroll
            for (int k = 0; k < Q; ++k) kz[k] = kp[Q2 * k];
        }
        const int et = tab_elem(ez, c.rz0, c.rz1);
        const ctab wnE = wnz + (int64_t)et * (S * Q), wdE = wdz + (int64_t)et * (S * Q);
#pragma unroll
        for (int bb = 0; bb <= P; ++bb) {
            const int sp = pair_index(P - e, bb);
            const ctab wn = wnE + sp * Q, wd = wdE + sp * Q;   // constant offsets
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                d0[e + bb] += wn[k] * kz[k];
                d1[e + bb] += wd[k] * kz[k];
            }
        }
        if constexpr (!FROM_REGS) __builtin_amdgcn_sched_barrier(0);
    }
    if (zt.item < T::NZI) {
        double* dp = D + zt.zr * T::DZR + zt.item;
#pragma unroll
        for (int o = 0; o < O; ++o) {
            dp[o * T::DOZ] = d0[o];
            dp[T::DT + o * T::DOZ] = d1[o];
        }
    }
}

// ---- stage y for wavefront w (< NWY): C of the y row w / WYI
template <class T>
__device__ __forceinline__ void y_stage(const TileCtx& c, int w, int lane, const double* D, double* C,
                                        int z0)
{
    constexpr int P = T::P, Q = T::Q, O = T::O, S = T::S, Q2 = T::Q2;
    const int yr = w / T::WYI;
    const int iy = c.iy0 + yr + z0;
    if (iy >= c.Ny) return;   // wave-uniform
    const int item = (w % T::WYI) * 64 + lane;
    const bool act = item < T::NYI;
    const int it = act ? item : T::NYI - 1;
    const int kx = it % Q, oz = (it / Q) % O, zr = it / (Q * O);
    double ca[O], cb[O];
#pragma unroll
    for (int o = 0; o < O; ++o) ca[o] = cb[o] = 0.0;
    const ctab wny = c.Wny + z0, wdy = c.Wdy + z0;
#pragma unroll
    for (int e = 0; e <= P; ++e) {
        const int ey = iy - P + e;
        if (ey < 0 || ey >= c.Ky) continue;   // wave-uniform
        const double* dp = D + zr * T::DZR + oz * T::DOZ + (yr + e) * Q2 + kx;
        double a[Q], b[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            a[k] = dp[k * Q];
            b[k] = dp[T::DT + k * Q];
        }
        const int et = tab_elem(ey, c.ry0, c.ry1);
        const ctab wnE = wny + (int64_t)et * (S * Q), wdE = wdy + (int64_t)et * (S * Q);
#pragma unroll
        for (int bb = 0; bb <= P; ++bb) {
            const int sp = pair_index(P - e, bb);
            const ctab wn = wnE + sp * Q, wd = wdE + sp * Q;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                ca[e + bb] += wn[k] * a[k];
                cb[e + bb] += wd[k] * a[k];
                cb[e + bb] += wn[k] * b[k];
            }
        }
        // sequential schedule: one y element's reads in flight at a time, for
        // the register budget (the pipelined stage-y wavefronts hold no ring)
        if constexpr (!T::PIPE) __builtin_amdgcn_sched_barrier(0);
    }
    if (act) {
        double* cp = C + (yr * T::TZ + zr) * T::CPEN + kx * T::CKX + oz;
#pragma unroll
        for (int o = 0; o < O; ++o) {
            cp[o * O] = ca[o];
            cp[T::CT + o * O] = cb[o];
        }
    }
}

// ring: C of elements ex-P .. ex (zero outside [0, Kx)) as [e][kx][NN | mixed];
// shift in the next element's C (null: an element past the end)
template <class T>
__device__ __forceinline__ void x_shift(const XThread<T>& xt, double (&ring)[T::P + 1][T::Q][2],
                                        const double* C)
{
    constexpr int P = T::P, Q = T::Q, O = T::O;
#pragma unroll
    for (int e = 0; e < P; ++e)
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            ring[e][k][0] = ring[e + 1][k][0];
            ring[e][k][1] = ring[e + 1][k][1];
        }
    if (C) {
        const double* cp = C + xt.pen * T::CPEN + xt.oy * O + xt.oz;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            ring[P][k][0] = cp[k * T::CKX];
            ring[P][k][1] = cp[T::CT + k * T::CKX];
        }
    } else {
#pragma unroll
        for (int k = 0; k < Q; ++k) ring[P][k][0] = ring[P][k][1] = 0.0;
    }
}

// row ix, ring elements E0 <= e < E1: every ox of the thread's (oy, oz)
// summed into m, k
template <class T, int E0, int E1>
__device__ __forceinline__ void x_row_sum(const TileCtx& c, const double (&ring)[T::P + 1][T::Q][2], int ix,
                                          double (&m)[T::O], double (&k)[T::O])
{
    constexpr int P = T::P, Q = T::Q, S = T::S;
#pragma unroll
    for (int e = E0; e < E1; ++e) {
        // the ring holds zeros outside the patch
        const int exc = tab_elem(clampi_t(ix - P + e, c.Kx - 1), c.rx0, c.rx1);
        const ctab wnE = c.Wnx + (int64_t)exc * (S * Q), wdE = c.Wdx + (int64_t)exc * (S * Q);
#pragma unroll
        for (int bb = 0; bb <= P; ++bb) {
            const int sp = pair_index(P - e, bb);
            const ctab wn = wnE + sp * Q, wd = wdE + sp * Q;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                m[e + bb] += wn[q] * ring[e][q][0];
                k[e + bb] += wd[q] * ring[e][q][0];
                k[e + bb] += wn[q] * ring[e][q][1];
            }
        }
    }
}

// row ix summed: staged at the row positions of the thread's (oy, oz)
template <class T>
__device__ __forceinline__ void x_row_put(const TileCtx& c, const XThread<T>& xt, int ix,
                                          const double (&m)[T::O], const double (&k)[T::O], double* STG)
{
    constexpr int P = T::P, O = T::O;
    const int Lx = band_len(ix, P, c.Nx);
    const int sub = xt.sub * Lx + (ix - P - band_lo(ix, P));   // + ox
    double* stM = STG + xt.pen * 2 * T::SROW;
    // branch-free stores (a branch per column would pull the column's
    // arithmetic, and all its table loads, apart)
#pragma unroll
    for (int ox = 0; ox < O; ++ox) {
        const int jx = ix + ox - P;
        const int pos = xt.row && jx >= 0 && jx < c.Nx ? sub + ox : T::SROW - 1;
        stM[pos] = m[ox];
        stM[T::SROW + pos] = k[ox];
    }
}

template <class T>
__device__ __forceinline__ void x_row(const TileCtx& c, const XThread<T>& xt,
                                      const double (&ring)[T::P + 1][T::Q][2], int ix, double* STG)
{
    double m[T::O], k[T::O];
#pragma unroll
    for (int o = 0; o < T::O; ++o) m[o] = k[o] = 0.0;
    x_row_sum<T, 0, T::P + 1>(c, ring, ix, m, k);
    x_row_put<T>(c, xt, ix, m, k, STG);
}

// One tile (pencils iy0.., iz0..) over the rows [seg*seglen, (seg+1)*seglen)
// of a patch, by one workgroup of T::NT threads with T::LDS doubles of LDS.
template <class T>
__device__ __forceinline__ void tile_run(const PatchDev& pd, const RowMap& rm,
                                         const double* __restrict__ kappa,
                                         double* __restrict__ Mv, double* __restrict__ Kv,
                                         int tile, int seg, int nty, int seglen, double* lds)
{
    constexpr int P = T::P, Q = T::Q;
    TileCtx c;
    c.kappa = kappa;
    c.Mv = Mv;
    c.Kv = Kv;
    c.Wnx = as_ctab(pd.d[0].Wnn);
    c.Wdx = as_ctab(pd.d[0].Wdd);
    c.Wny = as_ctab(pd.d[1].Wnn);
    c.Wdy = as_ctab(pd.d[1].Wdd);
    c.Wnz = as_ctab(pd.d[2].Wnn);
    c.Wdz = as_ctab(pd.d[2].Wdd);
    c.T0 = rm.T[0];
    c.T1 = rm.T[1];
    c.Kx = pd.d[0].K;
    c.Ky = pd.d[1].K;
    c.Kz = pd.d[2].K;
    c.Nx = pd.d[0].N;
    c.Ny = pd.d[1].N;
    c.Nz = pd.d[2].N;
    c.iy0 = (tile % nty) * T::TY;
    c.iz0 = (tile / nty) * T::TZ;
    tile_runs(c, pd);
    const int X0 = seg * seglen, X1 = min(c.Nx, X0 + seglen);   // rows emitted
    const int xs = max(0, X0 - P);                               // first element swept

    const int tid = threadIdx.x;
    // wave index made provably uniform, so that wave-derived addresses are scalar
    const int w = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    double* const D = lds;
    double* const C0 = lds + T::OFF_C;
    double* const STG = lds + T::OFF_S;

    if constexpr (!T::PIPE) {
        const ZThread<T> zt(c, w, lane);
        double kw[P + 1][Q];
        if constexpr (T::PREF) {
            if (w < T::NWZ && xs < c.Kx) z_load<T>(c, zt, xs, kw);
        }
        const XThread<T> xt(c, w * 64 + lane);
        int64_t pbase;
        int plen;
        pencil_rows<T>(c, lane, pbase, plen);
        double ring[P + 1][Q][2];
#pragma unroll
        for (int e = 0; e <= P; ++e)
#pragma unroll
            for (int k = 0; k < Q; ++k) ring[e][k][0] = ring[e][k][1] = 0.0;

        for (int ix = xs; ix < X1; ++ix) {
            const bool elem = ix < c.Kx;   // element ex = ix exists
            const bool emit = ix >= X0;    // row ix belongs to this segment
            const int z0 = opaque_zero_t();
            if (elem) {
                if (w < T::NWZ) {
                    z_stage<T, T::PREF>(c, zt, ix, kw, D, z0);
                    if constexpr (T::PREF) {
                        if (ix + 1 < c.Kx) z_load<T>(c, zt, ix + 1, kw);
                    }
                }
                __syncthreads();
                if (w < T::NWY) y_stage<T>(c, w, lane, D, C0, z0);
                __syncthreads();
            }
            if (w < T::WX) x_shift<T>(xt, ring, elem ? C0 : nullptr);
            if (emit) {
                if (w < T::WX) x_row<T>(c, xt, ring, ix, STG);
                __syncthreads();
                store_row<T>(c, STG, ix, tid, pbase, plen);
                __syncthreads();   // the next stage z rewrites the staged rows
            }
        }
    } else {
        // pipelined: iteration t computes element t on the stage-z/y
        // wavefronts and finishes row t-1 on the stage-x wavefronts; both
        // roles pass the same two barriers per iteration (split stage x: one
        // more iteration, which stores the last row)
        const int xe = min(c.Kx, X1);   // elements swept: [xs, xe)
        const int tend = X1 + (T::XS ? 1 : 0);
        if (w < T::NWZY) {
            const ZThread<T> zt(c, w, lane);
            double kw[P + 1][Q];
            if (w < T::NWZ && xs < xe) z_load<T>(c, zt, xs, kw);
            int64_t pbase = 0;
            int plen = 0;
            if (w >= T::HW0) pencil_rows<T>(c, lane, pbase, plen);
            const int ts = 64 * (T::WX + w - T::HW0) + lane;
            for (int t = xs; t <= tend; ++t) {
                const bool el = t < xe;
                const int z0 = 0;   // no ring here: table bases may stay in registers
                if (el && w < T::NWZ) {
                    z_stage<T, true>(c, zt, t, kw, D, z0);
                    if (t + 1 < xe) z_load<T>(c, zt, t + 1, kw);
                }
                __syncthreads();
                if (w < T::NWY) {
                    if (el) y_stage<T>(c, w, lane, D, C0, z0);
                } else if (w >= T::HW0 && t - 1 >= X0) {
                    store_row<T>(c, STG, t - 1, ts, pbase, plen);
                }
                __syncthreads();
            }
        } else {
            const int wx = w - T::XW0;
            const XThread<T> xt(c, wx * 64 + lane);
            int64_t pbase;
            int plen;
            pencil_rows<T>(c, lane, pbase, plen);
            double ring[P + 1][Q][2];
#pragma unroll
            for (int e = 0; e <= P; ++e)
#pragma unroll
                for (int k = 0; k < Q; ++k) ring[e][k][0] = ring[e][k][1] = 0.0;
            if constexpr (T::XS == 0) {
                for (int t = xs; t <= X1; ++t) {
                    const int r = t - 1;   // row finished in this iteration
                    const bool live = r >= xs, emit = r >= X0;
                    if (live) {
                        x_shift<T>(xt, ring, r < xe ? C0 : nullptr);
                        if (emit) x_row<T>(c, xt, ring, r, STG);
                    }
                    __syncthreads();
                    if (emit) store_row<T>(c, STG, r, wx * 64 + lane, pbase, plen);
                    __syncthreads();
                }
            } else {
                // row r = t-1 summed over both phases of iteration t into
                // buffer r & 1, stored in the first phase of iteration t+1
                for (int t = xs; t <= tend; ++t) {
                    const int r = t - 1;
                    const bool live = r >= xs && r < X1, emit = live && r >= X0;
                    if (live) x_shift<T>(xt, ring, r < xe ? C0 : nullptr);
                    if (r - 1 >= X0)
                        store_row<T>(c, STG + ((r - 1) & 1) * T::SSZ, r - 1, wx * 64 + lane, pbase, plen);
                    __builtin_amdgcn_sched_barrier(0);
                    double m[T::O], k[T::O];
#pragma unroll
                    for (int o = 0; o < T::O; ++o) m[o] = k[o] = 0.0;
                    if (emit) x_row_sum<T, 0, T::XS>(c, ring, r, m, k);
                    __syncthreads();
                    if (emit) {
                        x_row_sum<T, T::XS, P + 1>(c, ring, r, m, k);
                        x_row_put<T>(c, xt, r, m, k, STG + (r & 1) * T::SSZ);
                    }
                    __syncthreads();
                }
            }
        }
    }
}

template <class T>
__global__ __launch_bounds__(T::NT) __attribute__((amdgpu_waves_per_eu(T::WPE))) void k_rows_tile(
    PatchDev pd, RowMap rm, const double* __restrict__ kappa, double* __restrict__ Mv,
    double* __restrict__ Kv, int nty, int ntz, int nseg, int seglen, int nb8)
{
    __shared__ double lds[T::LDS];
    const int ntile = nty * ntz;
    const int b = xcd_tile(blockIdx.x, nb8);
    if (b >= ntile * nseg) return;   // whole workgroup
    tile_run<T>(pd, rm, kappa, Mv, Kv, b % ntile, b / ntile, nty, seglen, lds);
}

template <class T>
static int launch_rows_tile_t(const PatchDev& pd, const double* kappa, double* Mv, double* Kv,
                              hipStream_t st)
{
    RowMap rm = make_rowmap(pd);
    const int Nx = pd.d[0].N, Ny = pd.d[1].N, Nz = pd.d[2].N;
    const int nty = (Ny + T::TY - 1) / T::TY, ntz = (Nz + T::TZ - 1) / T::TZ;
    const int ntile = nty * ntz;
    // x segments: enough workgroups to keep every slot busy to the end, each
    // segment paying p warm-up elements (stages z and y only)
    const int slots = device_slots((const void*)k_rows_tile<T>, T::NT);
    if (!slots) return -3;
    // cost in element steps: the items spread over the slots, plus one item
    // as the tail; a segment pays ~4p/3 steps of warm-up and start-up (fitted
    // to sweeps of the segment count at 64^3 and 128^3)
    int nseg = 1;
    double best = 1e300;
    for (int s = 1; s <= 16 && (Nx + s - 1) / s >= 2 * T::P + 2; ++s) {
        const int64_t items = (int64_t)ntile * s;
        const double item = (Nx + s - 1) / s + 4.0 * T::P / 3.0;
        const double cost = (double)items * item / slots + item;
        if (cost < best - 1e-9) {
            best = cost;
            nseg = s;
        }
    }
    const int seglen = (Nx + nseg - 1) / nseg;
    const int nb = ntile * nseg, nb8 = (nb + 7) / 8;
    hipLaunchKernelGGL(k_rows_tile<T>, dim3(nb8 * 8), dim3(T::NT), 0, st, pd, rm, kappa, Mv, Kv,
                       nty, ntz, nseg, seglen, nb8);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_rows(const PatchDev& pd, const double* kappa, double* Mv, double* Kv, hipStream_t st)
{
    switch (pd.p) {
    case 1: return launch_rows_tile_t<TileCfg<1>::T>(pd, kappa, Mv, Kv, st);
    case 2: return launch_rows_tile_t<TileCfg<2>::T>(pd, kappa, Mv, Kv, st);
    case 3: return launch_rows_tile_t<TileCfg<3>::T>(pd, kappa, Mv, Kv, st);
    case 4: return launch_rows_tile_t<TileCfg<4>::T>(pd, kappa, Mv, Kv, st);
    case 5: return launch_rows_tile_t<TileCfg<5>::T>(pd, kappa, Mv, Kv, st);
    default: return -4;
    }
}

// ---------------------------------------------------------------------------
// Batched launch: one launch per degree present, each with that degree's
// tile, one workgroup per work item (patch, tile, x segment) of a list sorted
// longest first.  An item sweeps the rows of its pencils in its x segment
// (after p warm-up elements when it does not start at the patch boundary).

template <class Tp>
__device__ inline Tp uniform_ptr(Tp p)
{
    uint64_t v = reinterpret_cast<uint64_t>(p);
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<Tp>(((uint64_t)hi << 32) | lo);
}

__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// the patch record in scalar registers
__device__ inline void uniform_patch(const BatchPatch& src, PatchDev& pd, RowMap& rm,
                                     const double*& kappa, double*& Mv, double*& Kv)
{
    pd = src.pd;
    rm = src.rm;
    for (int d = 0; d < 3; ++d) {
        pd.d[d].Wnn = uniform_ptr(pd.d[d].Wnn);
        pd.d[d].Wdd = uniform_ptr(pd.d[d].Wdd);
        pd.d[d].K = uniform_int(pd.d[d].K);
        pd.d[d].N = uniform_int(pd.d[d].N);
        rm.T[d] = ((int64_t)uniform_int((int)(rm.T[d] >> 32)) << 32) | (uint32_t)uniform_int((int)rm.T[d]);
    }
    pd.p = uniform_int(pd.p);
    kappa = uniform_ptr(src.kappa);
    Mv = uniform_ptr(src.Mv);
    Kv = uniform_ptr(src.Kv);
}

template <class T>
__global__ __launch_bounds__(T::NT) __attribute__((amdgpu_waves_per_eu(T::WPE))) void k_rows_tile_items(
    const BatchPatch* __restrict__ patches, const int4* __restrict__ items, int nitems, int chunk)
{
    __shared__ double lds[T::LDS];
    // XCD x (which receives workgroups b = x mod 8) takes the item chunks
    // x, x+8, x+16, ...: neighbouring tiles share its L2, and the list stays
    // longest-first on every XCD
    const int x = blockIdx.x % 8, j = blockIdx.x / 8;
    const int b = ((j / chunk) * 8 + x) * chunk + j % chunk;
    if (b >= nitems) return;   // whole workgroup
    const int4 it = items[b];
    const int pid = uniform_int(it.x), tile = uniform_int(it.y);
    const int seg = uniform_int(it.z), seglen = uniform_int(it.w);
    PatchDev pd;
    RowMap rm;
    const double* kappa;
    double *Mv, *Kv;
    uniform_patch(patches[pid], pd, rm, kappa, Mv, Kv);
    if (pd.p != T::P) return;   // not an item of this degree (whole workgroup)
    tile_run<T>(pd, rm, kappa, Mv, Kv, tile, seg, (pd.d[1].N + T::TY - 1) / T::TY, seglen, lds);
}

template <class T>
static int launch_items_t(const BatchPatch* patches, const int4* items, int nitems, int chunk, hipStream_t st)
{
    hipLaunchKernelGGL(k_rows_tile_items<T>, dim3(rows_batch_grid(nitems, chunk)), dim3(T::NT), 0, st, patches,
                       items, nitems, chunk);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_rows_batch(int p, int variant, const BatchPatch* patches, const int4* items, int nitems, int chunk,
                      hipStream_t st)
{
    if (nitems <= 0) return 0;
    if (chunk < 1) return -4;
#define IGAF_RB(PP)                                                                                          \
    case PP:                                                                                                 \
        return variant ? launch_items_t<TileAlt<PP>::T>(patches, items, nitems, chunk, st)                   \
                       : launch_items_t<TileCfg<PP>::T>(patches, items, nitems, chunk, st);
    switch (p) {
        IGAF_RB(1)
        IGAF_RB(2)
        IGAF_RB(3)
        IGAF_RB(4)
        IGAF_RB(5)
    default: return -4;
    }
#undef IGAF_RB
}

int rows_batch_grid(int nitems, int chunk)
{
    return nitems <= 0 || chunk < 1 ? 0 : (nitems + 8 * chunk - 1) / (8 * chunk) * (8 * chunk);
}

// Tiles of a degree-p patch and the relative cost of one element step of a
// tile: fused-multiply-add issue slots of its wavefronts per x element (an
// item costs this times the elements it sweeps).  Used to sort each degree's
// items longest first.
template <class T>
static void tile_info_t(int Ny, int Nz, int* ntile, double* per_elem)
{
    *ntile = ((Ny + T::TY - 1) / T::TY) * ((Nz + T::TZ - 1) / T::TZ);
    constexpr double terms = (double)(T::P + 1) * (T::P + 1) * T::Q;
    *per_elem = T::NWZ * 2.0 * terms + T::NWY * 3.0 * terms + T::WX * 3.0 * terms;
}

int rows_tile_info(int p, int variant, int Ny, int Nz, int* ntile, double* per_elem)
{
#define IGAF_TI(PP)                                                                                          \
    case PP:                                                                                                 \
        if (variant) tile_info_t<TileAlt<PP>::T>(Ny, Nz, ntile, per_elem);                                  \
        else tile_info_t<TileCfg<PP>::T>(Ny, Nz, ntile, per_elem);                                          \
        return 0;
    switch (p) {
        IGAF_TI(1)
        IGAF_TI(2)
        IGAF_TI(3)
        IGAF_TI(4)
        IGAF_TI(5)
    default: return -4;
    }
#undef IGAF_TI
}

}  // namespace igaf
