// CSR values of the mass and stiffness matrices on a mapped geometry by
// owner-computed rows: one workgroup per tile of row pencils, no atomics, no
// workspace.
//
// With the per-point fields of a mapped geometry (cm = kappa det J and the
// symmetric tensor G = kappa det J J^-1 J^-T, given per quadrature point of
// every element) the global matrices are sums over the Gauss points of the
// elements in the common support of a row I and a column J (Sec. 3.1 summed
// over eq. (10) with J(x^n) varying per point):
//   M_IJ = sum_g cm[g] phi_I phi_J,   K_IJ = sum_g sum_{c,d} G_cd[g] d_c phi_I d_d phi_J.
// A cross term G_cd (c != d) puts N'_a N_b in direction c and N_a N'_b in
// direction d, so each direction works with ordered (test a, trial b) pairs.
// The contraction runs z -> y -> x (Algorithm 2's order) over global point
// sets, as for the identity geometry, with the nine stage-z and five stage-y
// products of the mapped-geometry element kernel:
//   stage z  D0 = nn.cm  D1 = nn.Gxx  D2 = nn.Gyy  D3 = dd.Gzz  D4 = nn.Gxy
//            D5 = nd.Gxz D6 = dn.Gxz  D7 = nd.Gyz  D8 = dn.Gyz
//   stage y  CM = nn D0, Cnn = dd D2 + nn D3 + dn D7 + nd D8, Cdd = nn D1,
//            Cdn = nd D4 + nn D5, Cnd = dn D4 + nn D6
//   stage x  M = nn CM,  K = nn Cnn + dd Cdd + dn Cdn + nd Cnd
// (nn[a][b][k] = w N_a N_b, dd = w N'_a N'_b, dn = w N'_a N_b, nd = w N_a N'_b
// at the Gauss points k of one element and direction).  Every product is
// taken as (weighted test value x input) folded over the test index first,
// then contracted with the plain trial values.
//
// A workgroup owns TY x TZ row pencils (iy in [iy0, iy0+TY), iz in
// [iz0, iz0+TZ)) and sweeps the x elements of one x segment in order.  Its
// wavefronts have two roles, pipelined one element apart (two barriers per
// element):
//   z/y wavefronts  element t: stage z, in units of one pass of three
//                   products and up to 64 points (ly, ky, kx) of the TY+p y
//                   elements of the window, for all TZ z rows of the tile
//                   (their z windows overlap: TZ+p z elements are loaded,
//                   the next element's while the current one is contracted);
//                   then stage y, in units of one y row, one output group
//                   and up to 64 (zr, oz, kx);
//   x wavefronts    element t-1: every (pencil, oy, oz) adds element t-1's
//                   contributions to the p+1 rows it touches.  Row ix is kept
//                   in slot ix mod (p+1) of the thread's accumulators; the
//                   sweep is unrolled by p+1 so that every slot index, test
//                   index and column offset is a compile-time constant.  After
//                   element ix the row ix is complete: it is staged in LDS at
//                   its CSR positions and stored as one contiguous segment per
//                   pencil, and its slot restarts at zero.  The slots are
//                   split over G groups of x wavefronts (register budget).
// Every unit is uniform over its wavefront (one pass, one y row and group),
// so every 1D table value (w N, w N', N, N' per element, the plan's
// Wg tables) is a scalar operand.
#include "common.h"
#include "launch.h"
#include "rows_common.h"

#include <type_traits>

namespace igaf {

template <int P_, int TY_, int TZ_, int NZW_, int G_, int WPE_, int ROUNDS_ = 1>
struct GeoTile {
    static constexpr int P = P_, TY = TY_, TZ = TZ_, G = G_, WPE = WPE_;
    // 1: all nine stage-z products of an element in LDS at once; 3: one pass
    // (three products) at a time, stage y accumulating over the three rounds
    static constexpr int ROUNDS = ROUNDS_;
    static constexpr int Q = P + 1, O = 2 * P + 1, Q2 = Q * Q, Q3 = Q2 * Q;
    static constexpr int NLY = TY + P;                       // y elements in the window
    static constexpr int NPEN = TY * TZ;                     // pencils per tile
    static constexpr int NLZ = TZ + P;                       // z elements of the tile's rows
    static constexpr int NZI = NLY * Q2, WZP = (NZI + 63) / 64;   // stage z items per pass
    static constexpr int NZU = (ROUNDS == 1 ? 3 : 1) * WZP;       // stage z units per round
    static constexpr int NYI = TZ * O * Q, WYP = (NYI + 63) / 64; // stage y items per (y row, group)
    static constexpr int NYU = TY * 3 * WYP;                      // stage y units
    static constexpr int NWZY = NZW_;                        // z/y wavefronts
    static constexpr bool ZPF = ROUNDS == 1 && NZU <= NWZY;  // one z unit per wavefront: prefetch
    static constexpr int NXI = NPEN * O * O, WXG = (NXI + 63) / 64;   // stage x: per slot group
    static constexpr int WX = G * WXG;
    static constexpr int NSL = (P + 1 + G - 1) / G;          // row slots per x thread
    static constexpr int NW = NWZY + WX, NT = 64 * NW, XW0 = NWZY;
    static constexpr int HW0 = NYU < NWZY ? NYU : NWZY;      // z/y wavefronts without y units
    static constexpr int NTS = 64 * (WX + NWZY - HW0);       // threads that store rows
    static constexpr int SROW = O * O * O + 1;
    static constexpr int SIT = (O * O * O + NTS - 1) / NTS;
    static constexpr int SGP = NPEN;
    // LDS (doubles): D[zr][9 or 3][O][DOZ] (DOZ >= NZI: [ly][ky][kx]);
    // C[5][NPEN][CP] (CP >= Q O O: [kx][oy][oz]); staged rows [NPEN][2][SROW]
    static constexpr int DOZ = pad16(NZI, Q), DD = O * DOZ, DZR = (ROUNDS == 1 ? 9 : 3) * DD, DSZ = TZ * DZR;
    static constexpr int CP = pad16(Q * O * O, O * O), CC = NPEN * CP, CSZ = 5 * CC;
    static constexpr int SSZ = NPEN * 2 * SROW;
    static constexpr int TBE = 4 * Q2;                       // one element's Wg table
    static constexpr int OFF_C = DSZ, OFF_S = OFF_C + CSZ;
    static constexpr int LDS = OFF_S + SSZ;
    static_assert(NW <= 16, "workgroup too large");
    static_assert(NZU <= 4 * NWZY && NYU <= 4 * NWZY, "units per wavefront");
    static_assert(ROUNDS == 1 || (ROUNDS == 3 && NZU <= NWZY && NYU <= 2 * NWZY), "units per wavefront (rounds)");
    static_assert(LDS * 8 <= 160 * 1024, "LDS");
};

// Tile shapes per degree: TZ rows fill the lanes of stage y, TY pencils share
// stage z; G slot groups bound the x wavefronts' accumulators ((p+1)/G slots
// of 2(2p+1) values).  At p = 3 a one-pencil tile (48 KB of LDS, four
// wavefronts) lets two workgroups share a CU, which measured faster than the
// larger tiles with one workgroup per CU.
template <int P> struct GeoCfg;
template <> struct GeoCfg<1> { using T = GeoTile<1, 4, 4, 6, 1, 2>; };
template <> struct GeoCfg<2> { using T = GeoTile<2, 2, 2, 6, 1, 2>; };
template <> struct GeoCfg<3> { using T = GeoTile<3, 1, 1, 3, 1, 2>; };
template <> struct GeoCfg<4> { using T = GeoTile<4, 1, 1, 6, 1, 2>; };
// p = 5: the nine products of one element would need 182 KB of LDS; three
// rounds of three (111 KB)
template <> struct GeoCfg<5> { using T = GeoTile<5, 1, 1, 4, 2, 2, 3>; };

struct GeoCtx {
    TileCtx c;
    const double* cm;
    const double* G;
    ctab Wx, Wy, Wz;   // Wg tables of the three directions
};

// products j = 0..2 of stage-z pass PASS: field (0 cm, 1..6 Gxx Gyy Gzz Gxy
// Gxz Gyz), test kind (0 w N, 1 w N'), trial kind (2 N, 3 N'); D index 3 PASS + j
//   pass 0: cm nn, Gxx nn, Gyy nn;  1: Gzz dd, Gxy nn, Gxz nd;  2: Gxz dn, Gyz nd, Gyz dn
template <int PASS> struct ZPass;
template <> struct ZPass<0> { static constexpr int f[3] = {0, 1, 2}, tk[3] = {0, 0, 0}, rk[3] = {2, 2, 2}; };
template <> struct ZPass<1> { static constexpr int f[3] = {3, 4, 5}, tk[3] = {1, 0, 0}, rk[3] = {3, 2, 3}; };
template <> struct ZPass<2> { static constexpr int f[3] = {5, 6, 6}, tk[3] = {1, 0, 1}, rk[3] = {2, 3, 2}; };

// ---- stage z, pass PASS for all TZ z rows of the tile: thread on point
// item (ly, ky, kx).  The rows' z windows overlap: the TZ+p z elements
// iz0-p .. iz0+TZ-1 are loaded once.  gz_load fetches the pass's three
// fields of element ex on them (z elements outside the patch are read at a
// clamped index and never used; a field the call does not need is read from
// the other one and its products are never stored); gz_unit contracts them.
template <class T, int PASS>
__device__ __forceinline__ void gz_load(const GeoCtx& g, int item, int ex, double (&pf)[3][T::NLZ][T::Q])
{
    constexpr int P = T::P, Q = T::Q, Q2 = T::Q2, Q3 = T::Q3;
    using PS = ZPass<PASS>;
    const TileCtx& c = g.c;
    const int it = item < T::NZI ? item : T::NZI - 1;
    const int ly = it / Q2, pq = it % Q2;   // pq = ky Q + kx
    const int ey = clampi_t(c.iy0 - P + ly, c.Ky - 1);   // y elements outside are never read
    const int64_t exy = (int64_t)ex + (int64_t)c.Kx * ey;   // element index without its z part
    const int64_t layer = (int64_t)c.Kx * c.Ky;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const bool gf = PS::f[j] > 0 && g.G;                      // a G component, present
        const double* src = PS::f[j] == 0 ? (g.cm ? g.cm : g.G) : (g.G ? g.G + (PS::f[j] - 1) * Q3 : g.cm);
        const int64_t es = gf ? 6 * Q3 : Q3;
#pragma unroll
        for (int m = 0; m < T::NLZ; ++m) {
            const int ezc = clampi_t(c.iz0 - P + m, c.Kz - 1);
            const double* sp = src + (exy + layer * ezc) * es + pq;
#pragma unroll
            for (int k = 0; k < Q; ++k) pf[j][m][k] = sp[Q2 * k];
        }
    }
}

template <class T, int PASS>
__device__ __forceinline__ void gz_unit(const GeoCtx& g, int item, const double (&pf)[3][T::NLZ][T::Q], double* D)
{
    constexpr int P = T::P, Q = T::Q, O = T::O, Q2 = T::Q2;
    using PS = ZPass<PASS>;
    const TileCtx& c = g.c;
#pragma unroll
    for (int zr = 0; zr < T::TZ; ++zr) {
        const int iz = c.iz0 + zr;
        if (iz >= c.Nz) break;   // rows outside: D never read (wave-uniform)
        double acc[3][O];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int o = 0; o < O; ++o) acc[j][o] = 0.0;
#pragma unroll
        for (int e = 0; e <= P; ++e) {
            const int ez = iz - P + e;
            if (ez < 0 || ez >= c.Kz) continue;   // wave-uniform
            const ctab tb = g.Wz + (int64_t)tab_elem(ez, c.rz0, c.rz1) * T::TBE;   // test index P - e, trial bb
            double gv[3][Q];
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int k = 0; k < Q; ++k) gv[j][k] = pf[j][zr + e][k] * tb[PS::tk[j] * Q2 + (P - e) * Q + k];
#pragma unroll
            for (int bb = 0; bb <= P; ++bb)
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int k = 0; k < Q; ++k) acc[j][e + bb] += tb[PS::rk[j] * Q2 + bb * Q + k] * gv[j][k];
        }
        if (item < T::NZI) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double* dp = D + zr * T::DZR + (T::ROUNDS == 1 ? 3 * PASS + j : j) * T::DD + item;
#pragma unroll
                for (int o = 0; o < O; ++o) dp[o * T::DOZ] = acc[j][o];
            }
        }
    }
}

// one stage-z unit u (several per wavefront when the units outnumber the
// z/y wavefronts): load and contract at once
template <class T>
__device__ __forceinline__ void gz_unit_direct(const GeoCtx& g, int u, int lane, int ex, double* D)
{
    const int pass = u / T::WZP;
    const int item = (u % T::WZP) * 64 + lane;
    double pf[3][T::NLZ][T::Q];
    if (pass == 0) {
        gz_load<T, 0>(g, item, ex, pf);
        gz_unit<T, 0>(g, item, pf, D);
    } else if (pass == 1) {
        gz_load<T, 1>(g, item, ex, pf);
        gz_unit<T, 1>(g, item, pf, D);
    } else {
        gz_load<T, 2>(g, item, ex, pf);
        gz_unit<T, 2>(g, item, pf, D);
    }
}

// stage z of pass PASS for the rounds schedule: the fields of one z element
// at a time are loaded and contracted (no prefetch: the register budget of
// the degree the rounds are for)
template <class T, int PASS>
__device__ __forceinline__ void gz_stream(const GeoCtx& g, int item, int ex, double* D)
{
    constexpr int P = T::P, Q = T::Q, O = T::O, Q2 = T::Q2, Q3 = T::Q3;
    using PS = ZPass<PASS>;
    const TileCtx& c = g.c;
    const int it = item < T::NZI ? item : T::NZI - 1;
    const int ly = it / Q2, pq = it % Q2;
    const int ey = clampi_t(c.iy0 - P + ly, c.Ky - 1);
    const int64_t exy = (int64_t)ex + (int64_t)c.Kx * ey;
    const int64_t layer = (int64_t)c.Kx * c.Ky;
    const double* src[3];
    int64_t es[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        src[j] = PS::f[j] == 0 ? (g.cm ? g.cm : g.G) : (g.G ? g.G + (PS::f[j] - 1) * Q3 : g.cm);
        es[j] = PS::f[j] > 0 && g.G ? 6 * Q3 : Q3;
    }
#pragma unroll
    for (int zr = 0; zr < T::TZ; ++zr) {
        const int iz = c.iz0 + zr;
        if (iz >= c.Nz) break;   // wave-uniform
        double acc[3][O];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int o = 0; o < O; ++o) acc[j][o] = 0.0;
#pragma unroll
        for (int e = 0; e <= P; ++e) {
            const int ez = iz - P + e;
            if (ez < 0 || ez >= c.Kz) continue;   // wave-uniform
            const ctab tb = g.Wz + (int64_t)tab_elem(ez, c.rz0, c.rz1) * T::TBE;
            double gv[3][Q];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double* sp = src[j] + (exy + layer * ez) * es[j] + pq;
#pragma unroll
                for (int k = 0; k < Q; ++k) gv[j][k] = sp[Q2 * k] * tb[PS::tk[j] * Q2 + (P - e) * Q + k];
            }
#pragma unroll
            for (int bb = 0; bb <= P; ++bb)
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int k = 0; k < Q; ++k) acc[j][e + bb] += tb[PS::rk[j] * Q2 + bb * Q + k] * gv[j][k];
        }
        if (item < T::NZI) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double* dp = D + zr * T::DZR + j * T::DD + item;
#pragma unroll
                for (int o = 0; o < O; ++o) dp[o * T::DOZ] = acc[j][o];
            }
        }
    }
}

// ---- stage y, output group GR of y row yr: thread on (zr, oz, kx)
//   GR 0: CM, Cdd;  GR 1: Cnn;  GR 2: Cdn, Cnd      (C index 0 CM, 1 Cnn, 2 Cdd, 3 Cdn, 4 Cnd)
template <class T, int GR>
__device__ __forceinline__ void gy_unit(const GeoCtx& g, int yr, int item, const double* D, double* C)
{
    constexpr int P = T::P, Q = T::Q, O = T::O, Q2 = T::Q2;
    const TileCtx& c = g.c;
    const int iy = c.iy0 + yr;
    if (iy >= c.Ny) return;   // wave-uniform
    const bool act = item < T::NYI;
    const int it = act ? item : T::NYI - 1;
    const int zr = it / (O * Q), oz = (it / Q) % O, kx = it % Q;
    double c0[O], c1[O];
#pragma unroll
    for (int o = 0; o < O; ++o) c0[o] = c1[o] = 0.0;
#pragma unroll
    for (int e = 0; e <= P; ++e) {
        const int ey = iy - P + e;
        if (ey < 0 || ey >= c.Ky) continue;   // wave-uniform
        const ctab tb = g.Wy + (int64_t)tab_elem(ey, c.ry0, c.ry1) * T::TBE;
        const ctab wN = tb + (P - e) * Q, wD = tb + Q2 + (P - e) * Q;
        const ctab Nb = tb + 2 * Q2, Db = tb + 3 * Q2;
        const double* dp = D + zr * T::DZR + oz * T::DOZ + (yr + e) * Q2 + kx;
        if constexpr (GR == 0) {
            double g0[Q], g1[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                g0[k] = wN[k] * dp[0 * T::DD + k * Q];
                g1[k] = wN[k] * dp[1 * T::DD + k * Q];
            }
#pragma unroll
            for (int bb = 0; bb <= P; ++bb)
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    c0[e + bb] += Nb[bb * Q + k] * g0[k];
                    c1[e + bb] += Nb[bb * Q + k] * g1[k];
                }
        } else if constexpr (GR == 1) {
            double hN[Q], hD[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                hN[k] = wN[k] * dp[3 * T::DD + k * Q] + wD[k] * dp[7 * T::DD + k * Q];
                hD[k] = wN[k] * dp[8 * T::DD + k * Q] + wD[k] * dp[2 * T::DD + k * Q];
            }
#pragma unroll
            for (int bb = 0; bb <= P; ++bb)
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    c0[e + bb] += Nb[bb * Q + k] * hN[k];
                    c0[e + bb] += Db[bb * Q + k] * hD[k];
                }
        } else {
            double b4[Q], c5[Q], d6[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const double d4 = dp[4 * T::DD + k * Q];
                b4[k] = wN[k] * d4;
                c5[k] = wN[k] * dp[5 * T::DD + k * Q];
                d6[k] = wD[k] * d4 + wN[k] * dp[6 * T::DD + k * Q];
            }
#pragma unroll
            for (int bb = 0; bb <= P; ++bb)
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    c0[e + bb] += Db[bb * Q + k] * b4[k];
                    c0[e + bb] += Nb[bb * Q + k] * c5[k];
                    c1[e + bb] += Nb[bb * Q + k] * d6[k];
                }
        }
    }
    if (act) {
        constexpr int o0 = GR == 0 ? 0 : (GR == 1 ? 1 : 3);
        constexpr int o1 = GR == 0 ? 2 : 4;
        double* cp = C + (yr * T::TZ + zr) * T::CP + kx * O * O + oz;
#pragma unroll
        for (int o = 0; o < O; ++o) cp[o0 * T::CC + o * O] = c0[o];
        if constexpr (GR != 1) {
#pragma unroll
            for (int o = 0; o < O; ++o) cp[o1 * T::CC + o * O] = c1[o];
        }
    }
}

// ---- stage y for the rounds schedule: round R adds the terms of output
// group GR whose stage-z products are pass R's (D slot j = product 3R + j);
// the accumulators c0, c1 stay in the thread's registers from round 0 (which
// clears them) to round 2 (which writes C)
//   round 0 (D0 D1 D2):  CM += nn D0, Cdd += nn D1, Cnn += dd D2
//   round 1 (D3 D4 D5):  Cnn += nn D3, Cdn += nd D4 + nn D5, Cnd += dn D4
//   round 2 (D6 D7 D8):  Cnn += dn D7 + nd D8, Cnd += nn D6
template <class T, int GR, int R>
__device__ __forceinline__ void gy_round(const GeoCtx& g, int yr, int item, const double* D, double* C,
                                         double (&c0)[T::O], double (&c1)[T::O])
{
    constexpr int P = T::P, Q = T::Q, O = T::O, Q2 = T::Q2;
    const TileCtx& c = g.c;
    const int iy = c.iy0 + yr;
    if (iy >= c.Ny) return;   // wave-uniform
    const bool act = item < T::NYI;
    const int it = act ? item : T::NYI - 1;
    const int zr = it / (O * Q), oz = (it / Q) % O, kx = it % Q;
    if constexpr (R == 0) {
#pragma unroll
        for (int o = 0; o < O; ++o) c0[o] = c1[o] = 0.0;
    }
    constexpr bool any = GR == 0 ? R == 0 : (GR == 1 ? true : R >= 1);
    if constexpr (any) {
#pragma unroll
        for (int e = 0; e <= P; ++e) {
            const int ey = iy - P + e;
            if (ey < 0 || ey >= c.Ky) continue;   // wave-uniform
            const ctab tb = g.Wy + (int64_t)tab_elem(ey, c.ry0, c.ry1) * T::TBE;
            const ctab wN = tb + (P - e) * Q, wD = tb + Q2 + (P - e) * Q;
            const ctab Nb = tb + 2 * Q2, Db = tb + 3 * Q2;
            const double* dp = D + zr * T::DZR + oz * T::DOZ + (yr + e) * Q2 + kx;
            // fa (trial N), fb (trial N') fold into c0; fc (trial N) into c1
            double fa[Q], fb[Q], fc[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const double d0 = dp[0 * T::DD + k * Q], d1 = dp[1 * T::DD + k * Q], d2 = dp[2 * T::DD + k * Q];
                if constexpr (GR == 0) {        // R == 0: CM += nn D0, Cdd += nn D1
                    fa[k] = wN[k] * d0;
                    fb[k] = 0.0;
                    fc[k] = wN[k] * d1;
                } else if constexpr (GR == 1) {
                    if constexpr (R == 0) {     // Cnn += dd D2
                        fa[k] = 0.0;
                        fb[k] = wD[k] * d2;
                    } else if constexpr (R == 1) {   // Cnn += nn D3
                        fa[k] = wN[k] * d0;
                        fb[k] = 0.0;
                    } else {                    // Cnn += dn D7 + nd D8
                        fa[k] = wD[k] * d1;
                        fb[k] = wN[k] * d2;
                    }
                    fc[k] = 0.0;
                } else {
                    if constexpr (R == 1) {     // Cdn += nd D4 + nn D5, Cnd += dn D4
                        fa[k] = wN[k] * d2;
                        fb[k] = wN[k] * d1;
                        fc[k] = wD[k] * d1;
                    } else {                    // Cnd += nn D6
                        fa[k] = 0.0;
                        fb[k] = 0.0;
                        fc[k] = wN[k] * d0;
                    }
                }
            }
            constexpr bool ua = !(GR == 1 && R == 0) && !(GR == 2 && R == 2);
            constexpr bool ub = (GR == 1 && R != 1) || (GR == 2 && R == 1);
            constexpr bool uc = GR == 0 || GR == 2;
#pragma unroll
            for (int bb = 0; bb <= P; ++bb)
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    if constexpr (ua) c0[e + bb] += Nb[bb * Q + k] * fa[k];
                    if constexpr (ub) c0[e + bb] += Db[bb * Q + k] * fb[k];
                    if constexpr (uc) c1[e + bb] += Nb[bb * Q + k] * fc[k];
                }
        }
    }
    if constexpr (R == 2 || T::ROUNDS == 1) {
        if (act) {
            constexpr int o0 = GR == 0 ? 0 : (GR == 1 ? 1 : 3);
            constexpr int o1 = GR == 0 ? 2 : 4;
            double* cp = C + (yr * T::TZ + zr) * T::CP + kx * O * O + oz;
#pragma unroll
            for (int o = 0; o < O; ++o) cp[o0 * T::CC + o * O] = c0[o];
            if constexpr (GR != 1) {
#pragma unroll
                for (int o = 0; o < O; ++o) cp[o1 * T::CC + o * O] = c1[o];
            }
        }
    }
}

// ---- stage x: element r (phase PH = r mod (p+1)) into the slots of group GG,
// then row r (slot PH) staged if emitted, and its slot cleared
template <class T, int GG, int PH>
__device__ __forceinline__ void gx_step(const GeoCtx& g, const XThread<T>& xt, double (&am)[T::NSL][T::O],
                                        double (&ak)[T::NSL][T::O], const double* C, int r, bool elem,
                                        bool emit, double* STG)
{
    constexpr int P = T::P, Q = T::Q, O = T::O, Q2 = T::Q2, G = T::G;
    if (elem) {
        const ctab tb = g.Wx + (int64_t)tab_elem(r, g.c.rx0, g.c.rx1) * T::TBE;
        double cM[Q], cN[Q], cD[Q], cDN[Q], cND[Q];
        const double* cp = C + xt.pen * T::CP + xt.oy * O + xt.oz;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            cM[k] = cp[0 * T::CC + k * O * O];
            cN[k] = cp[1 * T::CC + k * O * O];
            cD[k] = cp[2 * T::CC + k * O * O];
            cDN[k] = cp[3 * T::CC + k * O * O];
            cND[k] = cp[4 * T::CC + k * O * O];
        }
#pragma unroll
        for (int j = 0; j < T::NSL; ++j) {
            const int s = GG + j * G;   // compile-time after unrolling
            if (s > P) continue;
            const int a = (s - PH + (P + 1)) % (P + 1);   // test index of row r + a in element r
            const ctab wN = tb + a * Q, wD = tb + Q2 + a * Q;
            double m[Q], u[Q], v[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                m[k] = wN[k] * cM[k];
                u[k] = wN[k] * cN[k] + wD[k] * cDN[k];
                v[k] = wD[k] * cD[k] + wN[k] * cND[k];
            }
#pragma unroll
            for (int b = 0; b <= P; ++b) {
                const int ox = b - a + P;
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    am[j][ox] += tb[2 * Q2 + b * Q + k] * m[k];
                    ak[j][ox] += tb[2 * Q2 + b * Q + k] * u[k];
                    ak[j][ox] += tb[3 * Q2 + b * Q + k] * v[k];
                }
            }
        }
    }
    if constexpr (PH % G == GG) {
        constexpr int j = PH / G;
        if (emit) {
            const TileCtx& c = g.c;
            const int Lx = band_len(r, P, c.Nx);
            const int sub = xt.sub * Lx + (r - P - band_lo(r, P));
            double* st = STG + xt.pen * 2 * T::SROW;
#pragma unroll
            for (int ox = 0; ox < O; ++ox) {
                const int jx = r + ox - P;
                const int pos = xt.row && jx >= 0 && jx < c.Nx ? sub + ox : T::SROW - 1;
                st[pos] = am[j][ox];
                st[T::SROW + pos] = ak[j][ox];
            }
        }
#pragma unroll
        for (int ox = 0; ox < O; ++ox) am[j][ox] = ak[j][ox] = 0.0;
    }
}

// the x wavefronts of slot group GG over rows r = xs-1 .. X1-1 (iteration
// t = r + 1 of the z/y wavefronts), two barriers per row
template <class T, int GG>
__device__ __forceinline__ void gx_loop(const GeoCtx& g, int xi, int ts, int xs, int xe, int X0, int X1,
                                        const double* C, double* STG)
{
    constexpr int P = T::P, O = T::O;
    const XThread<T> xt(g.c, xi);
    int64_t pbase;
    int plen;
    pencil_rows<T>(g.c, ts % 64, pbase, plen);
    double am[T::NSL][O], ak[T::NSL][O];
#pragma unroll
    for (int j = 0; j < T::NSL; ++j)
#pragma unroll
        for (int o = 0; o < O; ++o) am[j][o] = ak[j][o] = 0.0;
    // first r rounded down to a multiple of p+1 (r >= -1)
    const int rf = xs - 1, r00 = rf < 0 ? -(P + 1) : rf - rf % (P + 1);
    auto row = [&](auto ph, int r) {
        constexpr int PH = decltype(ph)::value;
        if (r < rf || r > X1 - 1) return;   // uniform
        const bool live = r >= xs;
        if (live) gx_step<T, GG, PH>(g, xt, am, ak, C, r, r < xe, r >= X0, STG);
        __syncthreads();
        if (live && r >= X0) store_row<T>(g.c, STG, r, ts, pbase, plen);
        __syncthreads();
#pragma unroll
        for (int k = 1; k < T::ROUNDS; ++k) {   // the z/y wavefronts' later rounds
            __syncthreads();
            __syncthreads();
        }
    };
    for (int r0 = r00; r0 <= X1 - 1; r0 += P + 1) {
        row(std::integral_constant<int, 0>{}, r0);
        if constexpr (P >= 1) row(std::integral_constant<int, 1>{}, r0 + 1);
        if constexpr (P >= 2) row(std::integral_constant<int, 2>{}, r0 + 2);
        if constexpr (P >= 3) row(std::integral_constant<int, 3>{}, r0 + 3);
        if constexpr (P >= 4) row(std::integral_constant<int, 4>{}, r0 + 4);
        if constexpr (P >= 5) row(std::integral_constant<int, 5>{}, r0 + 5);
    }
}

// the z/y wavefronts over iterations t = xs .. X1: stage z and stage y of
// element t (t < xe), the row t-1 stored by the wavefronts without y units.
// PASS 0..2: the wavefront's one stage-z unit (prefetched fields), 3: none,
// -1: its units taken one by one without prefetch.
template <class T, int PASS>
__device__ __forceinline__ void gzy_loop(const GeoCtx& g, int w, int lane, int xs, int xe, int X0, int X1,
                                         double* D, double* C, double* STG)
{
    const TileCtx& c = g.c;
    int64_t pbase = 0;
    int plen = 0;
    if (w >= T::HW0) pencil_rows<T>(c, lane, pbase, plen);
    const int ts = 64 * (T::WX + w - T::HW0) + lane;
    constexpr int PP = PASS >= 0 && PASS < 3 ? PASS : 0;
    const int item = (w % T::WZP) * 64 + lane;
    double pf[3][T::NLZ][T::Q];
    if constexpr (PASS >= 0 && PASS < 3) {
        if (xs < xe) gz_load<T, PP>(g, item, xs, pf);
    }
    for (int t = xs; t <= X1; ++t) {
        const bool el = t < xe;
        if (el) {
            if constexpr (PASS >= 0 && PASS < 3) {
                gz_unit<T, PP>(g, item, pf, D);
                if (t + 1 < xe) gz_load<T, PP>(g, item, t + 1, pf);
            } else if constexpr (PASS < 0) {
                for (int u = w; u < T::NZU; u += T::NWZY) gz_unit_direct<T>(g, u, lane, t, D);
            }
        }
        __syncthreads();
        if (el) {
            for (int u = w; u < T::NYU; u += T::NWZY) {
                const int yr = u / (3 * T::WYP), gr = (u / T::WYP) % 3;
                const int yi = (u % T::WYP) * 64 + lane;
                if (gr == 0) gy_unit<T, 0>(g, yr, yi, D, C);
                else if (gr == 1) gy_unit<T, 1>(g, yr, yi, D, C);
                else gy_unit<T, 2>(g, yr, yi, D, C);
            }
        }
        if (w >= T::HW0 && t - 1 >= X0) store_row<T>(c, STG, t - 1, ts, pbase, plen);
        __syncthreads();
    }
}

// the z/y wavefronts under the rounds schedule: per iteration t, three
// rounds of (stage z of pass R | barrier | stage y, round R | barrier); the
// wavefront's stage-y units (at most two) keep their accumulators across the
// rounds; the row t-1 is stored in round 0 by the wavefronts without y units
template <class T>
__device__ __forceinline__ void gzy_loop_rounds(const GeoCtx& g, int w, int lane, int xs, int xe, int X0, int X1,
                                                double* D, double* C, double* STG)
{
    constexpr int O = T::O;
    const TileCtx& c = g.c;
    int64_t pbase = 0;
    int plen = 0;
    if (w >= T::HW0) pencil_rows<T>(c, lane, pbase, plen);
    const int ts = 64 * (T::WX + w - T::HW0) + lane;
    const int zitem = (w % T::WZP) * 64 + lane;
    double a0[2][O], a1[2][O];
    auto yround = [&](auto rr) {
        constexpr int R = decltype(rr)::value;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int u = w + k * T::NWZY;
            if (u >= T::NYU) break;   // wave-uniform
            const int yr = u / (3 * T::WYP), gr = (u / T::WYP) % 3;
            const int yi = (u % T::WYP) * 64 + lane;
            if (gr == 0) gy_round<T, 0, R>(g, yr, yi, D, C, a0[k], a1[k]);
            else if (gr == 1) gy_round<T, 1, R>(g, yr, yi, D, C, a0[k], a1[k]);
            else gy_round<T, 2, R>(g, yr, yi, D, C, a0[k], a1[k]);
        }
    };
    auto round = [&](auto rr, int t, bool el) {
        constexpr int R = decltype(rr)::value;
        if (el && w < T::NZU) gz_stream<T, R>(g, zitem, t, D);
        __syncthreads();
        if (el) yround(rr);
        if (R == 0 && w >= T::HW0 && t - 1 >= X0) store_row<T>(c, STG, t - 1, ts, pbase, plen);
        __syncthreads();
    };
    for (int t = xs; t <= X1; ++t) {
        const bool el = t < xe;
        round(std::integral_constant<int, 0>{}, t, el);
        round(std::integral_constant<int, 1>{}, t, el);
        round(std::integral_constant<int, 2>{}, t, el);
    }
}

// the x loop of slot group gg (wave-uniform), instantiated per group
template <class T, int GG>
__device__ __forceinline__ void gx_group(int gg, const GeoCtx& g, int xi, int ts, int xs, int xe, int X0, int X1,
                                         const double* C, double* STG)
{
    if constexpr (GG < T::G) {
        if (gg == GG) gx_loop<T, GG>(g, xi, ts, xs, xe, X0, X1, C, STG);
        else gx_group<T, GG + 1>(gg, g, xi, ts, xs, xe, X0, X1, C, STG);
    }
}

template <class T>
__device__ __forceinline__ void geo_tile_run(const PatchDev& pd, const RowMap& rm, const double* __restrict__ cm,
                                             const double* __restrict__ G, double* __restrict__ Mv,
                                             double* __restrict__ Kv, int tile, int seg, int nty, int seglen,
                                             double* lds)
{
    constexpr int P = T::P;
    GeoCtx g;
    TileCtx& c = g.c;
    c.kappa = nullptr;
    c.Mv = Mv;
    c.Kv = Kv;
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
    g.cm = Mv ? cm : nullptr;
    g.G = Kv ? G : nullptr;
    g.Wx = as_ctab(pd.d[0].Wg);
    g.Wy = as_ctab(pd.d[1].Wg);
    g.Wz = as_ctab(pd.d[2].Wg);
    const int X0 = seg * seglen, X1 = min(c.Nx, X0 + seglen);   // rows emitted
    const int xs = max(0, X0 - P);                               // first element swept
    const int xe = min(c.Kx, X1);                                // elements swept: [xs, xe)

    double* const D = lds;
    double* const C = lds + T::OFF_C;
    double* const STG = lds + T::OFF_S;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;

    if (w < T::NWZY) {
        if constexpr (T::ROUNDS == 3) {
            gzy_loop_rounds<T>(g, w, lane, xs, xe, X0, X1, D, C, STG);
        } else if constexpr (T::ZPF) {
            // one stage-z unit per wavefront: its pass is fixed, the next
            // element's fields are fetched while the current one is contracted
            const int pass = w < T::NZU ? w / T::WZP : 3;
            if (pass == 0) gzy_loop<T, 0>(g, w, lane, xs, xe, X0, X1, D, C, STG);
            else if (pass == 1) gzy_loop<T, 1>(g, w, lane, xs, xe, X0, X1, D, C, STG);
            else if (pass == 2) gzy_loop<T, 2>(g, w, lane, xs, xe, X0, X1, D, C, STG);
            else gzy_loop<T, 3>(g, w, lane, xs, xe, X0, X1, D, C, STG);
        } else {
            gzy_loop<T, -1>(g, w, lane, xs, xe, X0, X1, D, C, STG);
        }
    } else {
        const int wx = w - T::XW0;
        const int gg = wx / T::WXG, xi = (wx % T::WXG) * 64 + lane, ts = wx * 64 + lane;
        gx_group<T, 0>(gg, g, xi, ts, xs, xe, X0, X1, C, STG);
    }
}

template <class T>
__global__ __launch_bounds__(T::NT) __attribute__((amdgpu_waves_per_eu(T::WPE))) void k_rows_geo(
    PatchDev pd, RowMap rm, const double* __restrict__ cm, const double* __restrict__ G,
    double* __restrict__ Mv, double* __restrict__ Kv, int nty, int ntz, int nseg, int seglen, int nb8)
{
    __shared__ double lds[T::LDS];
    const int ntile = nty * ntz;
    const int b = xcd_tile(blockIdx.x, nb8);
    if (b >= ntile * nseg) return;   // whole workgroup
    geo_tile_run<T>(pd, rm, cm, G, Mv, Kv, b % ntile, b / ntile, nty, seglen, lds);
}

template <class T>
static int launch_rows_geo_t(const PatchDev& pd, const double* cm, const double* G, double* Mv, double* Kv,
                             hipStream_t st)
{
    RowMap rm = make_rowmap(pd);
    const int Nx = pd.d[0].N, Ny = pd.d[1].N, Nz = pd.d[2].N;
    const int nty = (Ny + T::TY - 1) / T::TY, ntz = (Nz + T::TZ - 1) / T::TZ;
    const int ntile = nty * ntz;
    const int slots = device_slots((const void*)k_rows_geo<T>, T::NT);
    if (!slots) return -3;
    // x segments as for the identity geometry: the items spread over the
    // slots plus one item as the tail, a segment paying ~4p/3 element steps
    // of warm-up and start-up
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
    hipLaunchKernelGGL(k_rows_geo<T>, dim3(nb8 * 8), dim3(T::NT), 0, st, pd, rm, cm, G, Mv, Kv, nty, ntz, nseg,
                       seglen, nb8);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_rows_geo(const PatchDev& pd, const double* cm, const double* G, double* Mv, double* Kv, hipStream_t st)
{
    if (!Mv && !Kv) return 0;
    switch (pd.p) {
    case 1: return launch_rows_geo_t<GeoCfg<1>::T>(pd, cm, G, Mv, Kv, st);
    case 2: return launch_rows_geo_t<GeoCfg<2>::T>(pd, cm, G, Mv, Kv, st);
    case 3: return launch_rows_geo_t<GeoCfg<3>::T>(pd, cm, G, Mv, Kv, st);
    case 4: return launch_rows_geo_t<GeoCfg<4>::T>(pd, cm, G, Mv, Kv, st);
    case 5: return launch_rows_geo_t<GeoCfg<5>::T>(pd, cm, G, Mv, Kv, st);
    default: return -4;
    }
}

}  // namespace igaf
