// Pieces shared by the owner-computed CSR rows kernels (identity and mapped
// geometry): the tile context, the row positions of a tile's pencils and the
// store of one staged CSR row per pencil as a contiguous segment.
//
// A tile owns the row pencils (iy, iz), iy in [iy0, iy0+TY), iz in
// [iz0, iz0+TZ) (pencil index pen = (iy - iy0) TZ + (iz - iz0)), for the rows
// ix of one x segment; o* in [0, 2p] are column offsets j = i + o - p, and a
// staged row holds the 2p+1 cubed values of one row at their CSR positions
// (columns outside the patch go to a junk slot at the end).
#pragma once

#include "common.h"

namespace igaf {

constexpr int cmax(int a, int b) { return a > b ? a : b; }
// smallest y >= x with y = r (mod 16): LDS strides that spread the lanes of a
// wavefront over the 64-bit banks
constexpr int pad16(int x, int r) { return x + (((r - x) % 16) + 16) % 16; }

__device__ inline int clampi_t(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// Number of structural entries in the rows before row i of one direction,
// sum_{i' < i} (min(N-1, i'+p) - max(0, i'-p) + 1), in closed form (the same
// prefix the plan tabulates): no memory round trip on the store path.
__device__ inline int64_t band_prefix(int i, int p, int N)
{
    auto tri = [](int64_t m) { return m > 0 ? m * (m + 1) / 2 : (int64_t)0; };
    const int64_t ii = i;
    return ii * (p + 1) + ii * (ii - 1) / 2 - tri(ii - 1 - p) - tri(ii + p - N);
}

// Per-workgroup constants of one tile.
struct TileCtx {
    const double* kappa;
    double* Mv;
    double* Kv;
    ctab Wnx, Wdx, Wny, Wdy, Wnz, Wdz;
    int64_t T0, T1;   // structural entries of one direction's 1D pattern
    int Kx, Ky, Kz, Nx, Ny, Nz;
    int iy0, iz0;
    int rx0, rx1, ry0, ry1, rz0, rz1;   // per direction: elements [r0, r1) read the tables of r0
};

__device__ inline void tile_runs(TileCtx& c, const PatchDev& pd)
{
    c.rx0 = pd.d[0].r0;
    c.rx1 = pd.d[0].r1;
    c.ry0 = pd.d[1].r0;
    c.ry1 = pd.d[1].r1;
    c.rz0 = pd.d[2].r0;
    c.rz1 = pd.d[2].r1;
}

// ---- stage x: thread xi = (stage-x wavefront)*64 + lane owns combo (pen, oy, oz)
template <class T>
struct XThread {
    int pen, oy, oz, sub;
    bool row;
    __device__ XThread(const TileCtx& c, int xi)
    {
        constexpr int P = T::P, O = T::O;
        const bool act = xi < T::NXI;
        const int it = act ? xi : T::NXI - 1;
        oz = it % O;
        oy = (it / O) % O;
        pen = it / (O * O);
        const int iy = c.iy0 + pen / T::TZ, iz = c.iz0 + pen % T::TZ;
        const int jy = iy + oy - P, jz = iz + oz - P;
        row = act && iy < c.Ny && iz < c.Nz && jy >= 0 && jy < c.Ny && jz >= 0 && jz < c.Nz;
        const int Ly = band_len(min(iy, c.Ny - 1), P, c.Ny);
        // row position of column (jx = band_lo(ix), jy, jz) without the Lx factor
        sub = row ? (jz - band_lo(iz, P)) * Ly + (jy - band_lo(iy, P)) : 0;
    }
};

// Row-start parts of pencil `lane` (lanes < NPEN): the row start without its
// x part, and Ly*Lz (0 for pencils outside the patch).
template <class T>
__device__ __forceinline__ void pencil_rows(const TileCtx& c, int lane, int64_t& pbase, int& plen)
{
    constexpr int P = T::P;
    pbase = 0;
    plen = 0;
    const int pl = lane < T::NPEN ? lane : 0;
    const int iy = c.iy0 + pl / T::TZ, iz = c.iz0 + pl % T::TZ;
    if (lane < T::NPEN && iy < c.Ny && iz < c.Nz) {
        const int Ly = band_len(iy, P, c.Ny), Lz = band_len(iz, P, c.Nz);
        plen = Ly * Lz;
        pbase = band_prefix(iz, P, c.Nz) * c.T1 * c.T0 + Lz * band_prefix(iy, P, c.Ny) * c.T0;
    }
}

// Each pencil's staged row ix as one contiguous segment, by the NTS storing
// threads (ts = 0..NTS-1).  The LDS reads of SGP pencils are issued before
// their stores: all pencils in the pipelined schedule (one wait per row),
// one at a time in the sequential one, whose registers hold the ring.  The
// stores are non-temporal: nothing in the kernel reads a CSR value back.
template <class T>
__device__ __forceinline__ void store_row(const TileCtx& c, const double* STG, int ix, int ts,
                                          int64_t pbase, int plen)
{
    constexpr int P = T::P, SIT = T::SIT, GP = T::SGP;
    const int Lx = band_len(ix, P, c.Nx);
    const int64_t px = band_prefix(ix, P, c.Nx);
#pragma unroll 1
    for (int p0 = 0; p0 < T::NPEN; p0 += GP) {
        double vm[GP][SIT], vk[GP][SIT];
#pragma unroll
        for (int g = 0; g < GP; ++g) {
            const double* st = STG + (p0 + g) * 2 * T::SROW;
#pragma unroll
            for (int j = 0; j < SIT; ++j) {
                const int i = min(ts + j * T::NTS, T::SROW - 1);
                vm[g][j] = st[i];
                vk[g][j] = st[T::SROW + i];
            }
        }
#pragma unroll
        for (int g = 0; g < GP; ++g) {
            const int pen = p0 + g;
            const int Lyz = __builtin_amdgcn_readlane(plen, pen);   // 0: pencil outside the patch
            const int L = Lx * Lyz;
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)pbase, pen);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(pbase >> 32), pen);
            const int64_t rs = (int64_t)(((uint64_t)hi << 32) | lo) + (int64_t)Lyz * px;
#pragma unroll
            for (int j = 0; j < SIT; ++j) {
                const int i = ts + j * T::NTS;
                if (i < L) {
                    if (c.Mv) __builtin_nontemporal_store(vm[g][j], c.Mv + rs + i);
                    if (c.Kv) __builtin_nontemporal_store(vk[g][j], c.Kv + rs + i);
                }
            }
        }
    }
}

// Logical workgroup index with XCD-aware order: the hardware hands workgroup
// b to XCD b % 8, so XCD x receives the contiguous logical range
// [x*nb8, (x+1)*nb8): neighbouring tiles (which share kappa) share one L2.
__device__ inline int xcd_tile(int b, int nb8) { return (b % 8) * nb8 + b / 8; }

}  // namespace igaf
