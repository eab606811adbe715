// Assembly of the global CSR values from stored element matrices (Sec. 3.1:
// the global matrix is the sum of the element matrices, each added at the
// positions of its functions), and a fill kernel for outputs that are
// accumulated into.
#include <map>
#include <mutex>
#include <utility>

#include "common.h"
#include "launch.h"

namespace igaf {

// ---------------------------------------------------------------------------
// Assembly from stored element matrices (A = sum over elements of A^gamma):
// one wavefront per CSR row I (several rows per wavefront for p <= 2).  For
// every element carrying I, in element order, the wavefront reads that
// element's matrix row I (n^3 contiguous values, lane = local trial index J)
// and adds each value into the row, held in LDS at the offsets of the
// structural pattern; the row is then written out contiguously.  Each stored
// value is read once, in coalesced runs.  Two elements can send values to the
// same column through different lanes, so the LDS adds are atomic; all adds
// of a row come from one wavefront, whose LDS operations execute in issue
// order, so every value is summed in element order.
template <int P>
__global__ __launch_bounds__(256) void k_gather(PatchDev pd, RowMap rm, const double* __restrict__ Me,
                                                const double* __restrict__ Ke, double* __restrict__ Mv,
                                                double* __restrict__ Kv)
{
    constexpr int n = P + 1, n3 = n * n * n, O = 2 * P + 1, O3 = O * O * O;
    constexpr int LPR = n3 < 64 ? n3 : 64;                   // lanes per row
    constexpr int RW = 64 / LPR;                             // rows per wavefront
    constexpr int NC = (n3 + LPR - 1) / LPR;                 // chunks of a matrix row
    constexpr int RB = 4 * RW;                               // rows per workgroup
    __shared__ double acc[2][RB][O3];
    const int tid = threadIdx.x, lane = tid % 64;
    const int rw = (tid / 64) * RW + lane / LPR, jl = lane % LPR;
    for (int i = tid; i < 2 * RB * O3; i += 256) (&acc[0][0][0])[i] = 0.0;
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * RB + rw;
    if (lane / LPR >= RW || g >= pd.ndof) return;
    const int Nx = pd.d[0].N, Ny = pd.d[1].N, Nz = pd.d[2].N;
    const int Kx = pd.d[0].K, Ky = pd.d[1].K, Kz = pd.d[2].K;
    const int ix = (int)(g % Nx), iy = (int)((g / Nx) % Ny), iz = (int)(g / ((int64_t)Nx * Ny));
    const int lox = band_lo(ix, P), loy = band_lo(iy, P), loz = band_lo(iz, P);
    const int Lx = band_len(ix, P, Nx), Ly = band_len(iy, P, Ny);
    const int elx = ix - P > 0 ? ix - P : 0, ehx = ix < Kx - 1 ? ix : Kx - 1;
    const int ely = iy - P > 0 ? iy - P : 0, ehy = iy < Ky - 1 ? iy : Ky - 1;
    const int elz = iz - P > 0 ? iz - P : 0, ehz = iz < Kz - 1 ? iz : Kz - 1;
    for (int ez = elz; ez <= ehz; ++ez)
        for (int ey = ely; ey <= ehy; ++ey)
            for (int ex = elx; ex <= ehx; ++ex) {
                const int64_t e = ex + (int64_t)Kx * (ey + (int64_t)Ky * ez);
                const int I = (ix - ex) + n * ((iy - ey) + n * (iz - ez));
                const int64_t row = e * (int64_t)n3 * n3 + (int64_t)I * n3;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const int J = c * LPR + jl;
                    if (J < n3) {
                        const int b1 = J % n, b2 = (J / n) % n, b3 = J / (n * n);
                        const int off = ((ez + b3 - loz) * Ly + (ey + b2 - loy)) * Lx + (ex + b1 - lox);
                        if (Mv) atomicAdd(&acc[0][rw][off], Me[row + J]);
                        if (Kv) atomicAdd(&acc[1][rw][off], Ke[row + J]);
                    }
                }
            }
    const int len = Lx * Ly * band_len(iz, P, Nz);
    const int64_t rs = rm.row_start(ix, iy, iz);
    for (int c = jl; c < len; c += LPR) {
        if (Mv) Mv[rs + c] = acc[0][rw][c];
        if (Kv) Kv[rs + c] = acc[1][rw][c];
    }
}

int launch_gather(const PatchDev& pd, const double* Me, const double* Ke, double* Mv, double* Kv,
                  hipStream_t st)
{
    RowMap rm = make_rowmap(pd);
    if (pd.ndof <= 0) return 0;
    switch (pd.p) {
#define IGAF_G(PP)                                                                                  \
    case PP: {                                                                                      \
        constexpr int n3 = (PP + 1) * (PP + 1) * (PP + 1), RB = 4 * (64 / (n3 < 64 ? n3 : 64));    \
        const int64_t blocks = (pd.ndof + RB - 1) / RB;                                             \
        hipLaunchKernelGGL(k_gather<PP>, dim3((unsigned)blocks), dim3(256), 0, st, pd, rm, Me, Ke, Mv, \
                           Kv);                                                                     \
        break;                                                                                      \
    }
        IGAF_G(1)
        IGAF_G(2)
        IGAF_G(3)
        IGAF_G(4)
        IGAF_G(5)
#undef IGAF_G
    default:
        return -4;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

__global__ void k_fill_zero(double* __restrict__ a, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = 0.0;
}

int launch_fill_zero(double* a, int64_t n, hipStream_t st)
{
    if (!a || n <= 0) return 0;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, a, n);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int device_slots(const void* kernel, int threads)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find({dev, kernel});
        if (it != cache.end()) return it->second;
    }
    int ncu = 0, per = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess)
        return 0;
    const int slots = ncu * (per > 0 ? per : 1);
    std::lock_guard<std::mutex> lock(mu);
    cache[{dev, kernel}] = slots;
    return slots;
}

}  // namespace igaf
