// One forward Euler step of the heat problem (Sec. 2.2, eq. Euler, in the
// matrix form of Sec. 2.4) with the coefficient kappa in both integrals:
//   M(kappa) mu_next = M(kappa) mu - dt K(kappa) mu.
// The right-hand side is one matrix-free operator apply; the mass system is
// solved by conjugate gradients (M is symmetric positive definite), each
// iteration one matrix-free mass apply.  Every vector operation runs in the
// kernels below; the CG scalars stay in device memory (alpha, beta computed
// on the device), and the host reads back only the residual norm for the
// convergence test.  Dot products are two-stage and in a fixed order, so the
// iteration is deterministic up to the atomics of the apply.
#include <cmath>

#include "common.h"
#include "launch.h"

namespace igaf {

namespace {

constexpr int kDotBlocks = 512;   // first-stage partial sums
constexpr int kDotThreads = 256;

// partial[b] = sum of a[i] * c[i] over the block-strided indices of block b
__global__ __launch_bounds__(kDotThreads) void k_dot_partial(const double* __restrict__ a,
                                                             const double* __restrict__ c,
                                                             int64_t n, double* __restrict__ partial)
{
    __shared__ double red[kDotThreads];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kDotThreads)
        s += a[i] * c[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kDotThreads / 2; h > 0; h /= 2) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// S[slot] = sum of the partials; then, by `mode`:
//   1: S[4] = S[0] / S[slot]           (alpha = r.r / p.Ap)
//   2: S[3] = S[slot] / S[0], S[0] = S[slot]   (beta, and the new r.r)
__global__ __launch_bounds__(kDotThreads) void k_dot_final(const double* __restrict__ partial,
                                                           int nb, double* __restrict__ S, int slot,
                                                           int mode)
{
    __shared__ double red[kDotThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kDotThreads) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kDotThreads / 2; h > 0; h /= 2) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = red[0];
        S[slot] = v;
        if (mode == 1) S[4] = v != 0.0 ? S[0] / v : 0.0;
        if (mode == 2) {
            S[3] = S[0] != 0.0 ? v / S[0] : 0.0;
            S[0] = v;
        }
    }
}

// x += alpha p, r -= alpha Ap (alpha = S[4])
__global__ __launch_bounds__(256) void k_cg_xr(double* __restrict__ x, double* __restrict__ r,
                                               const double* __restrict__ p,
                                               const double* __restrict__ Ap,
                                               const double* __restrict__ S, int64_t n)
{
    const double alpha = S[4];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        x[i] += alpha * p[i];
        r[i] -= alpha * Ap[i];
    }
}

// p = r + beta p (beta = S[3]); with first != 0: p = r
__global__ __launch_bounds__(256) void k_cg_p(double* __restrict__ p, const double* __restrict__ r,
                                              const double* __restrict__ S, int64_t n, int first)
{
    const double beta = first ? 0.0 : S[3];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = r[i] + beta * p[i];
}

// r = b - r (r holds M x on entry); x = mu
__global__ __launch_bounds__(256) void k_cg_init(double* __restrict__ r, const double* __restrict__ b,
                                                 double* __restrict__ x, const double* __restrict__ mu,
                                                 int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        r[i] = b[i] - r[i];
        x[i] = mu[i];
    }
}

int grid_for(int64_t n)
{
    const int64_t g = (n + 255) / 256;
    return (int)(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

int dot(const double* a, const double* c, int64_t n, double* partial, double* S, int slot, int mode,
        hipStream_t st)
{
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(kDotThreads), 0, st, a, c, n, partial);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kDotThreads), 0, st, partial, kDotBlocks, S, slot, mode);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace

int64_t euler_workspace_doubles(int64_t ndof) { return 4 * ndof + kDotBlocks + 8; }

// Workspace: b | r | p | Ap (ndof each) | dot partials | CG scalars S[8]:
// S[0] r.r, S[1] p.Ap, S[2] new r.r, S[3] beta, S[4] alpha.
// Returns 0 (converged), 1 (maxit reached) or -3 (launch failure).
int run_euler_step(const PatchDev& pd, int64_t ndof, const double* kappa, const double* mu, double dt,
                   double tol, int maxit, double* x, double* work, int* iters, double* relres,
                   hipStream_t st)
{
    double* b = work;
    double* r = b + ndof;
    double* p = r + ndof;
    double* Ap = p + ndof;
    double* partial = Ap + ndof;
    double* S = partial + kDotBlocks;
    const int gv = grid_for(ndof);
    auto mass_apply = [&](const double* v, double* out, double aK) {
        return launch_fill_zero(out, ndof, st) || launch_apply(pd, kappa, v, 1.0, aK, out, st) ? -3 : 0;
    };
    auto host_scalar = [&](int slot, double* out) {
        return hipMemcpyAsync(out, S + slot, sizeof(double), hipMemcpyDeviceToHost, st) == hipSuccess &&
                       hipStreamSynchronize(st) == hipSuccess
                   ? 0
                   : -3;
    };
    *iters = 0;
    *relres = 0.0;
    // right-hand side b = M mu - dt K mu; r = M mu (x starts at mu)
    if (mass_apply(mu, b, -dt) || mass_apply(mu, r, 0.0)) return -3;
    double bb = 0.0, rr = 0.0;
    if (dot(b, b, ndof, partial, S, 1, 0, st) || host_scalar(1, &bb)) return -3;
    hipLaunchKernelGGL(k_cg_init, dim3(gv), dim3(256), 0, st, r, b, x, mu, ndof);
    if (hipGetLastError() != hipSuccess) return -3;
    if (bb == 0.0) {   // zero right-hand side: the solution is zero
        return launch_fill_zero(x, ndof, st) ? -3 : 0;
    }
    if (dot(r, r, ndof, partial, S, 0, 0, st) || host_scalar(0, &rr)) return -3;
    *relres = std::sqrt(rr / bb);
    if (*relres <= tol) return 0;
    hipLaunchKernelGGL(k_cg_p, dim3(gv), dim3(256), 0, st, p, r, S, ndof, 1);
    for (int k = 1; k <= maxit; ++k) {
        if (mass_apply(p, Ap, 0.0)) return -3;
        if (dot(p, Ap, ndof, partial, S, 1, 1, st)) return -3;   // alpha
        hipLaunchKernelGGL(k_cg_xr, dim3(gv), dim3(256), 0, st, x, r, p, Ap, S, ndof);
        if (dot(r, r, ndof, partial, S, 2, 2, st)) return -3;    // beta, new r.r
        if (host_scalar(0, &rr)) return -3;
        *iters = k;
        *relres = std::sqrt(rr / bb);
        if (*relres <= tol) return 0;
        hipLaunchKernelGGL(k_cg_p, dim3(gv), dim3(256), 0, st, p, r, S, ndof, 0);
        if (hipGetLastError() != hipSuccess) return -3;
    }
    return 1;
}

}  // namespace igaf
