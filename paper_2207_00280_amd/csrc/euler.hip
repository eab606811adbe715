// One forward Euler step of the heat problem (Sec. 2.2, eq. Euler, in the
// matrix form of Sec. 2.4) with the coefficient kappa in both integrals:
//   M(kappa) mu_next = M(kappa) mu - dt K(kappa) mu.
// The right-hand side is one matrix-free operator apply; the mass system is
// solved by conjugate gradients (M is symmetric positive definite), each
// iteration one matrix-free mass apply, optionally preconditioned by the
// Kronecker product of the 1D mass matrices (kappa = 1), scaled on both
// sides so that its diagonal matches diag(M(kappa)): the product carries the
// B-spline basis (whose mass matrix conditioning grows quickly with p), the
// diagonal scaling the coefficient's variation, and it is applied by three
// sweeps of banded triangular solves along the grid lines.  Every vector operation runs in the
// kernels below; the CG scalars stay in device memory (alpha, beta computed
// on the device), and the host reads back only the residual norm for the
// convergence test.  Dot products are two-stage and in a fixed order and the
// apply sums every DOF in a fixed order, so the iteration is deterministic:
// repeated steps give the same bits.
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

// x += alpha p, r -= alpha Ap (alpha = S[4]), and the first stage of r.r:
// the grid and the order of k_dot_partial, so the partials are the same
__global__ __launch_bounds__(kDotThreads) void k_cg_xr_rr(double* __restrict__ x, double* __restrict__ r,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ Ap,
                                                          const double* __restrict__ S, int64_t n,
                                                          double* __restrict__ partial)
{
    __shared__ double red[kDotThreads];
    const double alpha = S[4];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kDotThreads) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * Ap[i];
        r[i] = ri;
        s += ri * ri;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kDotThreads / 2; h > 0; h /= 2) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// p = z + beta p (beta = S[3]); with first != 0: p = z
__global__ __launch_bounds__(256) void k_cg_p(double* __restrict__ p, const double* __restrict__ z,
                                              const double* __restrict__ S, int64_t n, int first)
{
    const double beta = first ? 0.0 : S[3];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = z[i] + beta * (first ? 0.0 : p[i]);
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

// s[I] <- sqrt(diag(Mz (x) My (x) Mx)_I / s[I]) (s holds diag(M(kappa)) on entry)
__global__ __launch_bounds__(256) void k_precond_scale(double* __restrict__ s, const double* __restrict__ Lx,
                                                       const double* __restrict__ Ly,
                                                       const double* __restrict__ Lz, int Nx, int Ny,
                                                       int W, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int ix = (int)(i % Nx), iy = (int)((i / Nx) % Ny), iz = (int)(i / ((int64_t)Nx * Ny));
        const double d0 = Lx[(int64_t)ix * W + W - 1] * Ly[(int64_t)iy * W + W - 1] * Lz[(int64_t)iz * W + W - 1];
        s[i] = sqrt(d0 / s[i]);
    }
}

// z = s * r (elementwise); with r == nullptr, z *= s
__global__ __launch_bounds__(256) void k_scale(double* __restrict__ z, const double* __restrict__ r,
                                               const double* __restrict__ s, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        z[i] = s[i] * (r ? r[i] : z[i]);
}

// In place v <- (L L^T)^-1 v along every grid line of one direction: a thread
// per line, forward then backward substitution over the line's N values with
// the banded factor (p sub-diagonals) kept as [1/L_ii, L_{i,i-1..i-p}, M_ii].
// Line t starts at (t % inner) + (t / inner) inner N and steps by `inner`
// (inner = 1, Nx, Nx Ny for x, y, z).  The substitution is serial along the
// line, so the line's values are read kLineChunk at a time, one chunk ahead of the
// arithmetic: each load then overlaps a chunk of steps instead of one.
constexpr int kLineChunk = 8;

template <int P>
__global__ __launch_bounds__(64) void k_line_solve(double* __restrict__ v, const double* __restrict__ Lm,
                                                   int N, int64_t nlines, int64_t inner)
{
    constexpr int W = P + 2, LSD = kLineChunk;
    const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (t >= nlines) return;
    double* line = v + (t % inner) + (t / inner) * inner * N;
    const int nch = (N + LSD - 1) / LSD;
    double cur[LSD], nxt[LSD];
    double ring[P];   // forward: y_{i-1-j}; backward: x_{i+1+j}
    // forward substitution, chunks in increasing i
#pragma unroll
    for (int j = 0; j < LSD; ++j) cur[j] = j < N ? line[(int64_t)j * inner] : 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) ring[j] = 0.0;
    for (int c = 0; c < nch; ++c) {
        const int i0 = c * LSD;
#pragma unroll
        for (int j = 0; j < LSD; ++j) {
            const int i = i0 + LSD + j;
            nxt[j] = i < N ? line[(int64_t)i * inner] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < LSD; ++j) {
            const int i = i0 + j;
            if (i < N) {
                const double* l = Lm + (int64_t)i * W;
                double s = cur[j];
#pragma unroll
                for (int k = 1; k <= P; ++k) s -= l[k] * ring[k - 1];
                s *= l[0];
#pragma unroll
                for (int q = P - 1; q > 0; --q) ring[q] = ring[q - 1];
                ring[0] = s;
                line[(int64_t)i * inner] = s;
            }
        }
#pragma unroll
        for (int j = 0; j < LSD; ++j) cur[j] = nxt[j];
    }
    // backward substitution, chunks in decreasing i; chunk c holds
    // i = N-1-c LSD-j, j = 0..LSD-1
#pragma unroll
    for (int j = 0; j < LSD; ++j) cur[j] = N - 1 - j >= 0 ? line[(int64_t)(N - 1 - j) * inner] : 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) ring[j] = 0.0;
    for (int c = 0; c < nch; ++c) {
        const int i0 = N - 1 - c * LSD;
#pragma unroll
        for (int j = 0; j < LSD; ++j) {
            const int i = i0 - LSD - j;
            nxt[j] = i >= 0 ? line[(int64_t)i * inner] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < LSD; ++j) {
            const int i = i0 - j;
            if (i >= 0) {
                double s = cur[j];
#pragma unroll
                for (int k = 1; k <= P; ++k) {
                    const int r = i + k < N ? i + k : N - 1;   // past the end the ring holds 0
                    s -= Lm[(int64_t)r * W + k] * ring[k - 1];
                }
                s *= Lm[(int64_t)i * W];
#pragma unroll
                for (int q = P - 1; q > 0; --q) ring[q] = ring[q - 1];
                ring[0] = s;
                line[(int64_t)i * inner] = s;
            }
        }
#pragma unroll
        for (int j = 0; j < LSD; ++j) cur[j] = nxt[j];
    }
}

template <int P>
int launch_line_solves_t(const PatchDev& pd, double* v, int64_t ndof, hipStream_t st)
{
    int64_t inner = 1;
    for (int a = 0; a < 3; ++a) {
        const int N = pd.d[a].N;
        const int64_t nlines = ndof / N;
        hipLaunchKernelGGL(k_line_solve<P>, dim3((unsigned)((nlines + 63) / 64)), dim3(64), 0, st, v,
                           pd.d[a].Lm, N, nlines, inner);
        inner *= N;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_line_solves(const PatchDev& pd, double* v, int64_t ndof, hipStream_t st)
{
    switch (pd.p) {
    case 1: return launch_line_solves_t<1>(pd, v, ndof, st);
    case 2: return launch_line_solves_t<2>(pd, v, ndof, st);
    case 3: return launch_line_solves_t<3>(pd, v, ndof, st);
    case 4: return launch_line_solves_t<4>(pd, v, ndof, st);
    case 5: return launch_line_solves_t<5>(pd, v, ndof, st);
    default: return -4;
    }
}

}  // namespace

int64_t euler_workspace_doubles(const PatchDev& pd, int64_t ndof)
{
    return 6 * ndof + kDotBlocks + 8 + apply_workspace_doubles(pd);
}

// Workspace: b | r | p | Ap | z | s (ndof each) | dot partials | CG scalars S[8]
// | the operator apply's run slots:
// S[0] r.z, S[1] p.Ap, S[2] new r.z, S[3] beta, S[4] alpha, S[5] r.r.
// Without a preconditioner z is r itself.  Returns 0 (converged), 1 (maxit
// reached) or -3 (launch failure).
// With G (a mapped geometry) `kappa` is the mass coefficient cm and G the
// stiffness tensor: only the right-hand side sees G, the mass system and its
// preconditioner take cm where the identity geometry takes kappa.
int run_euler_step(const PatchDev& pd, int64_t ndof, const double* kappa, const double* mu, double dt,
                   double tol, int maxit, int precond, double* x, double* work, int* iters, double* relres,
                   hipStream_t st, double* rb, hipEvent_t ev, const double* G)
{
    double* b = work;
    double* r = b + ndof;
    double* p = r + ndof;
    double* Ap = p + ndof;
    double* z = precond ? Ap + ndof : r;
    double* sc = Ap + 2 * ndof;
    double* partial = Ap + 3 * ndof;
    double* S = partial + kDotBlocks;
    double* Wap = S + 8;
    const int gv = grid_for(ndof);
    auto mass_apply = [&](const double* v, double* out) {
        return launch_apply(pd, kappa, v, 1.0, 0.0, out, Wap, st) ? -3 : 0;
    };
    auto host_scalar = [&](int slot, double* out) {
        return hipMemcpyAsync(out, S + slot, sizeof(double), hipMemcpyDeviceToHost, st) == hipSuccess &&
                       hipStreamSynchronize(st) == hipSuccess
                   ? 0
                   : -3;
    };
    // z = P^-1 r = S^-1 (Mz (x) My (x) Mx)^-1 S^-1 r, with sc = S^-1
    auto apply_precond = [&]() {
        if (!precond) return 0;
        hipLaunchKernelGGL(k_scale, dim3(gv), dim3(256), 0, st, z, r, sc, ndof);
        if (launch_line_solves(pd, z, ndof, st)) return -3;
        hipLaunchKernelGGL(k_scale, dim3(gv), dim3(256), 0, st, z, nullptr, sc, ndof);
        return hipGetLastError() == hipSuccess ? 0 : -3;
    };
    *iters = 0;
    *relres = 0.0;
    if (precond) {
        if (launch_apply(pd, kappa, nullptr, 1.0, 0.0, sc, Wap, st, nullptr, true)) return -3;   // diag(M)
        const int W = pd.p + 2;
        hipLaunchKernelGGL(k_precond_scale, dim3(gv), dim3(256), 0, st, sc, pd.d[0].Lm, pd.d[1].Lm,
                           pd.d[2].Lm, pd.d[0].N, pd.d[1].N, W, ndof);
    }
    // right-hand side b = M mu - dt K mu; r = M mu (x starts at mu)
    if (launch_apply(pd, kappa, mu, 1.0, -dt, b, Wap, st, G) || mass_apply(mu, r)) return -3;
    double bb = 0.0, rr = 0.0;
    if (dot(b, b, ndof, partial, S, 1, 0, st) || host_scalar(1, &bb)) return -3;
    hipLaunchKernelGGL(k_cg_init, dim3(gv), dim3(256), 0, st, r, b, x, mu, ndof);
    if (hipGetLastError() != hipSuccess) return -3;
    if (bb == 0.0) {   // zero right-hand side: the solution is zero
        return launch_fill_zero(x, ndof, st) ? -3 : 0;
    }
    if (dot(r, r, ndof, partial, S, 5, 0, st) || host_scalar(5, &rr)) return -3;
    *relres = std::sqrt(rr / bb);
    if (*relres <= tol) return 0;
    if (apply_precond() || dot(r, z, ndof, partial, S, 0, 0, st)) return -3;
    hipLaunchKernelGGL(k_cg_p, dim3(gv), dim3(256), 0, st, p, z, S, ndof, 1);
    if (mass_apply(p, Ap)) return -3;
    if (dot(p, Ap, ndof, partial, S, 1, 1, st)) return -3;       // alpha
    // Each iteration's r.r is read back through a pinned slot while the GPU
    // already runs the next iteration's work up to its update of x and r
    // (preconditioner, r.z, search direction, M p, p.Ap): the same kernels
    // in the same order, with the host's stopping test off the GPU's path.
    // After the last iteration that work is left unused.
    for (int k = 1; k <= maxit; ++k) {
        hipLaunchKernelGGL(k_cg_xr_rr, dim3(kDotBlocks), dim3(kDotThreads), 0, st, x, r, p, Ap, S, ndof,
                           partial);
        hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kDotThreads), 0, st, partial, kDotBlocks, S, 5, 0);
        if (hipGetLastError() != hipSuccess) return -3;
        if (hipMemcpyAsync(rb, S + 5, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipEventRecord(ev, st) != hipSuccess)
            return -3;
        if (k < maxit) {
            if (apply_precond()) return -3;
            if (dot(r, z, ndof, partial, S, 2, 2, st)) return -3;    // beta, new r.z
            hipLaunchKernelGGL(k_cg_p, dim3(gv), dim3(256), 0, st, p, z, S, ndof, 0);
            if (hipGetLastError() != hipSuccess) return -3;
            if (mass_apply(p, Ap)) return -3;
            if (dot(p, Ap, ndof, partial, S, 1, 1, st)) return -3;   // alpha
        }
        if (hipEventSynchronize(ev) != hipSuccess) return -3;
        rr = *rb;
        *iters = k;
        *relres = std::sqrt(rr / bb);
        if (*relres <= tol) return 0;
    }
    return 1;
}

}  // namespace igaf
