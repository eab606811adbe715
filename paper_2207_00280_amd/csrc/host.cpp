// C ABI of the library: argument checks, Gauss rule, plan objects (device
// tables), dispatch of the kernels.  See include/igafem.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "../../include/igafem.h"
#include "batch.h"
#include "common.h"
#include "launch.h"
#include "wq.h"

using namespace igaf;

namespace {

thread_local char g_err[512] = "";

igaf_status fail(igaf_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

// Gauss-Legendre rule on [-1, 1], nodes ascending: roots of P_q by Newton's
// method from the asymptotic first guess x ~ (1 - 1/(8q^2) + 1/(8q^3)) cos(pi (4i+3)/(4q+2)),
// weights 2 / ((1 - x^2) P_q'(x)^2).
void gauss_rule(int q, double* xi, double* wr)
{
    for (int i = 0; i < q; ++i) {
        double x = (1.0 - 1.0 / (8.0 * q * q) + 1.0 / (8.0 * q * q * q)) *
                   std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * q + 2.0));
        double dP = 1.0;
        for (int it = 0; it < 64; ++it) {
            double Pm1 = 1.0, Pk = x;     // P_0, P_1
            for (int k = 1; k < q; ++k) {
                double Pn = ((2.0 * k + 1.0) * x * Pk - k * Pm1) / (k + 1.0);
                Pm1 = Pk;
                Pk = Pn;
            }
            if (q == 1) { Pk = x; Pm1 = 1.0; }
            dP = q * (Pm1 - x * Pk) / (1.0 - x * x);
            double step = Pk / dP;
            x -= step;
            if (std::fabs(step) <= 1e-16 * std::fabs(x) + 1e-300) break;
        }
        double Pm1 = 1.0, Pk = x;
        for (int k = 1; k < q; ++k) {
            double Pn = ((2.0 * k + 1.0) * x * Pk - k * Pm1) / (k + 1.0);
            Pm1 = Pk;
            Pk = Pn;
        }
        if (q == 1) { Pk = x; Pm1 = 1.0; }
        dP = q * (Pm1 - x * Pk) / (1.0 - x * x);
        xi[q - 1 - i] = x;   // the guesses run from +1 downwards
        wr[q - 1 - i] = 2.0 / ((1.0 - x * x) * dP * dP);
    }
}

igaf_status check_desc(const igaf_patch_desc* d)
{
    if (!d) return fail(IGAF_EINVAL, "desc is NULL");
    int p = d->degree;
    if (p < 1) return fail(IGAF_EINVAL, "degree %d < 1", p);
    for (int a = 0; a < 3; ++a) {
        if (d->nelem[a] < 1) return fail(IGAF_EINVAL, "nelem[%d] = %d < 1", a, d->nelem[a]);
        if (d->nelem[a] > (1 << 20)) return fail(IGAF_EINVAL, "nelem[%d] = %d too large", a, d->nelem[a]);
        if (d->nquad[a] < 1 || d->nquad[a] > IGAF_MAX_QUAD)
            return fail(IGAF_EINVAL, "nquad[%d] = %d outside [1, %d]", a, d->nquad[a], IGAF_MAX_QUAD);
        const double* t = d->knots[a];
        if (!t) return fail(IGAF_EINVAL, "knots[%d] is NULL", a);
        int nk = d->nelem[a] + 2 * p + 1;
        for (int i = 0; i < nk; ++i)
            if (!std::isfinite(t[i])) return fail(IGAF_EINVAL, "knots[%d][%d] is not finite", a, i);
        for (int i = 0; i + 1 < nk; ++i)
            if (t[i] > t[i + 1]) return fail(IGAF_EINVAL, "knots[%d] decreases at %d", a, i);
        for (int i = 1; i <= p; ++i) {
            if (t[i] != t[0]) return fail(IGAF_EINVAL, "knots[%d]: first %d knots not equal (open vector)", a, p + 1);
            if (t[nk - 1 - i] != t[nk - 1]) return fail(IGAF_EINVAL, "knots[%d]: last %d knots not equal (open vector)", a, p + 1);
        }
        // interior knots may repeat (reduced continuity, C^{p-m} at a knot of
        // multiplicity m) as long as no basis function vanishes identically:
        // the support [t_i, t_{i+p+1}] of every function must be non-empty
        for (int i = 0; i + p + 1 < nk; ++i)
            if (!(t[i] < t[i + p + 1]))
                return fail(IGAF_EINVAL,
                            "knots[%d]: basis function %d has an empty support (a knot repeated more than "
                            "p+1 times)", a, i);
    }
    // the global sizes must fit the index types (int32 columns, int64 rows)
    double ndof = 1.0;
    for (int a = 0; a < 3; ++a) ndof *= (double)(d->nelem[a] + p);
    if (ndof >= 2147483647.0) return fail(IGAF_EINVAL, "ndof %.0f does not fit int32 column indices", ndof);
    return IGAF_OK;
}

int64_t band_total(int N, int p)
{
    int64_t T = 0;
    for (int i = 0; i < N; ++i) T += band_len(i, p, N);
    return T;
}

void sizes_of(const igaf_patch_desc* d, int64_t* ndof, int64_t* nelem, int64_t* nqp, int64_t* edim,
              int64_t* nnz)
{
    int p = d->degree;
    int64_t N = 1, E = 1, Qn = 1, T = 1;
    for (int a = 0; a < 3; ++a) {
        N *= d->nelem[a] + p;
        E *= d->nelem[a];
        Qn *= d->nquad[a];
        T *= band_total(d->nelem[a] + p, p);
    }
    if (ndof) *ndof = N;
    if (nelem) *nelem = E;
    if (nqp) *nqp = Qn;
    if (edim) *edim = (int64_t)(p + 1) * (p + 1) * (p + 1);
    if (nnz) *nnz = T;
}

// The longest run [r0, r1) of consecutive elements of one direction whose
// local knot windows agree: the values on span s = e+p depend on the 2p knots
// t_{e+1} .. t_{e+2p} only through their differences to the span's left end
// t_{e+p} (the recursion of Sec. 2.3), so element e may take the tables of r0
// when every difference t_{e+j} - t_{e+p} equals r0's up to the rounding of
// the knots (8 eps times the largest knot involved).  Uniform spacing gives
// one run over all elements away from the repeated end knots; r0 = r1 = 0
// when no two neighbours agree.
void shared_run(const double* t, int K, int p, int* r0, int* r1)
{
    const double eps = std::numeric_limits<double>::epsilon();
    auto same = [&](int e, int r) {
        for (int j = 1; j <= 2 * p; ++j) {
            const double de = t[e + j] - t[e + p], dr = t[r + j] - t[r + p];
            const double sc = std::max(std::max(std::fabs(t[e + j]), std::fabs(t[e + p])),
                                       std::max(std::fabs(t[r + j]), std::fabs(t[r + p])));
            if (!(std::fabs(de - dr) <= 8.0 * eps * sc)) return false;
        }
        return true;
    };
    int best0 = 0, best1 = 0;
    for (int s = 0; s < K;) {
        int e = s + 1;
        while (e < K && same(e, s)) ++e;
        if (e - s > best1 - best0) {
            best0 = s;
            best1 = e;
        }
        s = e;
    }
    if (best1 - best0 < 2) best0 = best1 = 0;
    *r0 = best0;
    *r1 = best1;
}

}  // namespace

struct igaf_plan {
    int p, n, S;
    int K[3], q[3], N[3];
    int64_t E, ndof, nnz, nqp;
    std::vector<double> xnode[3], wnode[3];   // host copies, [K][q]
    double* dmem = nullptr;
    int64_t* dpre = nullptr;
    PatchDev dev;
    int device = 0;
    int asm_mode = IGAF_ASM_ROWS;
    // opt-in kernel interval log of igaf_integrate_assemble (timing events)
    bool timing = false;
    std::vector<hipEvent_t> tev[2];   // [element | csr]: start, end, start, end, ...
    // Euler step: pinned slot and event for the residual read-back of CG
    double* rb_host = nullptr;
    hipEvent_t rb_ev = nullptr;
    // igaf_bilinear_form: per-wavefront partial sums (kLossParts, in dmem)
    double* dpart = nullptr;
    // weighted quadrature (igaf_wq_prepare): host knots, the points of every
    // direction and the rules in device memory
    std::vector<double> knots_h[3];
    std::vector<double> wq_x[3];
    std::vector<int> wq_lo0, wq_cnt0;
    void* wq_mem = nullptr;
    WqDev wq{};
    bool wq_ready = false;
};

namespace {
void timing_clear(igaf_plan* P)
{
    for (auto& v : P->tev) {
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
        v.clear();
    }
}

// Record one timing event of kernel `k` on stream `s` (skipped under capture).
void timing_mark(igaf_plan* P, int k, hipStream_t s)
{
    if (!P->timing) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, s) != hipSuccess) {
        (void)hipEventDestroy(e);
        return;
    }
    P->tev[k].push_back(e);
}
}  // namespace

namespace igaf {
const PatchDev& plan_dev(const igaf_plan* p) { return p->dev; }
int plan_degree(const igaf_plan* p) { return p->p; }
bool plan_hot_supported(const igaf_plan* p)
{
    return p->p >= 1 && p->p <= IGAF_MAX_DEGREE && p->q[0] == p->p + 1 && p->q[1] == p->p + 1 &&
           p->q[2] == p->p + 1;
}
}  // namespace igaf

extern "C" {

const char* igaf_version(void) { return "igafem 0.1 (gfx950, fp64)"; }

const char* igaf_last_error(void) { return g_err; }

igaf_status igaf_desc_check(const igaf_patch_desc* desc) { return check_desc(desc); }

igaf_status igaf_desc_sizes(const igaf_patch_desc* desc, int64_t* ndof, int64_t* nelem,
                            int64_t* nqp, int64_t* elem_dim, int64_t* nnz)
{
    igaf_status st = check_desc(desc);
    if (st) return st;
    sizes_of(desc, ndof, nelem, nqp, elem_dim, nnz);
    return IGAF_OK;
}

igaf_status igaf_desc_shared_run(const igaf_patch_desc* desc, int dir, int* first, int* end)
{
    igaf_status st = check_desc(desc);
    if (st) return st;
    if (dir < 0 || dir > 2) return fail(IGAF_EINVAL, "dir %d outside [0, 2]", dir);
    if (!first || !end) return fail(IGAF_EINVAL, "first / end is NULL");
    shared_run(desc->knots[dir], desc->nelem[dir], desc->degree, first, end);
    return IGAF_OK;
}

igaf_status igaf_csr_pattern_host(const igaf_patch_desc* desc, int64_t* row_ptr, int32_t* col)
{
    igaf_status st = check_desc(desc);
    if (st) return st;
    if (!row_ptr || !col) return fail(IGAF_EINVAL, "row_ptr_host / col_idx_host is NULL");
    int p = desc->degree;
    int Nx = desc->nelem[0] + p, Ny = desc->nelem[1] + p, Nz = desc->nelem[2] + p;
    int64_t o = 0, g = 0;
    for (int iz = 0; iz < Nz; ++iz)
        for (int iy = 0; iy < Ny; ++iy)
            for (int ix = 0; ix < Nx; ++ix) {
                row_ptr[g++] = o;
                for (int jz = band_lo(iz, p); jz <= band_hi(iz, p, Nz); ++jz)
                    for (int jy = band_lo(iy, p); jy <= band_hi(iy, p, Ny); ++jy)
                        for (int jx = band_lo(ix, p); jx <= band_hi(ix, p, Nx); ++jx)
                            col[o++] = (int32_t)(jx + (int64_t)Nx * (jy + (int64_t)Ny * jz));
            }
    row_ptr[g] = o;
    return IGAF_OK;
}

// The 1D mass matrix of every direction (kappa = 1, the plan's Gauss rule,
// from the device basis tables) and its banded Cholesky factor L L^T, for the
// preconditioner of the Euler step's mass solve.  Stored per DOF i as
// [1/L_ii, L_{i,i-1}, ..., L_{i,i-p}, M_ii] (entries left of column 0 are 0).
static igaf_status mass_factors(igaf_plan* P)
{
    const int p = P->p, n = P->n, B = p + 1, W = p + 2;
    for (int a = 0; a < 3; ++a) {
        const int K = P->K[a], Q = P->q[a], N = P->N[a];
        std::vector<double> Nv((size_t)K * n * Q), wq((size_t)K * Q);
        if (hipMemcpy(Nv.data(), P->dev.d[a].Nv, sizeof(double) * Nv.size(), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(wq.data(), P->dev.d[a].wq, sizeof(double) * wq.size(), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(IGAF_EDEVICE, "copy of basis tables failed");
        std::vector<double> A((size_t)N * B, 0.0);   // A[i*B + k] = M[i][i-k]
        for (int e = 0; e < K; ++e)
            for (int x = 0; x <= p; ++x)
                for (int y = 0; y <= x; ++y)
                    for (int k = 0; k < Q; ++k)
                        A[(size_t)(e + x) * B + (x - y)] +=
                            wq[(size_t)e * Q + k] * Nv[((size_t)e * n + x) * Q + k] * Nv[((size_t)e * n + y) * Q + k];
        std::vector<double> L((size_t)N * B, 0.0);   // L[i*B + k] = L[i][i-k]
        auto Lij = [&](int i, int j) { return L[(size_t)i * B + (i - j)]; };
        for (int i = 0; i < N; ++i)
            for (int j = std::max(0, i - p); j <= i; ++j) {
                double v = A[(size_t)i * B + (i - j)];
                for (int m = std::max(0, i - p); m < j; ++m) v -= Lij(i, m) * Lij(j, m);
                if (j == i) {
                    if (!(v > 0.0)) return fail(IGAF_EDEVICE, "1D mass matrix %d not positive definite", a);
                    L[(size_t)i * B] = std::sqrt(v);
                } else {
                    L[(size_t)i * B + (i - j)] = v / Lij(j, j);
                }
            }
        std::vector<double> out((size_t)N * W, 0.0);
        for (int i = 0; i < N; ++i) {
            out[(size_t)i * W] = 1.0 / L[(size_t)i * B];
            for (int k = 1; k <= p; ++k) out[(size_t)i * W + k] = i - k >= 0 ? L[(size_t)i * B + k] : 0.0;
            out[(size_t)i * W + p + 1] = A[(size_t)i * B];
        }
        if (hipMemcpy(const_cast<double*>(P->dev.d[a].Lm), out.data(), sizeof(double) * out.size(),
                      hipMemcpyHostToDevice) != hipSuccess)
            return fail(IGAF_EDEVICE, "upload of mass factors failed");
    }
    return IGAF_OK;
}

igaf_status igaf_plan_create(const igaf_patch_desc* desc, igaf_plan** out)
{
    if (!out) return fail(IGAF_EINVAL, "out is NULL");
    *out = nullptr;
    igaf_status st = check_desc(desc);
    if (st) return st;
    if (desc->degree > IGAF_MAX_DEGREE)
        return fail(IGAF_EUNSUPPORTED, "degree %d > %d", desc->degree, IGAF_MAX_DEGREE);

    igaf_plan* P = new (std::nothrow) igaf_plan();
    if (!P) return fail(IGAF_ENOMEM, "host allocation failed");
    P->p = desc->degree;
    P->n = P->p + 1;
    P->S = P->n * (P->n + 1) / 2;
    for (int a = 0; a < 3; ++a) {
        P->K[a] = desc->nelem[a];
        P->q[a] = desc->nquad[a];
        P->N[a] = P->K[a] + P->p;
    }
    sizes_of(desc, &P->ndof, &P->E, &P->nqp, nullptr, &P->nnz);

    // device layout: per direction [knots | xi | wr | Wnn | Wdd | Nv | dN | wq | Lm | Wg]
    int64_t dcount = 0, icount = 0;
    int64_t off[3][10];
    for (int a = 0; a < 3; ++a) {
        int K = P->K[a], Q = P->q[a], nk = K + 2 * P->p + 1;
        int64_t sz[10] = {nk, Q, Q, (int64_t)K * P->S * Q, (int64_t)K * P->S * Q,
                          (int64_t)K * P->n * Q, (int64_t)K * P->n * Q, (int64_t)K * Q,
                          (int64_t)P->N[a] * (P->p + 2), (int64_t)K * 4 * P->n * Q};
        for (int j = 0; j < 10; ++j) {
            off[a][j] = dcount;
            dcount += (sz[j] + 31) & ~int64_t(31);   // 256-byte aligned pieces
        }
        icount += P->N[a] + 1;
    }
    const int64_t part_off = dcount;
    dcount += kLossParts;
    if (hipGetDevice(&P->device) != hipSuccess) {
        delete P;
        return fail(IGAF_EDEVICE, "hipGetDevice failed (no GPU?)");
    }
    if (apply_scratch_init() != 0) {   // once per device: the static scratch's address
        delete P;
        return fail(IGAF_EDEVICE, "static scratch lookup failed: %s", hipGetErrorString(hipGetLastError()));
    }
    if (hipMalloc(&P->dmem, sizeof(double) * dcount) != hipSuccess) {
        delete P;
        return fail(IGAF_ENOMEM, "hipMalloc of %lld doubles failed", (long long)dcount);
    }
    if (hipMalloc(&P->dpre, sizeof(int64_t) * icount) != hipSuccess) {
        (void)hipFree(P->dmem);
        delete P;
        return fail(IGAF_ENOMEM, "hipMalloc of prefix tables failed");
    }
    int64_t ioff = 0;
    P->dpart = P->dmem + part_off;
    P->dev.p = P->p;
    // element kernels: two 256-lane workgroups per CU saturate the HBM store
    // path
    int ncu = 256;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess)
        ncu = 256;
    P->dev.elem_grid = 2 * ncu;
    if (const char* g = std::getenv("IGAF_ELEM_GRID")) {   // tuning override
        int v = std::atoi(g);
        if (v > 0) P->dev.elem_grid = v;
    }
    P->dev.E = P->E;
    P->dev.ndof = P->ndof;
    P->dev.nnz = P->nnz;
    igaf_status rc = IGAF_OK;
    for (int a = 0; a < 3 && rc == IGAF_OK; ++a) {
        int K = P->K[a], Q = P->q[a], nk = K + 2 * P->p + 1, N = P->N[a];
        std::vector<double> xi(Q), wr(Q);
        gauss_rule(Q, xi.data(), wr.data());
        const double* t = desc->knots[a];
        P->knots_h[a].assign(t, t + nk);
        P->xnode[a].resize((size_t)K * Q);
        P->wnode[a].resize((size_t)K * Q);
        for (int e = 0; e < K; ++e) {
            double x0 = t[e + P->p], h = t[e + P->p + 1] - x0;
            for (int k = 0; k < Q; ++k) {
                P->xnode[a][(size_t)e * Q + k] = x0 + 0.5 * (xi[k] + 1.0) * h;
                P->wnode[a][(size_t)e * Q + k] = 0.5 * wr[k] * h;
            }
        }
        std::vector<int64_t> pre(N + 1);
        pre[0] = 0;
        for (int i = 0; i < N; ++i) pre[i + 1] = pre[i] + band_len(i, P->p, N);
        P->dev.T[a] = pre[N];
        double* base = P->dmem;
        bool ok = hipMemcpy(base + off[a][0], t, sizeof(double) * nk, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(base + off[a][1], xi.data(), sizeof(double) * Q, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(base + off[a][2], wr.data(), sizeof(double) * Q, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(P->dpre + ioff, pre.data(), sizeof(int64_t) * (N + 1), hipMemcpyHostToDevice) == hipSuccess;
        if (!ok) {
            rc = fail(IGAF_EDEVICE, "hipMemcpy of tables failed");
            break;
        }
        DirTables& D = P->dev.d[a];
        D.Wnn = base + off[a][3];
        D.Wdd = base + off[a][4];
        D.Nv = base + off[a][5];
        D.dN = base + off[a][6];
        D.wq = base + off[a][7];
        D.Lm = base + off[a][8];
        D.Wg = base + off[a][9];
        D.pre = P->dpre + ioff;
        D.K = K;
        D.N = N;
        D.Q = Q;
        shared_run(t, K, P->p, &D.r0, &D.r1);
        ioff += N + 1;
        if (launch_basis_tables(P->p, base + off[a][0], K, base + off[a][1], base + off[a][2], Q,
                                base + off[a][3], base + off[a][4], base + off[a][5],
                                base + off[a][6], base + off[a][7], base + off[a][9], D.r0, D.r1, nullptr) != 0)
            rc = fail(IGAF_EDEVICE, "basis-table launch failed: %s", hipGetErrorString(hipGetLastError()));
    }
    if (rc == IGAF_OK && hipStreamSynchronize(nullptr) != hipSuccess)
        rc = fail(IGAF_EDEVICE, "basis-table kernel failed");
    if (rc == IGAF_OK) rc = mass_factors(P);
    if (rc == IGAF_OK && (hipHostMalloc((void**)&P->rb_host, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
                          hipEventCreateWithFlags(&P->rb_ev, hipEventDisableTiming) != hipSuccess))
        rc = fail(IGAF_EDEVICE, "pinned read-back slot or event creation failed");
    if (rc != IGAF_OK) {
        igaf_plan_destroy(P);
        return rc;
    }
    *out = P;
    return IGAF_OK;
}

void igaf_plan_destroy(igaf_plan* plan)
{
    if (!plan) return;
    timing_clear(plan);
    (void)hipFree(plan->dmem);
    (void)hipFree(plan->dpre);
    if (plan->wq_mem) (void)hipFree(plan->wq_mem);
    if (plan->rb_ev) (void)hipEventDestroy(plan->rb_ev);
    if (plan->rb_host) (void)hipHostFree(plan->rb_host);
    delete plan;
}

igaf_status igaf_plan_sizes(const igaf_plan* plan, int64_t* ndof, int64_t* nelem, int64_t* nqp,
                            int64_t* elem_dim, int64_t* nnz)
{
    if (!plan) return fail(IGAF_EINVAL, "plan is NULL");
    if (ndof) *ndof = plan->ndof;
    if (nelem) *nelem = plan->E;
    if (nqp) *nqp = plan->nqp;
    if (elem_dim) *elem_dim = (int64_t)plan->n * plan->n * plan->n;
    if (nnz) *nnz = plan->nnz;
    return IGAF_OK;
}

igaf_status igaf_quad_nodes(const igaf_plan* plan, int32_t dir, double* x, double* w)
{
    if (!plan) return fail(IGAF_EINVAL, "plan is NULL");
    if (dir < 0 || dir > 2) return fail(IGAF_EINVAL, "dir %d not in 0..2", dir);
    if (!x) return fail(IGAF_EINVAL, "x_host is NULL");
    std::memcpy(x, plan->xnode[dir].data(), sizeof(double) * plan->xnode[dir].size());
    if (w) std::memcpy(w, plan->wnode[dir].data(), sizeof(double) * plan->wnode[dir].size());
    return IGAF_OK;
}

igaf_status igaf_quad_points(const igaf_plan* plan, double* xyz)
{
    if (!plan) return fail(IGAF_EINVAL, "plan is NULL");
    if (!xyz) return fail(IGAF_EINVAL, "xyz_host is NULL");
    const int qx = plan->q[0], qy = plan->q[1], qz = plan->q[2];
    const int Kx = plan->K[0], Ky = plan->K[1];
    for (int64_t e = 0; e < plan->E; ++e) {
        const int ex = (int)(e % Kx), ey = (int)((e / Kx) % Ky), ez = (int)(e / ((int64_t)Kx * Ky));
        double* o = xyz + e * plan->nqp * 3;
        for (int kz = 0; kz < qz; ++kz)
            for (int ky = 0; ky < qy; ++ky)
                for (int kx = 0; kx < qx; ++kx, o += 3) {
                    o[0] = plan->xnode[0][(size_t)ex * qx + kx];
                    o[1] = plan->xnode[1][(size_t)ey * qy + ky];
                    o[2] = plan->xnode[2][(size_t)ez * qz + kz];
                }
    }
    return IGAF_OK;
}

igaf_status igaf_plan_set_assembly(igaf_plan* plan, int32_t mode)
{
    if (!plan) return fail(IGAF_EINVAL, "plan is NULL");
    if (mode != IGAF_ASM_ROWS && mode != IGAF_ASM_ATOMIC)
        return fail(IGAF_EINVAL, "assembly mode %d unknown", mode);
    plan->asm_mode = mode;
    return IGAF_OK;
}

igaf_status igaf_csr_pattern(const igaf_plan* plan, int64_t* row_ptr, int32_t* col, void* stream)
{
    if (!plan) return fail(IGAF_EINVAL, "plan is NULL");
    if (!row_ptr || !col) return fail(IGAF_EINVAL, "row_ptr / col_idx is NULL");
    if (launch_csr_pattern(plan->dev, row_ptr, col, (hipStream_t)stream))
        return fail(IGAF_EDEVICE, "pattern launch failed");
    return IGAF_OK;
}

static igaf_status check_hot(const igaf_plan* plan, int method)
{
    if (!plan) return fail(IGAF_EINVAL, "plan is NULL");
    if (method != IGAF_CLASSICAL && method != IGAF_SUMFACT)
        return fail(IGAF_EINVAL, "method %d unknown", method);
    if (!plan_hot_supported(plan))
        return fail(IGAF_EUNSUPPORTED, "kernels implement nquad = degree+1 in every direction "
                    "(got p=%d, q=%d,%d,%d)", plan->p, plan->q[0], plan->q[1], plan->q[2]);
    return IGAF_OK;
}

static igaf_status launched(int rc, const char* what)
{
    if (rc == -4) return fail(IGAF_EUNSUPPORTED, "%s: unsupported shape", what);
    if (rc) return fail(IGAF_EDEVICE, "%s: launch failed: %s", what, hipGetErrorString(hipGetLastError()));
    return IGAF_OK;
}

igaf_status igaf_element_matrices(const igaf_plan* plan, int32_t method, const double* kappa,
                                  double* Me, double* Ke, void* stream)
{
    igaf_status st = check_hot(plan, method);
    if (st) return st;
    if (!kappa) return fail(IGAF_EINVAL, "kappa is NULL");
    if (!Me && !Ke) return fail(IGAF_EINVAL, "Me and Ke are both NULL");
    return launched(launch_element(plan->dev, method, kappa, Me, Ke, nullptr, nullptr,
                                   (hipStream_t)stream), "element matrices");
}

igaf_status igaf_assemble(const igaf_plan* plan, const double* Me, const double* Ke, double* Mval,
                          double* Kval, void* stream)
{
    if (!plan) return fail(IGAF_EINVAL, "plan is NULL");
    if (!Mval && !Kval) return fail(IGAF_EINVAL, "Mval and Kval are both NULL");
    if ((Mval && !Me) || (Kval && !Ke)) return fail(IGAF_EINVAL, "an output has no input matrices");
    if (plan->p > IGAF_MAX_DEGREE) return fail(IGAF_EUNSUPPORTED, "degree too large");
    return launched(launch_gather(plan->dev, Mval ? Me : nullptr, Kval ? Ke : nullptr, Mval, Kval,
                                  (hipStream_t)stream), "assemble");
}

igaf_status igaf_integrate_assemble(const igaf_plan* plan, int32_t method, const double* kappa,
                                    double* Me, double* Ke, double* Mval, double* Kval,
                                    void* stream)
{
    igaf_status st = check_hot(plan, method);
    if (st) return st;
    if (!kappa) return fail(IGAF_EINVAL, "kappa is NULL");
    if (!Me && !Ke && !Mval && !Kval) return fail(IGAF_EINVAL, "all outputs are NULL");
    hipStream_t s = (hipStream_t)stream;
    if ((Mval || Kval) && plan->asm_mode == IGAF_ASM_ATOMIC) {
        st = launched(launch_fill_zero(Mval, Mval ? plan->nnz : 0, s), "zero");
        if (!st) st = launched(launch_fill_zero(Kval, Kval ? plan->nnz : 0, s), "zero");
        if (!st) st = launched(launch_element(plan->dev, method, kappa, Me, Ke, Mval, Kval, s),
                               "integrate+atomic assembly");
        return st;
    }
    // dense element matrices first, then the CSR rows kernel on the same
    // stream: one after the other measured faster than the two side by side
    // on two streams (they compete for the same CU slots)
    igaf_plan* mp = const_cast<igaf_plan*>(plan);
    if (Me || Ke) {
        timing_mark(mp, 0, s);
        st = launched(launch_element(plan->dev, method, kappa, Me, Ke, nullptr, nullptr, s),
                      "element matrices");
        timing_mark(mp, 0, s);
        if (st || !(Mval || Kval)) return st;
    }
    timing_mark(mp, 1, s);
    st = launched(launch_rows(plan->dev, kappa, Mval, Kval, s), "row assembly");
    timing_mark(mp, 1, s);
    return st;
}

igaf_status igaf_plan_set_timing(igaf_plan* plan, int32_t enable)
{
    if (!plan) return fail(IGAF_EINVAL, "plan is NULL");
    if (hipDeviceSynchronize() != hipSuccess) return fail(IGAF_EDEVICE, "device sync failed");
    timing_clear(plan);
    plan->timing = enable != 0;
    return IGAF_OK;
}

igaf_status igaf_plan_timing(igaf_plan* plan, int32_t kernel, double* avg_ms, int32_t* count)
{
    if (!plan) return fail(IGAF_EINVAL, "plan is NULL");
    if (kernel != 0 && kernel != 1) return fail(IGAF_EINVAL, "kernel %d not 0 or 1", kernel);
    const auto& v = plan->tev[kernel];
    double tot = 0.0;
    int n = 0;
    for (size_t i = 0; i + 1 < v.size(); i += 2) {
        float ms = 0.f;
        if (hipEventSynchronize(v[i + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, v[i], v[i + 1]) != hipSuccess)
            return fail(IGAF_EDEVICE, "timing event query failed");
        tot += ms;
        ++n;
    }
    if (avg_ms) *avg_ms = n ? tot / n : 0.0;
    if (count) *count = n;
    return IGAF_OK;
}

igaf_status igaf_integrate_assemble_geo(const igaf_plan* plan, const double* cm, const double* G,
                                        double* Me, double* Ke, double* Mval, double* Kval,
                                        void* stream)
{
    igaf_status st = check_hot(plan, IGAF_SUMFACT);
    if (st) return st;
    if (!Me && !Ke && !Mval && !Kval) return fail(IGAF_EINVAL, "all outputs are NULL");
    if ((Me || Mval) && !cm) return fail(IGAF_EINVAL, "cm is NULL but a mass output is requested");
    if ((Ke || Kval) && !G) return fail(IGAF_EINVAL, "G is NULL but a stiffness output is requested");
    hipStream_t s = (hipStream_t)stream;
    // dense element matrices into the caller's arrays, and the CSR values
    // that have theirs gathered from them (deterministic, no atomics)
    if (Me || Ke) {
        st = launched(launch_element_geo(plan->dev, Me ? cm : nullptr, Ke ? G : nullptr, Me, Ke, s),
                      "mapped-geometry integration");
        double* gm = Mval && Me ? Mval : nullptr;
        double* gk = Kval && Ke ? Kval : nullptr;
        if (!st && (gm || gk))
            st = launched(launch_gather(plan->dev, gm ? Me : nullptr, gk ? Ke : nullptr, gm, gk, s), "assemble");
        if (st) return st;
    }
    // the CSR values without stored element matrices: owner-computed rows
    // (no workspace, no atomics)
    double* sm = Mval && !Me ? Mval : nullptr;
    double* sk = Kval && !Ke ? Kval : nullptr;
    if (!sm && !sk) return IGAF_OK;
    return launched(launch_rows_geo(plan->dev, cm, G, sm, sk, s), "mapped-geometry rows");
}

igaf_status igaf_geo_prepare(igaf_plan* plan)
{
    // the mapped-geometry paths allocate nothing: only the checks remain
    return check_hot(plan, IGAF_SUMFACT);
}

igaf_status igaf_kappa_grad(const igaf_plan* plan, const double* u, const double* v,
                            double alphaM, double alphaK, double scale, const double* scale_dev,
                            double* grad, void* stream)
{
    igaf_status st = check_hot(plan, IGAF_SUMFACT);
    if (st) return st;
    if (!u || !v || !grad) return fail(IGAF_EINVAL, "u, v or grad is NULL");
    return launched(launch_kappa_grad(plan->dev, u, v, alphaM, alphaK, scale, scale_dev, grad,
                                      (hipStream_t)stream), "kappa gradient");
}

igaf_status igaf_bilinear_form(const igaf_plan* plan, const double* kappa, const double* u, const double* v,
                               double alphaM, double alphaK, double* L, void* stream)
{
    igaf_status st = check_hot(plan, IGAF_SUMFACT);
    if (st) return st;
    if (!kappa || !u || !v || !L) return fail(IGAF_EINVAL, "kappa, u, v or L is NULL");
    return launched(launch_bilinear(plan->dev, kappa, u, v, alphaM, alphaK, L, plan->dpart, (hipStream_t)stream),
                    "bilinear form");
}

int64_t igaf_apply_workspace(const igaf_plan* plan)
{
    return plan && plan_hot_supported(plan) ? apply_workspace_doubles(plan->dev) : 0;
}

igaf_status igaf_apply(const igaf_plan* plan, const double* kappa, const double* u,
                       double alphaM, double alphaK, double* y, double* work, void* stream)
{
    igaf_status st = check_hot(plan, IGAF_SUMFACT);
    if (st) return st;
    if (!kappa || !u || !y || !work) return fail(IGAF_EINVAL, "kappa, u, y or work is NULL");
    if (u == y) return fail(IGAF_EINVAL, "y must not overlap u");
    return launched(launch_apply(plan->dev, kappa, u, alphaM, alphaK, y, work, (hipStream_t)stream),
                    "operator apply");
}

igaf_status igaf_apply_static(const igaf_plan* plan, const double* kappa, const double* u, double alphaM,
                              double alphaK, double* y, void* stream)
{
    igaf_status st = check_hot(plan, IGAF_SUMFACT);
    if (st) return st;
    if (!kappa || !u || !y) return fail(IGAF_EINVAL, "kappa, u or y is NULL");
    if (u == y) return fail(IGAF_EINVAL, "y must not overlap u");
    int64_t cap = 0;
    double* w = apply_scratch(&cap);
    const int64_t need = apply_workspace_doubles(plan->dev);
    if (need > cap)
        return fail(IGAF_EUNSUPPORTED,
                    "igaf_apply_static: this patch needs %lld doubles of scratch, the static array holds %lld "
                    "(igaf_apply takes a workspace of any size)",
                    (long long)need, (long long)cap);
    if (!w) return fail(IGAF_EDEVICE, "igaf_apply_static: no scratch address on the current device");
    return launched(launch_apply(plan->dev, kappa, u, alphaM, alphaK, y, w, (hipStream_t)stream),
                    "operator apply (static scratch)");
}

igaf_status igaf_apply_geo(const igaf_plan* plan, const double* cm, const double* G, const double* u,
                           double alphaM, double alphaK, double* y, double* work, void* stream)
{
    igaf_status st = check_hot(plan, IGAF_SUMFACT);
    if (st) return st;
    if (!cm || !G || !u || !y || !work) return fail(IGAF_EINVAL, "cm, G, u, y or work is NULL");
    if (u == y) return fail(IGAF_EINVAL, "y must not overlap u");
    return launched(launch_apply(plan->dev, cm, u, alphaM, alphaK, y, work, (hipStream_t)stream, G),
                    "mapped-geometry apply");
}

igaf_status igaf_kappa_grad_geo(const igaf_plan* plan, const double* cm0, const double* G0, const double* u,
                                const double* v, double alphaM, double alphaK, double scale, double* grad,
                                void* stream)
{
    igaf_status st = check_hot(plan, IGAF_SUMFACT);
    if (st) return st;
    if (!cm0 || !G0 || !u || !v || !grad) return fail(IGAF_EINVAL, "cm0, G0, u, v or grad is NULL");
    return launched(launch_kappa_grad(plan->dev, u, v, alphaM, alphaK, scale, nullptr, grad, (hipStream_t)stream,
                                      cm0, G0),
                    "mapped-geometry kappa gradient");
}

igaf_status igaf_wq_prepare(igaf_plan* plan)
{
    igaf_status st = check_hot(plan, IGAF_SUMFACT);
    if (st) return st;
    if (plan->wq_ready) return IGAF_OK;
    WqHost H[3];
    for (int d = 0; d < 3; ++d) {
        const int rc = wq_build_dir(plan->p, plan->K[d], plan->knots_h[d].data(), plan->xnode[d].data(),
                                    plan->wnode[d].data(), H[d]);
        if (rc == -1)
            return fail(IGAF_EUNSUPPORTED, "weighted quadrature needs elements of positive length (direction %d)", d);
        if (rc) return fail(IGAF_EUNSUPPORTED, "weighted quadrature: a rule's system is singular (direction %d)", d);
    }
    const int PW = std::max(H[0].PW, std::max(H[1].PW, H[2].PW));
    // one buffer: per direction w00 | w11 (N x PW) | Bv | dB (npts x n) |
    // TN | TD (N x O x PW) doubles, then lo | cnt | eq ints
    const int n = plan->p + 1, O = 2 * plan->p + 1;
    int64_t nd = 0, ni = 0;
    for (int d = 0; d < 3; ++d) {
        nd += 2LL * H[d].N * PW + 2LL * H[d].npts * n + 2LL * H[d].N * O * PW;
        ni += 2LL * H[d].N + H[d].npts;
    }
    std::vector<double> hd((size_t)nd, 0.0);
    std::vector<int> hi((size_t)ni, 0);
    void* mem = nullptr;
    if (hipMalloc(&mem, sizeof(double) * nd + sizeof(int) * ni) != hipSuccess)
        return fail(IGAF_ENOMEM, "weighted quadrature tables: device allocation failed");
    double* dd = static_cast<double*>(mem);
    int* di = reinterpret_cast<int*>(dd + nd);
    WqDev w{};
    w.PW = PW;
    int64_t od = 0, oi = 0;
    for (int d = 0; d < 3; ++d) {
        const WqHost& h = H[d];
        for (int g = 0; g < h.N; ++g)
            for (int q = 0; q < h.PW; ++q) {
                hd[od + (size_t)g * PW + q] = h.w00[(size_t)g * h.PW + q];
                hd[od + (size_t)h.N * PW + (size_t)g * PW + q] = h.w11[(size_t)g * h.PW + q];
            }
        w.d[d].w00 = dd + od;
        w.d[d].w11 = dd + od + (int64_t)h.N * PW;
        od += 2LL * h.N * PW;
        std::copy(h.Bv.begin(), h.Bv.end(), hd.begin() + od);
        w.d[d].Bv = dd + od;
        od += (int64_t)h.npts * n;
        std::copy(h.dB.begin(), h.dB.end(), hd.begin() + od);
        w.d[d].dB = dd + od;
        od += (int64_t)h.npts * n;
        // TN, TD: the weighted test value times the trial value of the column
        // j = g + o - p at each point of g's support (zero outside the patch
        // and where x_q is outside supp(B_j))
        const int64_t otn = od, otd = od + (int64_t)h.N * O * PW;
        for (int g = 0; g < h.N; ++g)
            for (int o = 0; o < O; ++o) {
                const int j = g + o - plan->p;
                if (j < 0 || j >= h.N) continue;
                for (int q = 0; q < h.cnt[g]; ++q) {
                    const int pt = h.lo[g] + q, a = j - h.eq[pt];
                    if (a < 0 || a >= n) continue;
                    const size_t at = ((size_t)g * O + o) * PW + q;
                    hd[otn + at] = h.w00[(size_t)g * h.PW + q] * h.Bv[(size_t)pt * n + a];
                    hd[otd + at] = h.w11[(size_t)g * h.PW + q] * h.dB[(size_t)pt * n + a];
                }
            }
        w.d[d].TN = dd + otn;
        w.d[d].TD = dd + otd;
        od += 2LL * h.N * O * PW;
        std::copy(h.lo.begin(), h.lo.end(), hi.begin() + oi);
        w.d[d].lo = di + oi;
        oi += h.N;
        std::copy(h.cnt.begin(), h.cnt.end(), hi.begin() + oi);
        w.d[d].cnt = di + oi;
        oi += h.N;
        std::copy(h.eq.begin(), h.eq.end(), hi.begin() + oi);
        w.d[d].eq = di + oi;
        oi += h.npts;
        w.d[d].N = h.N;
        w.d[d].npts = h.npts;
    }
    if (hipMemcpy(dd, hd.data(), sizeof(double) * nd, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(di, hi.data(), sizeof(int) * ni, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(mem);
        return fail(IGAF_EDEVICE, "weighted quadrature tables: upload failed");
    }
    plan->wq_mem = mem;
    plan->wq_lo0 = H[0].lo;
    plan->wq_cnt0 = H[0].cnt;
    w.h_lo0 = plan->wq_lo0.data();
    w.h_cnt0 = plan->wq_cnt0.data();
    plan->wq = w;
    for (int d = 0; d < 3; ++d) plan->wq_x[d] = H[d].x;
    plan->wq_ready = true;
    return IGAF_OK;
}

igaf_status igaf_wq_points(const igaf_plan* plan, int32_t dir, int64_t* npts, double* x_host)
{
    if (!plan) return fail(IGAF_EINVAL, "plan is NULL");
    if (!plan->wq_ready) return fail(IGAF_EINVAL, "call igaf_wq_prepare first");
    if (dir < 0 || dir > 2) return fail(IGAF_EINVAL, "dir %d not in 0..2", dir);
    if (npts) *npts = (int64_t)plan->wq_x[dir].size();
    if (x_host) std::memcpy(x_host, plan->wq_x[dir].data(), sizeof(double) * plan->wq_x[dir].size());
    return IGAF_OK;
}

igaf_status igaf_wq_assemble(const igaf_plan* plan, const double* kappa, double* Mval, double* Kval,
                             void* stream)
{
    igaf_status st = check_hot(plan, IGAF_SUMFACT);
    if (st) return st;
    if (!plan->wq_ready) return fail(IGAF_EINVAL, "call igaf_wq_prepare first");
    if (!kappa) return fail(IGAF_EINVAL, "kappa is NULL");
    if (!Mval && !Kval) return fail(IGAF_EINVAL, "Mval and Kval are both NULL");
    return launched(launch_wq(plan->wq, plan->dev, kappa, Mval, Kval, (hipStream_t)stream),
                    "weighted-quadrature rows");
}

int64_t igaf_euler_workspace(const igaf_plan* plan)
{
    return plan && plan_hot_supported(plan) ? euler_workspace_doubles(plan->dev, plan->ndof) : 0;
}

static igaf_status euler_any(const igaf_plan* plan, const double* kappa, const double* G, const double* mu,
                             double dt, double tol, int32_t maxit, int32_t precond, double* mu_next,
                             double* work, int32_t* iters, double* relres, void* stream)
{
    igaf_status st = check_hot(plan, IGAF_SUMFACT);
    if (st) return st;
    if (!kappa || !mu || !mu_next || !work) return fail(IGAF_EINVAL, "coefficient, mu, mu_next or work is NULL");
    if (!(tol >= 0.0) || maxit < 0) return fail(IGAF_EINVAL, "tol < 0 or maxit < 0");
    if (precond != IGAF_PRECOND_NONE && precond != IGAF_PRECOND_KRON)
        return fail(IGAF_EINVAL, "precond %d unknown", precond);
    int it = 0;
    double rr = 0.0;
    int rc = run_euler_step(plan->dev, plan->ndof, kappa, mu, dt, tol, maxit, precond, mu_next, work, &it,
                            &rr, (hipStream_t)stream, plan->rb_host, plan->rb_ev, G);
    if (iters) *iters = it;
    if (relres) *relres = rr;
    if (rc < 0) return fail(IGAF_EDEVICE, "Euler step: %s", hipGetErrorString(hipGetLastError()));
    if (rc > 0) return fail(IGAF_ENOCONV, "Euler step: CG stopped at %d iterations, relative residual %.3e",
                            it, rr);
    return IGAF_OK;
}

igaf_status igaf_euler_step(const igaf_plan* plan, const double* kappa, const double* mu, double dt,
                            double tol, int32_t maxit, int32_t precond, double* mu_next, double* work,
                            int32_t* iters, double* relres, void* stream)
{
    return euler_any(plan, kappa, nullptr, mu, dt, tol, maxit, precond, mu_next, work, iters, relres, stream);
}

igaf_status igaf_euler_step_geo(const igaf_plan* plan, const double* cm, const double* G, const double* mu,
                                double dt, double tol, int32_t maxit, int32_t precond, double* mu_next,
                                double* work, int32_t* iters, double* relres, void* stream)
{
    if (!G) return fail(IGAF_EINVAL, "G is NULL");
    return euler_any(plan, cm, G, mu, dt, tol, maxit, precond, mu_next, work, iters, relres, stream);
}

}  // extern "C"

namespace igaf {
igaf_status set_error(igaf_status st, const char* msg) { return fail(st, "%s", msg); }
}  // namespace igaf
