// Weighted quadrature: the CSR values of the global mass and stiffness
// matrices with the test function moved into the quadrature weights (the
// variant the paper's sum-factorisation section names as reaching O(p^6);
// the method of F. Calabro, G. Sangalli, M. Tani, "Fast formation of
// isogeometric Galerkin matrices by weighted quadrature", CMAME 316, 2017).
//
// Per direction every basis function B_i has its own rule over the fixed
// points inside its support (two per element at its quarter points, p+1 in
// the first and the last element), with the minimum-norm weights that make
//   sum_q w00[i][q] B_j (x_q) = int B_i  B_j,   sum_q w11[i][q] B_j'(x_q) = int B_i' B_j'
// for every trial function j overlapping B_i.  With kappa given on the
// tensor grid of the points,
//   M_IJ = sum_q w00[i1][q1] w00[i2][q2] w00[i3][q3] kappa(q) B_j1(q1) B_j2(q2) B_j3(q3)
//   K_IJ = sum_q kappa(q) (w11 B' in one direction, w00 B in the other two, summed
//          over the three directions).
// No element matrix exists in this formulation: every CSR row is integrated
// directly over its own point box.
//
// Host side (wq_build_dir): points, per-function point ranges, trial values
// at the points, and the weights, each from a Householder QR of the
// transposed exactness matrix in long double (min-norm solution; the
// systems reach condition numbers of ~1e5 at p = 5).
//
// Kernel (k_wq_pencil): one workgroup per chunk of R consecutive rows along
// x of one pencil (i2, i3); the rows share the contractions over z and y,
// taken once for all the x points their supports cover, and each row then
// contracts x with its own weights (see the kernel).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "launch.h"
#include "wq.h"

namespace igaf {

namespace {

// Values and first derivatives of the p+1 functions non-zero on knot span
// s at x (the local Cox-de Boor triangle, as the basis-table kernel builds
// it), in long double.
void span_basis(const double* t, int p, int s, long double x, long double* N, long double* D)
{
    long double ndu[kWqMaxP + 1][kWqMaxP + 1], left[kWqMaxP + 1], right[kWqMaxP + 1];
    ndu[0][0] = 1.0L;
    for (int j = 1; j <= p; ++j) {
        left[j] = x - t[s + 1 - j];
        right[j] = t[s + j] - x;
        long double saved = 0.0L;
        for (int r = 0; r < j; ++r) {
            ndu[j][r] = right[r + 1] + left[j - r];
            const long double tmp = ndu[r][j - 1] / ndu[j][r];
            ndu[r][j] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        ndu[j][j] = saved;
    }
    for (int a = 0; a <= p; ++a) {
        N[a] = ndu[a][p];
        long double lo = 0.0L, hi = 0.0L;
        if (p >= 1 && a >= 1) lo = ndu[a - 1][p - 1] / ((long double)t[s + a] - t[s + a - p]);
        if (p >= 1 && a <= p - 1) hi = ndu[a][p - 1] / ((long double)t[s + a + 1] - t[s + a + 1 - p]);
        D[a] = p * (lo - hi);
    }
}

// The minimum-norm solution of A w = b (A: m x n row-major, m <= n, full row
// rank): Householder QR of A^T = Q R, R^T z = b, w = Q [z; 0].  Returns false
// if a pivot vanishes (rank-deficient system).
bool min_norm(int m, int n, const long double* A, const long double* b, long double* w)
{
    std::vector<long double> V(A, A + (size_t)m * n);   // row k of A = column k of A^T
    std::vector<long double> beta(m), rdiag(m);
    long double scale = 0.0L;
    for (size_t i = 0; i < V.size(); ++i) scale = fmaxl(scale, fabsl(V[i]));
    for (int k = 0; k < m; ++k) {
        long double* v = V.data() + (size_t)k * n;
        long double nrm = 0.0L;
        for (int i = k; i < n; ++i) nrm += v[i] * v[i];
        nrm = sqrtl(nrm);
        if (!(nrm > 1e-30L * scale)) return false;
        const long double alpha = v[k] > 0 ? -nrm : nrm;
        v[k] -= alpha;
        long double vn = 0.0L;
        for (int i = k; i < n; ++i) vn += v[i] * v[i];
        beta[k] = 2.0L / vn;
        rdiag[k] = alpha;
        for (int j = k + 1; j < m; ++j) {   // H_k applied to the later columns
            long double* c = V.data() + (size_t)j * n;
            long double s = 0.0L;
            for (int i = k; i < n; ++i) s += v[i] * c[i];
            s *= beta[k];
            for (int i = k; i < n; ++i) c[i] -= s * v[i];
        }
    }
    // R[k][j] (k < j) sits in V[j][k]; forward substitution R^T z = b
    std::vector<long double> y(n, 0.0L);
    for (int j = 0; j < m; ++j) {
        long double s = b[j];
        for (int k = 0; k < j; ++k) s -= V[(size_t)j * n + k] * y[k];
        y[j] = s / rdiag[j];
    }
    // w = H_0 H_1 ... H_{m-1} [z; 0]
    for (int k = m - 1; k >= 0; --k) {
        const long double* v = V.data() + (size_t)k * n;
        long double s = 0.0L;
        for (int i = k; i < n; ++i) s += v[i] * y[i];
        s *= beta[k];
        for (int i = k; i < n; ++i) y[i] -= s * v[i];
    }
    for (int i = 0; i < n; ++i) w[i] = y[i];
    return true;
}

}  // namespace

int wq_build_dir(int p, int K, const double* t, const double* xg, const double* wg, WqHost& out)
{
    const int n = p + 1, N = K + p;
    for (int e = 0; e < K; ++e)
        if (!(t[e + p + 1] > t[e + p])) return -1;   // an element of zero length
    // points: two per element at its quarter points, p+1 in the end elements
    std::vector<int> first(K + 1, 0);
    out.x.clear();
    out.eq.clear();
    for (int e = 0; e < K; ++e) {
        const int R = (e == 0 || e == K - 1) ? p + 1 : 2;
        const double a = t[e + p], h = t[e + p + 1] - t[e + p];
        for (int r = 0; r < R; ++r) {
            out.x.push_back(a + h * (r + 0.5) / R);
            out.eq.push_back(e);
        }
        first[e + 1] = first[e] + R;
    }
    const int np = first[K];
    out.npts = np;
    out.N = N;
    // trial values at the points (functions eq..eq+p)
    std::vector<long double> Bv((size_t)np * n), dB((size_t)np * n);
    for (int q = 0; q < np; ++q) span_basis(t, p, out.eq[q] + p, out.x[q], &Bv[(size_t)q * n], &dB[(size_t)q * n]);
    out.Bv.assign(Bv.begin(), Bv.end());
    out.dB.assign(dB.begin(), dB.end());
    // int B_i B_j, int B_i' B_j' by the (p+1)-point Gauss rule of the plan
    // (exact for these degree <= 2p products); banded [i][j - i + p]
    const int W = 2 * p + 1;
    std::vector<long double> Mg((size_t)N * W, 0.0L), Ag((size_t)N * W, 0.0L);
    long double Ng[kWqMaxP + 1], Dg[kWqMaxP + 1];
    for (int e = 0; e < K; ++e)
        for (int k = 0; k < n; ++k) {
            span_basis(t, p, e + p, xg[(size_t)e * n + k], Ng, Dg);
            const long double w = wg[(size_t)e * n + k];
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    Mg[(size_t)(e + a) * W + (b - a + p)] += w * Ng[a] * Ng[b];
                    Ag[(size_t)(e + a) * W + (b - a + p)] += w * Dg[a] * Dg[b];
                }
        }
    // the rules
    out.lo.assign(N, 0);
    out.cnt.assign(N, 0);
    int PW = 0;
    for (int g = 0; g < N; ++g) {
        const int lo = first[std::max(0, g - p)], hi = first[std::min(K - 1, g) + 1];
        out.lo[g] = lo;
        out.cnt[g] = hi - lo;
        PW = std::max(PW, hi - lo);
    }
    out.PW = PW;
    out.w00.assign((size_t)N * PW, 0.0);
    out.w11.assign((size_t)N * PW, 0.0);
    std::vector<long double> A, Ad, b, bd, w(PW);
    for (int g = 0; g < N; ++g) {
        const int lo = out.lo[g], c = out.cnt[g];
        const int j0 = std::max(0, g - p), j1 = std::min(N - 1, g + p), m = j1 - j0 + 1;
        A.assign((size_t)m * c, 0.0L);
        Ad.assign((size_t)m * c, 0.0L);
        b.resize(m);
        bd.resize(m);
        for (int r = 0; r < m; ++r) {
            const int j = j0 + r;
            b[r] = Mg[(size_t)g * W + (j - g + p)];
            bd[r] = Ag[(size_t)g * W + (j - g + p)];
            for (int q = 0; q < c; ++q) {
                const int pt = lo + q, a = j - out.eq[pt];
                if (a >= 0 && a <= p) {
                    A[(size_t)r * c + q] = Bv[(size_t)pt * n + a];
                    Ad[(size_t)r * c + q] = dB[(size_t)pt * n + a];
                }
            }
        }
        if (!min_norm(m, c, A.data(), b.data(), w.data())) return -2;
        for (int q = 0; q < c; ++q) out.w00[(size_t)g * PW + q] = (double)w[q];
        // the derivatives of the overlapping functions sum to zero on the
        // support: one condition is dependent and the system consistent; the
        // first m - 1 conditions have the same solutions
        if (!min_norm(m - 1, c, Ad.data(), bd.data(), w.data())) return -2;
        for (int q = 0; q < c; ++q) out.w11[(size_t)g * PW + q] = (double)w[q];
    }
    return 0;
}

template <int P>
struct WqShape {
    static constexpr int O = 2 * P + 1, n = P + 1;
};

// LDS doubles of the pencil kernel: T23 [2 dirs][2][O][PW], C [2][O][O][NX],
// KB [PW][PW][NX] (kappa of the chunk's point box)
template <int P>
static int64_t wq_lds_doubles(int PW, int NX)
{
    constexpr int O = WqShape<P>::O;
    return 4LL * O * PW + 2LL * O * O * NX + (int64_t)PW * PW * NX;
}

// One workgroup per (chunk of R rows along x, i2, i3): the rows (i1, i2,
// i3), i1 in [r0, r0 + R), share stages z and y over the x points their
// supports cover, [X0, X1), taken by one thread per (x, o3), the stage-z sums
// in registers:
//   Dn|Dd[q2]     = sum_q3 T3[n|d][o3][q3] kappa(X0 + x, lo2 + q2, lo3 + q3)
//   C0[o2][o3][x] = sum_q2 T2[n][o2][q2] Dn[q2]
//   C1[o2][o3][x] = sum_q2 (T2[d][o2][q2] Dn[q2] + T2[n][o2][q2] Dd[q2])
// and stage x gives each row's values from its own x tables:
//   M = sum_q1 T1[n][o1][q1] C0[.][lo1 - X0 + q1],  K = sum_q1 (T1[d] C0 + T1[n] C1)
// with T[d][n|d][o][q] = w00|w11[i_d][q] B_j|B_j'(x_q), j = i_d + o - p.
// A thread of stage x owns (row, o2, o3) and writes the row's O values of
// that (o2, o3), contiguous in the CSR row (columns jx fastest).
template <int P>
__global__ __launch_bounds__(256) void k_wq_pencil(WqDev w, RowMap rm, const double* __restrict__ kappa,
                                                   double* __restrict__ Mv, double* __restrict__ Kv, int R,
                                                   int NXM)
{
    using S = WqShape<P>;
    constexpr int O = S::O;
    extern __shared__ double sm[];
    const int PW = w.PW, tid = threadIdx.x;
    double* const T23 = sm;                         // [dir 0 = y, 1 = z][2][O][PW]
    double* const C = T23 + 4 * O * PW;             // [2][O][O][NXM]
    double* const KB = C + 2 * O * O * NXM;         // [q3][q2][x], strides PW, NXM
    const int N1 = w.d[0].N, N2 = w.d[1].N;
    const int np1 = w.d[0].npts, np2 = w.d[1].npts;
    const int nch = (N1 + R - 1) / R;
    const int ch = blockIdx.x % nch;
    const int i2 = (blockIdx.x / nch) % N2, i3 = blockIdx.x / (nch * N2);
    const int r0 = ch * R, nr = min(R, N1 - r0);
    const int X0 = w.d[0].lo[r0];
    const int NX = w.d[0].lo[r0 + nr - 1] + w.d[0].cnt[r0 + nr - 1] - X0;
    const int lo2 = w.d[1].lo[i2], c2 = w.d[1].cnt[i2];
    const int lo3 = w.d[2].lo[i3], c3 = w.d[2].cnt[i3];
    // weighted test values times trial values (the plan's TN, TD): the y and
    // z tables of the pencil (stage x reads its rows' own as scalars)
    for (int idx = tid; idx < 2 * O * PW; idx += 256) {
        const int t = idx / (O * PW), r = idx % (O * PW);
        const int ii = t == 0 ? i2 : i3;
        T23[(t * 2 + 0) * O * PW + r] = w.d[t + 1].TN[(int64_t)ii * O * PW + r];
        T23[(t * 2 + 1) * O * PW + r] = w.d[t + 1].TD[(int64_t)ii * O * PW + r];
    }
    // kappa of the chunk's point box, read once (consecutive x in
    // consecutive lanes): every stage-z thread of an x shares it
    const int64_t zs = (int64_t)np2 * np1;
    for (int idx = tid; idx < c3 * c2 * NX; idx += 256) {
        const int x = idx % NX, q2 = (idx / NX) % c2, q3 = idx / (NX * c2);
        KB[(q3 * PW + q2) * NXM + x] = kappa[((int64_t)lo3 + q3) * zs + (int64_t)(lo2 + q2) * np1 + X0 + x];
    }
    __syncthreads();
    // stages z and y: item (x, o3), consecutive x in consecutive lanes
    for (int it = tid; it < NX * O; it += 256) {
        const int x = it % NX, o3 = it / NX;
        const double* kp = KB + x;
        const double* t3n = T23 + (1 * 2 + 0) * O * PW + o3 * PW;
        const double* t3d = T23 + (1 * 2 + 1) * O * PW + o3 * PW;
        double c0[O], c1[O];
#pragma unroll
        for (int o = 0; o < O; ++o) c0[o] = c1[o] = 0.0;
        for (int q2 = 0; q2 < c2; ++q2) {
            double dn = 0.0, dd = 0.0;
            for (int q3 = 0; q3 < c3; ++q3) {
                const double k = kp[(q3 * PW + q2) * NXM];
                dn += t3n[q3] * k;
                dd += t3d[q3] * k;
            }
#pragma unroll
            for (int o = 0; o < O; ++o) {
                const double tn = T23[(0 * 2 + 0) * O * PW + o * PW + q2];
                const double td = T23[(0 * 2 + 1) * O * PW + o * PW + q2];
                c0[o] += tn * dn;
                c1[o] += td * dn;
                c1[o] += tn * dd;
            }
        }
#pragma unroll
        for (int o = 0; o < O; ++o) {
            C[((0 * O + o) * O + o3) * NXM + x] = c0[o];
            C[((1 * O + o) * O + o3) * NXM + x] = c1[o];
        }
    }
    __syncthreads();
    // stage x: each wavefront takes one row at a time, lanes on (o2, o3)
    // (ceil(O^2 / 64) wavefront passes per row), so that the row's own
    // tables TN, TD are the same in every lane (scalar operands); the row's
    // O values of (o2, o3) go out
    constexpr int WPR = (O * O + 63) / 64;
    const int bl2 = band_lo(i2, P), bl3 = band_lo(i3, P);
    const int Ly = band_len(i2, P, rm.N[1]);
    const int wv = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    for (int sl = wv; sl < nr * WPR; sl += 4) {
        const int r = sl / WPR, it = (sl % WPR) * 64 + lane;
        if (it >= O * O) continue;
        const int o2 = it % O, o3 = it / O;
        const int i1 = r0 + r, j2 = i2 + o2 - P, j3 = i3 + o3 - P;
        if (j2 < 0 || j2 >= rm.N[1] || j3 < 0 || j3 >= rm.N[2]) continue;
        const int xo = w.d[0].lo[i1] - X0, c1n = w.d[0].cnt[i1];
        const ctab tn = as_ctab(w.d[0].TN) + (int64_t)i1 * O * PW;
        const ctab td = as_ctab(w.d[0].TD) + (int64_t)i1 * O * PW;
        const double* a = C + ((0 * O + o2) * O + o3) * NXM + xo;
        const double* b = C + ((1 * O + o2) * O + o3) * NXM + xo;
        double m[O], k[O];
#pragma unroll
        for (int o = 0; o < O; ++o) m[o] = k[o] = 0.0;
        for (int q1 = 0; q1 < c1n; ++q1) {
            const double av = a[q1], bv = b[q1];
#pragma unroll
            for (int o = 0; o < O; ++o) {
                m[o] += tn[o * PW + q1] * av;
                k[o] += td[o * PW + q1] * av;
                k[o] += tn[o * PW + q1] * bv;
            }
        }
        const int bl1 = band_lo(i1, P), Lx = band_len(i1, P, rm.N[0]);
        const int64_t base = rm.row_start(i1, i2, i3) + ((int64_t)(j3 - bl3) * Ly + (j2 - bl2)) * Lx - bl1;
#pragma unroll
        for (int o = 0; o < O; ++o) {
            const int j1 = i1 + o - P;
            if (j1 >= 0 && j1 < rm.N[0]) {
                if (Mv) Mv[base + j1] = m[o];
                if (Kv) Kv[base + j1] = k[o];
            }
        }
    }
}

template <int P>
static int launch_wq_t(const WqDev& w, const PatchDev& pd, const double* kappa, double* Mv, double* Kv,
                       hipStream_t st)
{
    // rows per chunk: the most (8, 4, 2, 1) whose LDS fits a CU; NXM = the
    // most x points a chunk's rows cover
    const int N1 = w.d[0].N;
    for (int R = 8; R >= 1; R /= 2) {
        int NXM = 0;
        for (int r0 = 0; r0 < N1; r0 += R) {
            const int rl = std::min(N1, r0 + R) - 1;
            NXM = std::max(NXM, w.h_lo0[rl] + w.h_cnt0[rl] - w.h_lo0[r0]);
        }
        const int64_t lds = wq_lds_doubles<P>(w.PW, NXM) * (int64_t)sizeof(double);
        if (lds > 160 * 1024) continue;
        if (hipFuncSetAttribute((const void*)k_wq_pencil<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
            return -3;
        const int64_t blocks = (int64_t)((N1 + R - 1) / R) * w.d[1].N * w.d[2].N;
        hipLaunchKernelGGL(k_wq_pencil<P>, dim3((unsigned)blocks), dim3(256), (unsigned)lds, st, w, make_rowmap(pd),
                           kappa, Mv, Kv, R, NXM);
        return hipGetLastError() == hipSuccess ? 0 : -3;
    }
    return -4;
}

int launch_wq(const WqDev& w, const PatchDev& pd, const double* kappa, double* Mv, double* Kv, hipStream_t st)
{
    switch (pd.p) {
    case 1: return launch_wq_t<1>(w, pd, kappa, Mv, Kv, st);
    case 2: return launch_wq_t<2>(w, pd, kappa, Mv, Kv, st);
    case 3: return launch_wq_t<3>(w, pd, kappa, Mv, Kv, st);
    case 4: return launch_wq_t<4>(w, pd, kappa, Mv, Kv, st);
    case 5: return launch_wq_t<5>(w, pd, kappa, Mv, Kv, st);
    default: return -4;
    }
}

}  // namespace igaf
