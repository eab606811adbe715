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
// Kernel (k_wq_rows): one workgroup per CSR row, grid-stride over rows; the
// row's sums run by sum factorisation over its point box in LDS, x -> y -> z:
//   per direction d and column offset o: the weighted test values times the
//     trial values, T[d][n|d][o][q] = w00|w11[i_d][q] * B_j|B_j'(x_q);
//   stage x: E[n|d][o1][q3][q2]  = sum_q1 T[x][n|d][o1][q1] kappa(q1, q2, q3);
//   stage y: F0[o1][o2][q3]      = sum_q2 T[y][n][o2][q2] En,
//            F1[o1][o2][q3]      = sum_q2 (T[y][d][o2][q2] En + T[y][n][o2][q2] Ed);
//   stage z: M[o1][o2][o3]       = sum_q3 T[z][n][o3][q3] F0,
//            K[o1][o2][o3]       = sum_q3 (T[z][n][o3][q3] F1 + T[z][d][o3][q3] F0);
// then the row is staged in LDS at its CSR positions and written contiguously.
#include <cmath>
#include <vector>

#include "common.h"
#include "launch.h"

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
    static constexpr int O = 2 * P + 1, n = P + 1, O3 = O * O * O;
};

// LDS doubles of the row kernel for a largest point count PW per direction
template <int P>
static int64_t wq_lds_doubles(int PW)
{
    using S = WqShape<P>;
    const int64_t T = 6LL * S::O * PW, E = 2LL * S::O * PW * PW, F = 2LL * S::O * S::O * PW;
    const int64_t RW = 2LL * (S::O3 + 1);
    return T + (E > RW ? E : RW) + F;
}

template <int P>
__global__ __launch_bounds__(256) void k_wq_rows(WqDev w, RowMap rm, const double* __restrict__ kappa,
                                                 double* __restrict__ Mv, double* __restrict__ Kv, int64_t ndof)
{
    using S = WqShape<P>;
    constexpr int O = S::O, n = S::n, O3 = S::O3;
    extern __shared__ double sm[];
    const int PW = w.PW, tid = threadIdx.x;
    const int64_t sE = 2LL * O * PW * PW, sRW = 2LL * (O3 + 1);
    double* const T = sm;                                  // [3][2][O][PW]
    double* const E = T + 6 * O * PW;                      // [2][O][PW (q3)][PW (q2)]
    double* const RW = E;                                  // row staging [2][O3 + 1], after stage y
    double* const F = E + (sE > sRW ? sE : sRW);           // [2][O][O][PW]
    const int N1 = w.d[0].N, N2 = w.d[1].N;
    const int np1 = w.d[0].npts, np2 = w.d[1].npts;
    for (int64_t row = blockIdx.x; row < ndof; row += gridDim.x) {
        const int i1 = (int)(row % N1), i2 = (int)((row / N1) % N2), i3 = (int)(row / ((int64_t)N1 * N2));
        const int ii[3] = {i1, i2, i3};
        int lo[3], c[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = w.d[d].lo[ii[d]];
            c[d] = w.d[d].cnt[ii[d]];
        }
        // weighted test values times trial values, per direction and offset
        for (int idx = tid; idx < 3 * O * PW; idx += 256) {
            const int d = idx / (O * PW), o = (idx / PW) % O, q = idx % PW;
            const int j = ii[d] + o - P;
            double vn = 0.0, vd = 0.0;
            if (q < c[d] && j >= 0 && j < w.d[d].N) {
                const int pt = lo[d] + q, a = j - w.d[d].eq[pt];
                if (a >= 0 && a < n) {
                    vn = w.d[d].w00[(int64_t)ii[d] * PW + q] * w.d[d].Bv[(int64_t)pt * n + a];
                    vd = w.d[d].w11[(int64_t)ii[d] * PW + q] * w.d[d].dB[(int64_t)pt * n + a];
                }
            }
            T[(d * 2 + 0) * O * PW + o * PW + q] = vn;
            T[(d * 2 + 1) * O * PW + o * PW + q] = vd;
        }
        __syncthreads();
        // stage x: item (q2, q3)
        for (int it = tid; it < c[1] * c[2]; it += 256) {
            const int q2 = it % c[1], q3 = it / c[1];
            const double* kr = kappa + ((int64_t)(lo[2] + q3) * np2 + (lo[1] + q2)) * np1 + lo[0];
            double en[O], ed[O];
#pragma unroll
            for (int o = 0; o < O; ++o) en[o] = ed[o] = 0.0;
            for (int q1 = 0; q1 < c[0]; ++q1) {
                const double k = kr[q1];
#pragma unroll
                for (int o = 0; o < O; ++o) {
                    en[o] += T[(0 * 2 + 0) * O * PW + o * PW + q1] * k;
                    ed[o] += T[(0 * 2 + 1) * O * PW + o * PW + q1] * k;
                }
            }
#pragma unroll
            for (int o = 0; o < O; ++o) {
                E[(0 * O + o) * PW * PW + q3 * PW + q2] = en[o];
                E[(1 * O + o) * PW * PW + q3 * PW + q2] = ed[o];
            }
        }
        __syncthreads();
        // stage y: item (o1, q3)
        for (int it = tid; it < O * c[2]; it += 256) {
            const int o1 = it % O, q3 = it / O;
            const double* en = E + (0 * O + o1) * PW * PW + q3 * PW;
            const double* ed = E + (1 * O + o1) * PW * PW + q3 * PW;
            double f0[O], f1[O];
#pragma unroll
            for (int o = 0; o < O; ++o) f0[o] = f1[o] = 0.0;
            for (int q2 = 0; q2 < c[1]; ++q2) {
                const double a = en[q2], b = ed[q2];
#pragma unroll
                for (int o = 0; o < O; ++o) {
                    const double tn = T[(1 * 2 + 0) * O * PW + o * PW + q2];
                    const double td = T[(1 * 2 + 1) * O * PW + o * PW + q2];
                    f0[o] += tn * a;
                    f1[o] += td * a + tn * b;
                }
            }
#pragma unroll
            for (int o = 0; o < O; ++o) {
                F[(0 * O + o1) * O * PW + o * PW + q3] = f0[o];
                F[(1 * O + o1) * O * PW + o * PW + q3] = f1[o];
            }
        }
        __syncthreads();
        // stage z: item (o1, o2); the values go to their row positions
        const int bl1 = band_lo(i1, P), bl2 = band_lo(i2, P), bl3 = band_lo(i3, P);
        const int Lx = band_len(i1, P, rm.N[0]), Ly = band_len(i2, P, rm.N[1]), Lz = band_len(i3, P, rm.N[2]);
        for (int it = tid; it < O * O; it += 256) {
            const int o1 = it % O, o2 = it / O;
            const double* f0 = F + (0 * O + o1) * O * PW + o2 * PW;
            const double* f1 = F + (1 * O + o1) * O * PW + o2 * PW;
            double m[O], k[O];
#pragma unroll
            for (int o = 0; o < O; ++o) m[o] = k[o] = 0.0;
            for (int q3 = 0; q3 < c[2]; ++q3) {
                const double a = f0[q3], b = f1[q3];
#pragma unroll
                for (int o = 0; o < O; ++o) {
                    const double tn = T[(2 * 2 + 0) * O * PW + o * PW + q3];
                    const double td = T[(2 * 2 + 1) * O * PW + o * PW + q3];
                    m[o] += tn * a;
                    k[o] += tn * b + td * a;
                }
            }
            const int j1 = i1 + o1 - P, j2 = i2 + o2 - P;
            const bool ok12 = j1 >= 0 && j1 < rm.N[0] && j2 >= 0 && j2 < rm.N[1];
#pragma unroll
            for (int o = 0; o < O; ++o) {
                const int j3 = i3 + o - P;
                const int pos = ok12 && j3 >= 0 && j3 < rm.N[2] ? ((j3 - bl3) * Ly + (j2 - bl2)) * Lx + (j1 - bl1) : O3;
                RW[pos] = m[o];
                RW[O3 + 1 + pos] = k[o];
            }
        }
        __syncthreads();
        const int64_t rs = rm.row_start(i1, i2, i3);
        const int L = Lx * Ly * Lz;
        for (int i = tid; i < L; i += 256) {
            if (Mv) Mv[rs + i] = RW[i];
            if (Kv) Kv[rs + i] = RW[O3 + 1 + i];
        }
        __syncthreads();   // T, E, F and the staged row are rewritten by the next row
    }
}

template <int P>
static int launch_wq_t(const WqDev& w, const PatchDev& pd, const double* kappa, double* Mv, double* Kv,
                       hipStream_t st)
{
    const int64_t lds = wq_lds_doubles<P>(w.PW) * (int64_t)sizeof(double);
    if (lds > 160 * 1024) return -4;
    if (hipFuncSetAttribute((const void*)k_wq_rows<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
        return -3;
    int64_t blocks = pd.ndof < 16384 ? pd.ndof : 16384;
    hipLaunchKernelGGL(k_wq_rows<P>, dim3((unsigned)blocks), dim3(256), (unsigned)lds, st, w, make_rowmap(pd), kappa,
                       Mv, Kv, pd.ndof);
    return hipGetLastError() == hipSuccess ? 0 : -3;
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
