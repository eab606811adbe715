// Weighted quadrature (the rules of Calabro, Sangalli and Tani, 2017): the
// per-direction rules built on the host, their device tables and the CSR
// kernel's launch.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "common.h"

namespace igaf {

// ---- weighted quadrature
constexpr int kWqMaxP = 5;

// The rules of one direction on the host: points x (npts) with their
// element eq; per function g the points inside its support are
// [lo[g], lo[g] + cnt[g]) and its weights w00/w11[g * PW + q]; the trial
// values Bv/dB[q * (p+1) + a] of the functions eq[q] + a at every point.
struct WqHost {
    std::vector<double> x, w00, w11, Bv, dB;
    std::vector<int> eq, lo, cnt;
    int N = 0, npts = 0, PW = 0;
};
// Build them from the knots t and the plan's Gauss nodes/weights xg, wg
// ([K][p+1], for the exact integrals).  0, -1 (an element of zero length) or
// -2 (a rule's system is singular).
int wq_build_dir(int p, int K, const double* t, const double* xg, const double* wg, WqHost& out);

// The same tables in device memory (w00, w11 padded to the common width PW),
// and the products the kernel uses: TN[g][o][q] = w00[g][q] B_j(x_q),
// TD[g][o][q] = w11[g][q] B_j'(x_q) for the column j = g + o - p of every
// offset o (zero where j is outside the patch or x_q outside supp(B_j))
struct WqDir {
    const double* w00;
    const double* w11;
    const double* Bv;
    const double* dB;
    const double* TN;
    const double* TD;
    const int* lo;
    const int* cnt;
    const int* eq;
    int N, npts;
};
struct WqDev {
    WqDir d[3];
    int PW;
    const int* h_lo0;    // HOST copies of direction x's lo and cnt (launch sizing)
    const int* h_cnt0;
};
// CSR values (overwritten; either output may be null) by weighted
// quadrature, kappa [npts_z][npts_y][npts_x]; -4 if the LDS of a row exceeds
// the CU's.
int launch_wq(const WqDev& w, const PatchDev& pd, const double* kappa, double* Mv, double* Kv, hipStream_t st);

}  // namespace igaf
