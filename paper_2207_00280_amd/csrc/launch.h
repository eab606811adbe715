// Internal launchers (host side of each kernel file).  All return 0 on
// success, -3 on a launch failure, -4 for an unsupported shape.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace igaf {

int launch_basis_tables(int p, const double* t, int K, const double* xi, const double* wr, int Q,
                        double* Wnn, double* Wdd, double* Nv, double* dN, double* wq, double* Wg,
                        int r0, int r1, hipStream_t st);

int launch_csr_pattern(const PatchDev& pd, int64_t* row_ptr, int32_t* col, hipStream_t st);

// Element matrices (dense, [E][n^3][n^3]) by sum factorisation or classical
// quadrature; with Mval/Kval non-null the element values are also
// scatter-added into the CSR values with FP64 atomics (which must be zeroed
// first).
int launch_element(const PatchDev& pd, int method, const double* kappa, double* Me, double* Ke,
                   double* Mval_atomic, double* Kval_atomic, hipStream_t st);

// CSR values by owner-computes rows (no atomics), one workgroup per tile of
// row pencils: overwrites Mval / Kval.
int launch_rows(const PatchDev& pd, const double* kappa, double* Mval, double* Kval,
                hipStream_t st);

// The same on a mapped geometry (point fields cm [E][q^3], G [E][6][q^3]; a
// NULL output needs no field): overwrites Mval / Kval.  -4 for degrees whose
// tile does not fit the LDS of a CU (p = 5).
int launch_rows_geo(const PatchDev& pd, const double* cm, const double* G, double* Mval, double* Kval,
                    hipStream_t st);

// Batched CSR rows of the degree-p patches: one workgroup per (patch, tile,
// x segment, segment length) item of `items` (all of degree p), which the
// host sorts longest first, `chunk` consecutive items per XCD; `variant`
// selects the tile shape (0: the standalone kernel's, 1: the second shape of
// the degree, kTileVariants in all).  rows_batch_grid is the launch's workgroup count,
// rows_tile_info the tiles of a patch and the relative cost of one element
// step of a tile of that variant.
constexpr int kTileVariants = 2;
int launch_rows_batch(int p, int variant, const BatchPatch* patches, const int4* items, int nitems, int chunk,
                      hipStream_t st);
int rows_batch_grid(int nitems, int chunk);
int rows_tile_info(int p, int variant, int Ny, int Nz, int* ntile, double* per_elem);

// CSR values gathered from stored element matrices: overwrites Mval / Kval.
int launch_gather(const PatchDev& pd, const double* Me, const double* Ke, double* Mval,
                  double* Kval, hipStream_t st);

int launch_fill_zero(double* a, int64_t n, hipStream_t st);

// Workgroups of `kernel` (launched with `threads` threads and no dynamic LDS)
// that the current device runs at once: compute units times the occupancy.
// Cached per (device, kernel); returns 0 if the device cannot be queried.
int device_slots(const void* kernel, int threads);

// element matrices on a mapped geometry: cm [E][q^3], G [E][6][q^3]
int launch_element_geo(const PatchDev& pd, const double* cm, const double* G, double* Me, double* Ke,
                       hipStream_t st);
// y = alphaM M(kappa) u + alphaK K(kappa) u (overwritten; no atomics: each
// x-run of elements writes its DOF values to its slot of W, then one thread
// per DOF sums the slots in a fixed order); with G, kappa is the mass
// coefficient cm and G the stiffness tensor; with diag, y = alphaM
// diag(M(kappa)) and u is not read.  W: apply_workspace_doubles(pd) doubles.
int64_t apply_workspace_doubles(const PatchDev& pd);
// The static device scratch of the allocation-free apply: look up its
// address on the current device (once per device; 0 or -3), and get it
// (nullptr before the lookup) with its capacity in doubles.
int apply_scratch_init();
double* apply_scratch(int64_t* capacity);
int launch_apply(const PatchDev& pd, const double* kappa, const double* u, double alphaM, double alphaK,
                 double* y, double* W, hipStream_t st, const double* G = nullptr, bool diag = false);

// Forward Euler step: b = M mu - dt K mu, then CG on M x = b from x = mu.
// rb: pinned host slot for the residual read-back, ev: an event for it.
// Returns 0 (converged), 1 (maxit reached) or -3.
int64_t euler_workspace_doubles(const PatchDev& pd, int64_t ndof);
int run_euler_step(const PatchDev& pd, int64_t ndof, const double* kappa, const double* mu, double dt,
                   double tol, int maxit, int precond, double* x, double* work, int* iters, double* relres,
                   hipStream_t st, double* rb, hipEvent_t ev, const double* G = nullptr);

int launch_kappa_grad(const PatchDev& pd, const double* u, const double* v, double alphaM,
                      double alphaK, double scale, const double* scale_dev, double* grad, hipStream_t st,
                      const double* cm0 = nullptr, const double* G0 = nullptr);

// L[0] = alphaM u^T M(kappa) v + alphaK u^T K(kappa) v = sum_q kappa_q g_q by
// the adjoint's interpolation: per-wavefront partial sums into part
// (kLossParts doubles), then one workgroup sums them in a fixed order.
constexpr int kLossParts = 4096;
int launch_bilinear(const PatchDev& pd, const double* kappa, const double* u, const double* v, double alphaM,
                    double alphaK, double* L, double* part, hipStream_t st);

}  // namespace igaf
