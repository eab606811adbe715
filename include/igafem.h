/*
 * igafem.h -- C ABI of the MI355X (gfx950) B-spline element-integration library.
 *
 * The library integrates 3D tensor-product B-spline basis functions element
 * by element (Woźniak, Szyszka, Rojas: "A study of efficient concurrent
 * integration methods of B-Spline basis functions in IGA-FEM", arXiv
 * 2207.00280) and assembles the global matrices:
 *
 *   mass       M_IJ = int kappa phi_I phi_J            (Gram matrix, eq. mass_term / eq. 88)
 *   stiffness  K_IJ = int kappa grad phi_I . grad phi_J (from the weak form, eq. weak_space)
 *
 * with phi_I(x) = N_i(x1) N_j(x2) N_k(x3) (eq. basis_construction), each N a
 * Cox-de Boor B-spline (eqs. cox1/cox2) on an open knot vector (eq.
 * knot_vector), integrated by the tensor Gauss rule of eq. (10).  The
 * coefficient kappa is given at every quadrature point and enters eq. (10)
 * in the slot of J(x^n), next to the element Jacobian.  Around that it
 * provides the adjoint dL/dkappa, the matrix-free operator apply and one
 * forward Euler step of the heat problem (Sec. 2.2), a batched launch over
 * many patches, and the same calls on a mapped geometry (the *_geo entry
 * points, with the pulled-back coefficients given per point).
 *
 * CONVENTIONS (fixed where the paper leaves them open)
 *   - element e_d = 0..K_d-1 of direction d spans [t_d[e_d+p], t_d[e_d+p+1]]
 *     and carries the global functions e_d..e_d+p (Remark on element-by-element
 *     pre-computations); N_d = K_d + p functions per direction;
 *   - flat element index e = ex + Kx (ey + Ky ez);
 *   - local function index I = a1 + n (a2 + n a3), n = p+1 (x fastest);
 *   - global DOF index g = i + Nx (j + Ny k) (x fastest);
 *   - kappa and dL/dkappa: double [E][qz][qy][qx] (element-major, x fastest);
 *   - element matrices Me, Ke: double [E][n^3][n^3], row-major (row = test I);
 *   - CSR: row_ptr int64 [ndof+1], col_idx int32 [nnz], columns ascending.
 *     The pattern is structural: (I,J) is stored iff |i_d - j_d| <= p in every
 *     direction, numerically-zero entries included.  Values arrays are double
 *     [nnz] in that order.
 *
 * OWNERSHIP AND STREAMS
 *   The caller owns every array it passes.  Arguments named *_host are host
 *   memory; every other array is device memory on the current HIP device
 *   (e.g. from torch).  The library never frees caller memory.  A plan owns
 *   its device tables and releases them in igaf_plan_destroy.  Calls that
 *   take a `stream` (a hipStream_t, NULL = the legacy default stream) are
 *   asynchronous: argument checks run on the host and return before any
 *   launch; the kernels are queued on `stream` with no host synchronisation.
 *   A plan may be used from one host thread at a time.
 *
 * ERRORS
 *   Every igaf_status is IGAF_OK (0) or negative, and igaf_last_error()
 *   returns a thread-local message describing the last failure on this
 *   thread.  Argument errors (IGAF_EINVAL, IGAF_EUNSUPPORTED) are found
 *   before anything is launched, so outputs are untouched; after
 *   IGAF_EDEVICE the outputs are undefined; after IGAF_ENOCONV they hold the
 *   last iterate.
 *
 * PRECISION: FP64 throughout.  Supported hot-kernel shapes: 1 <= p <= 5 with
 * nquad = p+1 in every direction (other Gauss orders are rejected with
 * IGAF_EUNSUPPORTED by the integration calls; plan creation accepts 1..16).
 */
#ifndef IGAFEM_H
#define IGAFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t igaf_status;
#define IGAF_OK            0
#define IGAF_EINVAL       (-1) /* invalid argument (null pointer, bad size, bad knots) */
#define IGAF_ENOMEM       (-2) /* device or host allocation failed */
#define IGAF_EDEVICE      (-3) /* a HIP call or kernel launch failed */
#define IGAF_EUNSUPPORTED (-4) /* valid input outside what the kernels implement */
#define IGAF_ENOCONV      (-5) /* an iteration stopped at its limit before its tolerance */

#define IGAF_MAX_DEGREE 5
#define IGAF_MAX_QUAD   16

/* Integration algorithm (selects the algorithm, never the result). */
#define IGAF_CLASSICAL 0   /* Algorithm 1: every matrix value by a full q^3-point sum */
#define IGAF_SUMFACT   1   /* Algorithm 2 / eqs. finalsum, bufferC: contractions z, y, x */

/* How CSR values are formed (igaf_plan_set_assembly). */
#define IGAF_ASM_ROWS    0 /* default: owner-computes rows, on-chip reduction, no atomics */
#define IGAF_ASM_ATOMIC  1 /* element-by-element scatter-add with FP64 atomics */

typedef struct igaf_plan igaf_plan;
typedef struct igaf_batch igaf_batch;

/* One patch: the paper's problem statement (Sec. 2.3, 3.1): degree p, the
 * element grid, the knot vectors and the Gauss order per direction. */
typedef struct {
    int32_t degree;          /* p >= 1, the same in all directions */
    int32_t nelem[3];        /* K_x, K_y, K_z >= 1: knot spans between the end knots */
    const double* knots[3];  /* HOST, length nelem[d]+2p+1, nondecreasing: p+1 equal first
                                knots, p+1 equal last knots; an interior knot may repeat up to
                                p+1 times (continuity C^{p-m} at multiplicity m).  Element e_d
                                is the span [t[e_d+p], t[e_d+p+1]]; a span of zero length is
                                still an element (it keeps its kappa entries and its place in
                                every layout) but has zero Gauss weights and contributes
                                nothing. */
    int32_t nquad[3];        /* Gauss-Legendre points per direction, 1..IGAF_MAX_QUAD */
} igaf_patch_desc;

/* Library version string (static storage). */
const char* igaf_version(void);

/* Message for the last non-OK status returned on the calling thread
 * (static thread-local storage, valid until the next failing call). */
const char* igaf_last_error(void);

/* ---------------------------------------------------------------- host-only
 * These touch no GPU. */

/* Check a patch description (knot vector form, sizes, degree, Gauss order).
 * Returns IGAF_OK or IGAF_EINVAL. */
igaf_status igaf_desc_check(const igaf_patch_desc* desc);

/* Sizes implied by a description: ndof = prod_d (K_d+p); nelem = prod_d K_d;
 * nqp = prod_d q_d points per element; elem_dim = (p+1)^3; nnz of the
 * structural CSR pattern = prod_d (N_d (2p+1) - p (p+1)).  Any output may be
 * NULL. */
igaf_status igaf_desc_sizes(const igaf_patch_desc* desc, int64_t* ndof, int64_t* nelem,
                            int64_t* nqp, int64_t* elem_dim, int64_t* nnz);

/* The run of elements of direction `dir` (0..2) whose basis tables the plan
 * shares (Sec. 2.3: the values on an element depend only on the 2p knots
 * around its span, relative to the span): the longest run [*first, *end) of
 * consecutive elements whose knot differences t[e+j] - t[e+p], j = 1..2p,
 * agree with those of element *first up to 8 eps times the largest knot
 * involved.  A plan gives every element of the run the tables computed for
 * element *first, bit for bit (uniform spacing: all elements but the p - 1
 * nearest each end).  *first = *end = 0 when no two neighbours agree.
 * Returns IGAF_EINVAL for a bad description, dir or NULL output. */
igaf_status igaf_desc_shared_run(const igaf_patch_desc* desc, int dir, int* first, int* end);

/* The structural CSR pattern computed on the host into HOST arrays
 * row_ptr_host[ndof+1], col_idx_host[nnz]. */
igaf_status igaf_csr_pattern_host(const igaf_patch_desc* desc, int64_t* row_ptr_host,
                                  int32_t* col_idx_host);

/* ---------------------------------------------------------------- plans */

/* Validate `desc`, build the Gauss rule and the per-element 1D tables on the
 * current device (Cox-de Boor values and derivatives at the mapped Gauss
 * nodes, weights w*h/2 folded in, pair products N_a N_b and N_a' N_b' for the
 * (p+1)(p+2)/2 unordered pairs of each element and direction), and per
 * direction the banded Cholesky factor of the 1D mass matrix (the Euler
 * step's preconditioner).  The knot arrays are copied; the caller may free
 * them afterwards.  Synchronous (blocks until the tables are built).  *out
 * receives the plan. */
igaf_status igaf_plan_create(const igaf_patch_desc* desc, igaf_plan** out);

/* Release a plan and its device memory (NULL is ignored).  The caller must
 * make sure no queued work still uses the plan. */
void igaf_plan_destroy(igaf_plan* plan);

/* Sizes of the plan's patch (see igaf_desc_sizes). */
igaf_status igaf_plan_sizes(const igaf_plan* plan, int64_t* ndof, int64_t* nelem, int64_t* nqp,
                            int64_t* elem_dim, int64_t* nnz);

/* Mapped Gauss nodes x_host[K_d][q_d] of direction `dir` (0,1,2) and the
 * weights w_host[K_d][q_d] = w_k h_e/2 (w_host may be NULL), so that a caller
 * can evaluate kappa at the physical quadrature points (eq. 10). */
igaf_status igaf_quad_nodes(const igaf_plan* plan, int32_t dir, double* x_host, double* w_host);

/* Every quadrature point of the patch, xyz_host[E][qz][qy][qx][3] (HOST,
 * E q^3 3 doubles, caller-owned), in the layout of kappa: (x, y, z) of the
 * mapped Gauss nodes, e = ex + Kx (ey + Ky ez). */
igaf_status igaf_quad_points(const igaf_plan* plan, double* xyz_host);

/* Choose how CSR values are formed by the calls below (IGAF_ASM_ROWS or
 * IGAF_ASM_ATOMIC).  Both give the same matrix up to rounding order;
 * IGAF_ASM_ROWS is deterministic. */
igaf_status igaf_plan_set_assembly(igaf_plan* plan, int32_t mode);

/* Measurement: with enable != 0, igaf_integrate_assemble records HIP timing
 * events around each kernel it launches (element kernel on the caller's
 * stream, CSR kernel on the stream it runs on; nothing is recorded while a
 * stream is being captured).  Enabling or disabling waits for the device and
 * clears the log. */
igaf_status igaf_plan_set_timing(igaf_plan* plan, int32_t enable);

/* Average duration in ms and number of logged launches of `kernel`
 * (0 = element-matrix kernel, 1 = CSR kernel) since timing was enabled;
 * waits for the logged events. */
igaf_status igaf_plan_timing(igaf_plan* plan, int32_t kernel, double* avg_ms, int32_t* count);

/* ---------------------------------------------------------------- device calls */

/* Fill the structural CSR pattern into DEVICE arrays row_ptr[ndof+1] and
 * col_idx[nnz] (eq. mass_term gives the matrix; its pattern follows from the
 * (p+1)^3-function support of each element, Sec. 3.1 Remark). */
igaf_status igaf_csr_pattern(const igaf_plan* plan, int64_t* row_ptr, int32_t* col_idx,
                             void* stream);

/* Element matrices (eq. 88 integrated by eq. 10) for every element:
 * Me, Ke [E][n^3][n^3]; either may be NULL to skip it (not both).
 * kappa [E][q^3] is required.  method: IGAF_CLASSICAL (Algorithm 1) or
 * IGAF_SUMFACT (Algorithm 2). */
igaf_status igaf_element_matrices(const igaf_plan* plan, int32_t method, const double* kappa,
                                  double* Me, double* Ke, void* stream);

/* Global CSR values from stored element matrices (A = sum over elements of
 * A^gamma, Sec. 3.1; "insert local element into global"):  Mval, Kval [nnz]
 * are OVERWRITTEN.  A NULL output skips it; its input must then be NULL too.
 * Each CSR row is summed by one wavefront in element order (LDS adds in
 * issue order), so repeated calls give the same bits. */
igaf_status igaf_assemble(const igaf_plan* plan, const double* Me, const double* Ke,
                          double* Mval, double* Kval, void* stream);

/* The hot path: integrate and assemble in one call.  Any of Me, Ke, Mval,
 * Kval may be NULL (at least one non-NULL); with Me = Ke = NULL the element
 * matrices are never materialised (streamed mode).  Mval/Kval are
 * OVERWRITTEN.  method as in igaf_element_matrices (the CSR values are formed
 * with the sum-factorised contractions in both cases). */
igaf_status igaf_integrate_assemble(const igaf_plan* plan, int32_t method, const double* kappa,
                                    double* Me, double* Ke, double* Mval, double* Kval,
                                    void* stream);

/* Mapped geometry: the integrals of eq. (10) on x = F(xi), pulled back to
 * the parameter cube.  The per-point factor J(x^n) of eq. (10) becomes, for
 * the mass, cm = kappa det J and, for the stiffness, the symmetric tensor
 * G = kappa det J J^-1 J^-T (J = dF/dxi), which the caller evaluates at the
 * quadrature points (igaf_quad_nodes gives them):
 *   M_e[I][J] = sum_q w_q cm_q phi_I phi_J
 *   K_e[I][J] = sum_q w_q grad_xi phi_I^T G_q grad_xi phi_J
 * cm   DEVICE [E][q^3] (required when Me or Mval is requested)
 * G    DEVICE [E][6][q^3]: per element six [qz][qy][qx] blocks, the
 *      components xx, yy, zz, xy, xz, yz (required when Ke or Kval is)
 * Me, Ke   DEVICE [E][n^3][n^3] or NULL;  Mval, Kval DEVICE [nnz] or NULL,
 *      OVERWRITTEN with the assembled CSR values (structural pattern of
 *      igaf_csr_pattern).  At least one output.  A CSR output whose element
 *      matrices are requested too is summed from them as in igaf_assemble.
 *      One without is computed by owner-computed rows: every value summed
 *      by one thread over the Gauss points of the elements its row and
 *      column share, contracted z -> y -> x (no workspace, no atomics, the
 *      same bits on every call, capturable).  The two ways agree to
 *      rounding, not bit for bit.
 * Sum factorisation (Algorithm 2) with ordered per-direction pairs (the
 * cross terms of G are not symmetric in a pair); nquad = degree+1 in every
 * direction, else IGAF_EUNSUPPORTED.  cm = kappa, G = kappa I (the identity
 * geometry) gives the matrices of igaf_integrate_assemble.  Asynchronous on
 * `stream`. */
igaf_status igaf_integrate_assemble_geo(const igaf_plan* plan, const double* cm, const double* G,
                                        double* Me, double* Ke, double* Mval, double* Kval,
                                        void* stream);

/* Nothing to prepare: igaf_integrate_assemble_geo allocates nothing on any
 * path (its CSR-only values come from the owner-computed rows kernel).  Kept
 * so that callers that prepared a plan before capturing it still work; it
 * only checks the plan (IGAF_EINVAL for NULL, IGAF_EUNSUPPORTED for a
 * quadrature order other than degree+1). */
igaf_status igaf_geo_prepare(igaf_plan* plan);

/* Adjoint of L(kappa) = alphaM u^T M(kappa) v + alphaK u^T K(kappa) v with
 * respect to kappa at every quadrature point (L is linear in kappa through
 * the J(x^n) slot of eq. 10):
 *   grad[e][q] = s * w_q (alphaM u_h v_h + alphaK grad u_h . grad v_h)(x_q),
 * u_h = sum_I u_I phi_I, s = scale * (*scale_dev) with scale_dev a DEVICE
 * scalar (double[1], read on the device when the kernel runs, e.g. the
 * incoming gradient of an autograd backward) or s = scale when scale_dev is
 * NULL.  u, v: device [ndof]; grad: device [E][q^3], OVERWRITTEN.  No element
 * matrix is formed or stored. */
igaf_status igaf_kappa_grad(const igaf_plan* plan, const double* u, const double* v,
                            double alphaM, double alphaK, double scale, const double* scale_dev,
                            double* grad, void* stream);

/* The value of that bilinear form,
 *   L[0] = alphaM u^T M(kappa) v + alphaK u^T K(kappa) v = sum_q kappa_q dL/dkappa_q
 * (Euler's identity for a function linear in kappa), computed matrix-free
 * with the adjoint's interpolation: each wavefront sums kappa_q dL/dkappa_q
 * over its points into a partial-sum buffer the plan owns (4096 doubles,
 * allocated with the plan), and one workgroup adds the partials; every sum
 * runs in a fixed order, so repeated calls give the same bits.  kappa:
 * device [E][q^3]; u, v: device [ndof]; L: DEVICE double[1], OVERWRITTEN.
 * Calls on one plan that overlap (other streams or threads) race on the
 * partial sums. */
igaf_status igaf_bilinear_form(const igaf_plan* plan, const double* kappa, const double* u, const double* v,
                               double alphaM, double alphaK, double* L, void* stream);

/* Matrix-free operator apply, the step after assembly that an explicit time
 * step takes (the forward Euler step of Sec. 2.2, in the matrix form of
 * Sec. 2.4, needs M u and K u):
 *   y = alphaM M(kappa) u + alphaK K(kappa) u
 * computed element by element by sum factorisation (interpolate u and
 * grad u to the quadrature points, weight by kappa w, contract back against
 * the test functions; the element sum of Sec. 3.1), with no element or
 * global matrix formed.  kappa: device [E][q^3]; u, y: device [ndof]; y is
 * OVERWRITTEN and must not overlap u.  work: device scratch of
 * igaf_apply_workspace(plan) doubles, overwritten (each run of elements
 * along x writes its DOF values there; each y_I is then summed from them in
 * a fixed order, so repeated calls give the same bits).  Calls that overlap
 * on one `work` race.  alphaK == 0 takes a mass-only kernel that neither
 * interpolates nor contracts grad u (so non-finite gradients of u do not
 * reach y).  Needs nquad = degree + 1 in every direction. */
int64_t igaf_apply_workspace(const igaf_plan* plan);
igaf_status igaf_apply(const igaf_plan* plan, const double* kappa, const double* u,
                       double alphaM, double alphaK, double* y, double* work, void* stream);

/* The operator apply of igaf_apply (same kernels, same bits) for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops): the runs' slots live in a static device array of the library
 * (64 MiB, 8 388 608 doubles, one per device, held until the process ends;
 * its address is looked up when a plan is created on the device), so the
 * call allocates nothing and takes no workspace.  Patches needing more than
 * that (igaf_apply_workspace(plan) > 8 388 608, e.g. beyond about 480 000
 * elements at p = 3) are rejected with IGAF_EUNSUPPORTED before any launch.
 * Every call on one device shares the array and leaves its last contents
 * there (nothing in it needs clearing: each call writes every slot value it
 * reads): calls that overlap on one device (other streams or threads) race. */
igaf_status igaf_apply_static(const igaf_plan* plan, const double* kappa, const double* u,
                              double alphaM, double alphaK, double* y, void* stream);

/* The operator apply on a mapped geometry (the coefficients of
 * igaf_integrate_assemble_geo): y = alphaM M u + alphaK K u with
 *   M_IJ = sum_q w_q cm_q phi_I phi_J,  K_IJ = sum_q w_q grad_xi phi_I^T G_q grad_xi phi_J.
 * cm [E][q^3], G [E][6][q^3] (xx yy zz xy xz yz), u, y device [ndof]; y is
 * OVERWRITTEN and must not overlap u; work as in igaf_apply (same size,
 * same fixed-order sums). */
igaf_status igaf_apply_geo(const igaf_plan* plan, const double* cm, const double* G, const double* u,
                           double alphaM, double alphaK, double* y, double* work, void* stream);

/* The adjoint on a mapped geometry where kappa scales both coefficients,
 * cm = kappa cm0 and G = kappa G0 (cm0 = det J, G0 = det J J^-1 J^-T):
 * for L = alphaM u^T M(kappa) v + alphaK u^T K(kappa) v,
 *   grad[e][q] = scale * w_q (alphaM cm0 u_h v_h + alphaK grad u_h^T G0 grad v_h)(x_q).
 * cm0 [E][q^3], G0 [E][6][q^3], u, v device [ndof], grad device [E][q^3]
 * OVERWRITTEN. */
igaf_status igaf_kappa_grad_geo(const igaf_plan* plan, const double* cm0, const double* G0, const double* u,
                                const double* v, double alphaM, double alphaK, double scale, double* grad,
                                void* stream);

/* One forward Euler step of the heat problem (Sec. 2.2, eq. Euler; the
 * matrix form of Sec. 2.4) with the coefficient kappa in both integrals:
 *   M(kappa) mu_next = M(kappa) mu - dt K(kappa) mu.
 * The right-hand side is one igaf_apply; the mass system (symmetric positive
 * definite) is solved by conjugate gradients started from mu, each iteration
 * one matrix-free mass apply, until ||r|| <= tol ||b|| or after maxit
 * iterations (then IGAF_ENOCONV, mu_next holding the last iterate).
 * precond: IGAF_PRECOND_NONE (plain CG) or IGAF_PRECOND_KRON: CG
 * preconditioned by P = S (Mz (x) My (x) Mx) S, the Kronecker product of the
 * 1D mass matrices of the plan (kappa = 1; each applied through its banded
 * Cholesky factor, one sequential solve per grid line) scaled by
 * S = diag(M(kappa))^1/2 / diag(Mz (x) My (x) Mx)^1/2, which carries the
 * coefficient's variation.
 * kappa: device [E][q^3]; mu, mu_next: device [ndof] (may be the same
 * array); work: device scratch of igaf_euler_workspace(plan) doubles,
 * overwritten.  Every reduction (the applies, the diagonal of M(kappa), the
 * dot products) runs in a fixed order, so repeated steps give the same
 * bits.  iters, relres: HOST outputs (iterations taken, final
 * ||r|| / ||b|| of the recursively updated residual), either may be NULL.
 * Synchronous: it reads the residual of every iteration back through a
 * pinned slot of the plan (while the GPU runs the next iteration's work up
 * to its update of mu_next) and returns when the step is done; the work
 * after the last iteration may still run on `stream` then, touching only
 * `work`.  Calls on one plan that overlap (other threads or streams) race on
 * that slot.  Needs nquad = degree + 1 in every direction. */
enum { IGAF_PRECOND_NONE = 0, IGAF_PRECOND_KRON = 1 };
int64_t igaf_euler_workspace(const igaf_plan* plan);
igaf_status igaf_euler_step(const igaf_plan* plan, const double* kappa, const double* mu, double dt,
                            double tol, int32_t maxit, int32_t precond, double* mu_next, double* work,
                            int32_t* iters, double* relres, void* stream);

/* The same step on a mapped geometry: M from the mass coefficient cm, K from
 * the stiffness tensor G (the coefficients of igaf_integrate_assemble_geo);
 * the preconditioner's diagonal scaling takes diag(M(cm)).  Arguments as in
 * igaf_euler_step, with cm [E][q^3] and G [E][6][q^3] in place of kappa. */
igaf_status igaf_euler_step_geo(const igaf_plan* plan, const double* cm, const double* G, const double* mu,
                                double dt, double tol, int32_t maxit, int32_t precond, double* mu_next,
                                double* work, int32_t* iters, double* relres, void* stream);

/* ---------------------------------------------------------------- weighted quadrature
 * The variant of sum factorisation the paper names as reaching O(p^6)
 * (Sec. 1, "Sum factorization"): weighted quadrature, after F. Calabro,
 * G. Sangalli, M. Tani, "Fast formation of isogeometric Galerkin matrices by
 * weighted quadrature", CMAME 316 (2017).  The test function moves into the
 * weights: per direction every basis function B_i has its own rule over
 * fixed points inside its support (two per element at its quarter points,
 * p+1 points in the first and the last element, at a + h (r+1/2)/(p+1)),
 * with the minimum-norm weights exact for its products with every trial
 * function (sum_q w00_iq B_j(x_q) = int B_i B_j, sum_q w11_iq B_j'(x_q) =
 * int B_i' B_j').  With kappa given on the tensor grid of those points,
 *   M_IJ = sum_q w00[i1][q1] w00[i2][q2] w00[i3][q3] kappa(q) B_j1(q1) B_j2(q2) B_j3(q3)
 *   K_IJ = sum_q kappa(q) sum_d (w11 B' in direction d, w00 B in the other two)
 * (exact Galerkin matrices for kappa = 1).  Open knot vectors with elements
 * of positive length; nquad = degree+1 (the plan's Gauss rule forms the
 * exact 1D integrals). */

/* Build the rules of every direction (synchronous; host work O(N p^3) and
 * a device allocation the plan owns, released with it).  IGAF_EUNSUPPORTED
 * for a knot vector with a repeated interior knot.  Calling it again is a
 * no-op. */
igaf_status igaf_wq_prepare(igaf_plan* plan);

/* The points of direction dir (0, 1, 2) after igaf_wq_prepare: *npts
 * receives their number and x_host (HOST, may be NULL) the coordinates in
 * increasing order. */
igaf_status igaf_wq_points(const igaf_plan* plan, int32_t dir, int64_t* npts, double* x_host);

/* CSR values of M and K by weighted quadrature.  kappa: DEVICE
 * [npts_z][npts_y][npts_x] (x fastest) at the points of igaf_wq_points;
 * Mval, Kval: DEVICE [nnz], OVERWRITTEN (structural pattern of
 * igaf_csr_pattern), either may be NULL (not both).  One workgroup per CSR
 * row sums its values over the row's point box; deterministic.  Asynchronous
 * on `stream`; IGAF_EINVAL before igaf_wq_prepare. */
igaf_status igaf_wq_assemble(const igaf_plan* plan, const double* kappa, double* Mval, double* Kval,
                             void* stream);

/* ---------------------------------------------------------------- batches
 * Many independent patches (the paper's first concurrency level: parts of
 * the mesh computed concurrently) integrated and assembled to CSR (streamed
 * mode, M and K) by one kernel launch per degree present (each degree's tile
 * has its own block size and LDS): one workgroup per (patch, tile of row
 * pencils, x segment) item of that degree's work list, sorted longest first.
 * Per degree the launch has a configuration: the tile shape (0: the shape of
 * the single-patch kernel, 1: a second one, smaller for p <= 4 and for p = 5
 * three pencils without the split stage x), the x segments per tile (1, 2,
 * 4, 8) and the items per XCD chunk (4, 16, 64); every combination has its
 * own immutable work list, built at creation. */

/* Build per-patch plans, the device patch table and the work lists of every
 * configuration (synchronous; every degree starts with tile shape 0, one
 * segment per tile and 16 items per XCD chunk until igaf_batch_autotune or
 * igaf_batch_set_split / igaf_batch_set_degree_config choose others).  descs: HOST array of npatch
 * descriptions. */
igaf_status igaf_batch_create(const igaf_patch_desc* descs, int32_t npatch, igaf_batch** out);

/* Release a batch (NULL is ignored). */
void igaf_batch_destroy(igaf_batch* batch);

/* The plan of patch i (owned by the batch; do not destroy). */
const igaf_plan* igaf_batch_plan(const igaf_batch* batch, int32_t i);

/* The launch shape: family (kind of work item; 0 = a tile of row pencils,
 * the only kind), grid (workgroups launched over all degrees, each degree's
 * item count rounded up to whole XCD chunks), number of work items, with
 * every degree's current configuration.  Any output may be NULL. */
igaf_status igaf_batch_info(const igaf_batch* batch, int32_t* family, int32_t* grid,
                            int32_t* nitems);

/* One launch per degree present, in order on `stream`: for every patch i,
 * Mval[i], Kval[i] (device [nnz_i])
 * are OVERWRITTEN with the assembled mass and stiffness values for kappa[i]
 * (device [E_i][q_i^3]).  kappa, Mval, Kval are HOST arrays of npatch device
 * pointers; Mval[i] / Kval[i] may be NULL to skip that matrix.  The pointer
 * tables are copied to the device on `stream` from a pinned staging buffer
 * the batch owns; when they differ from the previous call the host first
 * waits for `stream`.  The call may be captured in a HIP graph once it has
 * run eagerly with the same pointers (changing them during capture returns
 * IGAF_EINVAL).  A replay keeps the configurations it was captured with
 * (each has its own immutable work list) but copies the pointer tables the
 * batch holds at replay time, i.e. those of the latest call: after an eager
 * call with other pointers, replays read and write those arrays.
 * Overlapping calls on one batch from different streams race. */
igaf_status igaf_batch_integrate_assemble(igaf_batch* batch, const double* const* kappa,
                                          double* const* Mval, double* const* Kval,
                                          void* stream);

/* The comparison path: the same work as npatch separate per-patch launches
 * of igaf_integrate_assemble (streamed mode) on `stream`. */
igaf_status igaf_batch_integrate_assemble_separate(igaf_batch* batch,
                                                   const double* const* kappa,
                                                   double* const* Mval, double* const* Kval,
                                                   void* stream);

/* Autotuner of the batched launch (synchronous; not under stream capture).
 * For every degree present, one at a time (the degrees' launches are
 * independent), every configuration is timed on the caller's arrays: tile
 * shape (0 or 1), x segments per tile (1, 2, 4 or 8, never below 2(p+1) rows
 * per segment; a segment that does not start at the patch boundary sweeps p
 * warm-up elements first: shorter items against more warm-up) and items per
 * XCD chunk (4, 16 or 64: L2 sharing between neighbouring tiles against
 * balance); one warm-up launch, then `reps` launches (1..100, HIP events on
 * `stream`), the median kept; the fastest configuration of each degree is
 * used by every later igaf_batch_integrate_assemble.  Mval, Kval are
 * overwritten, with the same values every time: each CSR value is summed in
 * one thread in a fixed order whatever the tile shape or split. */
igaf_status igaf_batch_autotune(igaf_batch* batch, const double* const* kappa, double* const* Mval,
                                double* const* Kval, int32_t reps, void* stream);

/* Set every degree to tile shape 0 with this split in {1, 2, 4, 8} and chunk
 * in {4, 16, 64} (else IGAF_EINVAL).  Host-only; later calls use it. */
igaf_status igaf_batch_set_split(igaf_batch* batch, int32_t split, int32_t chunk);

/* Set one degree's configuration (tile 0 or 1, split, chunk as above), e.g.
 * to reuse an earlier tuning.  Host-only. */
igaf_status igaf_batch_set_degree_config(igaf_batch* batch, int32_t degree, int32_t tile, int32_t split,
                                         int32_t chunk);

/* One degree's configuration, the autotuner's median launch time for it (0
 * when not tuned) and its number of work items.  Any output may be NULL. */
igaf_status igaf_batch_degree_config(const igaf_batch* batch, int32_t degree, int32_t* tile, int32_t* split,
                                     int32_t* chunk, double* tuned_ms, int32_t* nitems);

/* The split and chunk of the highest degree present and the sum of the
 * degrees' tuned launch times (0 before tuning).  Any output may be NULL. */
igaf_status igaf_batch_split(const igaf_batch* batch, int32_t* split, int32_t* chunk, double* tuned_ms);

#ifdef __cplusplus
}
#endif

#endif /* IGAFEM_H */
