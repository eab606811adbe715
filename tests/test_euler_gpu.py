"""One forward Euler step (igaf_euler_step): M(kappa) mu_next = M(kappa) mu -
dt K(kappa) mu, right-hand side by the matrix-free apply, mass system by
conjugate gradients.

Checked against a direct solve with the oracle's assembled matrices (the
error bound of a linear solve: relative error <= cond(M) x relative
residual), against the conservation law of the heat problem with the
Neumann boundary of Sec. 2.1 (1^T K = 0, so 1^T M mu is kept up to the CG
residual), and for its edge cases.
"""
import math

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import nonuniform_knots, relfro, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ig():
    import torch

    assert torch.cuda.is_available()
    from paper_2207_00280_amd import igafem

    return igafem


@pytest.mark.parametrize("precond", ["none", "kron"])
@pytest.mark.parametrize("p,K,uniform", [(1, (6, 5, 4), False), (2, (5, 4, 4), True),
                                         (3, (5, 4, 3), False), (4, (3, 3, 2), True),
                                         (5, (2, 3, 2), "repeated")])
def test_euler_vs_direct_solve(orc, ig, p, K, uniform, precond):
    """mu_next vs scipy's direct solve of M x = (M - dt K) mu with the oracle's
    matrices, within cond_2(M) times the CG's relative residual (+ rounding),
    with plain and with preconditioned CG."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    if uniform == "repeated":
        knots = [W.repeated_knots([0.4], [p], p), W.repeated_knots([0.3, 0.6], [1, p + 1], p),
                 W.open_uniform_knots(2, p)]
        K = tuple(len(t) - 2 * p - 1 for t in knots)
    else:
        knots = [W.open_uniform_knots(k, p) if uniform else nonuniform_knots(k, p, 7 * p + d)
                 for d, k in enumerate(K)]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    plan = ig.Plan(p, K, knots)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=21 + p)
    mu = W.normal_vector(P.ndof, 22 + p)
    rp, col, Mo, Ko = orc.assemble(P, kap)
    M = sp.csr_matrix((Mo, col, rp), shape=(P.ndof, P.ndof))
    Kk = sp.csr_matrix((Ko, col, rp), shape=(P.ndof, P.ndof))
    dt = 0.1 / max(K) ** 2
    ref = spla.spsolve(M.tocsc(), M @ mu - dt * (Kk @ mu))
    if p == 5 and precond == "none":
        # plain CG on the p = 5 mass matrix (condition number ~1e12) stalls far
        # above 1e-13: the step reports ENOCONV and leaves its last, finite,
        # iterate (the preconditioned solve covers p = 5 against the direct one)
        import torch

        out = torch.full((P.ndof,), float("nan"), dtype=torch.float64, device="cuda")
        with pytest.raises(ig.IgafError) as ei:
            plan.euler_step(to_dev(kap), to_dev(mu), dt, tol=1e-13, maxit=300, precond=ig.PRECOND_NONE, out=out)
        assert ei.value.status == ig.ENOCONV and "300 iterations" in str(ei.value)
        assert bool(torch.isfinite(out).all())
        return
    pc = ig.PRECOND_KRON if precond == "kron" else ig.PRECOND_NONE
    out, iters, relres = plan.euler_step(to_dev(kap), to_dev(mu), dt, tol=1e-13, maxit=5000, precond=pc)
    assert relres <= 1e-13 and iters > 0
    cond = np.linalg.cond(M.toarray())
    assert relfro(to_host(out), ref) <= cond * relres + 1e-13, (cond, relres)


def test_euler_conservation_and_edge_cases(ig):
    """48^3 elements, p=3, log-normal kappa: 1^T M mu_next = 1^T M mu up to
    |1^T r| <= sqrt(ndof) ||r||; in place equals out of place; a zero state
    stays zero; maxit reached raises ENOCONV."""
    import torch

    p, K = 3, (48, 48, 48)
    knots = [W.open_uniform_knots(k, p) for k in K]
    plan = ig.Plan(p, K, knots)
    kap = to_dev(W.kappa_lognormal(plan.nelem, plan.nqp, seed=31))
    mu = to_dev(W.normal_vector(plan.ndof, 32))
    dt = 0.1 / 48 ** 2
    tol = 1e-12
    out, iters, relres = plan.euler_step(kap, mu, dt, tol=tol, maxit=5000)
    assert relres <= tol
    m0 = to_host(plan.apply(kap, mu, 1.0, 0.0))
    m1 = to_host(plan.apply(kap, out, 1.0, 0.0))
    b = to_host(plan.apply(kap, mu, 1.0, -dt))
    s0, s1 = math.fsum(m0.tolist()), math.fsum(m1.tolist())
    bound = math.sqrt(plan.ndof) * relres * np.linalg.norm(b) + 1e-14 * math.fsum(np.abs(m0).tolist())
    assert abs(s1 - s0) <= bound, (s1 - s0, bound)
    # in place: mu_next over mu
    mu2 = mu.clone()
    _, it2, rr2 = plan.euler_step(kap, mu2, dt, tol=tol, maxit=5000, out=mu2)
    assert rr2 <= tol
    assert relfro(to_host(mu2), to_host(out)) <= 1e-11
    # zero state
    z, itz, rz = plan.euler_step(kap, torch.zeros_like(mu), dt)
    assert itz == 0 and float(torch.count_nonzero(z)) == 0
    # iteration limit
    with pytest.raises(ig.IgafError) as ei:
        plan.euler_step(kap, mu, dt, tol=1e-30, maxit=2)
    assert ei.value.status == ig.ENOCONV


def test_preconditioner_cuts_iterations(ig):
    """48^3 elements, p = 3, log-normal kappa: the Kronecker/diagonal-scaled
    preconditioner reaches the same tolerance in at most a fifth of plain
    CG's iterations, and both solutions agree within the bound of a linear
    solve (each within cond(M) times its residual of the exact solution;
    cond(M) is below 1e5 here)."""
    p, K = 3, (48, 48, 48)
    plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
    kap = to_dev(W.kappa_lognormal(plan.nelem, plan.nqp, seed=41))
    mu = to_dev(W.normal_vector(plan.ndof, 42))
    dt = 0.1 / 48 ** 2
    x0, it0, r0 = plan.euler_step(kap, mu, dt, tol=1e-11, maxit=20000, precond=ig.PRECOND_NONE)
    x1, it1, r1 = plan.euler_step(kap, mu, dt, tol=1e-11, maxit=20000, precond=ig.PRECOND_KRON)
    assert r0 <= 1e-11 and r1 <= 1e-11
    assert 5 * it1 <= it0, (it0, it1)
    assert relfro(to_host(x1), to_host(x0)) <= 2e5 * 1e-11


@pytest.mark.parametrize("p,K", [(1, (6, 5, 4)), (2, (5, 4, 4)), (3, (5, 4, 3)), (4, (3, 3, 2))])
def test_euler_geometry_vs_direct_solve(orc, ig, p, K):
    """Mapped geometry (curved map, log-normal kappa): mu_next vs scipy's direct
    solve with the oracle's geometry matrices, within cond_2(M) times the
    residual; 1^T M mu is conserved (K 1 = 0 on any geometry)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    knots = [nonuniform_knots(k, p, 40 * p + d) for d, k in enumerate(K)]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    plan = ig.Plan(p, K, knots)
    xs = [orc.quad_nodes(P, d)[0] for d in range(3)]
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=50 + p)
    cm, G = W.mapped_geometry(xs[0], xs[1], xs[2], kap, amp=0.1)
    mu = W.normal_vector(P.ndof, 60 + p)
    rp, col, Mo, Ko = orc.assemble(P, cm, G=G)
    M = sp.csr_matrix((Mo, col, rp), shape=(P.ndof, P.ndof))
    Kk = sp.csr_matrix((Ko, col, rp), shape=(P.ndof, P.ndof))
    dt = 0.1 / max(K) ** 2
    ref = spla.spsolve(M.tocsc(), M @ mu - dt * (Kk @ mu))
    out, iters, relres = plan.euler_step_geo(to_dev(cm), to_dev(G), to_dev(mu), dt, tol=1e-13, maxit=5000)
    assert relres <= 1e-13 and iters > 0
    cond = np.linalg.cond(M.toarray())
    x = to_host(out)
    assert relfro(x, ref) <= cond * relres + 1e-13, (cond, relres)
    s0, s1 = math.fsum((M @ mu).tolist()), math.fsum((M @ x).tolist())
    b = M @ mu - dt * (Kk @ mu)
    assert abs(s1 - s0) <= math.sqrt(P.ndof) * relres * np.linalg.norm(b) + 1e-13 * abs(s0)


def test_euler_overlapped_stop_leaves_result(ig):
    """The stopping test of CG reads r.r back while the GPU already prepares
    the next iteration (preconditioner, search direction, M p); that work
    must not touch mu_next.  Every reduction of the step runs in a fixed
    order (the applies and the diagonal of M sum each DOF from per-run slots,
    the dot products are two-stage with fixed grids), so a repeated step gives
    the same bits, and the converged result equals, bit for bit, the iterate
    of a run stopped by maxit at the same iteration count (no work past its
    last update of mu_next); one iteration fewer differs."""
    import torch

    p, K = 3, (40, 20, 16)   # two x-runs of the apply
    plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
    kap = to_dev(W.kappa_lognormal(plan.nelem, plan.nqp, seed=61))
    mu = to_dev(W.normal_vector(plan.ndof, 62))
    dt = 0.1 / 24 ** 2
    x1, it, rr = plan.euler_step(kap, mu, dt, tol=1e-10, maxit=5000, precond=ig.PRECOND_KRON)
    torch.cuda.synchronize()
    assert rr <= 1e-10 and it > 1
    x1b, itb, rrb = plan.euler_step(kap, mu, dt, tol=1e-10, maxit=5000, precond=ig.PRECOND_KRON)
    torch.cuda.synchronize()
    assert torch.equal(x1, x1b) and it == itb and rr == rrb
    x2 = torch.empty_like(mu)
    with pytest.raises(ig.IgafError) as ei:
        plan.euler_step(kap, mu, dt, tol=0.0, maxit=it, precond=ig.PRECOND_KRON, out=x2)
    assert ei.value.status == ig.ENOCONV
    x3 = torch.empty_like(mu)
    with pytest.raises(ig.IgafError):
        plan.euler_step(kap, mu, dt, tol=0.0, maxit=it - 1, precond=ig.PRECOND_KRON, out=x3)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2)
    assert not torch.equal(x1, x3)
    # plain CG: the same bits twice
    y1, jt, _ = plan.euler_step(kap, mu, dt, tol=1e-6, maxit=5000, precond=ig.PRECOND_NONE)
    y2, jt2, _ = plan.euler_step(kap, mu, dt, tol=1e-6, maxit=5000, precond=ig.PRECOND_NONE)
    torch.cuda.synchronize()
    assert jt == jt2 and torch.equal(y1, y2)
