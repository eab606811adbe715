"""Adjoint dL/dkappa (igaf_kappa_grad) parity.

L(kappa) = alphaM u^T M(kappa) v + alphaK u^T K(kappa) v is linear in kappa,
so: closed forms on special u, v; the oracle's point-by-point reference
gradient; Euler's identity L = <kappa, g> against the assembled CSR; and
central finite differences through the plain forward (assembled) path.
"""
import math

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import relfro, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ig():
    import torch

    assert torch.cuda.is_available()
    from paper_2207_00280_amd import igafem

    return igafem


def test_closed_forms(orc, ig):
    """u = v = 1: g = w_q;  u = v = Greville-x (u_h = x): g = w_q (x^2 + 1);
    u = Greville-x, v = 1: g = w_q x (expected weights/nodes from the oracle)."""
    from oracle import exact

    p, K = 3, (5, 3, 4)
    knots = [W.open_uniform_knots(k, p) for k in K]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    plan = ig.Plan(p, K, knots)
    xn = [orc.quad_nodes(P, d) for d in range(3)]
    wq = W.kappa_separable(xn[0][1], xn[1][1], xn[2][1])
    xq = W.kappa_separable(xn[0][0], np.ones_like(xn[1][0]), np.ones_like(xn[2][0]))
    gx = np.array([float(v) for v in exact.greville(list(knots[0]), p)])
    ux = np.tile(gx, P.N[1] * P.N[2])
    ones = np.ones(P.ndof)
    g1 = to_host(plan.kappa_grad(to_dev(ones), to_dev(ones)))
    g2 = to_host(plan.kappa_grad(to_dev(ux), to_dev(ux)))
    g3 = to_host(plan.kappa_grad(to_dev(ux), to_dev(ones)))
    assert relfro(g1, wq) <= 1e-13
    assert relfro(g2, wq * (xq ** 2 + 1)) <= 1e-13
    assert relfro(g3, wq * xq) <= 1e-13


@pytest.mark.parametrize("p,K", [(1, (4, 3, 5)), (2, (5, 4, 3)), (3, (6, 5, 4)), (4, (3, 3, 4)),
                                 (5, (2, 3, 2))])
def test_vs_oracle_small(orc, ig, p, K):
    """Every quadrature point vs the oracle's plain (no sum factorisation)
    reference gradient; also alphaM/alphaK/scale handling."""
    knots = [W.open_uniform_knots(k, p) for k in K]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    plan = ig.Plan(p, K, knots)
    u = W.normal_vector(P.ndof, 3)
    v = W.normal_vector(P.ndof, 4)
    for aM, aK, sc in [(1.0, 1.0, 1.0), (0.5, -2.0, 3.0), (1.0, 0.0, 1.0), (0.0, 1.0, 1.0)]:
        g = to_host(plan.kappa_grad(to_dev(u), to_dev(v), aM, aK, sc))
        go = orc.kappa_grad(P, u, v, aM, aK, sc)
        assert relfro(g, go) <= 1e-12


def _csr_bilinear(rp, col, val, u, v):
    """u^T A v with a compensated (fsum) reduction, host side."""
    import scipy.sparse as sp

    A = sp.csr_matrix((val, col, rp), shape=(len(u), len(v)))
    return math.fsum((u * (A @ v)).tolist())


def test_linearity_vs_assembled(ig):
    """Euler's identity: L(kappa) = sum_q kappa_q dL/dkappa_q, with L taken
    from the assembled CSR matrices (plain forward path), 24^3 elements."""
    p, K = 3, (24, 24, 24)
    knots = [W.open_uniform_knots(k, p) for k in K]
    plan = ig.Plan(p, K, knots)
    kap = W.kappa_lognormal(plan.nelem, plan.nqp, seed=2)
    u = W.normal_vector(plan.ndof, 3)
    v = W.normal_vector(plan.ndof, 4)
    _, _, Mv, Kv = plan.integrate_assemble(to_dev(kap), want_elem=False)
    rp, col = plan.csr_pattern()
    rp, col = to_host(rp), to_host(col)
    L = _csr_bilinear(rp, col, to_host(Mv) + to_host(Kv), u, v)
    g = to_host(plan.kappa_grad(to_dev(u), to_dev(v)))
    Lg = math.fsum((g * kap).reshape(-1).tolist())
    assert abs(Lg - L) <= 1e-12 * abs(L)


def test_w5_fullscale(orc, ig):
    """96^3 elements, p=3, log-normal kappa (seed 2), u, v ~ N(0,1) (seeds 3,4):
    (1) the oracle's reference gradient at all 56 623 104 points, relative L2
        <= 1e-12;
    (2) central finite differences on 100 seeded points through the plain
        forward path: g_fd = u^T (A(kappa + h e_q) - A(kappa - h e_q)) v / (2h),
        h = 0.1 kappa_q, A = M + K assembled to CSR by igaf_integrate_assemble
        (the row path is deterministic, so entries that kappa_q does not touch
        cancel exactly); relative L2 <= 1e-6."""
    import torch

    cfg = W.W5
    p, K = cfg["p"], cfg["K"]
    knots = [W.open_uniform_knots(k, p) for k in K]
    plan = ig.Plan(p, K, knots)
    kap = W.kappa_lognormal(plan.nelem, plan.nqp, seed=cfg["seed_kappa"])
    u = W.normal_vector(plan.ndof, cfg["seed_u"])
    v = W.normal_vector(plan.ndof, cfg["seed_v"])
    kd, ud, vd = to_dev(kap), to_dev(u), to_dev(v)
    g = plan.kappa_grad(ud, vd)
    gh = to_host(g).reshape(-1)
    # (1) oracle reference gradient at every point
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    go = orc.kappa_grad(P, u, v).reshape(-1)
    assert relfro(gh, go) <= 1e-12
    # (2) central differences through the assembled path
    pts = W.fd_points(plan.nelem * plan.nqp, cfg["npts"], cfg["seed_pts"])
    rp, col = plan.csr_pattern()
    rp_h = to_host(rp)
    col_h = to_host(col)
    Mp = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
    Kp = torch.empty_like(Mp)
    Mm = torch.empty_like(Mp)
    Km = torch.empty_like(Mp)
    flat = kd.view(-1)
    gfd = np.zeros(len(pts))
    for i, q in enumerate(pts):
        k0 = float(kap.reshape(-1)[q])
        h = 0.1 * k0
        flat[q] = k0 + h
        plan.integrate_assemble(kd, want_elem=False, Mval=Mp, Kval=Kp)
        flat[q] = k0 - h
        plan.integrate_assemble(kd, want_elem=False, Mval=Mm, Kval=Km)
        flat[q] = k0
        dA = (Mp - Mm) + (Kp - Km)
        nz = torch.nonzero(dA).view(-1)
        assert 0 < nz.numel() <= 2 * 4096
        idx = to_host(nz)
        vals = to_host(dA[nz])
        rows = np.searchsorted(rp_h, idx, side="right") - 1
        terms = u[rows] * vals * v[col_h[idx]]
        gfd[i] = math.fsum(terms.tolist()) / (2 * h)
    ga = gh[pts]
    assert np.linalg.norm(gfd - ga) / np.linalg.norm(gfd) <= 1e-6
    # the gradient is linear: the same value at any step (here far below 1e-6)
    assert np.linalg.norm(gfd - ga) / np.linalg.norm(gfd) <= 1e-10


def test_autograd_function(ig):
    """torch.autograd: loss.backward() gives the adjoint gradient scaled by
    the incoming gradient; the loss value is <kappa, g>."""
    import torch

    p, K = 2, (6, 5, 4)
    knots = [W.open_uniform_knots(k, p) for k in K]
    plan = ig.Plan(p, K, knots)
    kap = to_dev(W.kappa_lognormal(plan.nelem, plan.nqp, seed=9)).requires_grad_(True)
    u = to_dev(W.normal_vector(plan.ndof, 1))
    v = to_dev(W.normal_vector(plan.ndof, 2))
    loss = ig.kappa_bilinear_loss(kap, u, v, plan)
    (3.0 * loss).backward()
    g = plan.kappa_grad(u, v)
    assert relfro(to_host(kap.grad), 3.0 * to_host(g)) <= 1e-14
    assert abs(float(loss) - float((g * kap.detach()).sum())) <= 1e-12 * abs(float(loss))
