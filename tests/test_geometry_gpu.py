"""Mapped geometry (igaf_integrate_assemble_geo) parity.

On x = F(xi) the per-point factor of eq. (10) becomes cm = kappa det J for the
mass and the tensor G = kappa det J J^-1 J^-T for the stiffness; the caller's
side (workloads.mapped_geometry) evaluates them at the points.  The HIP path
(sum factorisation with ordered per-direction pairs; CSR values gathered from
the stored element matrices, or, when none are stored, computed by
owner-computed rows) is
compared with the oracle's classical quadrature of the same integrands, which
the CPU suite pins by scaled knots, exact affine Kronecker forms and linear
patch tests.
"""
import math

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import csr_close, nonuniform_knots, relfro, rowmax_rel, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def ig():
    import torch

    assert torch.cuda.is_available()
    from paper_2207_00280_amd import igafem

    return igafem


def _coeffs(orc, P, kap, **geo):
    xs = [orc.quad_nodes(P, d)[0] for d in range(3)]
    return W.mapped_geometry(xs[0], xs[1], xs[2], kap, **geo)


A_SHEAR = np.array([[1.3, 0.35, -0.2], [-0.1, 0.9, 0.25], [0.2, -0.15, 1.1]])

CASES = [
    # p, K, knots kind, geometry
    (1, (5, 4, 3), "nonuniform", dict(amp=0.1)),
    (2, (4, 5, 3), "uniform", dict(A=A_SHEAR, amp=0.05)),
    (3, (5, 3, 4), "nonuniform", dict(amp=0.1)),
    (3, None, "repeated", dict(A=A_SHEAR)),
    (4, (3, 3, 2), "nonuniform", dict(A=A_SHEAR, amp=0.08)),
    (5, (2, 3, 2), "uniform", dict(amp=0.1)),
]


def _knots(p, K, kind, seed):
    if kind == "repeated":
        ks = [W.random_repeated_knots(3, p, seed=seed + d)[0] for d in range(3)]
        return ks, tuple(len(t) - 2 * p - 1 for t in ks)
    if kind == "uniform":
        return [W.open_uniform_knots(k, p) for k in K], K
    return [nonuniform_knots(k, p, seed + d) for d, k in enumerate(K)], K


@pytest.mark.parametrize("p,K,kind,geo", CASES)
def test_geometry_vs_oracle(orc, ig, p, K, kind, geo):
    """Every element matrix and every CSR value vs the oracle (curved and
    sheared maps, non-uniform and repeated knots, log-normal kappa); mass-only
    and stiffness-only calls give the same values."""
    knots, K = _knots(p, K, kind, 70 + p)
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    plan = ig.Plan(p, K, knots)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=80 + p)
    cm, G = _coeffs(orc, P, kap, **geo)
    Me_o, Ke_o = orc.element_matrices(P, cm, G=G)
    rp_o, col_o, Mv_o, Kv_o = orc.assemble(P, cm, G=G)
    cmd, Gd = to_dev(cm), to_dev(G)
    Me, Ke, Mv, Kv = plan.integrate_assemble_geo(cmd, Gd)
    assert relfro(to_host(Me), Me_o) <= TOL and relfro(to_host(Ke), Ke_o) <= TOL
    em = np.abs(to_host(Ke) - Ke_o).reshape(P.nelem, -1).max(axis=1)
    assert em.max() <= TOL * np.abs(Ke_o).max()
    assert csr_close(to_host(Mv), Mv_o, rp_o, TOL) and csr_close(to_host(Kv), Kv_o, rp_o, TOL)
    rp, col = plan.csr_pattern()
    assert np.array_equal(to_host(rp), rp_o) and np.array_equal(to_host(col), col_o)
    # with the element matrices stored the CSR values are gathered: bitwise repeatable
    _, _, Mv_b, Kv_b = plan.integrate_assemble_geo(cmd, Gd)
    assert np.array_equal(to_host(Mv_b), to_host(Mv)) and np.array_equal(to_host(Kv_b), to_host(Kv))
    # one matrix at a time; element matrices only; CSR only (rows kernel):
    # both, each alone, repeated bit for bit
    Me2, Ke2, _, _ = plan.integrate_assemble_geo(cmd, None, want_k=False, want_csr=False)
    assert Ke2 is None and relfro(to_host(Me2), Me_o) <= TOL
    _, _, Mv3, Kv3 = plan.integrate_assemble_geo(None, Gd, want_m=False, want_elem=False)
    assert Mv3 is None and csr_close(to_host(Kv3), Kv_o, rp_o, TOL)
    _, _, Mv4, _ = plan.integrate_assemble_geo(cmd, None, want_k=False, want_elem=False)
    assert csr_close(to_host(Mv4), Mv_o, rp_o, TOL)
    _, _, Mv5, Kv5 = plan.integrate_assemble_geo(cmd, Gd, want_elem=False)
    assert csr_close(to_host(Mv5), Mv_o, rp_o, TOL) and csr_close(to_host(Kv5), Kv_o, rp_o, TOL)
    _, _, Mv6, Kv6 = plan.integrate_assemble_geo(cmd, Gd, want_elem=False)
    assert np.array_equal(to_host(Mv6), to_host(Mv5)) and np.array_equal(to_host(Kv6), to_host(Kv5))
    assert np.array_equal(to_host(Kv3), to_host(Kv5)) and np.array_equal(to_host(Mv4), to_host(Mv5))


ROWS_CASES = [
    # several tiles in y and z, several x segments, ragged tile edges
    (1, (37, 9, 6), "nonuniform", dict(amp=0.1)),
    (2, (29, 7, 5), "nonuniform", dict(A=A_SHEAR, amp=0.05)),
    (3, (26, 5, 5), "nonuniform", dict(A=A_SHEAR, amp=0.1)),
    (3, (21, 1, 2), "uniform", dict(amp=0.1)),
    (4, (20, 3, 2), "nonuniform", dict(amp=0.08)),
    (5, (16, 2, 2), "nonuniform", dict(A=A_SHEAR, amp=0.05)),
    (5, (13, 1, 3), "uniform", dict(amp=0.1)),
    (3, (1, 1, 1), "uniform", dict(amp=0.1)),
    (5, (1, 1, 1), "uniform", dict(amp=0.1)),
]


@pytest.mark.parametrize("p,K,kind,geo", ROWS_CASES)
def test_geometry_rows_kernel_vs_oracle(orc, ig, p, K, kind, geo):
    """The owner-computed CSR rows of a mapped geometry on meshes that span
    several tiles and x segments, and single elements: every CSR value of M
    and K vs the oracle (global and per-row relative error), repeated calls
    bit for bit."""
    knots, K = _knots(p, K, kind, 310 + p)
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    plan = ig.Plan(p, K, knots)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=320 + p)
    cm, G = _coeffs(orc, P, kap, **geo)
    rp_o, col_o, Mv_o, Kv_o = orc.assemble(P, cm, G=G)
    cmd, Gd = to_dev(cm), to_dev(G)
    _, _, Mv, Kv = plan.integrate_assemble_geo(cmd, Gd, want_elem=False)
    assert csr_close(to_host(Mv), Mv_o, rp_o, TOL) and csr_close(to_host(Kv), Kv_o, rp_o, TOL)
    _, _, Mv2, Kv2 = plan.integrate_assemble_geo(cmd, Gd, want_elem=False)
    assert np.array_equal(to_host(Mv2), to_host(Mv)) and np.array_equal(to_host(Kv2), to_host(Kv))


def test_identity_geometry_matches_plain_path(ig):
    """cm = kappa, G = kappa I: the same matrices as igaf_integrate_assemble
    (two different kernels; the plain one is checked against the oracle
    elsewhere), to rounding."""
    p, K = 3, (7, 6, 5)
    knots = [nonuniform_knots(k, p, 90 + d) for d, k in enumerate(K)]
    plan = ig.Plan(p, K, knots)
    kap = W.kappa_lognormal(plan.nelem, plan.nqp, seed=91)
    G = np.zeros((plan.nelem, 6, plan.nqp))
    G[:, 0], G[:, 1], G[:, 2] = kap, kap, kap
    kd = to_dev(kap)
    Me, Ke, Mv, Kv = plan.integrate_assemble_geo(kd, to_dev(G))
    Me_r, Ke_r, Mv_r, Kv_r = plan.integrate_assemble(kd)
    for a, b in ((Me, Me_r), (Ke, Ke_r), (Mv, Mv_r), (Kv, Kv_r)):
        assert relfro(to_host(a), to_host(b)) <= TOL


def test_geometry_fullscale(orc, ig):
    """64^3 elements, p=3, curved map (amp 0.1), kappa = 1 + 0.5 sin sin sin:
    (1) 32 seeded elements (first and last included): both matrices vs the
        oracle; (2) 32 seeded complete CSR rows (corners included) vs the
        oracle; (3) parametric linear functions u = c.xi* (Greville points):
        u^T K v = sum_q w_q c1^T G_q c2 and K 1 = 0."""
    import torch

    cfg = W.W6
    p, K = cfg["p"], cfg["K"]
    knots = [W.open_uniform_knots(k, p) for k in K]
    plan = ig.Plan(p, K, knots)
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    xs = [orc.quad_nodes(P, d) for d in range(3)]
    kap = W.kappa_sine(xs[0][0], xs[1][0], xs[2][0])
    cm, G = W.mapped_geometry(xs[0][0], xs[1][0], xs[2][0], kap, amp=cfg["amp"])
    cmd, Gd = to_dev(cm), to_dev(G)
    Me, Ke, Mv, Kv = plan.integrate_assemble_geo(cmd, Gd)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    els = np.concatenate([[0, plan.nelem - 1], rng.choice(plan.nelem, 30, replace=False)])
    idx = torch.from_numpy(els).cuda()
    Me_s, Ke_s = to_host(Me[idx]), to_host(Ke[idx])
    for i, e in enumerate(els):
        mo, ko = orc.element_matrices(P, cm, int(e), int(e) + 1, G=G)
        assert relfro(Me_s[i], mo[0]) <= TOL and relfro(Ke_s[i], ko[0]) <= TOL, e
    del Me, Ke
    torch.cuda.empty_cache()
    # CSR alone: the owner-computed rows kernel; the same values as the
    # gather from the element matrices to rounding, row by row
    _, _, Mv2, Kv2 = plan.integrate_assemble_geo(cmd, Gd, want_elem=False)
    rp = to_host(plan.csr_pattern()[0])
    Mv_h, Kv_h, Mv2_h, Kv2_h = to_host(Mv), to_host(Kv), to_host(Mv2), to_host(Kv2)
    del Mv2, Kv2
    assert rowmax_rel(Mv2_h, Mv_h, rp) <= TOL and rowmax_rel(Kv2_h, Kv_h, rp) <= TOL
    N = P.N
    corners = [0, N[0] - 1, plan.ndof - 1, plan.ndof - N[0]]
    dofs = np.concatenate([corners, rng.choice(plan.ndof, 28, replace=False)])
    for d, (c, m, k) in zip(dofs, orc.rows(P, cm, dofs, G=G)):
        seg = slice(rp[d], rp[d + 1])
        for mv, kv in ((Mv_h, Kv_h), (Mv2_h, Kv2_h)):
            assert np.abs(mv[seg] - m).max() <= TOL * np.abs(m).sum()
            assert np.abs(kv[seg] - k).max() <= TOL * np.abs(k).sum()
    del Mv2_h, Kv2_h
    # parametric linear functions through the assembled stiffness
    import scipy.sparse as sp

    col = to_host(plan.csr_pattern()[1])
    Kc = sp.csr_matrix((Kv_h, col, rp), shape=(plan.ndof, plan.ndof))
    gr = [np.array([sum(t[i + 1:i + p + 1]) / p for i in range(len(t) - p - 1)]) for t in knots]
    ii = np.arange(plan.ndof)
    XI = np.stack([gr[0][ii % N[0]], gr[1][(ii // N[0]) % N[1]], gr[2][ii // (N[0] * N[1])]], axis=1)
    c1, c2 = np.array([0.6, -1.1, 0.35]), np.array([-0.4, 0.8, 1.3])
    lhs = math.fsum(((XI @ c1) * (Kc @ (XI @ c2))).tolist())
    wq = W.kappa_separable(xs[0][1], xs[1][1], xs[2][1])
    comp = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    quad = sum((c1[r] * c2[t] + (c1[t] * c2[r] if r != t else 0.0)) * (wq * G[:, c, :])
               for c, (r, t) in enumerate(comp))
    rhs = math.fsum(quad.ravel().tolist())
    assert abs(lhs - rhs) <= 1e-11 * abs(rhs)
    k1 = Kc @ np.ones(plan.ndof)
    rowabs = np.abs(Kc) @ np.ones(plan.ndof)
    assert np.max(np.abs(k1)) <= 64 * np.finfo(float).eps * np.max(rowabs)


@pytest.mark.parametrize("p,K", [(2, (6, 5, 7)), (5, (3, 2, 4))])
def test_geometry_csr_under_capture(ig, p, K):
    """A CSR-only call under HIP graph capture: the rows kernel needs no
    workspace and captures at once (igaf_geo_prepare is a no-op); every
    replay (eager work between them) equals the eager result of another plan
    bit for bit."""
    import torch

    knots = [nonuniform_knots(k, p, 230 + d) for d, k in enumerate(K)]
    plan = ig.Plan(p, K, knots)
    xs = [plan.quad_nodes(d)[0] for d in range(3)]
    cm, G = W.mapped_geometry(xs[0], xs[1], xs[2], W.kappa_lognormal(plan.nelem, plan.nqp, seed=231), amp=0.1)
    cmd, Gd = to_dev(cm), to_dev(G)
    Mv = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
    Kv = torch.empty_like(Mv)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.integrate_assemble_geo(cmd, Gd, want_elem=False, Mval=Mv, Kval=Kv, stream=s)
    plan2 = ig.Plan(p, K, knots)
    _, _, Mr, Kr = plan2.integrate_assemble_geo(cmd, Gd, want_elem=False)
    for r in range(3):
        Mv.fill_(np.nan)
        Kv.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Mv, Mr) and torch.equal(Kv, Kr), r
        _ = torch.ones(1000, device="cuda").sum().item()


def test_geometry_errors(ig):
    """Missing coefficients for a requested output, no output and an
    unsupported quadrature order are refused before any launch."""
    p, K = 2, (3, 3, 3)
    plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
    L = ig.lib()
    cm = to_dev(np.ones((plan.nelem, plan.nqp)))
    Me = to_dev(np.zeros((plan.nelem, plan.elem_dim, plan.elem_dim)))
    assert L.igaf_integrate_assemble_geo(plan._h, None, None, Me.data_ptr(), None, None, None,
                                         None) == ig.EINVAL
    assert L.igaf_integrate_assemble_geo(plan._h, cm.data_ptr(), None, None, Me.data_ptr(), None,
                                         None, None) == ig.EINVAL
    assert L.igaf_integrate_assemble_geo(plan._h, cm.data_ptr(), None, None, None, None, None,
                                         None) == ig.EINVAL
    plan4 = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K], q=(4, 4, 4))
    with pytest.raises(ig.IgafError) as ei:
        plan4.integrate_assemble_geo(to_dev(np.ones((plan4.nelem, plan4.nqp))), None, want_k=False)
    assert ei.value.status == ig.EUNSUPPORTED


@pytest.mark.parametrize("p,K,kind,geo", CASES)
def test_geometry_apply_and_adjoint(orc, ig, p, K, kind, geo):
    """Matrix-free apply and adjoint on a mapped geometry: y vs the oracle's
    assembled geometry matrices times u; dL/dkappa (kappa scaling cm0 = det J
    and G0 = det J J^-1 J^-T) vs the oracle's point-wise gradient."""
    import scipy.sparse as sp

    knots, K = _knots(p, K, kind, 170 + p)
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    plan = ig.Plan(p, K, knots)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=180 + p)
    cm0, G0 = _coeffs(orc, P, W.kappa_constant(P.nelem, P.nq), **geo)
    cm, G = kap * cm0, kap[:, None, :] * G0
    u = W.normal_vector(P.ndof, 190 + p)
    v = W.normal_vector(P.ndof, 200 + p)
    rp, col, Mv, Kv = orc.assemble(P, cm, G=G)
    M = sp.csr_matrix((Mv, col, rp), shape=(P.ndof, P.ndof))
    Kk = sp.csr_matrix((Kv, col, rp), shape=(P.ndof, P.ndof))
    cmd, Gd, ud = to_dev(cm), to_dev(G), to_dev(u)
    for aM, aK in [(1.0, 0.0), (0.0, 1.0), (0.6, -1.4)]:
        y = to_host(plan.apply_geo(cmd, Gd, ud, aM, aK))
        assert relfro(y, aM * (M @ u) + aK * (Kk @ u)) <= TOL, (aM, aK)
    g = to_host(plan.kappa_grad_geo(to_dev(cm0), to_dev(G0), ud, to_dev(v), 0.8, 1.2, 1.5))
    go = orc.kappa_grad(P, u, v, 0.8, 1.2, 1.5, cm0=cm0, G0=G0)
    assert relfro(g, go) <= TOL


def test_identity_geometry_apply_adjoint_match_plain(ig):
    """cm = kappa, G = kappa I gives igaf_apply's y; cm0 = 1, G0 = I gives
    igaf_kappa_grad's gradient (different kernels' template branches)."""
    p, K = 3, (9, 5, 6)
    knots = [nonuniform_knots(k, p, 210 + d) for d, k in enumerate(K)]
    plan = ig.Plan(p, K, knots)
    kap = W.kappa_lognormal(plan.nelem, plan.nqp, seed=211)
    I6 = np.zeros((plan.nelem, 6, plan.nqp))
    I6[:, 0] = I6[:, 1] = I6[:, 2] = 1.0
    u, v = to_dev(W.normal_vector(plan.ndof, 212)), to_dev(W.normal_vector(plan.ndof, 213))
    kd = to_dev(kap)
    y0 = to_host(plan.apply(kd, u, 0.9, 1.1))
    y1 = to_host(plan.apply_geo(kd, to_dev(kap[:, None, :] * I6), u, 0.9, 1.1))
    assert relfro(y1, y0) <= TOL
    g0 = to_host(plan.kappa_grad(u, v, 0.9, 1.1, 2.0))
    g1 = to_host(plan.kappa_grad_geo(to_dev(np.ones_like(kap)), to_dev(I6), u, v, 0.9, 1.1, 2.0))
    assert relfro(g1, g0) <= TOL


def test_geometry_apply_adjoint_fullscale(orc, ig):
    """64^3 elements, p = 3, curved map: y = (M + K) u at 32 sampled DOFs vs
    the oracle's complete rows, and u^T (M + K) v from the apply equals
    <kappa, dL/dkappa> from the adjoint (L is linear in kappa), relative
    1e-12."""
    cfg = W.W6
    p, K = cfg["p"], cfg["K"]
    knots = [W.open_uniform_knots(k, p) for k in K]
    plan = ig.Plan(p, K, knots)
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    xs = [orc.quad_nodes(P, d)[0] for d in range(3)]
    kap = W.kappa_lognormal(plan.nelem, plan.nqp, seed=220)
    cm0, G0 = W.mapped_geometry(xs[0], xs[1], xs[2], W.kappa_constant(plan.nelem, plan.nqp), amp=cfg["amp"])
    cm, G = kap * cm0, kap[:, None, :] * G0
    u = W.normal_vector(plan.ndof, 221)
    v = W.normal_vector(plan.ndof, 222)
    ud, vd = to_dev(u), to_dev(v)
    y = to_host(plan.apply_geo(to_dev(cm), to_dev(G), ud, 1.0, 1.0))
    rng = np.random.default_rng(223)
    dofs = np.concatenate([[0, plan.ndof - 1], rng.choice(plan.ndof, 30, replace=False)])
    for d, (c, m, k) in zip(dofs, orc.rows(P, cm, dofs, G=G)):
        terms = (m + k) * u[c]
        assert abs(y[d] - math.fsum(terms.tolist())) <= TOL * np.sum(np.abs(terms))
    yv = to_host(plan.apply_geo(to_dev(cm), to_dev(G), vd, 1.0, 1.0))
    L = math.fsum((u * yv).tolist())
    g = to_host(plan.kappa_grad_geo(to_dev(cm0), to_dev(G0), ud, vd, 1.0, 1.0, 1.0))
    Lg = math.fsum((g.reshape(-1) * kap.reshape(-1)).tolist())
    assert abs(L - Lg) <= 1e-12 * abs(L)
