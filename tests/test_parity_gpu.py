"""GPU parity of the HIP path against the CPU oracle, element by element.

Bar (FP64): relative Frobenius error <= 1e-12 per output (element matrices,
CSR values); the CSR pattern bit-exact.  Inputs are seeded; every expected
value comes from oracle/.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import csr_close, nonuniform_knots, relfro, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def ig():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_00280_amd import igafem

    igafem.lib()
    return igafem


def _case(orc, ig, p, K, knots, kap):
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    plan = ig.Plan(p, K, knots)
    return P, plan, to_dev(kap)


def test_w1_mass_classical(orc, ig):
    """8^3 elements, p=2, 3-point Gauss, kappa=1, mass only, classical; CSR
    1000 x 1000 with 85 184 nonzeros."""
    p, K = 2, (8, 8, 8)
    knots = [W.open_uniform_knots(8, 2)] * 3
    P = orc.Patch(p, K, [3] * 3, knots)
    kap = W.kappa_constant(P.nelem, P.nq)
    plan = ig.Plan(p, K, knots)
    assert plan.nnz == 85184 and plan.ndof == 1000
    Me_o, _ = orc.element_matrices(P, kap, want_k=False)
    rp_o, col_o, Mv_o, _ = orc.assemble(P, kap)
    kd = to_dev(kap)
    Me, Ke, Mv, Kv = plan.integrate_assemble(kd, method=ig.CLASSICAL, want_k=False)
    assert Ke is None and Kv is None
    assert relfro(to_host(Me), Me_o) <= TOL
    assert csr_close(to_host(Mv), Mv_o, rp_o, TOL)
    rp, col = plan.csr_pattern()
    assert np.array_equal(to_host(rp), rp_o) and np.array_equal(to_host(col), col_o)
    # the sum-factorised path gives the same matrices
    Me2, _ = plan.element_matrices(kd, method=ig.SUMFACT, want_k=False)
    assert relfro(to_host(Me2), Me_o) <= TOL


CASES = [
    # p, K, nonuniform knots
    (1, (5, 3, 4), False),
    (2, (6, 5, 7), True),
    (3, (7, 6, 5), False),
    (3, (4, 9, 3), True),
    (4, (3, 4, 3), True),
    (5, (2, 3, 2), False),
]


@pytest.mark.parametrize("p,K,nonuni", CASES)
def test_element_matrices(orc, ig, p, K, nonuni):
    """Classical and sum-factorised element matrices (M and K) vs the oracle's
    classical quadrature, every element; seeded log-normal kappa."""
    knots = [nonuniform_knots(k, p, 10 + d) if nonuni else W.open_uniform_knots(k, p)
             for d, k in enumerate(K)]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=100 + p)
    plan = ig.Plan(p, K, knots)
    Me_o, Ke_o = orc.element_matrices(P, kap)
    kd = to_dev(kap)
    for method in (ig.CLASSICAL, ig.SUMFACT):
        Me, Ke = plan.element_matrices(kd, method=method)
        assert relfro(to_host(Me), Me_o) <= TOL, method
        assert relfro(to_host(Ke), Ke_o) <= TOL, method
        # per-element maximum too
        em = np.abs(to_host(Me) - Me_o).reshape(P.nelem, -1).max(axis=1)
        assert em.max() <= TOL * np.abs(Me_o).max()


@pytest.mark.parametrize("p,K", [(1, (9, 9, 8)), (3, (9, 9, 7)), (2, (9, 8, 8))])
def test_element_matrices_single_output(orc, ig, p, K):
    """Sum factorisation with one output requested (M only, then K only; the
    other pointer NULL) and more elements than workgroups, not a multiple of
    them (567-648 elements against 512 workgroups: some take two elements,
    some one), vs the oracle."""
    knots = [W.open_uniform_knots(k, p) for k in K]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=300 + p)
    plan = ig.Plan(p, K, knots)
    Me_o, Ke_o = orc.element_matrices(P, kap)
    kd = to_dev(kap)
    Me, Ke, _, _ = plan.integrate_assemble(kd, want_k=False, want_csr=False)
    assert Ke is None and relfro(to_host(Me), Me_o) <= TOL
    Me, Ke, _, _ = plan.integrate_assemble(kd, want_m=False, want_csr=False)
    assert Me is None and relfro(to_host(Ke), Ke_o) <= TOL


@pytest.mark.parametrize("p,K,nonuni", CASES)
def test_csr_assembly(orc, ig, p, K, nonuni):
    """CSR values by owner-computed rows, by FP64 atomics and by gathering the
    stored element matrices, vs the oracle's assembly; pattern bit-exact."""
    knots = [nonuniform_knots(k, p, 20 + d) if nonuni else W.open_uniform_knots(k, p)
             for d, k in enumerate(K)]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=200 + p)
    plan = ig.Plan(p, K, knots)
    rp_o, col_o, Mv_o, Kv_o = orc.assemble(P, kap)
    kd = to_dev(kap)
    rp, col = plan.csr_pattern()
    assert np.array_equal(to_host(rp), rp_o) and np.array_equal(to_host(col), col_o)
    _, _, Mv, Kv = plan.integrate_assemble(kd, want_elem=False)
    assert csr_close(to_host(Mv), Mv_o, rp_o, TOL) and csr_close(to_host(Kv), Kv_o, rp_o, TOL)
    plan.set_assembly(ig.ASM_ATOMIC)
    _, _, Mv2, Kv2 = plan.integrate_assemble(kd, want_elem=False)
    assert csr_close(to_host(Mv2), Mv_o, rp_o, TOL) and csr_close(to_host(Kv2), Kv_o, rp_o, TOL)
    plan.set_assembly(ig.ASM_ROWS)
    Me, Ke, Mv3, Kv3 = plan.integrate_assemble(kd, method=ig.CLASSICAL)
    assert csr_close(to_host(Mv3), Mv_o, rp_o, TOL) and csr_close(to_host(Kv3), Kv_o, rp_o, TOL)
    Mv4, Kv4 = plan.assemble(Me, Ke)
    assert csr_close(to_host(Mv4), Mv_o, rp_o, TOL) and csr_close(to_host(Kv4), Kv_o, rp_o, TOL)


@pytest.mark.parametrize("p,K", [(3, (13, 7, 12)), (4, (9, 8, 8)), (5, (10, 10, 4)), (5, (4, 4, 10))])
def test_csr_rows_shared_tables(orc, ig, p, K):
    """Owner-computed CSR rows on meshes long enough (K >= 2p) for the
    elements away from the ends of a direction to share one copy of the basis
    tables, which the rows kernels then read for the whole run (x, y and z
    runs covered; p = 3, 4: the ten- and five-pencil tiles over several tiles,
    p = 5: the split stage x): every CSR value vs the oracle's assembly."""
    knots = [W.open_uniform_knots(k, p) for k in K]
    d = ig.make_desc(p, K, knots)
    for a in range(3):
        lo, hi = p - 1, K[a] - p + 1
        assert ig.desc_shared_run(d, a) == ((lo, hi) if hi - lo >= 2 else (0, 0))
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    kap = W.kappa_lognormal(P.nelem, P.nq, seed=300 + p)
    plan = ig.Plan(p, K, knots)
    rp_o, col_o, Mv_o, Kv_o = orc.assemble(P, kap)
    _, _, Mv, Kv = plan.integrate_assemble(to_dev(kap), want_elem=False)
    assert csr_close(to_host(Mv), Mv_o, rp_o, TOL) and csr_close(to_host(Kv), Kv_o, rp_o, TOL)


def test_rows_deterministic(ig):
    """Owner-computed rows: bitwise identical results on repeated calls."""
    p, K = 3, (9, 7, 6)
    knots = [W.open_uniform_knots(k, p) for k in K]
    plan = ig.Plan(p, K, knots)
    kap = to_dev(W.kappa_lognormal(plan.nelem, plan.nqp, seed=5))
    _, _, a, b = plan.integrate_assemble(kap, want_elem=False)
    _, _, c, d = plan.integrate_assemble(kap, want_elem=False)
    assert np.array_equal(to_host(a), to_host(c)) and np.array_equal(to_host(b), to_host(d))


def test_quad_nodes_match_oracle(orc, ig):
    """The library's mapped Gauss nodes/weights equal the oracle's (used only
    to evaluate kappa; independent implementations of the same rule)."""
    p, K = 4, (3, 5, 2)
    knots = [nonuniform_knots(k, p, 3 + d) for d, k in enumerate(K)]
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    plan = ig.Plan(p, K, knots)
    for d in range(3):
        x, w = plan.quad_nodes(d)
        xo, wo = orc.quad_nodes(P, d)
        np.testing.assert_allclose(x, xo, rtol=0, atol=2e-16)
        np.testing.assert_allclose(w, wo, rtol=0, atol=2e-16)


def test_unsupported_quadrature(ig):
    """Valid input outside the kernels' shapes is refused, not miscomputed."""
    p, K = 2, (3, 3, 3)
    knots = [W.open_uniform_knots(3, 2)] * 3
    plan = ig.Plan(p, K, knots, q=(4, 4, 4))
    kap = to_dev(np.ones((plan.nelem, plan.nqp)))
    with pytest.raises(ig.IgafError) as ei:
        plan.element_matrices(kap)
    assert ei.value.status == ig.EUNSUPPORTED


def test_quad_points_and_one_shot_integrate(orc, ig):
    """igaf_quad_points gives every point in kappa's layout (kappa evaluated
    there equals kappa_sine on the per-direction nodes); the one-shot
    integrate() returns the same matrices as the plan path and the oracle."""
    import torch

    p, K = 2, (4, 3, 5)
    knots = [nonuniform_knots(k, p, 240 + d) for d, k in enumerate(K)]
    plan = ig.Plan(p, K, knots)
    xyz = plan.quad_points()
    xs = [plan.quad_nodes(d)[0] for d in range(3)]
    kap_nodes = W.kappa_sine(*xs)
    kap_pts = 1.0 + 0.5 * np.sin(2 * np.pi * xyz[..., 0]) * np.sin(2 * np.pi * xyz[..., 1]) * \
        np.sin(2 * np.pi * xyz[..., 2])
    np.testing.assert_allclose(kap_pts, kap_nodes, rtol=0, atol=1e-15)
    kd = to_dev(kap_nodes)
    r = ig.integrate(p, K, knots, kd)
    Me, Ke, Mv, Kv = plan.integrate_assemble(kd)
    for a, b in ((r["Me"], Me), (r["Ke"], Ke), (r["Mval"], Mv), (r["Kval"], Kv)):
        assert torch.equal(a, b)
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    rp_o, col_o, Mv_o, Kv_o = orc.assemble(P, kap_nodes)
    assert np.array_equal(to_host(r["row_ptr"]), rp_o) and np.array_equal(to_host(r["col"]), col_o)
    assert csr_close(to_host(r["Mval"]), Mv_o, rp_o, TOL) and csr_close(to_host(r["Kval"]), Kv_o, rp_o, TOL)
    assert ig.KappaBilinearLoss is ig.KappaBilinearLoss
