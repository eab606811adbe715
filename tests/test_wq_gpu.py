"""Weighted quadrature (igaf_wq_prepare / igaf_wq_points / igaf_wq_assemble)
against the oracle (oracle/wq.py, exact minimum-norm weights, plain triple
sums).

Small patches (p = 1..5, uniform and non-uniform knots, log-normal kappa on
the point grid): every CSR value vs the oracle's; kappa = 1: the exact
Galerkin matrices (Kronecker products of the 1D matrices of the oracle's
Gauss rule, exact for these integrands); 64^3, p = 3 (the headline mesh):
every one of the 95 443 993 values of M and K against the separable closed
form kappa = 1 + 0.5 s(x) s(y) s(z) admits (1D rule matrices from the
oracle), plus complete rows against the oracle.
"""
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


def _rows_cols(rp, col, N):
    Nx, Ny, Nz = N
    lens = np.diff(rp)
    rows = np.repeat(np.arange(len(rp) - 1, dtype=np.int64), lens)
    c = col.astype(np.int64)
    return (rows % Nx, (rows // Nx) % Ny, rows // (Nx * Ny)), (c % Nx, (c // Nx) % Ny, c // (Nx * Ny))


def _plan(ig, p, K, knots):
    plan = ig.Plan(p, K, knots)
    plan.wq_prepare()
    return plan


CASES = [(1, (4, 3, 5), False), (2, (5, 3, 4), True), (3, (4, 5, 3), False), (3, (3, 4, 4), True),
         (4, (3, 2, 3), False), (5, (1, 2, 2), True)]


@pytest.mark.parametrize("p,K,nonuni", CASES)
def test_wq_vs_oracle_small(orc, ig, p, K, nonuni):
    """Points, pattern and every CSR value of M and K vs the oracle."""
    from oracle import wq

    knots = [nonuniform_knots(k, p, 60 + 3 * p + d) if nonuni else W.open_uniform_knots(k, p)
             for d, k in enumerate(K)]
    plan = _plan(ig, p, K, knots)
    npts = []
    for d in range(3):
        x = plan.wq_points(d)
        xo, _ = wq.points_1d(knots[d], p)
        np.testing.assert_allclose(x, xo, rtol=0, atol=1e-15)
        npts.append(len(x))
    rng = np.random.default_rng(100 + p)
    kap = np.exp(0.5 * rng.standard_normal((npts[2], npts[1], npts[0])))
    rp_o, col_o, Mo, Ko = wq.assemble(knots, p, kap)
    rp, col = plan.csr_pattern()
    assert np.array_equal(to_host(rp), rp_o) and np.array_equal(to_host(col), col_o)
    Mv, Kv = plan.wq_assemble(to_dev(kap))
    assert csr_close(to_host(Mv), Mo, rp_o, TOL) and csr_close(to_host(Kv), Ko, rp_o, TOL)
    # one matrix at a time gives the same bits; repeated calls too
    Mv2, _ = plan.wq_assemble(to_dev(kap), want_k=False)
    _, Kv2 = plan.wq_assemble(to_dev(kap), want_m=False)
    import torch

    torch.cuda.synchronize()
    assert torch.equal(Mv, Mv2) and torch.equal(Kv, Kv2)


@pytest.mark.parametrize("p,K", [(2, (16, 14, 12)), (3, (20, 18, 16)), (4, (12, 11, 10)), (5, (10, 9, 8))])
def test_wq_constant_kappa_is_galerkin(orc, ig, p, K):
    """kappa = 1: the weighted-quadrature matrices are the exact Galerkin
    matrices; every value vs the Kronecker form of the oracle's 1D Gauss
    matrices (exact for kappa = 1)."""
    from oracle import wq

    knots = [nonuniform_knots(k, p, 7 * p + d) for d, k in enumerate(K)]
    plan = _plan(ig, p, K, knots)
    npts = [len(plan.wq_points(d)) for d in range(3)]
    Mv, Kv = plan.wq_assemble(to_dev(np.ones((npts[2], npts[1], npts[0]))))
    rp, col = plan.csr_pattern()
    rp, col = to_host(rp), to_host(col)
    G = [wq._gram_1d(knots[d], p) for d in range(3)]
    (ix, iy, iz), (jx, jy, jz) = _rows_cols(rp, col, [k + p for k in K])
    M1 = [G[d][0] for d in range(3)]
    A1 = [G[d][1] for d in range(3)]
    Mref = M1[0][ix, jx] * M1[1][iy, jy] * M1[2][iz, jz]
    Kref = (A1[0][ix, jx] * M1[1][iy, jy] * M1[2][iz, jz] + M1[0][ix, jx] * A1[1][iy, jy] * M1[2][iz, jz]
            + M1[0][ix, jx] * M1[1][iy, jy] * A1[2][iz, jz])
    assert csr_close(to_host(Mv), Mref, rp, TOL) and csr_close(to_host(Kv), Kref, rp, TOL)


def test_wq_headline_mesh_fullscale(orc, ig):
    """64^3, p = 3, kappa = 1 + 0.5 s(x) s(y) s(z) (s = sin 2 pi .) at the
    points: by linearity and the tensor structure of the rules,
    M = Mz My Mx + 0.5 Sz Sy Sx and K = the three derivative placements, with
    the oracle's 1D rule matrices (S_d, T_d with the weight s); all
    95 443 993 values of each matrix, plus 24 complete rows vs the oracle."""
    from oracle import wq

    p, K = W.W2["p"], W.W2["K"]
    knots = [W.open_uniform_knots(k, p) for k in K]
    plan = _plan(ig, p, K, knots)
    R = wq.rules(knots, p)
    xs = [plan.wq_points(d) for d in range(3)]
    s = [np.sin(2 * np.pi * x) for x in xs]
    kap = 1.0 + 0.5 * np.einsum("k,j,i->kji", s[2], s[1], s[0])
    Mv, Kv = plan.wq_assemble(to_dev(kap))
    rp, col = plan.csr_pattern()
    rp, col, Mvh, Kvh = to_host(rp), to_host(col), to_host(Mv), to_host(Kv)
    del Mv, Kv
    assert rp[-1] == 95443993
    m1 = [R[d].matrices() for d in range(3)]
    s1 = [R[d].matrices(s[d]) for d in range(3)]
    (ix, iy, iz), (jx, jy, jz) = _rows_cols(rp, col, [k + p for k in K])
    Mref = (m1[0][0][ix, jx] * m1[1][0][iy, jy] * m1[2][0][iz, jz]
            + 0.5 * s1[0][0][ix, jx] * s1[1][0][iy, jy] * s1[2][0][iz, jz])
    assert relfro(Mvh, Mref) <= TOL and rowmax_rel(Mvh, Mref, rp) <= TOL
    del Mref
    Kref = (m1[0][1][ix, jx] * m1[1][0][iy, jy] * m1[2][0][iz, jz]
            + m1[0][0][ix, jx] * m1[1][1][iy, jy] * m1[2][0][iz, jz]
            + m1[0][0][ix, jx] * m1[1][0][iy, jy] * m1[2][1][iz, jz]
            + 0.5 * (s1[0][1][ix, jx] * s1[1][0][iy, jy] * s1[2][0][iz, jz]
                     + s1[0][0][ix, jx] * s1[1][1][iy, jy] * s1[2][0][iz, jz]
                     + s1[0][0][ix, jx] * s1[1][0][iy, jy] * s1[2][1][iz, jz]))
    assert relfro(Kvh, Kref) <= TOL and rowmax_rel(Kvh, Kref, rp) <= TOL
    del Kref, ix, iy, iz, jx, jy, jz
    N = [k + p for k in K]
    rng = np.random.default_rng(13)
    dofs = [0, N[0] * N[1] * N[2] - 1, N[0] - 1, 2 + N[0] * (3 + N[1] * 4)] + list(rng.integers(0, N[0] * N[1] * N[2], 20))
    for d, (c, m, k) in zip(dofs, wq.rows(knots, p, kap, dofs)):
        a, b = rp[d], rp[d + 1]
        assert np.array_equal(col[a:b], c)
        assert relfro(Mvh[a:b], m) <= TOL and relfro(Kvh[a:b], k) <= TOL


def test_wq_errors(ig):
    """Before igaf_wq_prepare the calls are refused; a repeated interior knot
    (an element of zero length) is refused by the preparation."""
    import ctypes

    p, K = 2, (3, 3, 3)
    plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
    L = ig.lib()
    n = ctypes.c_int64()
    assert L.igaf_wq_points(plan.handle, 0, ctypes.byref(n), None) == ig.EINVAL
    dummy = to_dev(np.zeros(4))
    assert L.igaf_wq_assemble(plan.handle, dummy.data_ptr(), dummy.data_ptr(), None, None) == ig.EINVAL
    t = W.repeated_knots([0.5], [2], p)
    Kr = len(t) - 2 * p - 1
    plan2 = ig.Plan(p, (Kr, 2, 2), [t, W.open_uniform_knots(2, p), W.open_uniform_knots(2, p)])
    with pytest.raises(ig.IgafError) as ei:
        plan2.wq_prepare()
    assert ei.value.status == ig.EUNSUPPORTED
