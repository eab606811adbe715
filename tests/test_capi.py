"""C-ABI contract tests that need no GPU: the library loads, exports every
symbol include/igafem.h declares, and its host-side logic (argument checks,
sizes, the structural CSR pattern) is right.  Pattern pins come from the
oracle's brute-force union of element pairs."""
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2207_00280_amd import igafem as ig

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "igafem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(igaf_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = ig.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(ig.SYMBOLS) == names


def test_version():
    assert "gfx950" in ig.version()


@pytest.mark.parametrize("p,K", [(1, (3, 2, 4)), (2, (8, 8, 8)), (3, (5, 4, 3)), (4, (2, 3, 1)),
                                 (5, (1, 2, 2))])
def test_sizes_and_pattern_vs_oracle(orc, p, K):
    """nnz closed form prod_d (N_d (2p+1) - p (p+1)); the host pattern equals the
    oracle's brute-force union of element pairs, bit for bit."""
    knots = [W.open_uniform_knots(k, p) for k in K]
    d = ig.make_desc(p, K, knots)
    sz = ig.desc_sizes(d)
    N = [k + p for k in K]
    assert sz["ndof"] == N[0] * N[1] * N[2]
    assert sz["nelem"] == K[0] * K[1] * K[2]
    assert sz["nqp"] == (p + 1) ** 3
    assert sz["elem_dim"] == (p + 1) ** 3
    assert sz["nnz"] == np.prod([n * (2 * p + 1) - p * (p + 1) for n in N])
    rp, col = ig.csr_pattern_host(d)
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    rp_o, col_o, _, _ = orc.assemble(P, W.kappa_constant(P.nelem, P.nq))
    assert rp.dtype == np.int64 and col.dtype == np.int32
    assert np.array_equal(rp, rp_o)
    assert np.array_equal(col, col_o)


def test_headline_sizes():
    """64^3 elements, p=3: 67^3 DOFs and 95 443 993 structural nonzeros."""
    d = ig.make_desc(3, (64, 64, 64), [W.open_uniform_knots(64, 3)] * 3)
    sz = ig.desc_sizes(d)
    assert sz["ndof"] == 67 ** 3 and sz["nnz"] == 95443993


def _bad(p=2, K=(3, 3, 3), knots=None, q=None):
    if knots is None:
        knots = [W.open_uniform_knots(k, p) for k in K]
    return ig.make_desc(p, K, knots, q)


@pytest.mark.parametrize("case,frag", [
    ("p0", "degree"),
    ("K0", "nelem"),
    ("q0", "nquad"),
    ("q17", "nquad"),
    ("decreasing", "decreases"),
    ("not_open", "open"),
    ("knot_repeated_p_plus_2", "empty support"),
    ("nan", "finite"),
])
def test_desc_errors(case, frag):
    kn = W.open_uniform_knots(3, 2)
    if case == "p0":
        d = _bad(p=0, knots=[W.open_uniform_knots(3, 0)] * 3)
    elif case == "K0":
        d = _bad(K=(3, 0, 3), knots=[kn, W.open_uniform_knots(1, 2)[:5], kn])
    elif case == "q0":
        d = _bad(q=(3, 0, 3))
    elif case == "q17":
        d = _bad(q=(3, 3, 17))
    elif case == "decreasing":
        k2 = kn.copy()
        k2[3], k2[4] = k2[4], k2[3]
        d = _bad(knots=[kn, k2, kn])
    elif case == "not_open":
        k2 = kn.copy()
        k2[0] = -0.1
        d = _bad(knots=[kn, kn, k2])
    elif case == "knot_repeated_p_plus_2":
        k2 = kn.copy()
        k2[3] = k2[0]          # p+2 equal first knots: function 0 vanishes identically
        d = _bad(knots=[k2, kn, kn])
    elif case == "nan":
        k2 = kn.copy()
        k2[3] = float("nan")
        d = _bad(knots=[kn, k2, kn])
    st, msg = ig.desc_check(d)
    assert st == ig.EINVAL
    assert frag in msg
    with pytest.raises(ig.IgafError) as ei:
        ig.desc_sizes(d)
    assert ei.value.status == ig.EINVAL


@pytest.mark.parametrize("p", [1, 2, 3])
def test_repeated_interior_knots_accepted(orc, p):
    """Interior multiplicity up to p+1 (down to C^-1) is valid input: the
    sizes follow K = len - 2p - 1 spans (empty ones included), and the host
    CSR pattern equals the oracle's union of element pairs."""
    knots = [W.repeated_knots([0.3, 0.7], [p, p + 1], p), W.repeated_knots([0.5], [2], p),
             W.open_uniform_knots(2, p)]
    K = tuple(len(t) - 2 * p - 1 for t in knots)
    d = ig.make_desc(p, K, knots)
    assert ig.desc_check(d)[0] == ig.OK
    sz = ig.desc_sizes(d)
    P = orc.Patch(p, K, [p + 1] * 3, knots)
    assert sz["ndof"] == P.ndof and sz["nelem"] == P.nelem
    kap = np.ones((P.nelem, P.nq))
    rp_o, col_o, _, _ = orc.assemble(P, kap)
    rp, col = ig.csr_pattern_host(d)
    assert sz["nnz"] == len(col_o)
    assert np.array_equal(rp, rp_o) and np.array_equal(col, col_o)


def test_null_arguments():
    L = ig.lib()
    assert L.igaf_desc_check(None) == ig.EINVAL
    assert "NULL" in L.igaf_last_error().decode()
    assert L.igaf_plan_create(None, None) == ig.EINVAL
    assert L.igaf_plan_sizes(None, None, None, None, None, None) == ig.EINVAL
    assert L.igaf_element_matrices(None, 1, None, None, None, None) == ig.EINVAL
    assert L.igaf_integrate_assemble(None, 1, None, None, None, None, None, None) == ig.EINVAL
    assert L.igaf_kappa_grad(None, None, None, 1.0, 1.0, 1.0, None, None, None) == ig.EINVAL
    assert L.igaf_bilinear_form(None, None, None, None, 1.0, 1.0, None, None) == ig.EINVAL
    assert L.igaf_apply(None, None, None, 1.0, 1.0, None, None, None) == ig.EINVAL
    assert L.igaf_apply_workspace(None) == 0
    assert L.igaf_apply_static(None, None, None, 1.0, 1.0, None, None) == ig.EINVAL
    assert L.igaf_euler_step(None, None, None, 0.1, 1e-12, 10, 1, None, None, None, None, None) == ig.EINVAL
    assert L.igaf_euler_workspace(None) == 0
    assert L.igaf_assemble(None, None, None, None, None, None) == ig.EINVAL
    assert L.igaf_batch_create(None, 0, None) == ig.EINVAL
    L.igaf_plan_destroy(None)
    L.igaf_batch_destroy(None)


def test_plan_create_rejects_before_device():
    """Invalid descriptions fail on the host before any device call (so this
    runs without a GPU)."""
    import ctypes

    L = ig.lib()
    h = ctypes.c_void_p()
    d = _bad(p=0, knots=[W.open_uniform_knots(3, 0)] * 3)
    assert L.igaf_plan_create(ctypes.byref(d), ctypes.byref(h)) == ig.EINVAL
    assert h.value is None


def _local_values(orc, t, p, e):
    """Values and derivatives of the p+1 functions of element e at its Gauss
    nodes (oracle Cox-de Boor), derivatives scaled by the element length."""
    xi, _ = orc.gauss_legendre(p + 1)
    lo, hi = t[e + p], t[e + p + 1]
    out = []
    for x in lo + 0.5 * (xi + 1.0) * (hi - lo):
        B, dB = orc.basis_all(t, p, x)
        out.append(np.concatenate([B[e:e + p + 1], dB[e:e + p + 1] * (hi - lo)]))
    return np.array(out)


@pytest.mark.parametrize("p,K", [(1, 9), (2, 12), (3, 37), (5, 48), (3, 5), (4, 7)])
def test_shared_table_run(orc, p, K):
    """Uniform spacing: the run is every element but the p - 1 nearest each
    end (their windows hold the repeated end knots), it is the longest run of
    elements whose knot differences agree with its first element's, and the
    oracle's basis values on every element of the run equal those on its
    first element (the tables the plan shares); the elements just outside
    differ."""
    t = W.open_uniform_knots(K, p)
    d = ig.make_desc(p, (K, 4, 4), [t, W.open_uniform_knots(4, p), W.open_uniform_knots(4, p)])
    r0, r1 = ig.desc_shared_run(d, 0)
    lo, hi = p - 1, K - p + 1
    if hi - lo >= 2:
        assert (r0, r1) == (lo, hi)
    else:
        assert (r0, r1) == (0, 0)
        return
    ref = _local_values(orc, t, p, r0)
    for e in range(r0, r1):
        assert np.abs(_local_values(orc, t, p, e) - ref).max() <= 1e-12 * np.abs(ref).max()
    for e in (r0 - 1, r1):
        if 0 <= e < K:
            assert np.abs(_local_values(orc, t, p, e) - ref).max() > 1e-3


def test_shared_table_run_nonuniform():
    """Graded knots share nothing; one interior knot moved splits the uniform
    run, and the longer side is kept (brute force over all starting points)."""
    p, K = 3, 20
    g = np.concatenate([[0.0] * p, (np.arange(K + 1) / K) ** 2, [1.0] * p])
    d = ig.make_desc(p, (K, 4, 4), [g, W.open_uniform_knots(4, p), W.open_uniform_knots(4, p)])
    assert ig.desc_shared_run(d, 0) == (0, 0)
    t = W.open_uniform_knots(K, p)
    t[p + 6] += 0.3 / K   # knot p+6 lies in the windows t_{e+1} .. t_{e+2p} of e = 3 .. 8
    d = ig.make_desc(p, (K, 4, 4), [t, W.open_uniform_knots(4, p), W.open_uniform_knots(4, p)])
    r0, r1 = ig.desc_shared_run(d, 0)

    def same(e, r):
        for j in range(1, 2 * p + 1):
            sc = max(abs(t[e + j]), abs(t[e + p]), abs(t[r + j]), abs(t[r + p]))
            if abs((t[e + j] - t[e + p]) - (t[r + j] - t[r + p])) > 8 * np.finfo(float).eps * sc:
                return False
        return True

    best = max((e - s, s) for s in range(K) for e in range(s + 1, K + 1)
               if all(same(i, s) for i in range(s, e)))
    assert r1 - r0 == best[0] and (r0, r1) == (9, K - p + 1)
    for e in range(r0, r1):
        assert same(e, r0)
