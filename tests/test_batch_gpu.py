"""Batched launch (igaf_batch_integrate_assemble): many independent
patches of uneven sizes and degrees from one work list (one launch per
degree).

Checked against the oracle (small patches, every CSR value), against the
per-patch launches (the 256-patch workload, every value), and under HIP graph
capture (every replay equals the eager result bitwise).
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import csr_close, nonuniform_knots, relfro, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ig():
    import torch

    assert torch.cuda.is_available()
    from paper_2207_00280_amd import igafem

    return igafem


def _small_specs(seed):
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(12):
        p = int(rng.integers(1, 6))
        K = tuple(int(v) for v in rng.integers(1, 6 if p <= 3 else 4, size=3))
        knots = [nonuniform_knots(k, p, 1000 * seed + 10 * i + d) if i % 2 else W.open_uniform_knots(k, p)
                 for d, k in enumerate(K)]
        specs.append((p, K, knots))
    return specs


def test_batch_small_vs_oracle(orc, ig):
    """12 seeded patches (p = 1..5, K_d = 1..5 (1..3 at p >= 4), uniform and non-uniform knots)
    in one batched call, every CSR value vs the oracle's assembly."""
    import torch

    specs = _small_specs(3)
    B = ig.Batch(specs)
    kaps, Ms, Ks, refs = [], [], [], []
    for i, (p, K, knots) in enumerate(specs):
        P = orc.Patch(p, K, [p + 1] * 3, knots)
        kap = W.kappa_lognormal(P.nelem, P.nq, seed=50 + i)
        refs.append(orc.assemble(P, kap))
        kaps.append(to_dev(kap))
        Ms.append(torch.full((B.plans[i].nnz,), np.nan, dtype=torch.float64, device="cuda"))
        Ks.append(torch.full((B.plans[i].nnz,), np.nan, dtype=torch.float64, device="cuda"))
    B.integrate_assemble(kaps, Ms, Ks)
    torch.cuda.synchronize()
    for i, (rp, col, Mo, Ko) in enumerate(refs):
        assert csr_close(to_host(Ms[i]), Mo, rp), i
        assert csr_close(to_host(Ks[i]), Ko, rp), i
    info = B.info()
    assert info["family"] == 0 and info["grid"] >= info["nitems"] > 0
    # the second tile shape of every degree vs the oracle too
    for p in range(1, 6):
        B.set_degree_config(p, 1, 1, 16)
    Ma = [torch.full_like(m, np.nan) for m in Ms]
    Ka = [torch.full_like(k, np.nan) for k in Ks]
    B.integrate_assemble(kaps, Ma, Ka)
    torch.cuda.synchronize()
    for i, (rp, col, Mo, Ko) in enumerate(refs):
        assert csr_close(to_host(Ma[i]), Mo, rp) and csr_close(to_host(Ka[i]), Ko, rp), i
    B.set_split(1, 16)
    # mass only
    Ms2 = [torch.zeros_like(m) for m in Ms]
    B.integrate_assemble(kaps, Ms2, None)
    torch.cuda.synchronize()
    for a, b in zip(Ms, Ms2):
        assert torch.equal(a, b)


def test_batch_graph_replay(ig):
    """The batched launch captured in a HIP graph: three replays, with
    eager work between them, each equal to the eager result; a replay after a
    re-split (and an eager call with the new split) still equals it."""
    import torch

    specs = _small_specs(7)
    B = ig.Batch(specs)
    kaps = [to_dev(W.kappa_lognormal(pl.nelem, pl.nqp, seed=i)) for i, pl in enumerate(B.plans)]
    Ms = [torch.empty(pl.nnz, dtype=torch.float64, device="cuda") for pl in B.plans]
    Ks = [torch.empty(pl.nnz, dtype=torch.float64, device="cuda") for pl in B.plans]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B.integrate_assemble(kaps, Ms, Ks, stream=s)
    torch.cuda.synchronize()
    ref = [m.clone() for m in Ms] + [k.clone() for k in Ks]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        B.integrate_assemble(kaps, Ms, Ks, stream=s)
    for r in range(3):
        for t in Ms + Ks:
            t.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = Ms + Ks
        for a, b in zip(got, ref):
            assert torch.equal(a, b), r
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
    # a re-split after capture selects another work list; the graph keeps the
    # list it was captured with, and an eager call with the new split and the
    # same pointers gives the same bits
    B.set_split(8, 4)
    for t in Ms + Ks:
        t.fill_(-1.0)
    B.integrate_assemble(kaps, Ms, Ks)
    torch.cuda.synchronize()
    for a, b in zip(Ms + Ks, ref):
        assert torch.equal(a, b)
    for t in Ms + Ks:
        t.fill_(-1.0)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for a, b in zip(Ms + Ks, ref):
        assert torch.equal(a, b)


def test_batch_autotune(ig):
    """The autotuner times, per degree, every configuration (tile shape 0 or
    1, segments per tile 1, 2, 4, 8, items per XCD chunk 4, 16, 64) and keeps
    the fastest.  Patches long enough in x to be cut into segments (K_x up to
    40, p = 1..5): the values after tuning equal the untuned launch bit for
    bit (each CSR value is summed by one thread in a fixed order whatever the
    tile or split), and match the per-patch launches; forced splits and the
    second tile shape of every degree also give the same bits."""
    import torch

    rng = np.random.default_rng(17)
    specs = []
    for i in range(10):
        p = int(rng.integers(1, 6))
        K = (int(rng.integers(20, 41)), int(rng.integers(2, 7)), int(rng.integers(2, 6)))
        specs.append((p, K, [W.open_uniform_knots(k, p) for k in K]))
    B = ig.Batch(specs)
    assert B.split() == {"split": 1, "chunk": 16, "ms": 0.0}
    kaps = [to_dev(W.kappa_lognormal(pl.nelem, pl.nqp, seed=300 + i)) for i, pl in enumerate(B.plans)]
    Ms = [torch.empty(pl.nnz, dtype=torch.float64, device="cuda") for pl in B.plans]
    Ks = [torch.empty(pl.nnz, dtype=torch.float64, device="cuda") for pl in B.plans]
    B.integrate_assemble(kaps, Ms, Ks)
    torch.cuda.synchronize()
    ref = [m.clone() for m in Ms] + [k.clone() for k in Ks]
    n_untuned = B.info()["nitems"]
    sp = B.autotune(kaps, Ms, Ks, reps=1)
    assert sp["split"] in (1, 2, 4, 8) and sp["chunk"] in (4, 16, 64) and sp["ms"] > 0
    assert B.info()["nitems"] >= n_untuned
    for t in Ms + Ks:
        t.fill_(np.nan)
    B.integrate_assemble(kaps, Ms, Ks)
    torch.cuda.synchronize()
    for a, b in zip(Ms + Ks, ref):
        assert torch.equal(a, b)
    Ms2 = [torch.empty_like(m) for m in Ms]
    Ks2 = [torch.empty_like(k) for k in Ks]
    B.integrate_assemble(kaps, Ms2, Ks2, separate=True)
    torch.cuda.synchronize()
    for a, b in zip(Ms + Ks, Ms2 + Ks2):
        assert float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) <= 1e-12
    for p in range(1, 6):
        c = B.degree_config(p)
        assert c["tile"] in (0, 1) and c["split"] in (1, 2, 4, 8) and c["chunk"] in (4, 16, 64)
    for split, chunk in ((8, 4), (2, 64)):
        B.set_split(split, chunk)
        assert B.split()["split"] == split and B.info()["nitems"] > n_untuned
        for t in Ms + Ks:
            t.fill_(np.nan)
        B.integrate_assemble(kaps, Ms, Ks)
        torch.cuda.synchronize()
        for a, b in zip(Ms + Ks, ref):
            assert torch.equal(a, b), (split, chunk)
    # the second tile shape of every degree, forced: the same bits
    for p in range(1, 6):
        B.set_degree_config(p, 1, 2, 16)
        assert B.degree_config(p)["tile"] == 1
    for t in Ms + Ks:
        t.fill_(np.nan)
    B.integrate_assemble(kaps, Ms, Ks)
    torch.cuda.synchronize()
    for a, b in zip(Ms + Ks, ref):
        assert torch.equal(a, b)
    with pytest.raises(ig.IgafError):
        B.set_degree_config(3, 2, 1, 16)
    with pytest.raises(ig.IgafError):
        B.autotune(kaps, Ms, Ks, reps=0)
    with pytest.raises(ig.IgafError):
        B.set_split(3, 16)


def test_w4_batch_fullscale(orc, ig):
    """256 patches (seed 1): K_d ~ U{8..48}, p ~ U{2..5}, log-normal kappa.
    The batched launch equals the 256 per-patch launches value for value
    (same arithmetic per value; relative Frobenius <= 1e-12 per patch), and
    complete rows of 4 patches equal the oracle's."""
    import torch

    shapes = W.batch_patches(**{k: W.W4[k] for k in ("npatch", "seed", "kmin", "kmax", "ps")})
    kap_h = W.batch_kappas(shapes, seed=W.W4["seed"])
    specs = [(d["p"], d["K"], [W.open_uniform_knots(k, d["p"]) for k in d["K"]]) for d in shapes]
    B = ig.Batch(specs)
    kaps = [to_dev(k) for k in kap_h]
    Ms = [torch.empty(pl.nnz, dtype=torch.float64, device="cuda") for pl in B.plans]
    Ks = [torch.empty(pl.nnz, dtype=torch.float64, device="cuda") for pl in B.plans]
    B.integrate_assemble(kaps, Ms, Ks)
    torch.cuda.synchronize()
    Ms2 = [torch.empty_like(m) for m in Ms]
    Ks2 = [torch.empty_like(k) for k in Ks]
    B.integrate_assemble(kaps, Ms2, Ks2, separate=True)
    torch.cuda.synchronize()
    for i in range(len(Ms)):
        for a, b in ((Ms[i], Ms2[i]), (Ks[i], Ks2[i])):
            err = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
            assert err <= 1e-12, (i, err)
    del Ms2, Ks2
    rng = np.random.default_rng(4)
    for i in [int(np.argmax([d["p"] for d in shapes]))] + list(rng.integers(0, len(shapes), 3)):
        p, K, knots = specs[i]
        P = orc.Patch(p, K, [p + 1] * 3, knots)
        rp, col = B.plans[i].csr_pattern()
        rph = to_host(rp)
        dofs = np.concatenate([[0, P.ndof - 1], rng.integers(0, P.ndof, 6)])
        for d, (c, m, k) in zip(dofs, orc.rows(P, kap_h[i], dofs)):
            a, b = int(rph[d]), int(rph[d + 1])
            assert np.array_equal(to_host(col[a:b]), c)
            assert relfro(to_host(Ms[i][a:b]), m) <= 1e-12
            assert relfro(to_host(Ks[i][a:b]), k) <= 1e-12
