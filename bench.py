"""Benchmark of the B-spline element-integration hot path on one MI355X.

Headline workload: unit cube, 64^3 uniform elements, p=3 (C^2 open uniform
knots), 4-point Gauss rule per direction, kappa = 1 + 0.5 sin(2 pi x)
sin(2 pi y) sin(2 pi z) at the quadrature points, FP64.  One step = one
igaf_integrate_assemble call (sum factorisation) that produces the dense
element matrices M_e and K_e of all 262 144 elements AND the CSR values of
the global M and K (95 443 993 nonzeros each).  Inputs are resident in HBM
before the timed region; inputs are synthetic (seeded).

The same run also times, on the same GPU: the element kernel and the CSR
kernel alone (roofline of the dominant kernel), classical quadrature, the
atomic assembly, the 128^3 streamed workload (p = 2, 3, 4), the 256-patch
batched launches (one per degree) against 256 separate launches (eager and
graph-captured), the adjoint, the matrix-free operator apply and one forward
Euler step (conjugate gradients on M) against the plain forward assembly,
the headline mesh on a curved geometry map;
and the CPU oracle on a bounded sample of the headline workload.

Prints ONE JSON line on stdout.  --mode kernel:<name> runs one kernel only
(for profiler counter passes).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "element matrices/s (mass+stiffness, 64^3 p=3, FP64) + % HBM/FP64 roofline"
HBM_PEAK = 8.0e12        # bytes/s, MI355X published
FP64_PEAK = 78.6e12      # flop/s, MI355X published (vector = matrix)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_element_sumfact_64c_p3.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_fp64_and_rows.json")
ELEMENT_SRC = os.path.join(ROOT, "paper_2207_00280_amd", "csrc", "element.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sumfact_flops(p):
    """Minimum sum-factorisation flops per element (M and K) with symmetric
    pairs: stage z 4 S q^3, stage y 6 S^2 q^2, stage x 6 S^3 q."""
    n = p + 1
    q = p + 1
    S = n * (n + 1) // 2
    return 4 * S * q ** 3 + 6 * S * S * q * q + 6 * S ** 3 * q


def timed(fn, steps, warmup, stream):
    """fn() `warmup` times, then `steps` calls bracketed by HIP events recorded
    on `stream` (the stream the kernels run on); per-call milliseconds."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for i in range(steps):
        fn()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    return [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]


def src_hash(path):
    """Hash of a kernel source and the local headers it includes (one level
    deep, in include order): a profile taken on the kernel stays attached to
    it only while none of them changes."""
    import re

    h = hashlib.sha256()
    text = open(path, "rb").read()
    h.update(text)
    for inc in re.findall(rb'#include "([^"]+)"', text):
        h.update(open(os.path.join(os.path.dirname(path), inc.decode()), "rb").read())
    return h.hexdigest()[:16]


def element_src_hash():
    return src_hash(ELEMENT_SRC)


def classical_flops(p):
    """FP64 flops the classical kernel executes per element: for each of the
    S^3 distinct (M, K) value pairs, 3 fused multiply-adds and 2 multiplies
    at each of the q^3 points and 1 fused multiply-add and 2 multiplies per
    (ky, kz) point pair for the y-z factors (8 q^3 + 4 q^2 flops; the inner
    loop of k_element<P,0>, matched by the rocprofv3 FMA_F64/MUL_F64 counts)."""
    n = q = p + 1
    S = n * (n + 1) // 2
    return S ** 3 * (8 * q ** 3 + 4 * q ** 2)


def counters_for_current_sources():
    """Per-kernel rocprofv3 counter summaries (FP64 and instruction counts)
    from the committed passes, for kernels whose source (with its local
    headers) is unchanged since the counters were taken."""
    try:
        t = json.load(open(COUNTERS_FILE))
    except (OSError, ValueError):
        return None
    out = {}
    for name, e in t.get("kernels", {}).items():
        path = os.path.join(ROOT, e["source"])
        try:
            cur = src_hash(path)
        except OSError:
            continue
        if cur != e["src_sha256_16"]:
            continue
        c = e["counters_per_launch"]
        out[name] = {"workload": e["workload"], "fma_f64": c.get("SQ_INSTS_VALU_FMA_F64"),
                     "mul_f64": c.get("SQ_INSTS_VALU_MUL_F64"), "add_f64": c.get("SQ_INSTS_VALU_ADD_F64"),
                     "mfma": c.get("SQ_INSTS_MFMA"), "valu": c.get("SQ_INSTS_VALU"), "salu": c.get("SQ_INSTS_SALU"),
                     "smem": c.get("SQ_INSTS_SMEM"), "lds": c.get("SQ_INSTS_LDS"),
                     "lds_bank_conflict_cycles": c.get("SQ_LDS_BANK_CONFLICT"), "waves": c.get("SQ_WAVES"),
                     "fp64_flops_upper": e["fp64_flops_upper"]}
    return out


def traffic_for_current_kernel():
    """HBM bytes per launch of the element kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE passes, if they were taken on the
    current kernel source; else None."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("element_src_sha256_16") != element_src_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(nsample, chunk=4096):
    """The CPU oracle (classical quadrature, M_e and K_e) on the first
    `nsample` elements of the headline workload, all host threads; then, as
    context, one thread on 4 096 elements (per-core rate), the W1 mesh, the
    W3 degrees on 512-element meshes (rates extrapolated to 128^3) and the W5
    reference gradient on every point."""
    import oracle

    P = oracle.Patch(3, (64, 64, 64), (4, 4, 4), [W.open_uniform_knots(64, 3)] * 3)
    xs = [oracle.quad_nodes(P, d)[0] for d in range(3)]
    kap = W.kappa_sine(*xs)
    t0 = time.perf_counter()
    for e0 in range(0, nsample, chunk):
        oracle.element_matrices(P, kap, e0, min(nsample, e0 + chunk))
    dt = time.perf_counter() - t0
    cores = oracle.num_threads()
    out = {"value": nsample / dt, "unit": "element matrices/s", "cores": cores, "kind": "oracle",
           "sample": "first %d of the 262144 elements of the headline workload (classical "
                     "quadrature, M_e and K_e, no assembly), %.1f s" % (nsample, dt)}
    extra = {}
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.element_matrices(P, kap, 0, 4096)
    extra["w2_one_thread_elements_per_s"] = 4096 / (time.perf_counter() - t0)
    oracle.set_num_threads(cores)
    P1 = oracle.Patch(2, (8, 8, 8), (3, 3, 3), [W.open_uniform_knots(8, 2)] * 3)
    t0 = time.perf_counter()
    oracle.assemble(P1, W.kappa_constant(512, 27))
    extra["w1_full_mesh_s"] = time.perf_counter() - t0
    for p in (2, 3, 4):
        # the per-element cost does not depend on the mesh: 8^3 elements of the
        # same degree and rule stand for the 128^3 mesh
        Pp = oracle.Patch(p, (8, 8, 8), (p + 1,) * 3, [W.open_uniform_knots(8, p)] * 3)
        kp = W.kappa_lognormal(Pp.nelem, Pp.nq, seed=0)
        t0 = time.perf_counter()
        oracle.element_matrices(Pp, kp)
        rate = Pp.nelem / (time.perf_counter() - t0)
        extra["w3_p%d_elements_per_s_extrapolated" % p] = rate
        extra["w3_p%d_whole_mesh_s_extrapolated" % p] = 128 ** 3 / rate
    u = W.normal_vector(99 ** 3, 3)
    v = W.normal_vector(99 ** 3, 4)
    P5 = oracle.Patch(3, (96, 96, 96), (4, 4, 4), [W.open_uniform_knots(96, 3)] * 3)
    t0 = time.perf_counter()
    oracle.kappa_grad(P5, u, v)
    dt5 = time.perf_counter() - t0
    extra["w5_gradient_all_points_s"] = dt5
    extra["w5_gradient_points_per_s"] = P5.nelem * P5.nq / dt5
    out["context"] = extra
    return out


def measured_peaks(torch, stream):
    """Write and copy bandwidth of plain torch kernels on 8 GiB / 4 GiB
    buffers, and the FP64 rate of a library DGEMM (torch.matmul, 8192^2) on
    this GPU (context for the HBM and FP64 fractions)."""
    a = torch.empty(1 << 30, dtype=torch.float64, device="cuda")
    ms_f = min(timed(lambda: a.fill_(1.0), 5, 1, stream))
    b = a[: 1 << 29]
    c = a[1 << 29:]
    ms_c = min(timed(lambda: c.copy_(b), 5, 1, stream))
    del a, b, c
    torch.cuda.empty_cache()
    m = 8192
    x = torch.rand(m, m, dtype=torch.float64, device="cuda")
    y = torch.rand(m, m, dtype=torch.float64, device="cuda")
    z = torch.empty_like(x)
    ms_g = min(timed(lambda: torch.matmul(x, y, out=z), 3, 1, stream))
    del x, y, z
    torch.cuda.empty_cache()
    return {"write_GB/s": 8 * (1 << 30) / (ms_f * 1e-3) / 1e9,
            "copy_GB/s": 2 * 8 * (1 << 29) / (ms_c * 1e-3) / 1e9,
            "fp64_dgemm_TFLOP/s": 2.0 * m ** 3 / (ms_g * 1e-3) / 1e12}


class Headline:
    def __init__(self, ig, torch):
        p, K = 3, (64, 64, 64)
        self.p = p
        self.plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
        xs = [self.plan.quad_nodes(d)[0] for d in range(3)]
        self.kappa = torch.from_numpy(W.kappa_sine(*xs)).cuda()
        E, n3, nnz = self.plan.nelem, self.plan.elem_dim, self.plan.nnz
        self.Me = torch.empty(E, n3, n3, dtype=torch.float64, device="cuda")
        self.Ke = torch.empty_like(self.Me)
        self.Mval = torch.empty(nnz, dtype=torch.float64, device="cuda")
        self.Kval = torch.empty_like(self.Mval)
        self.ig = ig
        torch.cuda.synchronize()

    def step(self):
        self.plan.integrate_assemble(self.kappa, method=self.ig.SUMFACT, Me=self.Me, Ke=self.Ke,
                                     Mval=self.Mval, Kval=self.Kval)

    def element(self, method=None):
        self.plan.element_matrices(self.kappa, method=self.ig.SUMFACT if method is None else method,
                                   Me=self.Me, Ke=self.Ke)

    def csr(self):
        self.plan.integrate_assemble(self.kappa, want_elem=False, Mval=self.Mval, Kval=self.Kval)


def bench_w3(ig, torch, stream, steps):
    out = {}
    for p in W.W3["ps"]:
        K = W.W3["K"]
        plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
        kap = torch.from_numpy(W.kappa_lognormal(plan.nelem, plan.nqp, W.W3["seed"])).cuda()
        Mv = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
        Kv = torch.empty_like(Mv)
        ms = float(np.mean(timed(lambda: plan.integrate_assemble(kap, want_elem=False, Mval=Mv, Kval=Kv),
                                 steps, 2, stream)))
        b = plan.nelem * plan.nqp * 8 + 2 * plan.nnz * 8
        f = plan.nelem * sumfact_flops(p)
        troof = max(b / HBM_PEAK, f / FP64_PEAK)
        out["p%d" % p] = {"ms": ms, "elements_per_s": plan.nelem / (ms * 1e-3), "nnz": plan.nnz,
                          "bytes": b, "GB/s": b / (ms * 1e-3) / 1e9, "roofline_ms": troof * 1e3,
                          "frac": troof / (ms * 1e-3)}
        log("W3 p=%d: %.3f ms (%.1f%% of roofline)" % (p, ms, 100 * troof / (ms * 1e-3)))
        del kap, Mv, Kv, plan
        torch.cuda.empty_cache()
    return out


def bench_w4(ig, torch, stream, steps):
    shapes = W.batch_patches(**{k: W.W4[k] for k in ("npatch", "seed", "kmin", "kmax", "ps")})
    kap_h = W.batch_kappas(shapes, seed=W.W4["seed"])
    t0 = time.perf_counter()
    B = ig.Batch([(d["p"], d["K"], [W.open_uniform_knots(k, d["p"]) for k in d["K"]]) for d in shapes])
    t_create = time.perf_counter() - t0
    kaps = [torch.from_numpy(k).cuda() for k in kap_h]
    del kap_h
    Ms = [torch.empty(pl.nnz, dtype=torch.float64, device="cuda") for pl in B.plans]
    Ks = [torch.empty(pl.nnz, dtype=torch.float64, device="cuda") for pl in B.plans]
    E = sum(pl.nelem for pl in B.plans)
    nnz = sum(pl.nnz for pl in B.plans)
    b = sum(pl.nelem * pl.nqp * 8 for pl in B.plans) + 2 * nnz * 8
    f = sum(pl.nelem * sumfact_flops(pl.p) for pl in B.plans)
    troof = max(b / HBM_PEAK, f / FP64_PEAK)
    ms_untuned = float(np.mean(timed(lambda: B.integrate_assemble(kaps, Ms, Ks), steps, 2, stream)))
    t0 = time.perf_counter()
    tuned = B.autotune(kaps, Ms, Ks, reps=2, stream=stream)
    t_tune = time.perf_counter() - t0
    ms_b = float(np.mean(timed(lambda: B.integrate_assemble(kaps, Ms, Ks), steps, 2, stream)))
    ms_s = float(np.mean(timed(lambda: B.integrate_assemble(kaps, Ms, Ks, separate=True), steps, 2, stream)))
    # the 256 separate launches captured in one HIP graph and replayed
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B.integrate_assemble(kaps, Ms, Ks, separate=True, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        B.integrate_assemble(kaps, Ms, Ks, separate=True, stream=s)
    ms_g = float(np.mean(timed(g.replay, steps, 2, torch.cuda.current_stream())))
    # the batched launch captured and replayed
    with torch.cuda.stream(s):
        B.integrate_assemble(kaps, Ms, Ks, stream=s)
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=s):
        B.integrate_assemble(kaps, Ms, Ks, stream=s)
    ms_g2 = float(np.mean(timed(g2.replay, steps, 2, torch.cuda.current_stream())))
    info = B.info()
    info["degrees"] = {str(p): B.degree_config(p) for p in range(1, 6) if B.degree_config(p)["nitems"] > 0}
    out = {"patches": len(shapes), "elements": E, "nnz": nnz, "bytes": b, "flops": f,
           "roofline_ms": troof * 1e3,
           "batched": {"ms": ms_b, "elements_per_s": E / (ms_b * 1e-3), "frac": troof / (ms_b * 1e-3),
                       "work_split": tuned, "autotune_s": t_tune, "untuned_ms": ms_untuned},
           "batched_graph": {"ms": ms_g2, "elements_per_s": E / (ms_g2 * 1e-3)},
           "separate_eager": {"ms": ms_s, "elements_per_s": E / (ms_s * 1e-3)},
           "separate_graph": {"ms": ms_g, "elements_per_s": E / (ms_g * 1e-3)},
           "launch": info, "create_s": t_create}
    log("W4: batched %.2f ms (autotuned %s; %.2f ms untuned), graph %.2f ms, separate %.2f ms, "
        "separate graph %.2f ms (%s)" % (ms_b, tuned, ms_untuned, ms_g2, ms_s, ms_g, info))
    del Ms, Ks, kaps, B, g, g2
    torch.cuda.empty_cache()
    return out


def interp_fmas(p):
    """Fused multiply-adds per element of one field interpolated to the q^3
    points by sum factorisation with values and first derivatives, q = n =
    p+1: stage x 2n^4, stage y 3n^4, stage z 4n^4 (the transposed contraction
    of a weighted field back to the test functions costs the same)."""
    n = p + 1
    return 9 * n ** 4


def bench_w5(ig, torch, stream, steps):
    """W5 mesh: the adjoint dL/dkappa, and the matrix-free operator apply
    y = (M + K) u, each against the plain forward CSR assembly of the mesh;
    both are FP64-bound (about 10 kflop per element at p = 3)."""
    cfg = W.W5
    p, K = cfg["p"], cfg["K"]
    plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
    kap = torch.from_numpy(W.kappa_lognormal(plan.nelem, plan.nqp, cfg["seed_kappa"])).cuda()
    u = torch.from_numpy(W.normal_vector(plan.ndof, cfg["seed_u"])).cuda()
    v = torch.from_numpy(W.normal_vector(plan.ndof, cfg["seed_v"])).cuda()
    g = torch.empty_like(kap)
    y = torch.empty_like(u)
    Mv = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
    Kv = torch.empty_like(Mv)
    ms_a = float(np.mean(timed(lambda: plan.kappa_grad(u, v, grad=g), steps, 2, stream)))
    wk = torch.empty(plan.apply_workspace(), dtype=torch.float64, device="cuda")
    ms_y = float(np.mean(timed(lambda: plan.apply(kap, u, 1.0, 1.0, y=y, work=wk), steps, 2, stream)))
    ms_m = float(np.mean(timed(lambda: plan.apply(kap, u, 1.0, 0.0, y=y, work=wk), steps, 2, stream)))
    ms_f = float(np.mean(timed(lambda: plan.integrate_assemble(kap, want_elem=False, Mval=Mv, Kval=Kv),
                               steps, 2, stream)))
    q3, n3 = plan.nqp, (p + 1) ** 3
    # adjoint: two fields interpolated, combined at every point (6 FMA);
    # apply: one field interpolated and one contracted back, weighted at every point
    f_a = plan.nelem * 2.0 * (2 * interp_fmas(p) + 6 * q3)
    f_y = plan.nelem * 2.0 * (2 * interp_fmas(p) + 4 * q3)
    b_a = plan.nelem * q3 * 8 + 2 * plan.ndof * 8
    b_y = plan.nelem * q3 * 8 + 3 * plan.ndof * 8
    roof_a = max(b_a / HBM_PEAK, f_a / FP64_PEAK)
    roof_y = max(b_y / HBM_PEAK, f_y / FP64_PEAK)
    out = {"points": plan.nelem * plan.nqp, "forward_csr_ms": ms_f,
           "adjoint": {"ms": ms_a, "bytes": b_a, "flops": f_a, "roofline_ms": roof_a * 1e3,
                       "frac": roof_a / (ms_a * 1e-3), "bound": "fp64" if f_a / FP64_PEAK > b_a / HBM_PEAK else "hbm",
                       "speedup_vs_forward": ms_f / ms_a},
           "apply": {"ms": ms_y, "bytes": b_y, "flops": f_y, "roofline_ms": roof_y * 1e3,
                     "frac": roof_y / (ms_y * 1e-3), "bound": "fp64" if f_y / FP64_PEAK > b_y / HBM_PEAK else "hbm",
                     "speedup_vs_forward": ms_f / ms_y},
           "apply_mass_only_ms": ms_m}
    # one forward Euler step M mu_next = (M - dt K) mu: right-hand side by the
    # apply, conjugate gradients on M to a relative residual of 1e-10
    dt = 0.1 / max(K) ** 2
    mu_next = torch.empty_like(u)
    work = torch.empty(int(ig.lib().igaf_euler_workspace(plan._h)), dtype=torch.float64, device="cuda")
    for name, pc in (("euler_step", ig.PRECOND_KRON), ("euler_step_plain_cg", ig.PRECOND_NONE)):
        plan.euler_step(kap, u, dt, tol=1e-10, maxit=20000, precond=pc, out=mu_next, work=work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, iters, relres = plan.euler_step(kap, u, dt, tol=1e-10, maxit=20000, precond=pc, out=mu_next,
                                           work=work)
        torch.cuda.synchronize()
        ms_e = (time.perf_counter() - t0) * 1e3
        out[name] = {"ms": ms_e, "cg_iterations": iters, "relres": relres, "dt": dt,
                     "ms_per_iteration": ms_e / max(1, iters),
                     "preconditioner": "kronecker 1D mass, diagonal scaling" if pc else "none"}
    del mu_next, work
    log("W5: adjoint %.3f ms (%.0f%% of roofline), apply (M+K)u %.3f ms (%.0f%%), Mu %.3f ms, forward CSR %.3f ms, "
        "Euler step %.1f ms (%d PCG iterations; plain CG %.1f ms, %d iterations)"
        % (ms_a, 100 * out["adjoint"]["frac"], ms_y, 100 * out["apply"]["frac"], ms_m, ms_f,
           out["euler_step"]["ms"], out["euler_step"]["cg_iterations"], out["euler_step_plain_cg"]["ms"],
           out["euler_step_plain_cg"]["cg_iterations"]))
    del kap, u, v, g, y, wk, Mv, Kv, plan
    torch.cuda.empty_cache()
    return out


def geo_flops(p):
    """Flops per element of the mapped-geometry kernel (ordered pairs): stage z
    9 n^2 q^3, stage y 10 n^4 q^2, stage x 5 n^6 q fused multiply-adds."""
    n = q = p + 1
    return 2 * (9 * n ** 2 * q ** 3 + 10 * n ** 4 * q ** 2 + 5 * n ** 6 * q)


def bench_w6(ig, torch, stream, steps):
    """W6: the headline mesh on a curved map (mapped_geometry, amp 0.1): the
    element matrices from a per-point mass coefficient and stiffness tensor
    (7 q^3 doubles in, 2 n^6 out per element; HBM-bound), then with the CSR
    values gathered from them, the CSR values alone (owner-computed rows,
    no element matrices), and the
    matrix-free apply and adjoint on the same geometry."""
    cfg = W.W6
    p, K = cfg["p"], cfg["K"]
    plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
    xs = [plan.quad_nodes(d)[0] for d in range(3)]
    cm, G = W.mapped_geometry(xs[0], xs[1], xs[2], W.kappa_sine(*xs), amp=cfg["amp"])
    cmd, Gd = torch.from_numpy(cm).cuda(), torch.from_numpy(G).cuda()
    del cm, G
    n3 = plan.elem_dim
    Me = torch.empty(plan.nelem, n3, n3, dtype=torch.float64, device="cuda")
    Ke = torch.empty_like(Me)
    Mv = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
    Kv = torch.empty_like(Mv)
    ms_el = float(np.mean(timed(lambda: plan.integrate_assemble_geo(cmd, Gd, Me=Me, Ke=Ke, want_csr=False),
                                steps, 2, stream)))
    ms_all = float(np.mean(timed(lambda: plan.integrate_assemble_geo(cmd, Gd, Me=Me, Ke=Ke, Mval=Mv, Kval=Kv),
                                 steps, 1, stream)))
    ms_csr = float(np.mean(timed(lambda: plan.integrate_assemble_geo(cmd, Gd, want_elem=False, Mval=Mv, Kval=Kv),
                                 max(2, steps // 2), 1, stream)))
    del Me, Ke, Mv, Kv
    torch.cuda.empty_cache()
    # the matrix-free apply and the adjoint on the same geometry (kappa = 1
    # here, so cm, G double as the geometry factors cm0, G0)
    u = torch.from_numpy(W.normal_vector(plan.ndof, 3)).cuda()
    v = torch.from_numpy(W.normal_vector(plan.ndof, 4)).cuda()
    y = torch.empty_like(u)
    g = torch.empty(plan.nelem, plan.nqp, dtype=torch.float64, device="cuda")
    wk = torch.empty(plan.apply_workspace(), dtype=torch.float64, device="cuda")
    ms_ap = float(np.mean(timed(lambda: plan.apply_geo(cmd, Gd, u, 1.0, 1.0, y=y, work=wk), steps, 2, stream)))
    ms_ad = float(np.mean(timed(lambda: plan.kappa_grad_geo(cmd, Gd, u, v, grad=g), steps, 2, stream)))
    del u, v, y, g, wk
    b_el = plan.nelem * (7 * plan.nqp * 8 + 2 * n3 * n3 * 8)
    f_el = plan.nelem * geo_flops(p)
    roof = max(b_el / HBM_PEAK, f_el / FP64_PEAK)
    out = {"elements": plan.nelem,
           "element_matrices": {"ms": ms_el, "bytes": b_el, "flops": f_el, "GB/s": b_el / (ms_el * 1e-3) / 1e9,
                                "roofline_ms": roof * 1e3, "frac": roof / (ms_el * 1e-3), "bound": "hbm"},
           "element_matrices_and_csr_gathered_ms": ms_all,
           "csr_only_ms": ms_csr,
           "apply_ms": ms_ap, "adjoint_ms": ms_ad}
    log("W6 mapped geometry: element matrices %.3f ms (%.0f%% of HBM roofline), + CSR gathered %.3f ms, "
        "CSR alone %.3f ms, apply %.3f ms, adjoint %.3f ms"
        % (ms_el, 100 * out["element_matrices"]["frac"], ms_all, ms_csr, ms_ap, ms_ad))
    del cmd, Gd, plan
    torch.cuda.empty_cache()
    return out


def wq_fmas_per_row(p, w, R=8):
    """Fused multiply-adds per CSR row of the weighted-quadrature kernel for
    interior rows (w = 2(p+1) points per direction in a row's box): stages z
    and y once per chunk of R rows over its 2(R+p) x points, each point
    O w (2w + 3O), then stage x per row 3 O^3 w (O = 2p + 1)."""
    O = 2 * p + 1
    nx = 2 * (R + p)
    return nx * O * w * (2 * w + 3 * O) / R + 3 * O ** 3 * w


def bench_w7_wq(ig, torch, stream, steps):
    """Weighted quadrature on the headline mesh (64^3, p = 3): the CSR values
    of M and K from kappa = 1 + 0.5 sin sin sin at the weighted-quadrature
    points, against the sum-factorised Gauss path's CSR-only call on the same
    mesh (the same outputs, different quadrature)."""
    p, K = W.W2["p"], W.W2["K"]
    plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
    t0 = time.perf_counter()
    plan.wq_prepare()
    t_prep = time.perf_counter() - t0
    xs = [plan.wq_points(d) for d in range(3)]
    s = [np.sin(2 * np.pi * x) for x in xs]
    kap = torch.from_numpy(1.0 + 0.5 * np.einsum("k,j,i->kji", s[2], s[1], s[0])).cuda()
    Mv = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
    Kv = torch.empty_like(Mv)
    ms = float(np.mean(timed(lambda: plan.wq_assemble(kap, Mval=Mv, Kval=Kv), steps, 2, stream)))
    xg = [plan.quad_nodes(d)[0] for d in range(3)]
    kg = torch.from_numpy(W.kappa_sine(*xg)).cuda()
    ms_g = float(np.mean(timed(lambda: plan.integrate_assemble(kg, want_elem=False, Mval=Mv, Kval=Kv),
                               steps, 2, stream)))
    npts = [len(x) for x in xs]
    b = 8.0 * npts[0] * npts[1] * npts[2] + 2 * plan.nnz * 8
    f = 2.0 * plan.ndof * wq_fmas_per_row(p, 2 * (p + 1))   # interior rows: 2(p+1) points per direction
    roof = max(b / HBM_PEAK, f / FP64_PEAK)
    out = {"points": npts, "prepare_s": t_prep, "ms": ms, "rows_per_s": plan.ndof / (ms * 1e-3),
           "elements_per_s": plan.nelem / (ms * 1e-3), "bytes": b, "flops": f, "roofline_ms": roof * 1e3,
           "frac": roof / (ms * 1e-3), "bound": "fp64" if f / FP64_PEAK > b / HBM_PEAK else "hbm",
           "gauss_sumfact_csr_ms": ms_g}
    log("W7 weighted quadrature 64^3 p=3: CSR M+K %.3f ms (%.0f%% of roofline; Gauss sum-factorised CSR %.3f ms), "
        "rules built in %.2f s" % (ms, 100 * out["frac"], ms_g, t_prep))
    del kap, kg, Mv, Kv, plan
    torch.cuda.empty_cache()
    return out


def run_kernel_mode(name, ig, torch, steps):
    """Run one kernel `steps` times (no timing output) for profiler passes:
    copy (1 GiB device copy, the counter calibration), element, csr,
    classical, headline (W2), w3p<p> (W3 streamed CSR at degree p), w4 (the
    batched launches of W4), adjoint, apply, apply_mass (W5), geo (W6
    element matrices), geo_csr (W6 CSR values alone, owner-computed rows),
    wq (W7 weighted quadrature, CSR values)."""
    if name == "copy":
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(steps):
            b.copy_(a)
    elif name.startswith("w3p"):
        p, K = int(name[3:]), W.W3["K"]
        plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
        kap = torch.from_numpy(W.kappa_lognormal(plan.nelem, plan.nqp, W.W3["seed"])).cuda()
        Mv = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
        Kv = torch.empty_like(Mv)
        for _ in range(steps):
            plan.integrate_assemble(kap, want_elem=False, Mval=Mv, Kval=Kv)
    elif name == "w4":
        shapes = W.batch_patches(**{k: W.W4[k] for k in ("npatch", "seed", "kmin", "kmax", "ps")})
        B = ig.Batch([(d["p"], d["K"], [W.open_uniform_knots(k, d["p"]) for k in d["K"]]) for d in shapes])
        kaps = [torch.from_numpy(k).cuda() for k in W.batch_kappas(shapes, seed=W.W4["seed"])]
        Ms = [torch.empty(pl.nnz, dtype=torch.float64, device="cuda") for pl in B.plans]
        Ks = [torch.empty(pl.nnz, dtype=torch.float64, device="cuda") for pl in B.plans]
        for _ in range(steps):
            B.integrate_assemble(kaps, Ms, Ks)
    elif name in ("adjoint", "apply", "apply_mass"):
        cfg = W.W5
        p, K = cfg["p"], cfg["K"]
        plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
        kap = torch.from_numpy(W.kappa_lognormal(plan.nelem, plan.nqp, cfg["seed_kappa"])).cuda()
        u = torch.from_numpy(W.normal_vector(plan.ndof, cfg["seed_u"])).cuda()
        v = torch.from_numpy(W.normal_vector(plan.ndof, cfg["seed_v"])).cuda()
        g = torch.empty_like(kap)
        y = torch.empty_like(u)
        wk = torch.empty(plan.apply_workspace(), dtype=torch.float64, device="cuda")
        for _ in range(steps):
            if name == "adjoint":
                plan.kappa_grad(u, v, grad=g)
            else:
                plan.apply(kap, u, 1.0, 0.0 if name == "apply_mass" else 1.0, y=y, work=wk)
    elif name == "wq":
        p, K = W.W2["p"], W.W2["K"]
        plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
        plan.wq_prepare()
        xs = [plan.wq_points(d) for d in range(3)]
        s = [np.sin(2 * np.pi * x) for x in xs]
        kap = torch.from_numpy(1.0 + 0.5 * np.einsum("k,j,i->kji", s[2], s[1], s[0])).cuda()
        Mv = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
        Kv = torch.empty_like(Mv)
        for _ in range(steps):
            plan.wq_assemble(kap, Mval=Mv, Kval=Kv)
    elif name in ("geo", "geo_csr"):
        cfg = W.W6
        p, K = cfg["p"], cfg["K"]
        plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
        xs = [plan.quad_nodes(d)[0] for d in range(3)]
        cm, G = W.mapped_geometry(xs[0], xs[1], xs[2], W.kappa_sine(*xs), amp=cfg["amp"])
        cmd, Gd = torch.from_numpy(cm).cuda(), torch.from_numpy(G).cuda()
        if name == "geo_csr":
            Mv = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
            Kv = torch.empty_like(Mv)
            for _ in range(steps):
                plan.integrate_assemble_geo(cmd, Gd, want_elem=False, Mval=Mv, Kval=Kv)
        else:
            Me = torch.empty(plan.nelem, plan.elem_dim, plan.elem_dim, dtype=torch.float64, device="cuda")
            Ke = torch.empty_like(Me)
            for _ in range(steps):
                plan.integrate_assemble_geo(cmd, Gd, Me=Me, Ke=Ke, want_csr=False)
    else:
        h = Headline(ig, torch)
        fn = {"element": h.element, "csr": h.csr, "headline": h.step,
              "classical": lambda: h.element(ig.CLASSICAL)}[name]
        for _ in range(steps):
            fn()
    torch.cuda.synchronize()
    print(json.dumps({"mode": "kernel:" + name, "steps": steps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=262144,
                    help="elements of the CPU-oracle sample (0 = skip)")
    ap.add_argument("--mode", default="full",
                    help="full | headline | w3 | w4 | w5 | w6 | w7 | kernel:{element,csr,classical,headline,copy,"
                         "w3p<p>,w4,adjoint,apply,apply_mass,geo,geo_csr,wq}")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2207_00280_amd import igafem as ig

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.mode.startswith("kernel:"):
        run_kernel_mode(args.mode.split(":", 1)[1], ig, torch, args.steps)
        return
    if args.mode in ("w3", "w4", "w5", "w6", "w7"):
        # one secondary workload alone (its JSON object on stdout)
        fn = {"w3": bench_w3, "w4": bench_w4, "w5": bench_w5, "w6": bench_w6, "w7": bench_w7_wq}[args.mode]
        print(json.dumps({args.mode: fn(ig, torch, torch.cuda.current_stream(), args.steps)}), flush=True)
        return
    stream = torch.cuda.current_stream()
    h = Headline(ig, torch)
    plan = h.plan
    E, n3, nnz = plan.nelem, plan.elem_dim, plan.nnz
    log("plan ready: E=%d nnz=%d" % (E, nnz))

    for _ in range(args.warmup):
        h.step()
    plan.set_timing(True)        # HIP events around each kernel of every timed step
    ms = timed(h.step, args.steps, 0, stream)
    ms_step = float(np.mean(ms))
    el_ms, el_n = plan.timing(0)
    csr_ms, csr_n = plan.timing(1)
    plan.set_timing(False)
    log("headline: %.3f ms/step (min %.3f); in-step element kernel %.3f ms, CSR kernel %.3f ms"
        % (ms_step, min(ms), el_ms, csr_ms))

    bytes_kappa = E * plan.nqp * 8
    bytes_elem = 2 * E * n3 * n3 * 8
    bytes_csr = 2 * nnz * 8
    step_bytes = bytes_kappa + bytes_elem + bytes_csr
    step_flops = E * sumfact_flops(3)
    out = {
        "metric": METRIC,
        "value": E / (ms_step * 1e-3),
        "unit": "element matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_median": float(np.median(ms)),
        "ms_min": float(min(ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "unit cube 64^3 elements, p=3, 4-point Gauss, kappa=1+0.5 sin sin sin; "
                               "one igaf_integrate_assemble: dense M_e+K_e of all elements and CSR M,K "
                               "(95443993 nnz each), sum factorization",
                   "elements": E, "degree": 3, "nquad": 4, "nnz": nnz, "method": "sumfact",
                   "assembly": "rows"},
        "step_roofline": {"bound": "hbm", "bytes": step_bytes, "flops": step_flops,
                          "achieved": step_bytes / (ms_step * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                          "unit": "GB/s", "frac": step_bytes / (ms_step * 1e-3) / HBM_PEAK},
    }
    # roofline of the dominant kernel (the element-matrix kernel, HBM-store-bound), from
    # its HIP-event intervals inside the timed steps (the CSR kernel follows it on the
    # same stream)
    alg_el = bytes_kappa + bytes_elem
    out["roofline"] = {"bound": "hbm", "achieved": alg_el / (el_ms * 1e-3) / 1e9,
                       "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                       "frac": alg_el / (el_ms * 1e-3) / HBM_PEAK, "traffic": traffic_for_current_kernel(),
                       "kernel": "igaf::k_element_ws<3> (sum factorisation, dense M_e/K_e store)",
                       "bytes_per_launch": alg_el, "ms": el_ms, "launches": el_n,
                       "csr_kernel_in_step_ms": csr_ms}
    if args.mode == "full":
        # the same work kernel by kernel, each alone on the GPU
        ms_el = float(np.mean(timed(h.element, args.steps, args.warmup, stream)))
        ms_csr = float(np.mean(timed(h.csr, args.steps, args.warmup, stream)))
        ms_cl = float(np.mean(timed(lambda: h.element(ig.CLASSICAL), max(3, args.steps // 4), 1, stream)))
        plan.set_assembly(ig.ASM_ATOMIC)
        ms_at = float(np.mean(timed(h.csr, max(3, args.steps // 4), 1, stream)))
        plan.set_assembly(ig.ASM_ROWS)
        csr_b = bytes_kappa + bytes_csr
        out["kernels"] = {
            "element_sumfact": {"ms": ms_el, "bytes": alg_el, "GB/s": alg_el / (ms_el * 1e-3) / 1e9,
                                "frac_hbm": alg_el / (ms_el * 1e-3) / HBM_PEAK, "flops": step_flops},
            "csr_rows": {"ms": ms_csr, "bytes": csr_b, "GB/s": csr_b / (ms_csr * 1e-3) / 1e9,
                         "frac_hbm": csr_b / (ms_csr * 1e-3) / HBM_PEAK},
            "element_classical": {"ms": ms_cl, "elements_per_s": E / (ms_cl * 1e-3),
                                  "flops_executed": E * classical_flops(3),
                                  "TFLOP/s": E * classical_flops(3) / (ms_cl * 1e-3) / 1e12,
                                  "frac_fp64": E * classical_flops(3) / (ms_cl * 1e-3) / FP64_PEAK,
                                  "dense_equivalent_flops_8n6q3": E * 8 * 4 ** 6 * 4 ** 3,
                                  "note": "flops_executed = S^3 (8 q^3 + 4 q^2) per element (distinct values only); "
                                          "the dense-equivalent 8 n^6 q^3 count is context, not work done"},
            "csr_atomic": {"ms": ms_at, "GB/s": csr_b / (ms_at * 1e-3) / 1e9},
        }
        rp_t = torch.empty(plan.ndof + 1, dtype=torch.int64, device="cuda")
        col_t = torch.empty(nnz, dtype=torch.int32, device="cuda")
        out["kernels"]["csr_pattern"] = {"ms": float(np.mean(timed(
            lambda: plan.csr_pattern(rp_t, col_t), 3, 1, stream))), "note": "built once per plan, not in the step"}
        del rp_t, col_t
        log(json.dumps(out["kernels"]))
        del h
        torch.cuda.empty_cache()
        out["measured_peaks"] = measured_peaks(torch, stream)
        mp = out["measured_peaks"]
        out["kernels"]["element_sumfact"]["frac_measured_write"] = \
            out["kernels"]["element_sumfact"]["GB/s"] / mp["write_GB/s"]
        out["kernels"]["element_classical"]["frac_measured_dgemm"] = \
            out["kernels"]["element_classical"]["TFLOP/s"] / mp["fp64_dgemm_TFLOP/s"]
        log("measured peaks: %s" % json.dumps(out["measured_peaks"]))
        steps_x = max(3, args.steps // 4)
        out["w3_streamed_128c"] = bench_w3(ig, torch, stream, steps_x)
        out["w4_batched_256"] = bench_w4(ig, torch, stream, steps_x)
        out["w5_adjoint_apply_96c"] = bench_w5(ig, torch, stream, steps_x)
        out["w6_mapped_geometry_64c"] = bench_w6(ig, torch, stream, steps_x)
        out["w7_weighted_quadrature_64c"] = bench_w7_wq(ig, torch, stream, steps_x)
    else:
        del h
        torch.cuda.empty_cache()
    cnt = counters_for_current_sources()
    if cnt:
        out["counters"] = cnt
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
        log("cpu baseline: %s" % json.dumps(out["cpu_baseline"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
