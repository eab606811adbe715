"""Benchmark of the B-spline element-integration hot path on one MI355X.

Workload (the headline): unit cube, 64^3 uniform elements, p=3 (C^2 open
uniform knots), 4-point Gauss rule per direction, kappa = 1 + 0.5 sin(2 pi x)
sin(2 pi y) sin(2 pi z) at the quadrature points, FP64.  One step = one
igaf_integrate_assemble call, sum factorisation, producing the dense element
matrices M_e and K_e of all 262 144 elements AND the global CSR values of M
and K (95 443 993 nonzeros each).  Inputs are resident in HBM before timing.

Prints ONE JSON line (rank 0).  See --help.
"""
import argparse
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sumfact_flops(p):
    """Minimum sum-factorisation flops per element with symmetric pairs:
    stage z 4 S q^3, stage y 6 S^2 q^2, stage x 6 S^3 q (M and K)."""
    n = p + 1
    q = p + 1
    S = n * (n + 1) // 2
    return 4 * S * q ** 3 + 6 * S * S * q * q + 6 * S ** 3 * q


def timed(fn, steps, warmup, stream):
    """Run fn warmup times, then time `steps` calls with HIP events on `stream`;
    returns the list of per-call milliseconds."""
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


def cpu_baseline(nsample, chunk=4096):
    """The CPU oracle (classical quadrature, M_e and K_e) on the first
    `nsample` elements of the same workload, all host threads."""
    import oracle

    P = oracle.Patch(3, (64, 64, 64), (4, 4, 4), [W.open_uniform_knots(64, 3)] * 3)
    xs = [oracle.quad_nodes(P, d)[0] for d in range(3)]
    kap = W.kappa_sine(*xs)
    t0 = time.perf_counter()
    for e0 in range(0, nsample, chunk):
        oracle.element_matrices(P, kap, e0, min(nsample, e0 + chunk))
    dt = time.perf_counter() - t0
    return {"value": nsample / dt, "unit": "element matrices/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "first %d of the 262144 elements (classical quadrature, M_e and K_e, "
                      "no assembly), %.1f s" % (nsample, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=65536,
                    help="elements of the CPU-oracle sample (0 = skip)")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline step only (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2207_00280_amd import igafem as ig

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    p, K = 3, (64, 64, 64)
    knots = [W.open_uniform_knots(k, p) for k in K]
    plan = ig.Plan(p, K, knots)
    xs = [plan.quad_nodes(d)[0] for d in range(3)]
    kappa = torch.from_numpy(W.kappa_sine(*xs)).cuda()
    E, n3, nnz = plan.nelem, plan.elem_dim, plan.nnz
    Me = torch.empty(E, n3, n3, dtype=torch.float64, device="cuda")
    Ke = torch.empty_like(Me)
    Mval = torch.empty(nnz, dtype=torch.float64, device="cuda")
    Kval = torch.empty_like(Mval)
    torch.cuda.synchronize()
    log("plan ready: E=%d nnz=%d" % (E, nnz))

    def step():
        plan.integrate_assemble(kappa, method=ig.SUMFACT, Me=Me, Ke=Ke, Mval=Mval, Kval=Kval)

    ms = timed(step, args.steps, args.warmup, stream)
    ms_step = float(np.mean(ms))
    log("headline: %.3f ms/step (min %.3f)" % (ms_step, min(ms)))

    bytes_kappa = E * plan.nqp * 8
    bytes_elem = 2 * E * n3 * n3 * 8
    bytes_csr = 2 * nnz * 8
    out = {
        "metric": METRIC,
        "value": E / (ms_step * 1e-3),
        "unit": "element matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "unit cube 64^3 elements, p=3, 4-point Gauss, kappa=1+0.5sin sin sin, "
                               "sum factorization, M_e+K_e dense + CSR M,K (95443993 nnz)",
                   "elements": E, "degree": p, "nquad": 4, "nnz": nnz, "method": "sumfact",
                   "assembly": "rows"},
    }
    step_bytes = bytes_kappa + bytes_elem + bytes_csr
    out["step_roofline"] = {"bound": "hbm", "bytes": step_bytes,
                            "achieved": step_bytes / (ms_step * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                            "unit": "GB/s", "frac": step_bytes / (ms_step * 1e-3) / HBM_PEAK}

    if not args.only_headline:
        # per-kernel timing of the same work: element kernel, then the CSR kernel
        ms_el = timed(lambda: plan.element_matrices(kappa, method=ig.SUMFACT, Me=Me, Ke=Ke),
                      args.steps, args.warmup, stream)
        ms_csr = timed(lambda: plan.integrate_assemble(kappa, want_elem=False, Mval=Mval, Kval=Kval),
                       args.steps, args.warmup, stream)
        t_el = float(np.mean(ms_el)) * 1e-3
        t_csr = float(np.mean(ms_csr)) * 1e-3
        alg_el = bytes_kappa + bytes_elem
        out["roofline"] = {"bound": "hbm", "achieved": alg_el / t_el / 1e9, "peak": HBM_PEAK / 1e9,
                           "unit": "GB/s", "frac": alg_el / t_el / HBM_PEAK, "traffic": None,
                           "kernel": "k_element<3,SUMFACT> (dense M_e, K_e store)",
                           "ms": t_el * 1e3}
        out["kernels"] = {
            "element_sumfact": {"ms": t_el * 1e3, "bytes": alg_el, "GB/s": alg_el / t_el / 1e9,
                                "frac_hbm": alg_el / t_el / HBM_PEAK,
                                "flops": E * sumfact_flops(p)},
            "csr_rows": {"ms": t_csr * 1e3, "bytes": bytes_kappa + bytes_csr,
                         "GB/s": (bytes_kappa + bytes_csr) / t_csr / 1e9,
                         "frac_hbm": (bytes_kappa + bytes_csr) / t_csr / HBM_PEAK},
        }
        ms_cl = timed(lambda: plan.element_matrices(kappa, method=ig.CLASSICAL, Me=Me, Ke=Ke),
                      max(3, args.steps // 4), 1, stream)
        t_cl = float(np.mean(ms_cl)) * 1e-3
        out["kernels"]["element_classical"] = {"ms": t_cl * 1e3, "elements_per_s": E / t_cl}
        plan.set_assembly(ig.ASM_ATOMIC)
        ms_at = timed(lambda: plan.integrate_assemble(kappa, want_elem=False, Mval=Mval, Kval=Kval),
                      max(3, args.steps // 4), 1, stream)
        plan.set_assembly(ig.ASM_ROWS)
        out["kernels"]["csr_atomic"] = {"ms": float(np.mean(ms_at))}
        log(json.dumps(out["kernels"]))

    del Me, Ke
    torch.cuda.empty_cache()
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
        log("cpu baseline: %s" % json.dumps(out["cpu_baseline"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
