"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np

import workloads as W


def relfro(a, b):
    """Relative Frobenius error ||a - b|| / ||b||."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rowmax_rel(a, b, row_ptr):
    """max over CSR rows of ||a_row - b_row|| / ||b_row|| (every structural
    row holds at least its diagonal entry)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    rp = np.asarray(row_ptr, dtype=np.int64)
    starts = rp[:-1]
    dn = np.sqrt(np.add.reduceat((a - b) ** 2, starts))
    bn = np.sqrt(np.add.reduceat(b * b, starts))
    return float(np.max(dn / np.maximum(bn, np.finfo(np.float64).tiny)))


def csr_close(a, b, row_ptr, tol=1e-12):
    """CSR values a vs the reference b: relative Frobenius error over the
    whole matrix AND the largest relative error of a single row, each <= tol
    (a wrong row of small entries cannot hide under the global norm)."""
    g, r = relfro(a, b), rowmax_rel(a, b, row_ptr)
    return g <= tol and r <= tol


def nonuniform_knots(K, p, seed):
    """Open knot vector with K distinct, randomly placed interior spans."""
    if K == 1:
        return W.open_uniform_knots(1, p)
    rng = np.random.default_rng(seed)
    while True:
        inner = np.sort(rng.uniform(0.02, 0.98, K - 1))
        if np.min(np.diff(np.concatenate([[0.0], inner, [1.0]]))) > 0.2 / K:
            break
    return np.concatenate([[0.0] * (p + 1), inner, [1.0] * (p + 1)])


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()
