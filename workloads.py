"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no integration arithmetic: it only produces the inputs the
method takes (knot vectors, the coefficient kappa at given quadrature points,
random vectors, random patch descriptions).  Quadrature nodes are passed IN
by the caller (each side computes its own), so nothing here depends on
either the HIP path or the CPU oracle.

Workloads (unit cube, open uniform knots, Gauss rule with q = p+1):
  W1  8^3 elements,   p=2, q=3, kappa = 1, mass only
  W2  64^3 elements,  p=3, q=4, kappa = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z)
  W3  128^3 elements, p in {2,3,4}, kappa log-normal(0, 0.5) i.i.d., seed 0
  W4  256 patches (seed 1): K_d ~ U{8..48}, p ~ U{2..5}, kappa log-normal(0, 0.5)
  W5  96^3 elements,  p=3, kappa log-normal (seed 2), u, v ~ N(0,1) (seeds 3, 4),
      100 finite-difference points (seed 5)
  W6  64^3 elements,  p=3, mapped geometry (mapped_geometry, amp 0.1, A = I),
      kappa as W2
"""
import numpy as np

W1 = dict(name="W1", K=(8, 8, 8), p=2)
W2 = dict(name="W2", K=(64, 64, 64), p=3)
W3 = dict(name="W3", K=(128, 128, 128), ps=(2, 3, 4), seed=0)
W4 = dict(name="W4", npatch=256, seed=1, kmin=8, kmax=48, ps=(2, 3, 4, 5))
W5 = dict(name="W5", K=(96, 96, 96), p=3, seed_kappa=2, seed_u=3, seed_v=4, seed_pts=5, npts=100)
W6 = dict(name="W6", K=(64, 64, 64), p=3, amp=0.1)


def open_uniform_knots(K, p, lo=0.0, hi=1.0):
    """p+1 copies of lo, the K-1 uniform interior breakpoints, p+1 copies of hi."""
    inner = [lo + (hi - lo) * k / K for k in range(1, K)]
    return np.array([lo] * (p + 1) + inner + [hi] * (p + 1), dtype=np.float64)


def repeated_knots(breaks, mults, p, lo=0.0, hi=1.0):
    """Open knot vector with interior breakpoints `breaks` (increasing, inside
    (lo, hi)), breakpoint i repeated mults[i] times (1 <= mults[i] <= p+1):
    the basis is C^{p - mults[i]} there.  K = len - 2p - 1 spans, the empty
    ones included."""
    inner = [b for b, m in zip(breaks, mults) for _ in range(int(m))]
    return np.array([lo] * (p + 1) + list(inner) + [hi] * (p + 1), dtype=np.float64)


def random_repeated_knots(nbreak, p, seed, max_mult=None):
    """Seeded breakpoints (uniform, kept apart) with multiplicities drawn
    uniformly from 1..max_mult (default p+1).  Returns (knots, K)."""
    rng = np.random.default_rng(seed)
    max_mult = p + 1 if max_mult is None else max_mult
    while True:
        breaks = np.sort(rng.uniform(0.03, 0.97, nbreak))
        if nbreak == 0 or np.min(np.diff(np.concatenate([[0.0], breaks, [1.0]]))) > 0.2 / (nbreak + 1):
            break
    mults = rng.integers(1, max_mult + 1, nbreak)
    t = repeated_knots(breaks, mults, p)
    return t, len(t) - 2 * p - 1


def kappa_layout(fx, fy, fz):
    """Evaluate a separable-looking field given per-direction node values.

    fx, fy, fz: arrays [K_d, q_d] of some per-coordinate quantity.  Returns the
    array indexed [E][qz][qy][qx] with e = ex + Kx (ey + Ky ez) and the value at
    (ex,kx),(ey,ky),(ez,kz) taken from the callable-free broadcast product
    fx*fy*fz.  Used with log/sine factors by the callers below."""
    Kx, qx = fx.shape
    Ky, qy = fy.shape
    Kz, qz = fz.shape
    # axes: ez, ey, ex, kz, ky, kx
    v = (fz[:, None, None, :, None, None] * fy[None, :, None, None, :, None]
         * fx[None, None, :, None, None, :])
    return np.ascontiguousarray(v.reshape(Kz * Ky * Kx, qz * qy * qx))


def kappa_sine(xn, yn, zn):
    """kappa = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z) at the given nodes
    (xn, yn, zn: [K_d, q_d] node coordinates).  Layout [E][qz][qy][qx]."""
    s = kappa_layout(np.sin(2 * np.pi * np.asarray(xn)), np.sin(2 * np.pi * np.asarray(yn)),
                     np.sin(2 * np.pi * np.asarray(zn)))
    return 1.0 + 0.5 * s


def kappa_separable(fx, fy, fz):
    """kappa = fx(x) fy(y) fz(z) from per-direction node values [K_d, q_d]."""
    return kappa_layout(np.asarray(fx, dtype=np.float64), np.asarray(fy, dtype=np.float64),
                        np.asarray(fz, dtype=np.float64))


def mapped_geometry(xn, yn, zn, kappa, A=None, b=None, amp=0.0):
    """Per-point coefficients of a mapped geometry x = F(xi) of the unit cube,

        F(xi) = A xi + b + amp (sin(pi y) sin(pi z), sin(pi z) sin(pi x), sin(pi x) sin(pi y)),

    at the parametric nodes xn, yn, zn ([K_d, q_d] per direction).  This is the
    caller's side of the geometry (the pull-back of the physical integrals to
    the parameter cube); the integration itself takes the result as input:

        cm = kappa det J                 [E][q^3]      (mass)
        G  = kappa det J J^-1 J^-T       [E][6][q^3]   (stiffness; xx yy zz xy xz yz)

    with J = dF/dxi.  A defaults to the identity; det J must stay positive
    (|amp| pi small against A)."""
    A = np.eye(3) if A is None else np.asarray(A, dtype=np.float64)
    one = [np.ones_like(np.asarray(v, dtype=np.float64)) for v in (xn, yn, zn)]
    X = kappa_layout(np.asarray(xn, dtype=np.float64), one[1], one[2])
    Y = kappa_layout(one[0], np.asarray(yn, dtype=np.float64), one[2])
    Z = kappa_layout(one[0], one[1], np.asarray(zn, dtype=np.float64))
    sx, cx = np.sin(np.pi * X), np.cos(np.pi * X)
    sy, cy = np.sin(np.pi * Y), np.cos(np.pi * Y)
    sz, cz = np.sin(np.pi * Z), np.cos(np.pi * Z)
    a = amp * np.pi
    zero = np.zeros_like(X)
    # J[r][c] = d F_r / d xi_c
    J = [[A[0, 0] + zero, A[0, 1] + a * cy * sz, A[0, 2] + a * sy * cz],
         [A[1, 0] + a * cx * sz, A[1, 1] + zero, A[1, 2] + a * sx * cz],
         [A[2, 0] + a * cx * sy, A[2, 1] + a * sx * cy, A[2, 2] + zero]]
    # adjugate: J^-1 = adj / det
    adj = [[J[1][1] * J[2][2] - J[1][2] * J[2][1], J[0][2] * J[2][1] - J[0][1] * J[2][2],
            J[0][1] * J[1][2] - J[0][2] * J[1][1]],
           [J[1][2] * J[2][0] - J[1][0] * J[2][2], J[0][0] * J[2][2] - J[0][2] * J[2][0],
            J[0][2] * J[1][0] - J[0][0] * J[1][2]],
           [J[1][0] * J[2][1] - J[1][1] * J[2][0], J[0][1] * J[2][0] - J[0][0] * J[2][1],
            J[0][0] * J[1][1] - J[0][1] * J[1][0]]]
    det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0]
    if np.min(det) <= 0:
        raise ValueError("geometry map folds over (det J <= 0)")
    kappa = np.asarray(kappa, dtype=np.float64)
    f = kappa / det             # kappa det J (adj/det)(adj/det)^T = kappa/det adj adj^T
    G = np.empty((X.shape[0], 6, X.shape[1]))
    for c, (r, t) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        G[:, c, :] = f * (adj[r][0] * adj[t][0] + adj[r][1] * adj[t][1] + adj[r][2] * adj[t][2])
    return kappa * det, G


def kappa_lognormal(nelem, nq, seed, sigma=0.5):
    """kappa_q = exp(sigma Z), Z ~ N(0,1) i.i.d., drawn in layout order."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal((nelem, nq)))


def kappa_constant(nelem, nq, value=1.0):
    return np.full((nelem, nq), float(value))


def normal_vector(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


def fd_points(total, count, seed):
    """`count` distinct flat quadrature-point indices in [0, total)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(total, size=count, replace=False)).astype(np.int64)


def batch_patches(npatch=256, seed=1, kmin=8, kmax=48, ps=(2, 3, 4, 5)):
    """Draw patch shapes: for each patch (Kx, Ky, Kz, p) in that order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(npatch):
        Kx, Ky, Kz = (int(v) for v in rng.integers(kmin, kmax + 1, size=3))
        p = int(rng.choice(ps))
        out.append(dict(K=(Kx, Ky, Kz), p=p, q=p + 1))
    return out


def batch_kappas(patches, seed=1, sigma=0.5):
    """Log-normal kappa per patch, drawn after the shapes from a stream
    derived from the same seed (patch i uses seed (seed, i))."""
    out = []
    for i, d in enumerate(patches):
        rng = np.random.default_rng([seed, i])
        E = d["K"][0] * d["K"][1] * d["K"][2]
        out.append(np.exp(sigma * rng.standard_normal((E, d["q"] ** 3))))
    return out
