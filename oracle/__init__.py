"""CPU oracle for the B-spline element-integration path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (plain FP64,
classical quadrature of Algorithm 1, assembly by brute-force union of
element pairs) through ctypes and holds the exact-rational module
``exact.py`` and the weighted-quadrature oracle ``wq.py`` (numpy).  It
shares no code with the HIP path.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=False):
    """Compile oracle.c with gcc (OpenMP) into liboracle.so next to it."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.orc_basis_all.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_basis_all.restype = None
        patch = [ctypes.c_int, ip, ip, dp, dp, dp]
        L.orc_validate.argtypes = patch
        L.orc_quad_nodes.argtypes = patch + [ctypes.c_int, dp, dp]
        L.orc_element_matrices.argtypes = patch + [dp, ctypes.c_int64, ctypes.c_int64, dp, dp]
        L.orc_assemble.argtypes = patch + [dp, i64p, i32p, dp, dp, i64p]
        L.orc_rows.argtypes = patch + [dp, i64p, ctypes.c_int64, i32p, dp, dp, i32p, ctypes.c_int64]
        L.orc_element_matrices_geo.argtypes = patch + [dp, dp, ctypes.c_int64, ctypes.c_int64, dp, dp]
        L.orc_assemble_geo.argtypes = patch + [dp, dp, i64p, i32p, dp, dp, i64p]
        L.orc_rows_geo.argtypes = patch + [dp, dp, i64p, ctypes.c_int64, i32p, dp, dp, i32p,
                                           ctypes.c_int64]
        L.orc_kappa_grad.argtypes = patch + [dp, dp, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, dp]
        L.orc_kappa_grad_geo.argtypes = patch + [dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Patch:
    """A patch as the oracle sees it: degree p, elements K[3], Gauss orders q[3],
    knot vectors t[3] (each K_d+2p+1 long)."""

    def __init__(self, p, K, q, knots):
        self.p = int(p)
        self.K = [int(k) for k in K]
        self.q = [int(x) for x in q]
        self.t = [_f64(k) for k in knots]
        self._Ka = (ctypes.c_int * 3)(*self.K)
        self._qa = (ctypes.c_int * 3)(*self.q)

    @property
    def n(self):
        return self.p + 1

    @property
    def N(self):
        return [k + self.p for k in self.K]

    @property
    def ndof(self):
        N = self.N
        return N[0] * N[1] * N[2]

    @property
    def nelem(self):
        return self.K[0] * self.K[1] * self.K[2]

    @property
    def nq(self):
        return self.q[0] * self.q[1] * self.q[2]

    def args(self):
        return (self.p, self._Ka, self._qa, _dp(self.t[0]), _dp(self.t[1]), _dp(self.t[2]))


def gauss_legendre(q):
    x = np.zeros(q)
    w = np.zeros(q)
    if lib().orc_gauss_legendre(q, _dp(x), _dp(w)) != 0:
        raise ValueError("bad q")
    return x, w


def basis_all(t, p, x):
    t = _f64(t)
    nb = len(t) - p - 1
    B = np.zeros(nb)
    dB = np.zeros(nb)
    lib().orc_basis_all(_dp(t), len(t), p, float(x), _dp(B), _dp(dB))
    return B, dB


def validate(P):
    return lib().orc_validate(*P.args()) == 0


def quad_nodes(P, d):
    """Mapped Gauss nodes and weights (w*h/2) of direction d: arrays [K_d, q_d]."""
    x = np.zeros(P.K[d] * P.q[d])
    w = np.zeros(P.K[d] * P.q[d])
    if lib().orc_quad_nodes(*P.args(), d, _dp(x), _dp(w)) != 0:
        raise ValueError("invalid patch")
    return x.reshape(P.K[d], P.q[d]), w.reshape(P.K[d], P.q[d])


def _geo_arg(P, G):
    if G is None:
        return None
    G = _f64(G).reshape(-1)
    assert G.size == P.nelem * 6 * P.nq
    return G


def element_matrices(P, kappa, e0=0, e1=None, want_m=True, want_k=True, G=None):
    """Classical (Algorithm 1) element matrices for elements [e0, e1):
    arrays [e1-e0, n^3, n^3] (None where not wanted).  With G (mapped
    geometry, [E][6][q^3], components xx yy zz xy xz yz) kappa is the mass
    coefficient cm = kappa det J and G the stiffness tensor kappa det J J^-1 J^-T."""
    if e1 is None:
        e1 = P.nelem
    kappa = _f64(kappa).reshape(-1)
    assert kappa.size == P.nelem * P.nq
    G = _geo_arg(P, G)
    n3 = P.n ** 3
    Me = np.zeros((e1 - e0, n3, n3)) if want_m else None
    Ke = np.zeros((e1 - e0, n3, n3)) if want_k else None
    if G is not None:
        rc = lib().orc_element_matrices_geo(*P.args(), _dp(kappa), _dp(G), e0, e1, _dp(Me), _dp(Ke))
    else:
        rc = lib().orc_element_matrices(*P.args(), _dp(kappa), e0, e1, _dp(Me), _dp(Ke))
    if rc != 0:
        raise ValueError("invalid patch or range")
    return Me, Ke


def assemble(P, kappa, G=None):
    """Global CSR (row_ptr int64, col int32, Mval, Kval) by brute-force union
    (with G: mapped geometry, as in element_matrices)."""
    kappa = _f64(kappa).reshape(-1)
    assert kappa.size == P.nelem * P.nq
    G = _geo_arg(P, G)
    L = lib()
    if G is not None:
        call = lambda *a: L.orc_assemble_geo(*P.args(), _dp(kappa), _dp(G), *a)
    else:
        call = lambda *a: L.orc_assemble(*P.args(), _dp(kappa), *a)
    row_ptr = np.zeros(P.ndof + 1, dtype=np.int64)
    nnz = ctypes.c_int64(0)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    rc = call(row_ptr.ctypes.data_as(i64p), None, None, None, ctypes.byref(nnz))
    if rc != 0:
        raise ValueError("invalid patch")
    col = np.zeros(nnz.value, dtype=np.int32)
    Mv = np.zeros(nnz.value)
    Kv = np.zeros(nnz.value)
    call(row_ptr.ctypes.data_as(i64p), col.ctypes.data_as(i32p), _dp(Mv), _dp(Kv), ctypes.byref(nnz))
    return row_ptr, col, Mv, Kv


def rows(P, kappa, dofs, G=None):
    """Complete global rows for the given DOFs: list of (cols, mvals, kvals)
    (with G: mapped geometry, as in element_matrices)."""
    kappa = _f64(kappa).reshape(-1)
    G = _geo_arg(P, G)
    dofs = np.ascontiguousarray(dofs, dtype=np.int64)
    stride = (2 * P.p + 1) ** 3
    cols = np.zeros((len(dofs), stride), dtype=np.int32)
    mv = np.zeros((len(dofs), stride))
    kv = np.zeros((len(dofs), stride))
    ln = np.zeros(len(dofs), dtype=np.int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    if G is not None:
        rc = lib().orc_rows_geo(*P.args(), _dp(kappa), _dp(G), dofs.ctypes.data_as(i64p), len(dofs),
                                cols.ctypes.data_as(i32p), _dp(mv), _dp(kv), ln.ctypes.data_as(i32p),
                                stride)
    else:
        rc = lib().orc_rows(*P.args(), _dp(kappa), dofs.ctypes.data_as(i64p), len(dofs),
                            cols.ctypes.data_as(i32p), _dp(mv), _dp(kv), ln.ctypes.data_as(i32p), stride)
    if rc != 0:
        raise ValueError("invalid patch")
    return [(cols[r, :ln[r]].copy(), mv[r, :ln[r]].copy(), kv[r, :ln[r]].copy()) for r in range(len(dofs))]


def kappa_grad(P, u, v, alphaM=1.0, alphaK=1.0, scale=1.0, cm0=None, G0=None):
    """Reference dL/dkappa at every quadrature point, [E, q^3].  With cm0, G0
    (mapped geometry, kappa scaling both coefficients: cm = kappa cm0,
    G = kappa G0) the geometry's factors enter the point values."""
    u = _f64(u)
    v = _f64(v)
    assert u.size == P.ndof and v.size == P.ndof
    g = np.zeros((P.nelem, P.nq))
    if G0 is not None:
        cm0 = _f64(cm0).reshape(-1)
        G0 = _geo_arg(P, G0)
        rc = lib().orc_kappa_grad_geo(*P.args(), _dp(cm0), _dp(G0), _dp(u), _dp(v), alphaM, alphaK,
                                      scale, _dp(g))
    else:
        rc = lib().orc_kappa_grad(*P.args(), _dp(u), _dp(v), alphaM, alphaK, scale, _dp(g))
    if rc != 0:
        raise ValueError("invalid patch")
    return g


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))
