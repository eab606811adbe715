"""Python binding of libigafem.so (the C ABI in include/igafem.h).

Argument marshalling only: every step of the integration runs in the HIP
kernels of the library; torch provides device memory and streams.  Importing
this module loads the library and raises if it has not been built; the
integration calls raise if no GPU is present.  There is no CPU fallback.
"""
import contextlib
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigafem.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ENOCONV = 0, -1, -2, -3, -4, -5
PRECOND_NONE, PRECOND_KRON = 0, 1
CLASSICAL, SUMFACT = 0, 1
ASM_ROWS, ASM_ATOMIC = 0, 1
MAX_DEGREE = 5

SYMBOLS = [
    "igaf_version", "igaf_last_error", "igaf_desc_check", "igaf_desc_sizes", "igaf_desc_shared_run",
    "igaf_csr_pattern_host",
    "igaf_plan_create", "igaf_plan_destroy", "igaf_plan_sizes", "igaf_quad_nodes", "igaf_quad_points",
    "igaf_plan_set_assembly", "igaf_plan_set_timing", "igaf_plan_timing", "igaf_csr_pattern", "igaf_element_matrices", "igaf_assemble",
    "igaf_integrate_assemble", "igaf_integrate_assemble_geo", "igaf_geo_prepare", "igaf_kappa_grad", "igaf_bilinear_form",
    "igaf_apply_workspace",
    "igaf_apply", "igaf_apply_static",
    "igaf_apply_geo", "igaf_kappa_grad_geo", "igaf_euler_step_geo", "igaf_euler_workspace", "igaf_euler_step",
    "igaf_batch_create", "igaf_batch_destroy",
    "igaf_batch_plan", "igaf_batch_info", "igaf_batch_integrate_assemble",
    "igaf_batch_integrate_assemble_separate", "igaf_batch_autotune", "igaf_batch_split",
    "igaf_batch_set_split", "igaf_batch_set_degree_config", "igaf_batch_degree_config", "igaf_wq_prepare", "igaf_wq_points", "igaf_wq_assemble",
]


class IgafError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("igafem status %d: %s" % (status, msg))
        self.status = status


class PatchDesc(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("nelem", ctypes.c_int32 * 3),
                ("knots", ctypes.POINTER(ctypes.c_double) * 3), ("nquad", ctypes.c_int32 * 3)]


_lib = None
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


def lib():
    """Load libigafem.so (raises if it is missing: build it with
    ``python -m paper_2207_00280_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libigafem.so not built (run python -m paper_2207_00280_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    L.igaf_version.restype = ctypes.c_char_p
    L.igaf_last_error.restype = ctypes.c_char_p
    st = ctypes.c_int32
    L.igaf_desc_check.argtypes = [ctypes.POINTER(PatchDesc)]
    L.igaf_desc_sizes.argtypes = [ctypes.POINTER(PatchDesc)] + [_i64p] * 5
    L.igaf_desc_shared_run.argtypes = [ctypes.POINTER(PatchDesc), ctypes.c_int32, _i32p, _i32p]
    L.igaf_csr_pattern_host.argtypes = [ctypes.POINTER(PatchDesc), _i64p, _i32p]
    L.igaf_plan_create.argtypes = [ctypes.POINTER(PatchDesc), ctypes.POINTER(_vp)]
    L.igaf_plan_destroy.argtypes = [_vp]
    L.igaf_plan_destroy.restype = None
    L.igaf_plan_sizes.argtypes = [_vp] + [_i64p] * 5
    L.igaf_quad_nodes.argtypes = [_vp, ctypes.c_int32, _dp, _dp]
    L.igaf_quad_points.argtypes = [_vp, _dp]
    L.igaf_plan_set_assembly.argtypes = [_vp, ctypes.c_int32]
    L.igaf_plan_set_timing.argtypes = [_vp, ctypes.c_int32]
    L.igaf_plan_timing.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _i32p]
    L.igaf_csr_pattern.argtypes = [_vp, _vp, _vp, _vp]
    L.igaf_element_matrices.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp]
    L.igaf_assemble.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    L.igaf_integrate_assemble.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]
    L.igaf_kappa_grad.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, _vp, _vp, _vp]
    L.igaf_bilinear_form.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp]
    L.igaf_apply_workspace.argtypes = [_vp]
    L.igaf_apply_workspace.restype = ctypes.c_int64
    L.igaf_apply.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp, _vp]
    L.igaf_apply_static.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp]
    L.igaf_integrate_assemble_geo.argtypes = [_vp] * 8
    L.igaf_geo_prepare.argtypes = [_vp]
    L.igaf_apply_geo.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp, _vp]
    L.igaf_kappa_grad_geo.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, _vp, _vp]
    L.igaf_euler_workspace.argtypes = [_vp]
    L.igaf_euler_workspace.restype = ctypes.c_int64
    L.igaf_euler_step.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                  ctypes.c_int32, _vp, _vp, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_double), _vp]
    L.igaf_euler_step_geo.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_int32, _vp, _vp, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_double), _vp]
    L.igaf_batch_create.argtypes = [ctypes.POINTER(PatchDesc), ctypes.c_int32, ctypes.POINTER(_vp)]
    L.igaf_batch_destroy.argtypes = [_vp]
    L.igaf_batch_destroy.restype = None
    L.igaf_batch_plan.argtypes = [_vp, ctypes.c_int32]
    L.igaf_batch_plan.restype = _vp
    L.igaf_batch_info.argtypes = [_vp, _i32p, _i32p, _i32p]
    ptrs = ctypes.POINTER(_vp)
    L.igaf_batch_integrate_assemble.argtypes = [_vp, ptrs, ptrs, ptrs, _vp]
    L.igaf_batch_integrate_assemble_separate.argtypes = [_vp, ptrs, ptrs, ptrs, _vp]
    L.igaf_batch_autotune.argtypes = [_vp, ptrs, ptrs, ptrs, ctypes.c_int32, _vp]
    L.igaf_batch_split.argtypes = [_vp, _i32p, _i32p, ctypes.POINTER(ctypes.c_double)]
    L.igaf_batch_set_split.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
    L.igaf_batch_set_degree_config.argtypes = [_vp] + [ctypes.c_int32] * 4
    L.igaf_batch_degree_config.argtypes = [_vp, ctypes.c_int32, _i32p, _i32p, _i32p,
                                           ctypes.POINTER(ctypes.c_double), _i32p]
    L.igaf_wq_prepare.argtypes = [_vp]
    L.igaf_wq_points.argtypes = [_vp, ctypes.c_int32, _i64p, _dp]
    L.igaf_wq_assemble.argtypes = [_vp, _vp, _vp, _vp, _vp]
    for name in SYMBOLS:
        f = getattr(L, name)
        if f.restype is ctypes.c_int:   # default restype -> status
            f.restype = st
    _lib = L
    return L


def _check(status):
    if status != OK:
        raise IgafError(status, lib().igaf_last_error().decode())


def version():
    return lib().igaf_version().decode()


def make_desc(p, K, knots, q=None):
    """Build a PatchDesc; keeps the knot arrays alive on the returned object."""
    if q is None:
        q = (p + 1,) * 3
    d = PatchDesc()
    d.degree = int(p)
    keep = []
    for a in range(3):
        d.nelem[a] = int(K[a])
        d.nquad[a] = int(q[a])
        t = np.ascontiguousarray(knots[a], dtype=np.float64)
        keep.append(t)
        d.knots[a] = t.ctypes.data_as(_dp)
    d._keep = keep
    return d


def desc_sizes(desc):
    v = [ctypes.c_int64() for _ in range(5)]
    _check(lib().igaf_desc_sizes(ctypes.byref(desc), *[ctypes.byref(x) for x in v]))
    return dict(zip(["ndof", "nelem", "nqp", "elem_dim", "nnz"], [x.value for x in v]))


def desc_check(desc):
    """Returns (status, message)."""
    s = lib().igaf_desc_check(ctypes.byref(desc))
    return s, (lib().igaf_last_error().decode() if s else "")


def desc_shared_run(desc, d):
    """(first, end): the elements [first, end) of direction d that share the
    basis tables of element `first` (equal local knot windows)."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().igaf_desc_shared_run(ctypes.byref(desc), int(d), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def csr_pattern_host(desc):
    sz = desc_sizes(desc)
    rp = np.zeros(sz["ndof"] + 1, dtype=np.int64)
    col = np.zeros(sz["nnz"], dtype=np.int32)
    _check(lib().igaf_csr_pattern_host(ctypes.byref(desc), rp.ctypes.data_as(_i64p),
                                       col.ctypes.data_as(_i32p)))
    return rp, col


def _torch():
    import torch

    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _need_f64_cuda(t, name, numel=None):
    torch = _torch()
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64 (got %s)" % (name, t.dtype))
    if not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))


class Plan:
    """A patch bound to the current device: tables built at construction."""

    def __init__(self, p, K, knots, q=None):
        self.desc = make_desc(p, K, knots, q)
        h = _vp()
        _check(lib().igaf_plan_create(ctypes.byref(self.desc), ctypes.byref(h)))
        self._h = h
        self.p = int(p)
        self.K = tuple(int(k) for k in K)
        self.q = tuple(int(x) for x in (q if q is not None else (p + 1,) * 3))
        v = [ctypes.c_int64() for _ in range(5)]
        _check(lib().igaf_plan_sizes(h, *[ctypes.byref(x) for x in v]))
        self.ndof, self.nelem, self.nqp, self.elem_dim, self.nnz = [x.value for x in v]

    @classmethod
    def _wrap(cls, handle, desc):
        self = cls.__new__(cls)
        self.desc = desc
        self._h = _vp(handle)
        self._owned = False
        self.p = desc.degree
        self.K = tuple(desc.nelem)
        self.q = tuple(desc.nquad)
        v = [ctypes.c_int64() for _ in range(5)]
        _check(lib().igaf_plan_sizes(self._h, *[ctypes.byref(x) for x in v]))
        self.ndof, self.nelem, self.nqp, self.elem_dim, self.nnz = [x.value for x in v]
        return self

    def close(self):
        if getattr(self, "_h", None) and getattr(self, "_owned", True):
            lib().igaf_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def quad_points(self):
        """Every quadrature point, [E, q^3, 3] (x, y, z), in kappa's layout."""
        xyz = np.zeros((self.nelem, self.nqp, 3))
        _check(lib().igaf_quad_points(self._h, xyz.ctypes.data_as(_dp)))
        return xyz

    def quad_nodes(self, d):
        x = np.zeros(self.K[d] * self.q[d])
        w = np.zeros(self.K[d] * self.q[d])
        _check(lib().igaf_quad_nodes(self._h, d, x.ctypes.data_as(_dp), w.ctypes.data_as(_dp)))
        return x.reshape(self.K[d], self.q[d]), w.reshape(self.K[d], self.q[d])

    def set_assembly(self, mode):
        _check(lib().igaf_plan_set_assembly(self._h, int(mode)))

    def set_timing(self, enable=True):
        """Log HIP-event intervals of every kernel igaf_integrate_assemble launches."""
        _check(lib().igaf_plan_set_timing(self._h, 1 if enable else 0))

    def timing(self, kernel):
        """(average ms, count) of the logged launches; kernel 0 = element, 1 = CSR."""
        a = ctypes.c_double()
        n = ctypes.c_int32()
        _check(lib().igaf_plan_timing(self._h, int(kernel), ctypes.byref(a), ctypes.byref(n)))
        return a.value, n.value

    def csr_pattern(self, row_ptr=None, col=None, stream=None):
        """The structural CSR pattern into (new, or the given) device arrays."""
        torch = _torch()
        with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
            if row_ptr is None:
                row_ptr = torch.empty(self.ndof + 1, dtype=torch.int64, device="cuda")
            if col is None:
                col = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        rp = row_ptr
        _check(lib().igaf_csr_pattern(self._h, _ptr(rp), _ptr(col), _stream(stream)))
        return rp, col

    def _alloc(self, *shape, stream=None):
        """A float64 device tensor; with an explicit stream it is allocated on
        that stream, so that the caching allocator does not hand its memory to
        other streams while work queued on `stream` may still use it."""
        torch = _torch()
        if stream is None:
            return torch.empty(*shape, dtype=torch.float64, device="cuda")
        with torch.cuda.stream(stream):
            return torch.empty(*shape, dtype=torch.float64, device="cuda")

    def element_matrices(self, kappa, method=SUMFACT, want_m=True, want_k=True, Me=None, Ke=None,
                         stream=None):
        _need_f64_cuda(kappa, "kappa", self.nelem * self.nqp)
        n3 = self.elem_dim
        if want_m and Me is None:
            Me = self._alloc(self.nelem, n3, n3, stream=stream)
        if want_k and Ke is None:
            Ke = self._alloc(self.nelem, n3, n3, stream=stream)
        Me = Me if want_m else None
        Ke = Ke if want_k else None
        for t, nm in ((Me, "Me"), (Ke, "Ke")):
            if t is not None:
                _need_f64_cuda(t, nm, self.nelem * n3 * n3)
        _check(lib().igaf_element_matrices(self._h, int(method), _ptr(kappa), _ptr(Me), _ptr(Ke),
                                           _stream(stream)))
        return Me, Ke

    def assemble(self, Me, Ke, Mval=None, Kval=None, stream=None):
        if Me is not None and Mval is None:
            Mval = self._alloc(self.nnz, stream=stream)
        if Ke is not None and Kval is None:
            Kval = self._alloc(self.nnz, stream=stream)
        _check(lib().igaf_assemble(self._h, _ptr(Me), _ptr(Ke), _ptr(Mval), _ptr(Kval),
                                   _stream(stream)))
        return Mval, Kval

    def integrate_assemble(self, kappa, method=SUMFACT, want_elem=True, want_csr=True, want_m=True,
                           want_k=True, Me=None, Ke=None, Mval=None, Kval=None, stream=None):
        _need_f64_cuda(kappa, "kappa", self.nelem * self.nqp)
        n3 = self.elem_dim
        if want_elem:
            if want_m and Me is None:
                Me = self._alloc(self.nelem, n3, n3, stream=stream)
            if want_k and Ke is None:
                Ke = self._alloc(self.nelem, n3, n3, stream=stream)
        if want_csr:
            if want_m and Mval is None:
                Mval = self._alloc(self.nnz, stream=stream)
            if want_k and Kval is None:
                Kval = self._alloc(self.nnz, stream=stream)
        Me = Me if (want_elem and want_m) else None
        Ke = Ke if (want_elem and want_k) else None
        Mval = Mval if (want_csr and want_m) else None
        Kval = Kval if (want_csr and want_k) else None
        for t, nm, ne in ((Me, "Me", self.nelem * n3 * n3), (Ke, "Ke", self.nelem * n3 * n3),
                          (Mval, "Mval", self.nnz), (Kval, "Kval", self.nnz)):
            if t is not None:
                _need_f64_cuda(t, nm, ne)
        _check(lib().igaf_integrate_assemble(self._h, int(method), _ptr(kappa), _ptr(Me), _ptr(Ke),
                                             _ptr(Mval), _ptr(Kval), _stream(stream)))
        return Me, Ke, Mval, Kval

    def integrate_assemble_geo(self, cm, G, want_elem=True, want_csr=True, want_m=True, want_k=True,
                               Me=None, Ke=None, Mval=None, Kval=None, stream=None):
        """Mapped geometry (igaf_integrate_assemble_geo): cm = kappa det J [E, q^3],
        G = kappa det J J^-1 J^-T [E, 6, q^3] (xx yy zz xy xz yz).  Returns
        (Me, Ke, Mval, Kval), None where not requested."""
        if want_m:
            _need_f64_cuda(cm, "cm", self.nelem * self.nqp)
        if want_k:
            _need_f64_cuda(G, "G", self.nelem * 6 * self.nqp)
        n3 = self.elem_dim
        if want_elem:
            if want_m and Me is None:
                Me = self._alloc(self.nelem, n3, n3, stream=stream)
            if want_k and Ke is None:
                Ke = self._alloc(self.nelem, n3, n3, stream=stream)
        if want_csr:
            if want_m and Mval is None:
                Mval = self._alloc(self.nnz, stream=stream)
            if want_k and Kval is None:
                Kval = self._alloc(self.nnz, stream=stream)
        Me = Me if (want_elem and want_m) else None
        Ke = Ke if (want_elem and want_k) else None
        Mval = Mval if (want_csr and want_m) else None
        Kval = Kval if (want_csr and want_k) else None
        for t, nm, ne in ((Me, "Me", self.nelem * n3 * n3), (Ke, "Ke", self.nelem * n3 * n3),
                          (Mval, "Mval", self.nnz), (Kval, "Kval", self.nnz)):
            if t is not None:
                _need_f64_cuda(t, nm, ne)
        _check(lib().igaf_integrate_assemble_geo(self._h, _ptr(cm if want_m else None),
                                                 _ptr(G if want_k else None), _ptr(Me), _ptr(Ke),
                                                 _ptr(Mval), _ptr(Kval), _stream(stream)))
        return Me, Ke, Mval, Kval

    def apply_workspace(self):
        """Doubles of scratch igaf_apply needs (the runs' slots)."""
        return int(lib().igaf_apply_workspace(self._h))

    def _apply_work(self, work, stream):
        nw = self.apply_workspace()
        if work is None:
            work = self._alloc(nw, stream=stream)
        _need_f64_cuda(work, "work", None)
        if work.numel() < nw:
            raise ValueError("work has %d elements, needs %d" % (work.numel(), nw))
        return work

    def geo_prepare(self):
        """igaf_geo_prepare: checks the plan; the mapped-geometry calls allocate
        nothing, so there is nothing to prepare before a capture."""
        _check(lib().igaf_geo_prepare(self._h))

    def apply(self, kappa, u, alphaM=1.0, alphaK=1.0, y=None, work=None, stream=None):
        """y = alphaM M(kappa) u + alphaK K(kappa) u, matrix-free (igaf_apply)."""
        _need_f64_cuda(kappa, "kappa", self.nelem * self.nqp)
        _need_f64_cuda(u, "u", self.ndof)
        if y is None:
            y = self._alloc(self.ndof, stream=stream)
        _need_f64_cuda(y, "y", self.ndof)
        work = self._apply_work(work, stream)
        _check(lib().igaf_apply(self._h, _ptr(kappa), _ptr(u), float(alphaM), float(alphaK),
                                _ptr(y), _ptr(work), _stream(stream)))
        return y

    def euler_step(self, kappa, mu, dt, tol=1e-12, maxit=1000, precond=None, out=None, work=None,
                   stream=None):
        """One forward Euler step M(kappa) mu_next = M(kappa) mu - dt K(kappa) mu
        (igaf_euler_step, conjugate gradients on M; precond PRECOND_KRON (the
        default) or PRECOND_NONE).  Returns (mu_next, iterations, relative
        residual); raises IgafError with status ENOCONV if maxit is reached
        first."""
        return self._euler(kappa, None, mu, dt, tol, maxit, precond, out, work, stream)

    def euler_step_geo(self, cm, G, mu, dt, tol=1e-12, maxit=1000, precond=None, out=None, work=None,
                       stream=None):
        """The Euler step on a mapped geometry (igaf_euler_step_geo)."""
        return self._euler(cm, G, mu, dt, tol, maxit, precond, out, work, stream)

    def _euler(self, kappa, G, mu, dt, tol, maxit, precond, out, work, stream):
        """Shared body of euler_step / euler_step_geo (G None: identity geometry)."""
        precond = PRECOND_KRON if precond is None else int(precond)
        _need_f64_cuda(kappa, "kappa", self.nelem * self.nqp)
        _need_f64_cuda(mu, "mu", self.ndof)
        if out is None:
            out = self._alloc(self.ndof, stream=stream)
        _need_f64_cuda(out, "out", self.ndof)
        nw = int(lib().igaf_euler_workspace(self._h))
        if work is None:
            # work after the last iteration may still run on `stream`: allocate there
            work = self._alloc(nw, stream=stream)
        _need_f64_cuda(work, "work", nw)
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        if G is None:
            _check(lib().igaf_euler_step(self._h, _ptr(kappa), _ptr(mu), float(dt), float(tol), int(maxit),
                                         precond, _ptr(out), _ptr(work), ctypes.byref(it), ctypes.byref(rr),
                                         _stream(stream)))
        else:
            _need_f64_cuda(G, "G", self.nelem * 6 * self.nqp)
            _check(lib().igaf_euler_step_geo(self._h, _ptr(kappa), _ptr(G), _ptr(mu), float(dt), float(tol),
                                             int(maxit), precond, _ptr(out), _ptr(work), ctypes.byref(it),
                                             ctypes.byref(rr), _stream(stream)))
        return out, it.value, rr.value

    def apply_static(self, kappa, u, y, alphaM=1.0, alphaK=1.0, stream=None):
        """igaf_apply_static: the apply with the library's static scratch (no
        workspace, nothing allocated); y must be given."""
        _need_f64_cuda(kappa, "kappa", self.nelem * self.nqp)
        _need_f64_cuda(u, "u", self.ndof)
        _need_f64_cuda(y, "y", self.ndof)
        _check(lib().igaf_apply_static(self._h, _ptr(kappa), _ptr(u), float(alphaM), float(alphaK), _ptr(y),
                                       _stream(stream)))
        return y

    def apply_geo(self, cm, G, u, alphaM=1.0, alphaK=1.0, y=None, work=None, stream=None):
        """Mapped-geometry apply (igaf_apply_geo): y = alphaM M u + alphaK K u."""
        _need_f64_cuda(cm, "cm", self.nelem * self.nqp)
        _need_f64_cuda(G, "G", self.nelem * 6 * self.nqp)
        _need_f64_cuda(u, "u", self.ndof)
        if y is None:
            y = self._alloc(self.ndof, stream=stream)
        _need_f64_cuda(y, "y", self.ndof)
        work = self._apply_work(work, stream)
        _check(lib().igaf_apply_geo(self._h, _ptr(cm), _ptr(G), _ptr(u), float(alphaM), float(alphaK),
                                    _ptr(y), _ptr(work), _stream(stream)))
        return y

    def kappa_grad_geo(self, cm0, G0, u, v, alphaM=1.0, alphaK=1.0, scale=1.0, grad=None, stream=None):
        """Mapped-geometry adjoint (igaf_kappa_grad_geo): dL/dkappa when kappa
        scales cm0 and G0."""
        _need_f64_cuda(cm0, "cm0", self.nelem * self.nqp)
        _need_f64_cuda(G0, "G0", self.nelem * 6 * self.nqp)
        _need_f64_cuda(u, "u", self.ndof)
        _need_f64_cuda(v, "v", self.ndof)
        if grad is None:
            grad = self._alloc(self.nelem, self.nqp, stream=stream)
        _need_f64_cuda(grad, "grad", self.nelem * self.nqp)
        _check(lib().igaf_kappa_grad_geo(self._h, _ptr(cm0), _ptr(G0), _ptr(u), _ptr(v), float(alphaM),
                                         float(alphaK), float(scale), _ptr(grad), _stream(stream)))
        return grad

    def kappa_grad(self, u, v, alphaM=1.0, alphaK=1.0, scale=1.0, grad=None, scale_dev=None, stream=None):
        """dL/dkappa [E, q^3] (igaf_kappa_grad), times scale and, if given, the
        device scalar scale_dev (a one-element float64 CUDA tensor)."""
        _need_f64_cuda(u, "u", self.ndof)
        _need_f64_cuda(v, "v", self.ndof)
        if scale_dev is not None:
            _need_f64_cuda(scale_dev, "scale_dev", 1)
        if grad is None:
            grad = self._alloc(self.nelem, self.nqp, stream=stream)
        _need_f64_cuda(grad, "grad", self.nelem * self.nqp)
        _check(lib().igaf_kappa_grad(self._h, _ptr(u), _ptr(v), float(alphaM), float(alphaK),
                                     float(scale), _ptr(scale_dev), _ptr(grad), _stream(stream)))
        return grad

    def bilinear_form(self, kappa, u, v, alphaM=1.0, alphaK=1.0, out=None, stream=None):
        """L = alphaM u^T M(kappa) v + alphaK u^T K(kappa) v as a 0-dim CUDA
        tensor (igaf_bilinear_form: matrix-free, fixed-order sums)."""
        _need_f64_cuda(kappa, "kappa", self.nelem * self.nqp)
        _need_f64_cuda(u, "u", self.ndof)
        _need_f64_cuda(v, "v", self.ndof)
        if out is None:
            out = self._alloc((), stream=stream)
        _need_f64_cuda(out, "out", 1)
        _check(lib().igaf_bilinear_form(self._h, _ptr(kappa), _ptr(u), _ptr(v), float(alphaM), float(alphaK),
                                        _ptr(out), _stream(stream)))
        return out


    # ---- weighted quadrature
    def wq_prepare(self):
        """Build the weighted-quadrature rules (igaf_wq_prepare)."""
        _check(lib().igaf_wq_prepare(self._h))

    def wq_points(self, d):
        """The weighted-quadrature points of direction d (numpy array)."""
        n = ctypes.c_int64()
        _check(lib().igaf_wq_points(self._h, int(d), ctypes.byref(n), None))
        x = np.zeros(n.value)
        _check(lib().igaf_wq_points(self._h, int(d), None, x.ctypes.data_as(_dp)))
        return x

    def wq_assemble(self, kappa, want_m=True, want_k=True, Mval=None, Kval=None, stream=None):
        """CSR values of M and K by weighted quadrature (igaf_wq_assemble);
        kappa: CUDA float64 on the point grid [npts_z, npts_y, npts_x]."""
        npts = [len(self.wq_points(d)) for d in range(3)]
        _need_f64_cuda(kappa, "kappa", npts[0] * npts[1] * npts[2])
        if want_m and Mval is None:
            Mval = self._alloc(self.nnz, stream=stream)
        if want_k and Kval is None:
            Kval = self._alloc(self.nnz, stream=stream)
        Mval = Mval if want_m else None
        Kval = Kval if want_k else None
        for t, nm in ((Mval, "Mval"), (Kval, "Kval")):
            if t is not None:
                _need_f64_cuda(t, nm, self.nnz)
        _check(lib().igaf_wq_assemble(self._h, _ptr(kappa), _ptr(Mval), _ptr(Kval), _stream(stream)))
        return Mval, Kval


def _ptr_array(tensors):
    arr = (_vp * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr() if t is not None else None
    return arr


class Batch:
    """Many independent patches integrated and assembled (CSR, streamed) together."""

    def __init__(self, specs):
        """specs: list of (p, K, knots[, q])."""
        self.descs_keep = [make_desc(*s) for s in specs]
        arr = (PatchDesc * len(specs))()
        for i, d in enumerate(self.descs_keep):
            arr[i] = d
        self._arr = arr
        h = _vp()
        _check(lib().igaf_batch_create(arr, len(specs), ctypes.byref(h)))
        self._h = h
        self.plans = [Plan._wrap(lib().igaf_batch_plan(h, i), self.descs_keep[i])
                      for i in range(len(specs))]

    def close(self):
        if getattr(self, "_h", None):
            lib().igaf_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        v = [ctypes.c_int32() for _ in range(3)]
        _check(lib().igaf_batch_info(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(["family", "grid", "nitems"], [x.value for x in v]))

    def split(self):
        """The work split in use: segments per tile, items per XCD chunk, and
        the autotuner's median time for it (0 before tuning)."""
        a, b, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().igaf_batch_split(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(t)))
        return dict(split=a.value, chunk=b.value, ms=t.value)

    def set_split(self, split, chunk):
        _check(lib().igaf_batch_set_split(self._h, int(split), int(chunk)))

    def set_degree_config(self, degree, tile, split, chunk):
        _check(lib().igaf_batch_set_degree_config(self._h, int(degree), int(tile), int(split), int(chunk)))

    def degree_config(self, degree):
        """One degree's launch configuration: tile shape, split, chunk, the
        autotuner's median ms (0 if not tuned) and the number of items."""
        v = [ctypes.c_int32() for _ in range(3)]
        t = ctypes.c_double()
        n = ctypes.c_int32()
        _check(lib().igaf_batch_degree_config(self._h, int(degree), *[ctypes.byref(x) for x in v],
                                              ctypes.byref(t), ctypes.byref(n)))
        return dict(tile=v[0].value, split=v[1].value, chunk=v[2].value, ms=t.value, nitems=n.value)

    def autotune(self, kappas, Mvals, Kvals, reps=3, stream=None):
        """Time every work split on these arrays and keep the fastest
        (igaf_batch_autotune); returns split()."""
        _check(lib().igaf_batch_autotune(self._h, _ptr_array(kappas),
                                         _ptr_array(Mvals) if Mvals is not None else None,
                                         _ptr_array(Kvals) if Kvals is not None else None, int(reps),
                                         _stream(stream)))
        return self.split()

    def integrate_assemble(self, kappas, Mvals, Kvals, separate=False, stream=None):
        f = lib().igaf_batch_integrate_assemble_separate if separate else lib().igaf_batch_integrate_assemble
        _check(f(self._h, _ptr_array(kappas), _ptr_array(Mvals) if Mvals is not None else None,
                 _ptr_array(Kvals) if Kvals is not None else None, _stream(stream)))


def _autograd():
    torch = _torch()

    class KappaBilinearLoss(torch.autograd.Function):
        """L(kappa) = alphaM u^T M(kappa) v + alphaK u^T K(kappa) v.

        The value comes from igaf_bilinear_form and the gradient from the
        adjoint kernel (igaf_kappa_grad), with the incoming gradient passed to
        the library as a device scalar: no arithmetic in Python and no host
        synchronisation, so forward and backward can be captured in a HIP
        graph.  Neither recomputes nor stores element matrices.  Gradients
        with respect to u and v are not provided (an error if they require
        grad)."""

        @staticmethod
        def forward(ctx, kappa, u, v, plan, alphaM=1.0, alphaK=1.0):
            if u.requires_grad or v.requires_grad:
                raise ValueError("KappaBilinearLoss differentiates with respect to kappa only; "
                                 "u and v must not require grad")
            L = plan.bilinear_form(kappa.detach().reshape(-1), u, v, alphaM, alphaK)
            ctx.save_for_backward(u, v)
            ctx.plan, ctx.alphaM, ctx.alphaK, ctx.kshape = plan, alphaM, alphaK, kappa.shape
            return L

        @staticmethod
        def backward(ctx, grad_out):
            u, v = ctx.saved_tensors
            go = grad_out
            if go.dtype != torch.float64 or not go.is_cuda or not go.is_contiguous():
                go = go.to(dtype=torch.float64, device=u.device).contiguous()
            g = ctx.plan.kappa_grad(u, v, ctx.alphaM, ctx.alphaK, 1.0, scale_dev=go.reshape(1))
            return g.view(ctx.kshape), None, None, None, None, None

    return KappaBilinearLoss


_KBL = None


def integrate(p, K, knots, kappa, method=SUMFACT, want_elem=True, want_csr=True, q=None):
    """One-shot integration and assembly of a patch: builds the plan, runs
    igaf_integrate_assemble and returns torch tensors as a dict with keys
    Me, Ke ([E, n^3, n^3] or None), row_ptr, col, Mval, Kval (CSR; None when
    want_csr is False) and the plan.  kappa: CUDA float64 [E, q^3]."""
    plan = Plan(p, K, knots, q)
    Me, Ke, Mv, Kv = plan.integrate_assemble(kappa, method=method, want_elem=want_elem, want_csr=want_csr)
    rp, col = plan.csr_pattern() if want_csr else (None, None)
    return dict(Me=Me, Ke=Ke, row_ptr=rp, col=col, Mval=Mv, Kval=Kv, plan=plan)


def __getattr__(name):
    # the autograd class needs torch; it is built on first access
    if name == "KappaBilinearLoss":
        global _KBL
        if _KBL is None:
            _KBL = _autograd()
        return _KBL
    raise AttributeError(name)


def kappa_bilinear_loss(kappa, u, v, plan, alphaM=1.0, alphaK=1.0):
    global _KBL
    if _KBL is None:
        _KBL = _autograd()
    return _KBL.apply(kappa, u, v, plan, alphaM, alphaK)
