"""Thin Python binding of libvdsolve.so (argument marshalling only).

Every computation runs in the HIP library; torch is used only to own device
memory and to name the HIP stream.  Function names mirror the C ABI in
include/vdsolve.h; ``Grid`` is a convenience wrapper around them.  A missing
library is an error: there is no fallback path.
"""
import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvdsolve.so")

VD_OK, VD_NOT_CONVERGED = 0, 1
VD_GMRES, VD_CG, VD_RMR = 0, 1, 2
VD_FP64, VD_FP32_REFINE = 0, 1
VD_OP_PRESSURE, VD_OP_HELMHOLTZ, VD_OP_PRESSURE_K = 0, 1, 2
VD_FORM_L, VD_FORM_K = 0, 1
VD_FOURIER, VD_CHEB_GL = 0, 1
OP_KINDS = {"pressure": VD_OP_PRESSURE, "helmholtz": VD_OP_HELMHOLTZ, "pressure_k": VD_OP_PRESSURE_K}
FORMULATIONS = {"L": VD_FORM_L, "K": VD_FORM_K}
SOLVERS = {"gmres": VD_GMRES, "cg": VD_CG, "rmr": VD_RMR}
PRECISIONS = {"fp64": VD_FP64, "fp32_refine": VD_FP32_REFINE, "fp32": VD_FP32_REFINE}


class vd_grid_desc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("basis", ctypes.c_int * 3),
                ("length", ctypes.c_double * 3)]


class vd_solve_opts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int), ("restart", ctypes.c_int), ("rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("precond", ctypes.c_int), ("precision", ctypes.c_int),
                ("inner_rtol", ctypes.c_double), ("max_outer", ctypes.c_int), ("rho0", ctypes.c_double),
                ("use_x0", ctypes.c_int), ("formulation", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int)]


class vd_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int), ("refinements", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("rhs_null_norm", ctypes.c_double),
                ("seconds", ctypes.c_double), ("gs_second_passes", ctypes.c_int), ("history_len", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class VdError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {vd_status_string(status)} ({status})")


class vd_request(ctypes.Structure):
    _fields_ = [("desc", vd_grid_desc), ("kind", ctypes.c_int), ("dt_nu", ctypes.c_double),
                ("ncomp", ctypes.c_int), ("rho", ctypes.c_void_p), ("f", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("opts", vd_solve_opts), ("user_tag", ctypes.c_ulonglong)]


class vd_result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_ulonglong), ("user_tag", ctypes.c_ulonglong), ("status", ctypes.c_int),
                ("iterations", ctypes.c_int), ("refinements", ctypes.c_int), ("slot", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("t_arrive", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vd_server_stats_t(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_longlong), ("in_flight", ctypes.c_longlong), ("busy_slots", ctypes.c_int),
                ("grids", ctypes.c_int), ("hbm_used", ctypes.c_size_t), ("hbm_peak", ctypes.c_size_t),
                ("peak_busy_slots", ctypes.c_int)]


class vd_ns_params(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("sc", ctypes.c_double), ("dt", ctypes.c_double), ("s", ctypes.c_double),
                ("visc_rtol", ctypes.c_double), ("pres_rtol", ctypes.c_double), ("restart", ctypes.c_int),
                ("max_iter", ctypes.c_int), ("pres_solver", ctypes.c_int), ("pres_form", ctypes.c_int)]


class vd_ns_info(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("steps", ctypes.c_int), ("visc_iters", ctypes.c_int),
                ("pres_iters", ctypes.c_int), ("visc_status", ctypes.c_int), ("pres_status", ctypes.c_int),
                ("visc_rel_residual", ctypes.c_double), ("pres_rel_residual", ctypes.c_double),
                ("pres_seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int

_SIGS = {
    "vd_default_opts": (None, [ctypes.POINTER(vd_solve_opts)]),
    "vd_grid_create": (_I, [ctypes.POINTER(_P), ctypes.POINTER(vd_grid_desc), _P]),
    "vd_grid_destroy": (_I, [_P]),
    "vd_set_density": (_I, [_P, _P]),
    "vd_apply_operator": (_I, [_P, _I, _I, _D, _P, _P]),
    "vd_apply_precond": (_I, [_P, _I, _I, _D, _D, _P, _P]),
    "vd_solve_pressure": (_I, [_P, _P, _P, ctypes.POINTER(vd_solve_opts), ctypes.POINTER(vd_solve_info)]),
    "vd_solve_helmholtz": (_I, [_P, _D, _I, _P, _P, ctypes.POINTER(vd_solve_opts),
                                ctypes.POINTER(vd_solve_info)]),
    "vd_solve_pressure_batch": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                     ctypes.POINTER(vd_solve_opts), ctypes.POINTER(vd_solve_info)]),
    "vd_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(vd_grid_desc), ctypes.POINTER(vd_solve_opts)]),
    "vd_workspace_bytes_helmholtz": (ctypes.c_size_t, [ctypes.POINTER(vd_grid_desc), ctypes.POINTER(vd_solve_opts),
                                                       ctypes.c_int]),
    "vd_profile_enable": (_I, [_P, _I]),
    "vd_profile_read": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_D), _I]),
    "vd_status_string": (ctypes.c_char_p, [_I]),
    "vd_dense_matmul": (_I, [_I, _P, _P, _P, _I, _I, _I, _P]),
    "vd_visc1d_create": (_I, [ctypes.POINTER(_P), _I, _I, _D, _D, _P]),
    "vd_visc1d_destroy": (_I, [_P]),
    "vd_pres1d_create": (_I, [ctypes.POINTER(_P), _I, _I, _P]),
    "vd_visc1d_apply": (_I, [_P, _I, _P, _P, _P, _I]),
    "vd_visc1d_solve": (_I, [_P, _I, _P, _P, _P, ctypes.POINTER(vd_solve_opts), _P, _P,
                             ctypes.POINTER(vd_solve_info)]),
    "vd_ns_default_params": (None, [ctypes.POINTER(vd_ns_params)]),
    "vd_ns_create": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(vd_ns_params), _P]),
    "vd_ns_destroy": (_I, [_P]),
    "vd_ns_set_state": (_I, [_P, _P, _P, _P, _D]),
    "vd_ns_init_taylor_green": (_I, [_P]),
    "vd_ns_step": (_I, [_P, _I, ctypes.POINTER(vd_ns_info)]),
    "vd_ns_get_state": (_I, [_P, _P, _P, _P, ctypes.POINTER(_D)]),
    "vd_ns_errors": (_I, [_P, ctypes.POINTER(_D)]),
    "vd_ns_project": (_I, [_P, _P, _P, _P, ctypes.POINTER(vd_solve_info)]),
    "vd_ns_profile_enable": (_I, [_P, _I]),
    "vd_ns_profile_read": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_D), _I]),
    "vd_visc1d_kernel_ms": (_I, [_P, ctypes.POINTER(_D)]),
    "vd_visc1d_solve_noalloc": (_I, [_P, _I, _P, _P, _P, ctypes.POINTER(vd_solve_opts), _P, _P,
                                     ctypes.POINTER(vd_solve_info)]),
    "vd_server_create": (_I, [ctypes.POINTER(_P), ctypes.c_size_t, _I]),
    "vd_server_create_dry": (_I, [ctypes.POINTER(_P), ctypes.c_size_t, _I, _D]),
    "vd_server_submit": (_I, [_P, ctypes.POINTER(vd_request), ctypes.POINTER(ctypes.c_ulonglong)]),
    "vd_server_set_batch": (_I, [_P, _I]),
    "vd_server_poll": (_I, [_P, ctypes.POINTER(vd_result), _I, ctypes.POINTER(_I)]),
    "vd_server_wait": (_I, [_P, ctypes.POINTER(vd_result), _I, ctypes.POINTER(_I), _D]),
    "vd_server_stats": (_I, [_P, ctypes.POINTER(vd_server_stats_t)]),
    "vd_server_destroy": (_I, [_P]),
}


def lib():
    """Load libvdsolve.so (built in-tree by paper_2403_06654_amd.build)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2403_06654_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def vd_status_string(s):
    return lib().vd_status_string(int(s)).decode()


def make_desc(shape, lengths=None, cheb=False):
    """Descriptor of a grid of C-order ``shape`` (x last).  Fourier on every
    axis, or with ``cheb`` a 2D grid (nz, nx) whose first axis holds the nz
    Chebyshev-Gauss-Lobatto points of [-1, 1] (row 0 at z = +1)."""
    nd = len(shape)
    if lengths is None:
        lengths = (2 * math.pi,) * nd
    d = vd_grid_desc()
    d.ndim = nd
    for i in range(nd):  # n[0] = nx (last C axis)
        d.n[i] = int(shape[nd - 1 - i])
        d.length[i] = float(lengths[nd - 1 - i])
        d.basis[i] = 0
    if cheb:
        if nd != 2:
            raise ValueError("a Chebyshev axis needs a 2D grid (nz, nx)")
        d.basis[1] = 1
        d.length[1] = 2.0
    return d


def dense_matmul(A, B, precision="fp64"):
    """C = A @ B on the device with the library's MFMA contraction."""
    import torch
    M, K = A.shape
    K2, N = B.shape
    assert K == K2 and A.is_contiguous() and B.is_contiguous() and A.dtype == B.dtype
    C = torch.empty((M, N), dtype=A.dtype, device=A.device)
    st = torch.cuda.current_stream().cuda_stream
    _check(lib().vd_dense_matmul(PRECISIONS[precision], A.data_ptr(), B.data_ptr(), C.data_ptr(), M, N, K, st),
           "vd_dense_matmul", False)
    return C


def make_opts(solver="gmres", restart=30, rtol=1e-10, max_iter=2000, precond=True, precision="fp64",
              inner_rtol=1e-5, max_outer=10, rho0=float("nan"), use_x0=False, formulation="L", history=None):
    """history: a contiguous float64 numpy array that receives the residual
    history (its length is the capacity), or None."""
    o = vd_solve_opts()
    lib().vd_default_opts(ctypes.byref(o))
    o.solver = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    o.restart = int(restart)
    o.rtol = float(rtol)
    o.max_iter = int(max_iter)
    o.precond = 1 if precond else 0
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.inner_rtol = float(inner_rtol)
    o.max_outer = int(max_outer)
    o.rho0 = float(rho0)
    o.use_x0 = 1 if use_x0 else 0
    o.formulation = FORMULATIONS[formulation] if isinstance(formulation, str) else int(formulation)
    if history is not None:
        import numpy as np
        if not (isinstance(history, np.ndarray) and history.dtype == np.float64 and history.flags.c_contiguous):
            raise TypeError("history must be a contiguous float64 numpy array")
        o.history = history.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.history_cap = int(history.size)
    return o


def workspace_bytes(shape, lengths=None, cheb=False, helmholtz_ncomp=None, **opts):
    """Device bytes of a grid plus one solve; helmholtz_ncomp: of a velocity
    solve with that many components (several are solved together)."""
    d = make_desc(shape, lengths, cheb)
    o = make_opts(**opts)
    if helmholtz_ncomp is not None:
        return int(lib().vd_workspace_bytes_helmholtz(ctypes.byref(d), ctypes.byref(o), int(helmholtz_ncomp)))
    return int(lib().vd_workspace_bytes(ctypes.byref(d), ctypes.byref(o)))


def _with_history(info, opts):
    d = info.as_dict()
    h = opts.get("history")
    if h is not None:
        d["history"] = h.reshape(-1)[: d["history_len"]].copy() if h.ndim == 1 else h.copy()
    return d


def _check(st, where, allow_nc=True):
    if st == VD_OK or (allow_nc and st == VD_NOT_CONVERGED):
        return st
    raise VdError(st, where)


def _dev_f64(t, shape, what):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{what} must be a float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous with shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Grid:
    """A periodic grid with its device resources (vd_grid_create)."""

    def __init__(self, shape, lengths=None, stream=None, cheb=False):
        import torch
        self.shape = tuple(int(s) for s in shape)
        self.lengths = lengths
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        d = make_desc(self.shape, lengths, cheb)
        h = ctypes.c_void_p()
        _check(lib().vd_grid_create(ctypes.byref(h), ctypes.byref(d), ctypes.c_void_p(self._stream.cuda_stream)),
               "vd_grid_create", False)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().vd_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_density(self, rho):
        _check(lib().vd_set_density(self._h, _dev_f64(rho, self.shape, "rho")), "vd_set_density", False)

    def apply_operator(self, kind, x, precision="fp64", nu=0.0, out=None):
        import torch
        y = out if out is not None else torch.empty_like(x)
        k = OP_KINDS[kind]
        _check(lib().vd_apply_operator(self._h, k, PRECISIONS[precision], float(nu), _dev_f64(x, self.shape, "x"),
                                       _dev_f64(y, self.shape, "y")), "vd_apply_operator", False)
        return y

    def apply_precond(self, kind, r, precision="fp64", nu=0.0, rho0=float("nan"), out=None):
        import torch
        z = out if out is not None else torch.empty_like(r)
        k = OP_KINDS[kind]
        _check(lib().vd_apply_precond(self._h, k, PRECISIONS[precision], float(nu), float(rho0),
                                      _dev_f64(r, self.shape, "r"), _dev_f64(z, self.shape, "z")),
               "vd_apply_precond", False)
        return z

    def solve_pressure(self, f, p=None, **opts):
        import torch
        if p is None:
            p = torch.zeros_like(f)
        o = make_opts(**opts)
        info = vd_solve_info()
        st = lib().vd_solve_pressure(self._h, _dev_f64(f, self.shape, "f"), _dev_f64(p, self.shape, "p"),
                                     ctypes.byref(o), ctypes.byref(info))
        _check(st, "vd_solve_pressure")
        return p, _with_history(info, opts)

    def solve_helmholtz(self, g, dt_nu, u=None, **opts):
        import torch
        ncomp = 1 if g.dim() == len(self.shape) else g.shape[0]
        shp = self.shape if ncomp == 1 and g.dim() == len(self.shape) else (ncomp,) + self.shape
        if u is None:
            u = torch.zeros_like(g)
        o = make_opts(**opts)
        info = vd_solve_info()
        st = lib().vd_solve_helmholtz(self._h, float(dt_nu), int(ncomp), _dev_f64(g, shp, "g"),
                                      _dev_f64(u, shp, "u"), ctypes.byref(o), ctypes.byref(info))
        _check(st, "vd_solve_helmholtz")
        return u, _with_history(info, opts)

    @staticmethod
    def solve_pressure_batch(grids, fs, ps=None, **opts):
        """L_rho p = f on up to three grids of one shape together
        (vd_solve_pressure_batch); returns the fields and one info per grid."""
        import torch
        n = len(grids)
        if len(fs) != n or (ps is not None and len(ps) != n):
            raise ValueError("one f (and p) per grid")
        if ps is None:
            ps = [torch.zeros_like(f) for f in fs]
        hs = (_P * n)(*[g._h.value for g in grids])
        fp = (_P * n)(*[_dev_f64(f, g.shape, "f").value for f, g in zip(fs, grids)])
        pp = (_P * n)(*[_dev_f64(p, g.shape, "p").value for p, g in zip(ps, grids)])
        o = make_opts(**opts)
        infos = (vd_solve_info * n)()
        st = lib().vd_solve_pressure_batch(hs, n, fp, pp, ctypes.byref(o), infos)
        _check(st, "vd_solve_pressure_batch")
        return ps, [_with_history(infos[k], opts if k == 0 else {}) for k in range(n)]

    def profile_enable(self, on=True):
        """on: True (every kernel class), False, or a bit mask of classes."""
        mask = -1 if on is True else (0 if on is False else int(on))
        _check(lib().vd_profile_enable(self._h, mask), "vd_profile_enable", False)

    def profile_read(self, nclass=12):
        ms = (ctypes.c_double * nclass)()
        cnt = (ctypes.c_longlong * nclass)()
        nb = (ctypes.c_double * nclass)()
        _check(lib().vd_profile_read(self._h, ms, cnt, nb, nclass), "vd_profile_read", False)
        return list(ms), list(cnt), list(nb)


class Visc1d:
    """Batched 1D implicit viscous systems V_rho u = b (vd_visc1d_*)."""

    @classmethod
    def pressure(cls, n, form="K", stream=None):
        """Batched 1D Chebyshev-collocation pressure operators with Neumann
        walls, L_rho or K_rho (vd_pres1d_create); same methods."""
        import torch
        self = cls.__new__(cls)
        self.n = int(n)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().vd_pres1d_create(ctypes.byref(h), self.n, FORMULATIONS[form],
                                      ctypes.c_void_p(self._stream.cuda_stream)), "vd_pres1d_create", False)
        self._h = h
        return self

    def __init__(self, basis, n, a, length=2 * math.pi, stream=None):
        import torch
        self.n = int(n)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        b = {"cheb": VD_CHEB_GL, "fourier": VD_FOURIER}[basis]
        h = ctypes.c_void_p()
        _check(lib().vd_visc1d_create(ctypes.byref(h), b, self.n, float(length), float(a),
                                      ctypes.c_void_p(self._stream.cuda_stream)), "vd_visc1d_create", False)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().vd_visc1d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _batch(self, t, name):
        if t.dtype != __import__("torch").float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name}: contiguous float64 CUDA tensor expected")
        if t.shape[-1] != self.n:
            raise ValueError(f"{name}: last dimension must be {self.n}")
        return t.numel() // self.n

    def apply(self, rho, u, precond=False, out=None):
        import torch
        y = out if out is not None else torch.empty_like(u)
        nb = self._batch(u, "u")
        if self._batch(rho, "rho") != nb:
            raise ValueError("rho and u batch sizes differ")
        _check(lib().vd_visc1d_apply(self._h, nb, rho.data_ptr(), u.data_ptr(), y.data_ptr(), 1 if precond else 0),
               "vd_visc1d_apply", False)
        return y

    def solve(self, rho, b, u=None, **opts):
        return self._solve(lib().vd_visc1d_solve, "vd_visc1d_solve", rho, b, u, **opts)

    def solve_noalloc(self, rho, b, u=None, **opts):
        """vd_visc1d_solve_noalloc: the same solve on the library's static
        device scratch (no device allocation in the call)."""
        return self._solve(lib().vd_visc1d_solve_noalloc, "vd_visc1d_solve_noalloc", rho, b, u, **opts)

    def _solve(self, fn, name, rho, b, u=None, **opts):
        import numpy as np
        import torch
        if u is None:
            u = torch.zeros_like(b)
        nb = self._batch(b, "b")
        if self._batch(rho, "rho") != nb or self._batch(u, "u") != nb:
            raise ValueError("batch sizes differ")
        # history: entries per system (int), or a (batch, cap) float64 array
        hist = opts.pop("history", None)
        if hist is not None and not isinstance(hist, np.ndarray):
            hist = np.zeros((nb, int(hist)))
        o = make_opts(**opts)
        if hist is not None:
            if hist.dtype != np.float64 or hist.ndim != 2 or hist.shape[0] != nb or not hist.flags.c_contiguous:
                raise ValueError("history must be a contiguous float64 array of shape (batch, cap)")
            o.history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            o.history_cap = int(hist.shape[1])
        it = np.zeros(nb, dtype=np.int32)
        rr = np.zeros(nb, dtype=np.float64)
        info = vd_solve_info()
        st = fn(self._h, nb, rho.data_ptr(), b.data_ptr(), u.data_ptr(), ctypes.byref(o),
                it.ctypes.data, rr.ctypes.data, ctypes.byref(info))
        _check(st, name)
        d = info.as_dict()
        if hist is not None:
            d["history"] = hist
        return u, it, rr, d

    def kernel_ms(self):
        """Duration of the last apply/solve kernel (HIP events around the launch)."""
        ms = ctypes.c_double()
        _check(lib().vd_visc1d_kernel_ms(self._h, ctypes.byref(ms)), "vd_visc1d_kernel_ms", False)
        return ms.value


class FractionalStep:
    """Fractional-step time integration of the variable-density Navier-Stokes
    equations on [0, 2 pi)^3 (vd_ns_*)."""

    def __init__(self, n, re=1.0, sc=1.0, dt=0.01, s=0.0, visc_rtol=1e-12, pres_rtol=1e-12, restart=30,
                 max_iter=2000, pres_solver="gmres", pres_form="L", stream=None):
        import torch
        self.n = int(n)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        prm = vd_ns_params()
        lib().vd_ns_default_params(ctypes.byref(prm))
        prm.re, prm.sc, prm.dt, prm.s = float(re), float(sc), float(dt), float(s)
        prm.visc_rtol, prm.pres_rtol = float(visc_rtol), float(pres_rtol)
        prm.restart, prm.max_iter = int(restart), int(max_iter)
        prm.pres_solver = SOLVERS[pres_solver]
        prm.pres_form = FORMULATIONS[pres_form]
        h = ctypes.c_void_p()
        _check(lib().vd_ns_create(ctypes.byref(h), self.n, ctypes.byref(prm),
                                  ctypes.c_void_p(self._stream.cuda_stream)), "vd_ns_create", False)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().vd_ns_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_taylor_green(self):
        _check(lib().vd_ns_init_taylor_green(self._h), "vd_ns_init_taylor_green", False)

    def set_state(self, u, rho, p, t=0.0):
        n = self.n
        _check(lib().vd_ns_set_state(self._h, _dev_f64(u, (3, n, n, n), "u"), _dev_f64(rho, (n, n, n), "rho"),
                                     _dev_f64(p, (n, n, n), "p"), float(t)), "vd_ns_set_state", False)

    def step(self, nsteps=1):
        info = vd_ns_info()
        _check(lib().vd_ns_step(self._h, int(nsteps), ctypes.byref(info)), "vd_ns_step", False)
        return info.as_dict()

    def state(self):
        import torch
        n = self.n
        u = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
        rho = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
        p = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
        t = ctypes.c_double()
        _check(lib().vd_ns_get_state(self._h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(rho.data_ptr()),
                                     ctypes.c_void_p(p.data_ptr()), ctypes.byref(t)), "vd_ns_get_state", False)
        return u, rho, p, t.value

    def errors(self):
        e = (ctypes.c_double * 4)()
        _check(lib().vd_ns_errors(self._h, e), "vd_ns_errors", False)
        return {"u": e[0], "p": e[1], "rho": e[2], "div": e[3]}

    def project(self, rho, u, out=None):
        """P_rho(u) = u - grad(phi) / rho, L_rho phi = div u (Sec. 2)."""
        import torch
        n = self.n
        out = out if out is not None else torch.empty_like(u)
        info = vd_solve_info()
        _check(lib().vd_ns_project(self._h, _dev_f64(rho, (n, n, n), "rho"), _dev_f64(u, (3, n, n, n), "u"),
                                   _dev_f64(out, (3, n, n, n), "out"), ctypes.byref(info)), "vd_ns_project")
        return out, info.as_dict()

    def profile_enable(self, on=True):
        _check(lib().vd_ns_profile_enable(self._h, 1 if on else 0), "vd_ns_profile_enable", False)

    def profile_read(self):
        ms = (ctypes.c_double * 3)()
        cnt = (ctypes.c_longlong * 3)()
        by = (ctypes.c_double * 3)()
        _check(lib().vd_ns_profile_read(self._h, ms, cnt, by, 3), "vd_ns_profile_read", False)
        names = ("transforms", "pressure_solves", "viscous_krylov_vector_ops")
        return {names[c]: {"ms": ms[c], "count": cnt[c], "bytes": by[c]} for c in range(3)}


class Server:
    """Continuous-batching solve server (vd_server_*)."""

    def __init__(self, hbm_budget, max_slots=8, dry_seconds=None, batch=3):
        h = ctypes.c_void_p()
        if dry_seconds is None:
            st = lib().vd_server_create(ctypes.byref(h), int(hbm_budget), int(max_slots))
        else:
            st = lib().vd_server_create_dry(ctypes.byref(h), int(hbm_budget), int(max_slots), float(dry_seconds))
        _check(st, "vd_server_create", False)
        self._h = h
        self._keep = {}   # ticket -> tensors the server reads or writes
        _check(lib().vd_server_set_batch(h, int(batch)), "vd_server_set_batch", False)

    def submit(self, shape, rho=None, f=None, x=None, lengths=None, kind="pressure", dt_nu=0.0, ncomp=1,
               user_tag=0, cheb=False, **opts):
        r = vd_request()
        r.desc = make_desc(shape, lengths, cheb)
        r.kind = VD_OP_PRESSURE if kind == "pressure" else VD_OP_HELMHOLTZ
        r.dt_nu = float(dt_nu)
        r.ncomp = int(ncomp)
        # the server reads rho and f and writes x on the device with no shape
        # information beyond the descriptor: check them here (a wrong dtype,
        # shape or layout would otherwise be read or written out of bounds)
        shp = tuple(int(v) for v in shape)
        fshp = (r.ncomp,) + shp if r.kind == VD_OP_HELMHOLTZ and r.ncomp > 1 else shp
        for t, want, what in ((rho, shp, "rho"), (f, fshp, "f"), (x, fshp, "x")):
            if t is not None:
                _dev_f64(t, want, what)
        r.rho = rho.data_ptr() if rho is not None else None
        r.f = f.data_ptr() if f is not None else None
        r.x = x.data_ptr() if x is not None else None
        r.opts = make_opts(**opts)
        r.user_tag = int(user_tag)
        t = ctypes.c_ulonglong()
        _check(lib().vd_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)), "vd_server_submit", False)
        self._keep[t.value] = (rho, f, x)
        return t.value

    def _collect(self, fn, cap, *extra):
        buf = (vd_result * cap)()
        n = ctypes.c_int()
        _check(fn(self._h, buf, cap, ctypes.byref(n), *extra), "vd_server_poll", False)
        out = []
        for i in range(n.value):
            d = buf[i].as_dict()
            self._keep.pop(d["ticket"], None)
            out.append(d)
        return out

    def poll(self, cap=256):
        return self._collect(lib().vd_server_poll, cap)

    def wait(self, timeout=1.0, cap=256):
        return self._collect(lib().vd_server_wait, cap, float(timeout))

    def stats(self):
        st = vd_server_stats_t()
        _check(lib().vd_server_stats(self._h, ctypes.byref(st)), "vd_server_stats", False)
        return {k: getattr(st, k) for k, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().vd_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
