"""libnuht: nonuniform fast Hankel transform on AMD MI355X (gfx950).

Python binding of the C ABI in ``include/nuht.h``: argument marshalling only.
Every step of the transform runs in the HIP kernels of ``libnuht.so``; PyTorch
supplies device memory (float64 tensors on the GPU) and the current stream.
There is no CPU fallback: without the built library, or without a GPU, the
calls raise.

    g_j = sum_k c_k J_nu(omega_j r_k)        (Beckman & O'Neil, Sec. 1, eq. DHT)
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnuht.so")

NUHT_OK = 0
NUHT_FP64 = 0
NUHT_FP32_SPREAD = 1
NUHT_FB_TRANSFORM = 0
NUHT_FB_DIRECT = 1

_ERRORS = {
    -1: "NUHT_EINVAL", -2: "NUHT_EDOMAIN", -3: "NUHT_EPRECISION", -4: "NUHT_ENOMEM",
    -5: "NUHT_EHIP", -6: "NUHT_ECAPACITY", -7: "NUHT_ENOTREADY",
}


class NuhtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class NuhtOpts(ctypes.Structure):
    _fields_ = [("min_size", ctypes.c_int64), ("M_override", ctypes.c_int32),
                ("split_candidates", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("dft_max", ctypes.c_int32), ("spread_chunk", ctypes.c_int32), ("tune", ctypes.c_int32),
                ("vector_spread", ctypes.c_int32), ("local_rank", ctypes.c_int32), ("margin", ctypes.c_double),
                ("tune_cache", ctypes.c_char_p)]


class NuhtInfo(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_int32), ("M", ctypes.c_int32), ("L", ctypes.c_int32),
                ("es_width", ctypes.c_int32),
                ("eps", ctypes.c_double), ("z", ctypes.c_double), ("es_beta", ctypes.c_double),
                ("levels", ctypes.c_int32), ("n_nodes", ctypes.c_int32), ("n_local", ctypes.c_int32),
                ("n_asy", ctypes.c_int32), ("n_direct", ctypes.c_int32), ("n_fft_blocks", ctypes.c_int32),
                ("local_row_members", ctypes.c_int64), ("local_col_members", ctypes.c_int64),
                ("asy_row_members", ctypes.c_int64), ("asy_col_members", ctypes.c_int64),
                ("direct_entries", ctypes.c_int64), ("grid_cells", ctypes.c_int64),
                ("fft_points", ctypes.c_int64), ("dft_row_cells", ctypes.c_int64),
                ("fft_row_members", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("min_size", ctypes.c_int64), ("dft_max", ctypes.c_int32), ("spread_chunk", ctypes.c_int32),
                ("spread_items", ctypes.c_int32), ("dense_items", ctypes.c_int32),
                ("split_candidates", ctypes.c_int32), ("half_order", ctypes.c_int32)]


# every symbol include/nuht.h declares
EXPORTS = ("nuht_plan", "nuht_plan_half", "nuht_execute", "nuht_adjoint", "nuht_gradient", "nuht_gradient_noalloc",
           "nuht_plan_set_order",
           "nuht_plan_info", "nuht_plan_order", "nuht_tune", "nuht_plan_many", "nuht_execute_many", "nuht_batch_info",
           "nuht_batch_destroy", "nuht_destroy", "nuht_strerror", "nuht_direct", "nuht_profile",
           "nuht_profile_stages", "nuht_profile_read",
           "nuht_fb_plan", "nuht_fb_analysis", "nuht_fb_synthesis", "nuht_fb_helmholtz", "nuht_fb_destroy")

STAGES = ("gather", "local_moments", "spread", "grid_assembly", "fft", "direct", "rows_asymptotic", "rows_local")

_lib = None


def load_library():
    """Load libnuht.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2411_09583_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.nuht_plan.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_double, ctypes.c_int64, vp,
                              ctypes.c_int64, vp, ctypes.POINTER(NuhtOpts), vp]
    lib.nuht_plan_half.argtypes = lib.nuht_plan.argtypes
    lib.nuht_execute.argtypes = [vp, vp, vp, vp]
    lib.nuht_adjoint.argtypes = [vp, vp, vp, vp]
    lib.nuht_gradient.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.nuht_gradient_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.nuht_tune.argtypes = [vp, vp, ctypes.c_int, ctypes.POINTER(NuhtOpts), ctypes.POINTER(ctypes.c_double), vp]
    lib.nuht_plan_many.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(vp), ctypes.POINTER(NuhtOpts), vp]
    lib.nuht_execute_many.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.nuht_batch_info.argtypes = [vp, ctypes.c_int, ctypes.POINTER(NuhtInfo)]
    lib.nuht_batch_destroy.argtypes = [vp]
    lib.nuht_plan_set_order.argtypes = [vp, ctypes.c_int, vp]
    lib.nuht_plan_info.argtypes = [vp, ctypes.POINTER(NuhtInfo)]
    lib.nuht_plan_order.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.nuht_destroy.argtypes = [vp]
    lib.nuht_strerror.argtypes = [ctypes.c_int]
    lib.nuht_strerror.restype = ctypes.c_char_p
    lib.nuht_direct.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, vp, vp, ctypes.c_int64, vp, vp, vp]
    lib.nuht_profile.argtypes = [vp, ctypes.c_int]
    lib.nuht_profile_stages.argtypes = [vp, ctypes.c_uint32]
    lib.nuht_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.nuht_fb_plan.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int64, vp, vp, ctypes.c_int64,
                                 ctypes.c_int64, vp, ctypes.c_double, ctypes.c_int32, vp]
    lib.nuht_fb_analysis.argtypes = [vp, vp, vp, vp]
    lib.nuht_fb_synthesis.argtypes = [vp, vp, vp, vp]
    lib.nuht_fb_helmholtz.argtypes = [vp, ctypes.c_double, vp, vp, vp, vp, vp]
    lib.nuht_fb_destroy.argtypes = [vp]
    for name in ("nuht_plan", "nuht_plan_half", "nuht_execute", "nuht_adjoint", "nuht_gradient", "nuht_gradient_noalloc",
                 "nuht_plan_set_order", "nuht_plan_info", "nuht_plan_order",
                 "nuht_tune", "nuht_plan_many", "nuht_execute_many", "nuht_batch_info", "nuht_batch_destroy",
                 "nuht_destroy", "nuht_direct", "nuht_profile", "nuht_profile_stages", "nuht_profile_read",
                 "nuht_fb_plan",
                 "nuht_fb_analysis", "nuht_fb_synthesis", "nuht_fb_helmholtz", "nuht_fb_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code):
    if code != NUHT_OK:
        raise NuhtError(code, load_library().nuht_strerror(code).decode())


def _dev_f64(x, name):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if x.device.type != "cuda" or x.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor on the GPU")
    if x.dim() != 1:
        raise ValueError(f"{name} must be one-dimensional")
    return x.contiguous()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


class Plan:
    """A planned transform r (n points) -> omega (m frequencies) of order nu
    (an integer, or a positive half-integer such as 0.5 or 1.5).

    The plan sorts and subdivides once; ``execute`` and ``adjoint`` then run
    asynchronously on the current stream.  ``execute(c)`` returns
    g_j = sum_k c_k J_nu(omega_j r_k); ``adjoint(y)`` returns
    cbar_k = sum_j y_j J_nu(omega_j r_k).
    """

    def __init__(self, r, omega, nu: int, eps: float, *, min_size: int = 0, M: int = 0,
                 split_candidates: int = 0, precision: int = NUHT_FP64, dft_max: int = 0,
                 spread_chunk: int = 0, vector_spread: bool = False, local_rank: int = 0, margin: float = 0.0,
                 tune_cache: str = None):
        lib = load_library()
        r = _dev_f64(r, "r")
        omega = _dev_f64(omega, "omega")
        self.n = r.numel()
        self.m = omega.numel()
        self.device = r.device
        opts = NuhtOpts(min_size, M, split_candidates, precision, dft_max, spread_chunk, 0,
                        1 if vector_spread else 0, int(local_rank), float(margin),
                        os.fsencode(tune_cache) if tune_cache else None)
        nu2 = 2.0 * float(nu)
        if nu2 != round(nu2):
            raise ValueError("the order must be an integer or a half-integer")
        self.nu = nu
        h = ctypes.c_void_p()
        _check(lib.nuht_plan_half(ctypes.byref(h), int(round(nu2)), float(eps), self.n, _ptr(r), self.m,
                                  _ptr(omega), ctypes.byref(opts), _stream()))
        self._h = h

    def execute(self, c, out=None):
        c = _dev_f64(c, "c")
        if c.numel() != self.n:
            raise ValueError("c must have n entries")
        g = out if out is not None else torch.empty(self.m, dtype=torch.float64, device=self.device)
        _check(load_library().nuht_execute(self._h, _ptr(c), _ptr(g), _stream()))
        return g

    def adjoint(self, y, out=None):
        y = _dev_f64(y, "y")
        if y.numel() != self.m:
            raise ValueError("y must have m entries")
        cb = out if out is not None else torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(load_library().nuht_adjoint(self._h, _ptr(y), _ptr(cb), _stream()))
        return cb

    def gradient(self, c, gbar, *, want_c=True, want_r=True, want_omega=True, out=None):
        """(dL/dc, dL/dr, dL/domega) for g = execute(c) and gbar = dL/dg; entries
        not wanted are None."""
        return self._gradient("nuht_gradient", c, gbar, want_c, want_r, want_omega, out)

    def gradient_noalloc(self, c, gbar, *, want_c=True, want_r=True, want_omega=True, out=None):
        """The same through nuht_gradient_noalloc: no device allocation inside
        the library (the temporaries live in its per-device array; the
        partitions must have been built by an earlier gradient, adjoint or
        set_order call).  ``out`` = (dc, dr, domega) preallocated tensors (None
        entries are allocated here by torch)."""
        return self._gradient("nuht_gradient_noalloc", c, gbar, want_c, want_r, want_omega, out)

    def _gradient(self, entry, c, gbar, want_c, want_r, want_omega, out):
        gbar = _dev_f64(gbar, "gbar")
        if gbar.numel() != self.m:
            raise ValueError("gbar must have m entries")
        if want_r or want_omega:
            c = _dev_f64(c, "c")
            if c.numel() != self.n:
                raise ValueError("c must have n entries")
        new = lambda k: torch.empty(k, dtype=torch.float64, device=self.device)
        o_c, o_r, o_w = out if out is not None else (None, None, None)
        dc = (o_c if o_c is not None else new(self.n)) if want_c else None
        dr = (o_r if o_r is not None else new(self.n)) if want_r else None
        dw = (o_w if o_w is not None else new(self.m)) if want_omega else None
        null = ctypes.c_void_p(0)
        _check(getattr(load_library(), entry)(self._h, _ptr(c) if (want_r or want_omega) else null, _ptr(gbar),
                                             _ptr(dc) if dc is not None else null,
                                             _ptr(dr) if dr is not None else null,
                                             _ptr(dw) if dw is not None else null, _stream()))
        return dc, dr, dw

    def tune(self, c=None, reps: int = 3) -> dict:
        """Autotune this plan's spreading item size, min_size and dft_max (see
        nuht_tune); the plan adopts the best options.  Returns them with the
        best time per execute in ms."""
        best = NuhtOpts()
        ms = ctypes.c_double()
        cp = _ptr(_dev_f64(c, "c")) if c is not None else ctypes.c_void_p(0)
        _check(load_library().nuht_tune(self._h, cp, int(reps), ctypes.byref(best), ctypes.byref(ms), _stream()))
        out = {f: getattr(best, f) for f, _ in NuhtOpts._fields_ if f != "tune_cache"}
        out["ms"] = ms.value
        return out

    def set_order(self, nu: int):
        _check(load_library().nuht_plan_set_order(self._h, int(nu), _stream()))

    def info(self) -> dict:
        inf = NuhtInfo()
        _check(load_library().nuht_plan_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in NuhtInfo._fields_}

    def order(self):
        """The plan's sorted geometry (nuht_plan_order): r sorted, the caller
        index of each sorted point, omega sorted and its indices."""
        f64 = dict(dtype=torch.float64, device=self.device)
        i32 = dict(dtype=torch.int32, device=self.device)
        rs, pr = torch.empty(self.n, **f64), torch.empty(self.n, **i32)
        ws, pw = torch.empty(self.m, **f64), torch.empty(self.m, **i32)
        _check(load_library().nuht_plan_order(self._h, _ptr(rs), _ptr(pr), _ptr(ws), _ptr(pw), _stream()))
        return rs, pr, ws, pw

    def profile(self, enable: bool = True, stages=None):
        """Start (clearing earlier records) or stop per-stage event timing;
        stages: names from STAGES to time only those (all by default)."""
        if stages is None:
            _check(load_library().nuht_profile(self._h, 1 if enable else 0))
        else:
            mask = sum(1 << STAGES.index(s) for s in stages) if enable else 0
            _check(load_library().nuht_profile_stages(self._h, mask))

    def profile_read(self):
        """Per-stage totals in ms over the profiled calls, and the call count."""
        ms = (ctypes.c_double * len(STAGES))()
        calls = ctypes.c_int64()
        _check(load_library().nuht_profile_read(self._h, ms, ctypes.byref(calls)))
        return dict(zip(STAGES, list(ms))), calls.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().nuht_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent transforms (uneven n, m and order), planned together
    and executed as one captured graph (nuht_plan_many / nuht_execute_many)."""

    def __init__(self, rs, omegas, nus, eps: float, *, tune: bool = False, min_size: int = 0,
                 dft_max: int = 0, spread_chunk: int = 0, margin: float = 0.0, tune_cache: str = None):
        lib = load_library()
        if not (len(rs) == len(omegas) == len(nus)):
            raise ValueError("rs, omegas and nus must have the same length")
        self.count = len(rs)
        self._keep = [(_dev_f64(r, "r"), _dev_f64(w, "omega")) for r, w in zip(rs, omegas)]
        self.n = [r.numel() for r, _ in self._keep]
        self.m = [w.numel() for _, w in self._keep]
        self.device = self._keep[0][0].device if self.count else torch.device("cuda")
        k = self.count
        nu_a = (ctypes.c_int * k)(*[int(v) for v in nus])
        n_a = (ctypes.c_int64 * k)(*self.n)
        m_a = (ctypes.c_int64 * k)(*self.m)
        r_a = (ctypes.c_void_p * k)(*[_ptr(r).value for r, _ in self._keep])
        w_a = (ctypes.c_void_p * k)(*[_ptr(w).value for _, w in self._keep])
        opts = NuhtOpts(min_size, 0, 0, NUHT_FP64, dft_max, spread_chunk, 1 if tune else 0, 0, 0, float(margin),
                        os.fsencode(tune_cache) if tune_cache else None)
        h = ctypes.c_void_p()
        _check(lib.nuht_plan_many(ctypes.byref(h), k, nu_a, float(eps), n_a, r_a, m_a, w_a, ctypes.byref(opts),
                                  _stream()))
        self._h = h
        self._keep = None          # the plans hold sorted copies

    def execute(self, cs, gs=None):
        if len(cs) != self.count:
            raise ValueError("one weight vector per transform")
        cs = [_dev_f64(c, "c") for c in cs]
        for c, n in zip(cs, self.n):
            if c.numel() != n:
                raise ValueError("weight vector of the wrong length")
        if gs is None:
            gs = [torch.empty(m, dtype=torch.float64, device=self.device) for m in self.m]
        k = self.count
        c_a = (ctypes.c_void_p * k)(*[_ptr(c).value for c in cs])
        g_a = (ctypes.c_void_p * k)(*[_ptr(g).value for g in gs])
        self._io = (cs, gs)        # alive until the next call
        _check(load_library().nuht_execute_many(self._h, c_a, g_a, _stream()))
        return gs

    def info(self, i: int) -> dict:
        inf = NuhtInfo()
        _check(load_library().nuht_batch_info(self._h, int(i), ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in NuhtInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load_library().nuht_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DiskSolver:
    """Fourier-Bessel expansions and the Helmholtz solver on the unit disk
    (nuht_fb_*): m radii r with radial weights wr, t equispaced angles, orders
    -L .. L and J radial modes per order; zeros is an (L + 1) x J tensor of the
    first J positive zeros of J_0 .. J_L.  method "transform" (the default)
    takes the radial sums with this library's transforms, "direct" sums the
    m J terms per order with J_l evaluated in place."""

    METHODS = {"transform": NUHT_FB_TRANSFORM, "direct": NUHT_FB_DIRECT}

    def __init__(self, r, wr, t: int, zeros, eps: float, method: str = "transform"):
        if method not in self.METHODS:
            raise ValueError(f"method must be one of {sorted(self.METHODS)}")
        lib = load_library()
        r = _dev_f64(r, "r")
        wr = _dev_f64(wr, "wr")
        if zeros.dim() != 2 or zeros.device.type != "cuda" or zeros.dtype != torch.float64:
            raise TypeError("zeros must be an (L + 1) x J float64 tensor on the GPU")
        zeros = zeros.contiguous()
        self.L, self.J = zeros.shape[0] - 1, zeros.shape[1]
        self.m, self.t = r.numel(), int(t)
        if wr.numel() != self.m:
            raise ValueError("r and wr must have the same length")
        self.device = r.device
        h = ctypes.c_void_p()
        _check(lib.nuht_fb_plan(ctypes.byref(h), self.L, self.m, _ptr(r), _ptr(wr), self.t, self.J, _ptr(zeros),
                                float(eps), self.METHODS[method], _stream()))
        self._h = h
        self.method = method

    def _grid(self, f, name):
        if f.shape != (self.m, self.t) or f.device.type != "cuda" or f.dtype != torch.float64:
            raise ValueError(f"{name} must be an m x t float64 tensor on the GPU")
        return f.contiguous()

    def _coef(self, a, name):
        if a.shape != (2 * self.L + 1, self.J) or a.device.type != "cuda" or a.dtype != torch.complex128:
            raise ValueError(f"{name} must be a (2L + 1) x J complex128 tensor on the GPU")
        return a.contiguous()

    def analysis(self, f):
        """alpha[l + L, j - 1]: the Fourier-Bessel coefficients of the samples f."""
        f = self._grid(f, "f")
        alpha = torch.empty((2 * self.L + 1, self.J), dtype=torch.complex128, device=self.device)
        _check(load_library().nuht_fb_analysis(self._h, _ptr(f), _ptr(alpha), _stream()))
        return alpha

    def synthesis(self, beta):
        """The real part of the expansion with coefficients beta on the grid."""
        beta = self._coef(beta, "beta")
        u = torch.empty((self.m, self.t), dtype=torch.float64, device=self.device)
        _check(load_library().nuht_fb_synthesis(self._h, _ptr(beta), _ptr(u), _stream()))
        return u

    def helmholtz(self, kappa: float, f, return_coefficients: bool = False):
        """u with (Delta + kappa^2) u = f on the disk and u = 0 on the circle."""
        f = self._grid(f, "f")
        u = torch.empty((self.m, self.t), dtype=torch.float64, device=self.device)
        alpha = beta = None
        if return_coefficients:
            alpha = torch.empty((2 * self.L + 1, self.J), dtype=torch.complex128, device=self.device)
            beta = torch.empty_like(alpha)
        _check(load_library().nuht_fb_helmholtz(self._h, float(kappa), _ptr(f),
                                                _ptr(alpha) if alpha is not None else None,
                                                _ptr(beta) if beta is not None else None, _ptr(u), _stream()))
        return (u, alpha, beta) if return_coefficients else u

    def close(self):
        if getattr(self, "_h", None):
            load_library().nuht_fb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NuhtFunction(torch.autograd.Function):
    """g = A(r, omega) c, differentiable in c, r and omega.

    The forward pass plans on (r, omega) (the method needs no precomputation
    beyond the plan) and keeps the plan for the backward pass, which runs
    nuht_gradient: A^T gbar for c, and the order nu -+ 1 transforms of
    J_nu' = (J_{nu-1} - J_{nu+1}) / 2 for r and omega.  The plan lives as
    long as the autograd graph that holds it (freed with the graph, not by
    the first backward), so a graph kept with retain_graph=True can be
    differentiated again.
    """

    @staticmethod
    def forward(ctx, c, r, omega, nu, eps=1e-12):
        plan = Plan(r.detach(), omega.detach(), nu, eps)
        g = plan.execute(c.detach())
        ctx.plan = plan
        ctx.save_for_backward(c)
        return g

    @staticmethod
    def backward(ctx, gbar):
        (c,) = ctx.saved_tensors
        want = ctx.needs_input_grad
        dc, dr, dw = ctx.plan.gradient(c.detach(), gbar.contiguous(), want_c=want[0], want_r=want[1],
                                       want_omega=want[2])
        return dc, dr, dw, None, None


def nuht(c, r, omega, nu: int, eps: float = 1e-12, **opts):
    """One-shot transform: plan, execute, free."""
    p = Plan(r, omega, nu, eps, **opts)
    try:
        return p.execute(c)
    finally:
        p.close()


def direct(c, r, omega, nu: int, eps: float = 1e-12):
    """Brute-force O(nm) evaluation on the GPU with the library's J_nu."""
    lib = load_library()
    r = _dev_f64(r, "r")
    c = _dev_f64(c, "c")
    omega = _dev_f64(omega, "omega")
    g = torch.empty(omega.numel(), dtype=torch.float64, device=omega.device)
    _check(lib.nuht_direct(int(nu), float(eps), r.numel(), _ptr(r), _ptr(c), omega.numel(), _ptr(omega),
                           _ptr(g), _stream()))
    return g
