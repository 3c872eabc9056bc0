"""Python binding of the HIP Helmholtz solver library (``libhz.so``).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels. PyTorch supplies device memory (tensors passed by data pointer) and
the stream the work is ordered on. Importing fails loudly when the built
library is missing; there is no CPU fallback.

The functions mirror the C ABI in ``include/hz.h`` (same names without the
``hz_`` prefix on the methods of :class:`Context`).
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhz.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built: run `python -m paper_1712_08743_amd.build` "
        "(hipcc for gfx950) before using the solver")

_lib = ctypes.CDLL(LIB_PATH)

HZ_OK, HZ_WARN_NOCONV = 0, 1
HZ_ERR_ARG, HZ_ERR_SHAPE, HZ_ERR_NOMEM, HZ_ERR_DEVICE, HZ_ERR_STATE = -1, -2, -3, -4, -5
HZ_BICGSTAB, HZ_GMRES = 0, 1
HZ_PRECOND_MG, HZ_PRECOND_EXACT, HZ_PRECOND_NONE = 0, 1, 2
HZ_RHS_CONVERGED, HZ_RHS_MAXIT, HZ_RHS_BREAKDOWN, HZ_RHS_NONFINITE = 0, 1, 2, 3
HZ_MAX_LEVELS = 12
HZ_COARSE_AUTO, HZ_COARSE_EXACT, HZ_COARSE_JACOBI = 0, 1, 2
COARSE = {"auto": HZ_COARSE_AUTO, "exact": HZ_COARSE_EXACT, "jacobi": HZ_COARSE_JACOBI}
HZ_KERNEL = {"smooth": 0, "apply": 1, "restrict": 2, "prolong": 3, "update": 4, "coarse": 5, "presmooth": 6,
             "presmooth_s": 7, "apply_s": 8, "levels": 9}

PRECOND = {"mg": HZ_PRECOND_MG, "exact": HZ_PRECOND_EXACT, "none": HZ_PRECOND_NONE}
KRYLOV = {"bicgstab": HZ_BICGSTAB, "gmres": HZ_GMRES}


class CtxOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hip_stream", ctypes.c_void_p),
                ("workspace_budget_bytes", ctypes.c_size_t)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("krylov", ctypes.c_int), ("gmres_m", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("precond", ctypes.c_int), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("levels", ctypes.c_int), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("jacobi_w", ctypes.c_double),
                ("jacobi_w_level", ctypes.POINTER(ctypes.c_double)), ("autotune", ctypes.c_int),
                ("chunk_rows", ctypes.c_int), ("coarse", ctypes.c_int), ("coarse_sweeps", ctypes.c_int),
                ("graphs", ctypes.c_int), ("restart_at", ctypes.c_int), ("plain", ctypes.c_int)]


class RhsInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("relres", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_size_t), ("slots", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nz", ctypes.c_int), ("nx", ctypes.c_int), ("h", ctypes.c_double),
                ("m_dev", ctypes.c_void_p), ("nfreq", ctypes.c_int), ("freq_hz", ctypes.POINTER(ctypes.c_double)),
                ("alpha", ctypes.c_double), ("nrhs", ctypes.c_int), ("b_dev", ctypes.c_void_p),
                ("u_dev", ctypes.c_void_p), ("opts", ctypes.POINTER(SolveOpts))]


_vp, _ip, _dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
_i, _d = ctypes.c_int, ctypes.c_double

_SIGS = {
    "hz_default_opts": (None, [ctypes.POINTER(SolveOpts)]),
    "hz_create": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(CtxOpts)]),
    "hz_destroy": (None, [_vp]),
    "hz_set_model": (_i, [_vp, _i, _i, _i, _d, _vp]),
    "hz_set_density": (_i, [_vp, _vp]),
    "hz_point_rhs": (_i, [_vp, _i, _ip, _ip, _vp, _vp]),
    "hz_set_model_3d": (_i, [_vp, _i, _i, _i, _d, _vp]),
    "hz_point_rhs_3d": (_i, [_vp, _i, _ip, _ip, _ip, _vp, _vp]),
    "hz_solve": (_i, [_vp, ctypes.POINTER(SolveOpts), _i, _dp, _d, _i, _vp, _vp,
                      ctypes.POINTER(RhsInfo)]),
    "hz_solve_noalloc": (_i, [_vp, ctypes.POINTER(SolveOpts), _i, _dp, _d, _i, _vp, _vp,
                              ctypes.POINTER(RhsInfo)]),
    "hz_misfit": (_i, [_vp, ctypes.POINTER(SolveOpts), _i, _dp, _d, _i, _ip, _ip, _vp, _i, _ip,
                       _ip, _vp, _d, _dp, _vp, ctypes.POINTER(RhsInfo)]),
    "hz_gradient": (_i, [_vp, ctypes.POINTER(SolveOpts), _i, _dp, _d, _i, _ip, _ip, _vp, _i, _ip,
                         _ip, _vp, _d, _dp, _vp, ctypes.POINTER(RhsInfo)]),
    "hz_gn_step": (_i, [_vp, ctypes.POINTER(SolveOpts), _i, _dp, _d, _i, _ip, _ip, _vp, _i, _ip,
                        _ip, _vp, _d, _i, _d, _dp, _vp, _ip, ctypes.POINTER(RhsInfo)]),
    "hz_misfit_3d": (_i, [_vp, ctypes.POINTER(SolveOpts), _i, _dp, _d, _i, _ip, _ip, _ip, _vp, _i, _ip,
                          _ip, _ip, _vp, _d, _dp, _vp, ctypes.POINTER(RhsInfo)]),
    "hz_gradient_3d": (_i, [_vp, ctypes.POINTER(SolveOpts), _i, _dp, _d, _i, _ip, _ip, _ip, _vp, _i, _ip,
                            _ip, _ip, _vp, _d, _dp, _vp, ctypes.POINTER(RhsInfo)]),
    "hz_gn_step_3d": (_i, [_vp, ctypes.POINTER(SolveOpts), _i, _dp, _d, _i, _ip, _ip, _ip, _vp, _i, _ip,
                           _ip, _ip, _vp, _d, _i, _d, _dp, _vp, _ip, ctypes.POINTER(RhsInfo)]),
    "hz_plan": (_i, [_vp, ctypes.POINTER(SolveOpts), _d, _ip, _dp]),
    "hz_plan_grid": (_i, [_i, _i, _i, _d, _d, _d, ctypes.POINTER(SolveOpts), _d, _ip, _dp]),
    "hz_apply": (_i, [_vp, _i, _i, _d, _d, _d, _d, _i, _vp, _vp]),
    "hz_smooth": (_i, [_vp, _i, _d, _d, _d, _d, _i, _vp, _vp, _vp]),
    "hz_restrict": (_i, [_vp, _i, _d, _d, _d, _i, _vp, _vp, _vp]),
    "hz_prolong": (_i, [_vp, _i, _i, _vp, _vp]),
    "hz_precond": (_i, [_vp, ctypes.POINTER(SolveOpts), _d, _i, _vp, _vp]),
    "hz_timing_start": (_i, [_vp, ctypes.c_uint]),
    "hz_timing_read": (_i, [_vp, _i, _ip, _dp]),
    "hz_footprint": (ctypes.c_size_t, [_i, _i, _i, _i, _i, ctypes.POINTER(SolveOpts)]),
    "hz_server_footprint": (ctypes.c_size_t, [_i, _i, _i, _i, _i, ctypes.POINTER(SolveOpts)]),
    "hz_server_create": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(ServerOpts)]),
    "hz_server_destroy": (None, [_vp]),
    "hz_server_submit": (_i, [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_longlong)]),
    "hz_server_wait": (_i, [_vp, ctypes.c_longlong, ctypes.POINTER(RhsInfo), _dp]),
    "hz_server_stats": (_i, [_vp, _ip, _ip, _ip, ctypes.POINTER(ctypes.c_size_t)]),
    "hz_status_str": (ctypes.c_char_p, [_i]),
    "hz_last_error": (ctypes.c_char_p, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class HzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_lib.hz_status_str(code).decode()} ({code}): {msg}")
        self.code = code


def default_opts():
    o = SolveOpts()
    _lib.hz_default_opts(ctypes.byref(o))
    return o


def make_opts(krylov="bicgstab", gmres_m=30, tol=1e-8, maxit=10000, precond="mg", beta=(1.0, 0.5),
              levels=0, nu=(2, 2), jacobi_w=0.8, jacobi_w_level=None, autotune=True, chunk_rows=0,
              graphs=False, coarse="auto", coarse_sweeps=2, restart_at=0, plain=False):
    """Build an hz_solve_opts; returns (opts, keepalive)."""
    o = default_opts()
    o.krylov = KRYLOV[krylov] if isinstance(krylov, str) else int(krylov)
    o.gmres_m = int(gmres_m)
    o.tol = float(tol)
    o.maxit = int(maxit)
    o.precond = PRECOND[precond] if isinstance(precond, str) else int(precond)
    o.beta1, o.beta2 = float(beta[0]), float(beta[1])
    o.levels = int(levels)
    o.nu1, o.nu2 = int(nu[0]), int(nu[1])
    o.jacobi_w = float(jacobi_w)
    o.autotune = 1 if autotune else 0
    o.chunk_rows = int(chunk_rows)
    o.graphs = 1 if graphs else 0
    o.restart_at = int(restart_at)
    o.plain = 1 if plain else 0
    o.coarse = COARSE[coarse] if isinstance(coarse, str) else int(coarse)
    o.coarse_sweeps = int(coarse_sweeps)
    keep = None
    if jacobi_w_level is not None:
        keep = (ctypes.c_double * max(1, len(jacobi_w_level)))(*[float(w) for w in jacobi_w_level])
        o.jacobi_w_level = ctypes.cast(keep, ctypes.POINTER(ctypes.c_double))
    return o, keep


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _int_array(vals):
    return (ctypes.c_int * len(vals))(*[int(v) for v in vals])


class Context:
    """One library context bound to a device and torch's current stream there."""

    def __init__(self, device=0, budget_bytes=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        co = CtxOpts(device, ctypes.c_void_p(stream.cuda_stream), budget_bytes)
        h = ctypes.c_void_p()
        rc = _lib.hz_create(ctypes.byref(h), ctypes.byref(co))
        if rc != HZ_OK:
            raise HzError(rc, "hz_create failed")
        self._h = h
        self.shape = None
        self.h = None

    def close(self):
        if getattr(self, "_h", None):
            _lib.hz_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_warn=False):
        if rc < 0 or (rc > 0 and not allow_warn):
            raise HzError(rc, _lib.hz_last_error(self._h).decode())
        return rc

    # -- model and sources -------------------------------------------------
    def set_model(self, m, h):
        """m: float64 tensor (n,) for 1D, (nz, nx) for 2D or (nz, ny, nx) for 3D, slowness in s/m."""
        t = self.torch
        m = m.to(device=self.device, dtype=t.float64).contiguous()
        if m.dim() == 1:
            dim, nz, nx = 1, 1, m.shape[0]
        elif m.dim() == 2:
            dim, nz, nx = 2, m.shape[0], m.shape[1]
        elif m.dim() == 3:
            dim = 3
        else:
            raise ValueError("m must be 1D, 2D or 3D")
        if dim == 3:
            self._check(_lib.hz_set_model_3d(self._h, m.shape[0], m.shape[1], m.shape[2], float(h), _ptr(m)))
        else:
            self._check(_lib.hz_set_model(self._h, dim, nz, nx, float(h), _ptr(m)))
        self.shape = tuple(m.shape)
        self.dim = dim
        self.h = float(h)
        self._m = m
        self._rho = None
        return self

    def set_density(self, rho):
        """Density of Eq. (1) on the model (float64 tensor of the model's
        shape, finite and positive); None returns to constant density."""
        if rho is None:
            self._check(_lib.hz_set_density(self._h, None))
            self._rho = None
            return self
        t = self.torch
        rho = rho.to(device=self.device, dtype=t.float64).contiguous()
        if tuple(rho.shape) != self.shape:
            raise ValueError(f"density shape {tuple(rho.shape)} is not the model's {self.shape}")
        self._check(_lib.hz_set_density(self._h, _ptr(rho)))
        self._rho = rho
        return self

    @property
    def n(self):
        n = 1
        for s in self.shape:
            n *= s
        return n

    def point_rhs(self, iz, ix, amp=None):
        """Weighted point sources, complex128 tensor [nsrc, *shape]."""
        t = self.torch
        nsrc = len(ix)
        b = t.empty((nsrc,) + self.shape, dtype=t.complex128, device=self.device)
        ampbuf = None
        if amp is not None:
            ampbuf = (ctypes.c_double * (2 * nsrc))()
            for k, a in enumerate(amp):
                ampbuf[2 * k], ampbuf[2 * k + 1] = complex(a).real, complex(a).imag
        self._check(_lib.hz_point_rhs(self._h, nsrc, _int_array(iz), _int_array(ix),
                                      ctypes.cast(ampbuf, ctypes.c_void_p) if ampbuf is not None else None,
                                      _ptr(b)))
        return b

    def point_rhs_3d(self, iz, iy, ix, amp=None):
        """Weighted point sources on a 3D model, complex128 tensor [nsrc, nz, ny, nx]."""
        t = self.torch
        nsrc = len(ix)
        b = t.empty((nsrc,) + self.shape, dtype=t.complex128, device=self.device)
        ampbuf = None
        if amp is not None:
            ampbuf = (ctypes.c_double * (2 * nsrc))()
            for k, a in enumerate(amp):
                ampbuf[2 * k], ampbuf[2 * k + 1] = complex(a).real, complex(a).imag
        self._check(_lib.hz_point_rhs_3d(self._h, nsrc, _int_array(iz), _int_array(iy), _int_array(ix),
                                         ctypes.cast(ampbuf, ctypes.c_void_p) if ampbuf is not None else None,
                                         _ptr(b)))
        return b

    # -- solves ------------------------------------------------------------
    def solve(self, freqs, alpha, b, out=None, noalloc=False, **opt):
        """Solve for every frequency and every right-hand side.

        b: complex128 tensor [nfreq, nrhs, *shape] (or [nrhs, *shape] for one
        frequency). Returns (u, info) with info a list of (status, iters, relres).
        noalloc=True calls hz_solve_noalloc (the workspace from the library's
        static device array; pass ``out`` to allocate nothing on this side either).
        """
        t = self.torch
        freqs = [float(f) for f in freqs]
        nf = len(freqs)
        b = b.to(self.device).contiguous()
        if b.dim() == len(self.shape) + 1:
            b = b.reshape((1,) + tuple(b.shape))
        if b.dtype != t.complex128 or b.shape[0] != nf or tuple(b.shape[2:]) != self.shape:
            raise ValueError(f"b must be complex128 [{nf}, nrhs, {self.shape}], got {b.dtype} {tuple(b.shape)}")
        nrhs = b.shape[1]
        u = out if out is not None else t.empty_like(b)
        if u.shape != b.shape or u.dtype != b.dtype or not u.is_contiguous() or u.device != b.device:
            raise ValueError("out must be a contiguous tensor like b")
        o, keep = make_opts(**opt)
        info = (RhsInfo * (nf * nrhs))()
        fa = (ctypes.c_double * nf)(*freqs)
        call = _lib.hz_solve_noalloc if noalloc else _lib.hz_solve
        rc = call(self._h, ctypes.byref(o), nf, fa, float(alpha), nrhs, _ptr(b), _ptr(u), info)
        self._check(rc, allow_warn=True)
        del keep
        self.last_seconds = [i.seconds for i in info]
        return u, [(i.status, i.iters, i.relres) for i in info]

    def _fwi_call(self, name, three_d, freqs, src, rec, d_obs, src_amp, nrec_info):
        """Marshal the arguments shared by the misfit, gradient and
        Gauss-Newton calls: (function, leading args, trailing arg builder)."""
        t = self.torch
        freqs = [float(f) for f in freqs]
        nf, ns, nr = len(freqs), len(src), len(rec)
        d_obs = d_obs.to(self.device, t.complex128).contiguous()
        assert tuple(d_obs.shape) == (nf, ns, nr)
        ampbuf = None
        if src_amp is not None:
            ampbuf = (ctypes.c_double * (2 * ns))()
            for k, a in enumerate(src_amp):
                ampbuf[2 * k], ampbuf[2 * k + 1] = complex(a).real, complex(a).imag
        naxes = 3 if three_d else 2
        for q in list(src) + list(rec):
            if len(q) != naxes:
                raise ValueError(f"sources and receivers are {naxes}-tuples of node indices, got {q}")
        src_axes = [_int_array([q[a] for q in src]) for a in range(naxes)]
        rec_axes = [_int_array([q[a] for q in rec]) for a in range(naxes)]
        amp = ctypes.cast(ampbuf, ctypes.c_void_p) if ampbuf is not None else None
        fa = (ctypes.c_double * nf)(*freqs)
        fn = getattr(_lib, name + ("_3d" if three_d else ""))
        head = [nf, fa]
        pts = [ns] + src_axes + [amp, nr] + rec_axes + [_ptr(d_obs)]
        info = (RhsInfo * (nrec_info * nf * ns))()
        return fn, head, pts, info, d_obs, (ampbuf, src_axes, rec_axes, fa)

    def _misfit(self, three_d, freqs, alpha, src, rec, d_obs, lam, src_amp, opt):
        fn, head, pts, info, d_obs, keep_args = self._fwi_call("hz_misfit", three_d, freqs, src, rec, d_obs,
                                                               src_amp, 1)
        d_cal = self.torch.empty_like(d_obs)
        o, keep = make_opts(**opt)
        J = ctypes.c_double()
        rc = fn(self._h, ctypes.byref(o), *head, float(alpha), *pts, float(lam), ctypes.byref(J), _ptr(d_cal), info)
        self._check(rc, allow_warn=True)
        del keep, keep_args
        return J.value, d_cal, [(i.status, i.iters, i.relres) for i in info]

    def _gradient(self, three_d, freqs, alpha, src, rec, d_obs, lam, src_amp, opt):
        fn, head, pts, info, d_obs, keep_args = self._fwi_call("hz_gradient", three_d, freqs, src, rec, d_obs,
                                                               src_amp, 2)
        grad = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        o, keep = make_opts(**opt)
        J = ctypes.c_double()
        rc = fn(self._h, ctypes.byref(o), *head, float(alpha), *pts, float(lam), ctypes.byref(J), _ptr(grad), info)
        self._check(rc, allow_warn=True)
        del keep, keep_args
        return J.value, grad, [(i.status, i.iters, i.relres) for i in info]

    def _gn_step(self, three_d, freqs, alpha, src, rec, d_obs, lam, cg_iters, cg_tol, src_amp, opt):
        fn, head, pts, info, d_obs, keep_args = self._fwi_call("hz_gn_step", three_d, freqs, src, rec, d_obs,
                                                               src_amp, 1)
        dm = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        o, keep = make_opts(**opt)
        J = ctypes.c_double()
        done = ctypes.c_int()
        rc = fn(self._h, ctypes.byref(o), *head, float(alpha), *pts, float(lam), int(cg_iters), float(cg_tol),
                ctypes.byref(J), _ptr(dm), ctypes.byref(done), info)
        self._check(rc, allow_warn=True)
        del keep, keep_args
        return dm, J.value, done.value, [(i.status, i.iters, i.relres) for i in info]

    def misfit(self, freqs, alpha, src, rec, d_obs, lam, src_amp=None, **opt):
        """J(m) of Eq. (4); src, rec: lists of (iz, ix). Returns (J, d_cal, info)."""
        return self._misfit(False, freqs, alpha, src, rec, d_obs, lam, src_amp, opt)

    def misfit_3d(self, freqs, alpha, src, rec, d_obs, lam, src_amp=None, **opt):
        """misfit on a 3D model; src, rec: lists of (iz, iy, ix)."""
        return self._misfit(True, freqs, alpha, src, rec, d_obs, lam, src_amp, opt)

    def gradient(self, freqs, alpha, src, rec, d_obs, lam, src_amp=None, **opt):
        """J(m) and dJ/dm (float64 tensor shaped like m) by the adjoint-state
        method. Returns (J, grad, info) with 2 * nfreq * nsrc info records
        (forward solves, then adjoint solves)."""
        return self._gradient(False, freqs, alpha, src, rec, d_obs, lam, src_amp, opt)

    def gradient_3d(self, freqs, alpha, src, rec, d_obs, lam, src_amp=None, **opt):
        """gradient on a 3D model; src, rec: lists of (iz, iy, ix)."""
        return self._gradient(True, freqs, alpha, src, rec, d_obs, lam, src_amp, opt)

    def gn_step(self, freqs, alpha, src, rec, d_obs, lam, cg_iters, cg_tol=0.0, src_amp=None, **opt):
        """One Gauss-Newton update (Eq. (9)) of the current model by CG on the
        Gauss-Newton system. Returns (dm, J, cg_iterations, info)."""
        return self._gn_step(False, freqs, alpha, src, rec, d_obs, lam, cg_iters, cg_tol, src_amp, opt)

    def gn_step_3d(self, freqs, alpha, src, rec, d_obs, lam, cg_iters, cg_tol=0.0, src_amp=None, **opt):
        """gn_step on a 3D model; src, rec: lists of (iz, iy, ix)."""
        return self._gn_step(True, freqs, alpha, src, rec, d_obs, lam, cg_iters, cg_tol, src_amp, opt)

    def plan(self, freq, **opt):
        o, keep = make_opts(**opt)
        L = ctypes.c_int()
        w = (ctypes.c_double * HZ_MAX_LEVELS)()
        self._check(_lib.hz_plan(self._h, ctypes.byref(o), float(freq), ctypes.byref(L), w))
        return L.value, [w[i] for i in range(L.value - 1)]

    # -- measurement -------------------------------------------------------
    def timing_start(self, kernels=()):
        """Time every launch of the named kernel classes (names in HZ_KERNEL) with HIP events."""
        mask = 0
        for k in kernels:
            mask |= 1 << (HZ_KERNEL[k] if isinstance(k, str) else int(k))
        self._check(_lib.hz_timing_start(self._h, mask))

    def timing_read(self, kernel):
        n = ctypes.c_int()
        ms = ctypes.c_double()
        k = HZ_KERNEL[kernel] if isinstance(kernel, str) else int(kernel)
        self._check(_lib.hz_timing_read(self._h, k, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    # -- single steps ------------------------------------------------------
    def level_shape(self, level):
        shp = self.shape
        for _ in range(level):
            shp = tuple((s - 1) // 2 + 1 for s in shp)
        return shp

    def _vecs(self, v, level):
        """Device complex128 [nrhs, *level_shape] (the library reads exactly that)."""
        t = self.torch
        v = v.to(self.device)
        if v.dtype != t.complex128 or tuple(v.shape[1:]) != self.level_shape(level) or v.shape[0] < 1:
            raise ValueError(f"expected complex128 [nrhs, {self.level_shape(level)}], got {v.dtype} {tuple(v.shape)}")
        return v.contiguous()

    def apply(self, op, level, freq, x, alpha=0.0, beta=(1.0, 0.5)):
        """y = B x (op 'B') or M x (op 'M') on a level; x: [nrhs, *level_shape]."""
        x = self._vecs(x, level)
        y = self.torch.empty_like(x)
        opi = {"B": 0, "M": 1}[op]
        self._check(_lib.hz_apply(self._h, opi, level, float(freq), float(alpha), float(beta[0]),
                                  float(beta[1]), x.shape[0], _ptr(x), _ptr(y)))
        return y

    def smooth(self, level, freq, b, u_in=None, w=0.8, beta=(1.0, 0.5)):
        b = self._vecs(b, level)
        out = self.torch.empty_like(b)
        if u_in is not None:
            u_in = self._vecs(u_in, level)
            assert u_in.shape == b.shape
        uin = _ptr(u_in) if u_in is not None else None
        self._check(_lib.hz_smooth(self._h, level, float(freq), float(beta[0]), float(beta[1]), float(w),
                                   b.shape[0], _ptr(b), uin, _ptr(out)))
        return out

    def restrict(self, level, freq, b, u, beta=(1.0, 0.5)):
        b = self._vecs(b, level)
        u = self._vecs(u, level)
        assert u.shape == b.shape
        bc = self.torch.empty((b.shape[0],) + self.level_shape(level + 1), dtype=b.dtype, device=self.device)
        self._check(_lib.hz_restrict(self._h, level, float(freq), float(beta[0]), float(beta[1]),
                                     b.shape[0], _ptr(b), _ptr(u), _ptr(bc)))
        return bc

    def prolong(self, level, e, u):
        """Returns u + P e (u is not modified)."""
        e = self._vecs(e, level + 1)
        out = self._vecs(u, level).clone()
        assert out.shape[0] == e.shape[0]
        self._check(_lib.hz_prolong(self._h, level, e.shape[0], _ptr(e), _ptr(out)))
        return out

    def precond(self, freq, b, **opt):
        b = self._vecs(b, 0)
        u = self.torch.empty_like(b)
        o, keep = make_opts(**opt)
        self._check(_lib.hz_precond(self._h, ctypes.byref(o), float(freq), b.shape[0], _ptr(b), _ptr(u)))
        del keep
        return u


def plan_grid(shape, h, m_min, m_max, freq, **opt):
    """Level count and Jacobi weights for a grid (host computation, no device)."""
    o, keep = make_opts(**opt)
    dim = len(shape)
    nz, nx = (1, shape[0]) if dim == 1 else shape
    L = ctypes.c_int()
    w = (ctypes.c_double * HZ_MAX_LEVELS)()
    rc = _lib.hz_plan_grid(dim, nz, nx, float(h), float(m_min), float(m_max), ctypes.byref(o),
                           float(freq), ctypes.byref(L), w)
    if rc != HZ_OK:
        raise HzError(rc, "hz_plan_grid failed")
    del keep
    return L.value, [w[i] for i in range(L.value - 1)]


def footprint(shape, nfreq, nrhs, **opt):
    """Device bytes a solve of this shape holds (host computation)."""
    o, keep = make_opts(**opt)
    dim = len(shape)
    nz, nx = (1, shape[0]) if dim == 1 else shape
    return int(_lib.hz_footprint(dim, nz, nx, nfreq, nrhs, ctypes.byref(o)))


def server_footprint(shape, nfreq, nrhs, **opt):
    """Device bytes the server reserves to run a request of this shape (host computation)."""
    o, keep = make_opts(**opt)
    dim = len(shape)
    nz, nx = (1, shape[0]) if dim == 1 else shape
    return int(_lib.hz_server_footprint(dim, nz, nx, nfreq, nrhs, ctypes.byref(o)))


class Server:
    """Continuous-batching solve server (see hz_server_* in include/hz.h).

    submit() queues a request and returns a ticket; wait() returns
    (u, info, times) with times = (queued s, running s, latency s). Tensors
    of a request are kept referenced until it is waited for."""

    def __init__(self, device=0, budget_bytes=0, slots=4):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        rc = _lib.hz_server_create(ctypes.byref(h), ctypes.byref(ServerOpts(device, budget_bytes, slots)))
        if rc != HZ_OK:
            raise HzError(rc, "hz_server_create failed")
        self._h = h
        self._live = {}

    def submit(self, m, h, freqs, alpha, b, **opt):
        """m: slowness (n,) or (nz, nx); b: complex128 [nfreq, nrhs, *m.shape]."""
        t = self.torch
        m = m.to(self.device, t.float64).contiguous()
        b = b.to(self.device, t.complex128).contiguous()
        freqs = [float(f) for f in freqs]
        if b.dim() != m.dim() + 2 or b.shape[0] != len(freqs) or tuple(b.shape[2:]) != tuple(m.shape):
            raise ValueError("b must be [nfreq, nrhs, *m.shape]")
        u = t.empty_like(b)
        o, keep = make_opts(**opt)
        fa = (ctypes.c_double * len(freqs))(*freqs)
        dim = m.dim()
        nz, nx = (1, m.shape[0]) if dim == 1 else (m.shape[0], m.shape[1])
        rq = Request(dim, nz, nx, float(h), ctypes.c_void_p(m.data_ptr()), len(freqs),
                     ctypes.cast(fa, ctypes.POINTER(ctypes.c_double)), float(alpha), b.shape[1],
                     ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(u.data_ptr()), ctypes.pointer(o))
        tk = ctypes.c_longlong()
        torch_stream = t.cuda.current_stream(self.device)
        torch_stream.synchronize()  # inputs written on torch's stream are complete before a slot reads them
        rc = _lib.hz_server_submit(self._h, ctypes.byref(rq), ctypes.byref(tk))
        if rc != HZ_OK:
            raise HzError(rc, "hz_server_submit failed")
        self._live[tk.value] = (m, b, u, len(freqs) * b.shape[1], keep)
        return tk.value

    def wait(self, ticket):
        m, b, u, nrec, keep = self._live.pop(ticket)
        info = (RhsInfo * nrec)()
        times = (ctypes.c_double * 3)()
        rc = _lib.hz_server_wait(self._h, ctypes.c_longlong(ticket), info, times)
        if rc < 0:
            raise HzError(rc, "request failed")
        return u, [(i.status, i.iters, i.relres) for i in info], tuple(times)

    def stats(self):
        q, r, pk = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        by = ctypes.c_size_t()
        _lib.hz_server_stats(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(pk), ctypes.byref(by))
        return {"queued": q.value, "running": r.value, "peak_running": pk.value, "bytes": by.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.hz_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Misfit:
    """J(m) of Eq. (4) as a differentiable function of the slowness tensor.

    ``Misfit(ctx, freqs, alpha, src, rec, d_obs, lam)(m)`` returns a 0-d
    float64 tensor; its backward pass returns dJ/dm from the adjoint-state
    gradient (Eq. (7)) computed by the library (forward and adjoint solves on
    the GPU). When autograd will need the gradient (``m.requires_grad`` under
    grad mode) the forward call forms it together with J, where the forward
    wavefields are at hand; otherwise (a line search, ``torch.no_grad()``)
    the forward call runs the forward solves alone. With ``lazy=True`` the
    forward call always computes J alone and the backward pass computes the
    gradient, solving the forward problems again (nothing is kept between
    the two passes). A 3D slowness tensor takes (iz, iy, ix) sources and
    receivers.
    """

    def __init__(self, ctx, freqs, alpha, src, rec, d_obs, lam, lazy=False, **opt):
        import torch
        self.ctx, self.freqs, self.alpha = ctx, list(freqs), float(alpha)
        self.src, self.rec, self.d_obs, self.lam, self.opt = src, rec, d_obs, float(lam), opt
        self.lazy = bool(lazy)
        self.last_info = None
        self.calls = {"misfit": 0, "gradient": 0}
        outer = self

        def gradient(m):
            outer.ctx.set_model(m, outer.ctx.h)
            call = outer.ctx.gradient_3d if m.dim() == 3 else outer.ctx.gradient
            outer.calls["gradient"] += 1
            J, grad, info = call(outer.freqs, outer.alpha, outer.src, outer.rec, outer.d_obs, outer.lam, **outer.opt)
            outer.last_info = info
            return J, grad

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(fctx, m):
                m = m.detach()
                if outer._need_grad and not outer.lazy:
                    J, grad = gradient(m)
                    fctx.save_for_backward(grad)
                    fctx.grad_ready = True
                else:
                    outer.ctx.set_model(m, outer.ctx.h)
                    call = outer.ctx.misfit_3d if m.dim() == 3 else outer.ctx.misfit
                    outer.calls["misfit"] += 1
                    J, _, info = call(outer.freqs, outer.alpha, outer.src, outer.rec, outer.d_obs, outer.lam,
                                      **outer.opt)
                    outer.last_info = info
                    fctx.save_for_backward(m)
                    fctx.grad_ready = False
                return torch.tensor(J, dtype=torch.float64, device=m.device)

            @staticmethod
            def backward(fctx, gJ):
                (saved,) = fctx.saved_tensors
                grad = saved if fctx.grad_ready else gradient(saved)[1]
                return gJ * grad

        self._fn = _Fn

    def __call__(self, m):
        # forward() runs with grad mode off: decide here whether autograd will ask for dJ/dm
        self._need_grad = bool(self.torch_grad_enabled() and m.requires_grad)
        return self._fn.apply(m)

    @staticmethod
    def torch_grad_enabled():
        import torch
        return torch.is_grad_enabled()


def exported_symbols():
    """Names of the C-ABI functions this binding resolves."""
    return sorted(_SIGS)
