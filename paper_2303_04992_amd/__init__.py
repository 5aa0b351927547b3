"""Python binding of libkfbi (ctypes; argument marshalling only).

Every step of the operator runs in the HIP library; PyTorch supplies device memory and
streams.  Importing this package loads ``libkfbi.so`` from the package directory and fails
loudly if it is missing (build it with ``python paper_2303_04992_amd/build.py``).

Names follow include/kfbi.h: ``Operator.eval`` is kfbi_eval (K phi = 1/2 phi - M phi read off
the double-layer interface problem in the context's trace form), ``Operator.eval_adjoint`` its
transpose, ``Operator.solve_bvp`` the Dirichlet boundary-value solve (GMRES on the
second-kind integral equation), ``Operator.interface_solve`` the grid solution of the
unified interface problem, ``Operator.probe`` the velocity at interior probes.  ``BIEEval``,
``BIESolve`` and ``ProbeEval`` wrap them as autograd functions with hand-written transposes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkfbi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libkfbi.so not found at {LIB_PATH}; build it with python paper_2303_04992_amd/build.py")

# PyTorch owns the device memory and streams the library works on: load it first so that the
# process has a single HIP runtime (libkfbi.so binds to the one already loaded).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

STOKES, NAVIER = 0, 1
FP64, MIXED_FP32 = 0, 1
DCT2, DST2, DCT3, DST3, DST1, K_GEMM_X = 0, 1, 2, 3, 4, 10
TRACE_AVERAGE, TRACE_INTERIOR = 0, 1
_TRACE = {"interior": TRACE_INTERIOR, "average": TRACE_AVERAGE}
OK, EINVAL, ENOMEM, EGEOM, ENOCONV, EDEVICE = 0, -1, -2, -3, -4, -5
_STATUS = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EGEOM: "EGEOM", ENOCONV: "ENOCONV", EDEVICE: "EDEVICE"}


class KfbiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Shape(C.Structure):
    _fields_ = [("kind", C.c_int), ("center", C.c_double * 3), ("param", C.c_double * 6), ("rot_z_deg", C.c_double)]


class Config(C.Structure):
    _fields_ = [("N", C.c_int32), ("lo", C.c_double), ("hi", C.c_double), ("pde", C.c_int), ("mu", C.c_double),
                ("lam", C.c_double), ("shape", Shape), ("precision", C.c_int), ("cg_rtol", C.c_double),
                ("cg_maxit", C.c_int32), ("inner_rtol", C.c_double), ("gmres_rtol", C.c_double),
                ("gmres_maxit", C.c_int32), ("stream", C.c_void_p), ("trace", C.c_int)]


class Info(C.Structure):
    _fields_ = [("cg_iters", C.c_int32), ("refine_rounds", C.c_int32), ("gmres_iters", C.c_int32),
                ("final_rel_residual", C.c_double), ("ms_total", C.c_double), ("ms_stage", C.c_double * 6),
                ("model_bytes", C.c_double)]

    STAGES = ("jumps", "corrections", "rhs", "cg", "backsub", "interp")

    def as_dict(self):
        return {"cg_iters": self.cg_iters, "refine_rounds": self.refine_rounds, "gmres_iters": self.gmres_iters,
                "final_rel_residual": self.final_rel_residual, "ms_total": self.ms_total,
                "ms_stage": dict(zip(self.STAGES, self.ms_stage)), "model_bytes": self.model_bytes}


VecFn = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_double), C.c_void_p)

_P = C.c_void_p
_sig = {
    "kfbi_create": (C.c_int, [C.POINTER(Config), C.POINTER(_P)]),
    "kfbi_destroy": (None, [_P]),
    "kfbi_last_error": (C.c_char_p, [_P]),
    "kfbi_create_error": (C.c_char_p, []),
    "kfbi_num_points": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "kfbi_get_points": (C.c_int, [_P, _P, _P]),
    "kfbi_sizes": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "kfbi_eval": (C.c_int, [_P, _P, _P, C.POINTER(Info)]),
    "kfbi_eval_adjoint": (C.c_int, [_P, _P, _P, C.POINTER(Info)]),
    "kfbi_eval_noalloc": (C.c_int, [_P, _P, _P, C.POINTER(Info)]),
    "kfbi_eval_batch": (C.c_int, [_P, C.c_int32, _P, _P, C.POINTER(Info)]),
    "kfbi_solve_bvp": (C.c_int, [_P, _P, VecFn, _P, _P, _P, _P, C.POINTER(Info)]),
    "kfbi_interface_solve": (C.c_int, [_P, _P, C.c_int32, _P, _P, C.POINTER(Info)]),
    "kfbi_set_probes": (C.c_int, [_P, _P, C.c_int64]),
    "kfbi_probe": (C.c_int, [_P, _P, C.c_int32, _P, C.POINTER(Info)]),
    "kfbi_probe_adjoint": (C.c_int, [_P, _P, _P, C.POINTER(Info)]),
    "kfbi_solve_adjoint": (C.c_int, [_P, _P, _P, C.POINTER(Info)]),
    "kfbi_solve_bvp_adjoint": (C.c_int, [_P, _P, _P, _P, C.POINTER(Info)]),
    "kfbi_apply_pass": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P]),
    "kfbi_time_pass": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double)]),
    "kfbi_profile_pass": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "kfbi_plan_create": (C.c_int, [C.POINTER(Config), C.POINTER(_P)]),
    "kfbi_plan_destroy": (None, [_P]),
    "kfbi_plan_get": (C.c_int64, [_P, C.c_char_p, _P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def make_config(cfg, precision=FP64, cg_rtol=0.0, cg_maxit=0, inner_rtol=0.0, gmres_rtol=0.0, gmres_maxit=0,
                stream=None, trace="average") -> Config:
    """Marshal a workload description (kfbi_inputs.Config-like object) into kfbi_config.
    trace: "average" (1/2 phi + mean of the two limits, default) or "interior" (K phi = u+)."""
    sh = Shape(int(cfg.shape.kind), (C.c_double * 3)(*cfg.shape.center), (C.c_double * 6)(*cfg.shape.param),
               float(cfg.shape.rot_z_deg))
    return Config(int(cfg.N), float(cfg.lo), float(cfg.hi), int(cfg.pde), float(cfg.mu), float(cfg.lam), sh,
                  int(precision), float(cg_rtol), int(cg_maxit), float(inner_rtol), float(gmres_rtol),
                  int(gmres_maxit), stream, _TRACE[trace])


class Plan:
    """Host-only setup (no device): geometry and sparse maps, for inspection."""

    _dtypes = {"xyz": np.float64, "normal": np.float64, "t1": np.float64, "t2": np.float64, "kappa": np.float64,
               "fam": np.int32, "line1": np.int32, "line2": np.int32, "cp_target": np.int64, "nb_ptr": np.int64,
               "nb_idx": np.int32, "fitw": np.float64, "jmap": np.float64, "jfmap": np.float64, "emap": np.float64,
               "irr_node": np.int64, "irr_ptr": np.int64, "arm_t": np.int32, "arm_o": np.int8, "arm_a": np.float64,
               "itp_idx": np.int64, "itp_w": np.float64, "side0": np.uint8, "side1": np.uint8, "side2": np.uint8,
               "sidep": np.uint8, "stab_a": np.float64, "sv_ptr": np.int64, "sv_idx": np.int32, "sv_w": np.float64}

    def __init__(self, cfg, **kw):
        c = make_config(cfg, **kw)
        h = C.c_void_p()
        st = _lib.kfbi_plan_create(C.byref(c), C.byref(h))
        if st != OK:
            raise KfbiError(st, _lib.kfbi_create_error().decode())
        self._h = h

    def get(self, name):
        n = _lib.kfbi_plan_get(self._h, name.encode(), None)
        if n < 0:
            raise KeyError(name)
        out = np.empty(n, dtype=self._dtypes[name])
        _lib.kfbi_plan_get(self._h, name.encode(), out.ctypes.data_as(C.c_void_p))
        return out

    def __del__(self, _destroy=_lib.kfbi_plan_destroy):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None


def _torch():
    import torch
    return torch


def _ptr(t):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


class Operator:
    """One geometry + grid + PDE: K phi, K^T w, the BVP solve."""

    def __init__(self, cfg, precision=FP64, cg_rtol=0.0, cg_maxit=0, inner_rtol=0.0, gmres_rtol=0.0, gmres_maxit=0,
                 device=None, trace="average"):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("kfbi needs a HIP device (torch.cuda.is_available() is False)")
        self.device = torch.device(device or "cuda:0")
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            self.stream = stream
            c = make_config(cfg, precision, cg_rtol, cg_maxit, inner_rtol, gmres_rtol, gmres_maxit,
                            C.c_void_p(stream.cuda_stream), trace)
            h = C.c_void_p()
            st = _lib.kfbi_create(C.byref(c), C.byref(h))
        if st != OK:
            raise KfbiError(st, _lib.kfbi_create_error().decode())
        self._h = h
        self.cfg = cfg
        self.trace = trace
        n = C.c_int64()
        _lib.kfbi_num_points(h, C.byref(n))
        self.n = int(n.value)
        nt, ni = C.c_int64(), C.c_int64()
        _lib.kfbi_sizes(h, C.byref(nt), C.byref(ni))
        self.n_crossings, self.n_irregular = int(nt.value), int(ni.value)
        self.last_info = None

    def __del__(self, _destroy=_lib.kfbi_destroy):
        # the destroy function is bound at definition time: module globals may already be
        # cleared when the interpreter finalises
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def _check(self, st):
        if st != OK:
            raise KfbiError(st, _lib.kfbi_last_error(self._h).decode())

    def points(self):
        xyz = np.empty((self.n, 3))
        nrm = np.empty((self.n, 3))
        self._check(_lib.kfbi_get_points(self._h, xyz.ctypes.data_as(C.c_void_p), nrm.ctypes.data_as(C.c_void_p)))
        return xyz, nrm

    def _vec(self, v):
        torch = _torch()
        v = torch.as_tensor(v, dtype=torch.float64, device=self.device).reshape(self.n, 3).contiguous()
        return v

    def eval(self, phi):
        torch = _torch()
        phi = self._vec(phi)
        out = torch.empty_like(phi)
        info = Info()
        self._check(_lib.kfbi_eval(self._h, _ptr(phi), _ptr(out), C.byref(info)))
        self.last_info = info.as_dict()
        return out

    def eval_batch(self, phis):
        """K phi[r] for a stack of densities (nrhs, n, 3) in one call (kfbi_eval_batch)."""
        torch = _torch()
        phis = torch.as_tensor(phis, dtype=torch.float64, device=self.device)
        nrhs = phis.shape[0] if phis.dim() == 3 else 1
        phis = phis.reshape(nrhs, self.n, 3).contiguous()
        out = torch.empty_like(phis)
        info = Info()
        self._check(_lib.kfbi_eval_batch(self._h, int(nrhs), _ptr(phis), _ptr(out), C.byref(info)))
        self.last_info = info.as_dict()
        return out

    def eval_noalloc(self, phi, out=None):
        """K phi through kfbi_eval_noalloc (work buffers in the library's static device scratch;
        the caller provides phi and out)."""
        torch = _torch()
        phi = self._vec(phi)
        out = torch.empty_like(phi) if out is None else out
        info = Info()
        self._check(_lib.kfbi_eval_noalloc(self._h, _ptr(phi), _ptr(out), C.byref(info)))
        self.last_info = info.as_dict()
        return out

    def eval_adjoint(self, w):
        torch = _torch()
        w = self._vec(w)
        out = torch.empty_like(w)
        info = Info()
        self._check(_lib.kfbi_eval_adjoint(self._h, _ptr(w), _ptr(out), C.byref(info)))
        self.last_info = info.as_dict()
        return out

    def solve_bvp(self, g, f=None, return_fields=True):
        """Returns (phi, u packed (3, N+1, N, N)-ish flat, p (N,N,N)) as CUDA tensors."""
        torch = _torch()
        g = self._vec(g)
        phi = torch.empty_like(g)
        N = self.cfg.N
        u = torch.empty(3 * (N + 1) * N * N, dtype=torch.float64, device=self.device) if return_fields else None
        p = torch.empty((N, N, N), dtype=torch.float64, device=self.device) if return_fields else None
        cb = VecFn(0)
        if f is not None:
            def _f(xyz, m, out, user):
                X = np.ctypeslib.as_array(xyz, shape=(m, 3))
                O = np.ctypeslib.as_array(out, shape=(m, 3))
                O[:] = f(X[:, 0], X[:, 1], X[:, 2])
            cb = VecFn(_f)
        info = Info()
        st = _lib.kfbi_solve_bvp(self._h, _ptr(g), cb, None, _ptr(phi), _ptr(u) if u is not None else None,
                                 _ptr(p) if p is not None else None, C.byref(info))
        self.last_info = info.as_dict()
        self._check(st)
        return phi, u, p

    def interface_solve(self, phi, use_force=False):
        torch = _torch()
        phi = self._vec(phi)
        N = self.cfg.N
        u = torch.empty(3 * (N + 1) * N * N, dtype=torch.float64, device=self.device)
        p = torch.empty((N, N, N), dtype=torch.float64, device=self.device)
        info = Info()
        self._check(_lib.kfbi_interface_solve(self._h, _ptr(phi), int(bool(use_force)), _ptr(u), _ptr(p),
                                              C.byref(info)))
        self.last_info = info.as_dict()
        return u, p

    def set_probes(self, xyz):
        xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
        self._check(_lib.kfbi_set_probes(self._h, xyz.ctypes.data_as(C.c_void_p), len(xyz)))
        self.nprobe = len(xyz)

    def probe(self, phi, use_force=False):
        """Velocity at the probes of the unified interface solve with density phi."""
        torch = _torch()
        phi = self._vec(phi)
        out = torch.empty((self.nprobe, 3), dtype=torch.float64, device=self.device)
        info = Info()
        self._check(_lib.kfbi_probe(self._h, _ptr(phi), int(bool(use_force)), _ptr(out), C.byref(info)))
        self.last_info = info.as_dict()
        return out

    def probe_adjoint(self, vbar):
        torch = _torch()
        vbar = torch.as_tensor(vbar, dtype=torch.float64, device=self.device).reshape(self.nprobe, 3).contiguous()
        out = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        info = Info()
        self._check(_lib.kfbi_probe_adjoint(self._h, _ptr(vbar), _ptr(out), C.byref(info)))
        self.last_info = info.as_dict()
        return out

    def solve_adjoint(self, rhs):
        """y = K^{-T} rhs (GMRES with the transposed operator)."""
        torch = _torch()
        rhs = self._vec(rhs)
        out = torch.empty_like(rhs)
        info = Info()
        st = _lib.kfbi_solve_adjoint(self._h, _ptr(rhs), _ptr(out), C.byref(info))
        self.last_info = info.as_dict()
        self._check(st)
        return out

    def solve_bvp_adjoint(self, vbar, want_g=True, want_phi=True):
        """(g_bar, phi_bar) for the cotangent vbar of the probe values of the BVP solution:
        phi_bar = P^T vbar, g_bar = K^{-T} phi_bar (kfbi_solve_bvp_adjoint)."""
        torch = _torch()
        vbar = torch.as_tensor(vbar, dtype=torch.float64, device=self.device).reshape(self.nprobe, 3).contiguous()
        gb = torch.empty((self.n, 3), dtype=torch.float64, device=self.device) if want_g else None
        pb = torch.empty((self.n, 3), dtype=torch.float64, device=self.device) if want_phi else None
        info = Info()
        st = _lib.kfbi_solve_bvp_adjoint(self._h, _ptr(vbar), _ptr(gb) if gb is not None else None,
                                         _ptr(pb) if pb is not None else None, C.byref(info))
        self.last_info = info.as_dict()
        self._check(st)
        return gb, pb

    def apply_pass(self, kind, axis, field):
        """One transform pass (kfbi_apply_pass) of an N^3 field ([x][y][z], float64) along axis,
        in the context's inner precision; returns a new float64 CUDA tensor."""
        torch = _torch()
        N = self.cfg.N
        f = torch.as_tensor(field, dtype=torch.float64, device=self.device).reshape(N, N, N).contiguous()
        out = torch.empty_like(f)
        self._check(_lib.kfbi_apply_pass(self._h, int(kind), int(axis), _ptr(f), _ptr(out)))
        return out

    def time_pass(self, kind=1, axis=1, reps=20):
        """Mean duration (ms) and algorithmic bytes of one transform-pass launch."""
        ms, by = C.c_double(), C.c_double()
        self._check(_lib.kfbi_time_pass(self._h, int(kind), int(axis), int(reps), C.byref(ms), C.byref(by)))
        return ms.value, by.value

    def profile_pass(self, kind=3, axis=1, enable=True):
        """Start (enable) or stop live event timing of one transform pass inside evaluations;
        returns (launches, total_ms, bytes_per_launch) recorded since the previous call."""
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        self._check(_lib.kfbi_profile_pass(self._h, int(kind), int(axis), int(bool(enable)), C.byref(n),
                                           C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def split_u(self, u):
        """Packed exported velocity -> (u1 (N+1,N,N), u2 (N,N+1,N), u3 (N,N,N+1))."""
        N = self.cfg.N
        s = (N + 1) * N * N
        return (u[:s].reshape(N + 1, N, N), u[s:2 * s].reshape(N, N + 1, N), u[2 * s:].reshape(N, N, N + 1))


def _autograd():
    torch = _torch()

    class BIEEval(torch.autograd.Function):
        """K phi with the hand-written transpose (kfbi_eval_adjoint) as backward."""

        @staticmethod
        def forward(ctx, phi, op):
            ctx.op = op
            return op.eval(phi.detach())

        @staticmethod
        def backward(ctx, gout):
            return ctx.op.eval_adjoint(gout.contiguous()), None

    class BIESolve(torch.autograd.Function):
        """phi = K^{-1}(g - b) by GMRES (b = volume trace of the body force f, if any);
        backward: g_bar = K^{-T} phi_bar (GMRES with the transposed operator)."""

        @staticmethod
        def forward(ctx, g, op, f=None):
            ctx.op = op
            phi, _, _ = op.solve_bvp(g.detach(), f, return_fields=False)
            return phi

        @staticmethod
        def backward(ctx, gphi):
            return ctx.op.solve_adjoint(gphi.contiguous()), None, None

    class ProbeEval(torch.autograd.Function):
        """Velocity at the interior probes of the unified interface solve with density phi."""

        @staticmethod
        def forward(ctx, phi, op, use_force=False):
            ctx.op = op
            return op.probe(phi.detach(), use_force)

        @staticmethod
        def backward(ctx, gv):
            return ctx.op.probe_adjoint(gv.contiguous()), None, None

    return BIEEval, BIESolve, ProbeEval


def __getattr__(name):
    if name in ("BIEEval", "BIESolve", "ProbeEval"):
        E, S, P = _autograd()
        globals()["BIEEval"], globals()["BIESolve"], globals()["ProbeEval"] = E, S, P
        return globals()[name]
    raise AttributeError(name)
