"""MI355X phonon-BTE source-iteration solver: Python binding of libbte_hip.so.

A thin ctypes layer over the C ABI declared in ``include/bte.h``: it marshals
arguments (host arrays as numpy, device arrays as torch tensors' data
pointers, streams as torch's current HIP stream) and does no computation of
its own. Every step of the solve runs in the library's HIP kernels; if the
library has not been built the import fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbte_hip.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python {os.path.join(_HERE, 'build.py')}`")

# torch carries its own HIP runtime; it must be loaded before the library so
# that the library binds to the same runtime (one device context, shared
# streams and allocations).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

(BTE_OK, BTE_ERR_INVALID, BTE_ERR_HIP, BTE_ERR_NOT_CONVERGED, BTE_ERR_NONFINITE, BTE_ERR_STATE,
 BTE_ERR_WORKSPACE) = range(7)
STATUS_NAMES = {0: "ok", 1: "invalid", 2: "hip", 3: "not_converged", 4: "nonfinite", 5: "state",
                6: "workspace"}
BC_ISOTHERMAL, BC_DIFFUSE, BC_SPECULAR = 0, 1, 2
PREC_FP64, PREC_FP32 = 0, 1


class Geometry(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double * 3),
                ("h_mask", ctypes.c_void_p), ("h_face_bc", ctypes.c_void_p), ("n_bc", ctypes.c_int),
                ("h_bc_kind", ctypes.c_void_p), ("h_bc_T", ctypes.c_void_p)]


class Bands(ctypes.Structure):
    _fields_ = [("n_bands", ctypes.c_int), ("h_v", ctypes.c_void_p), ("h_tau", ctypes.c_void_p),
                ("h_C", ctypes.c_void_p)]


class Quadrature(ctypes.Structure):
    _fields_ = [("n_dirs", ctypes.c_int), ("h_s", ctypes.c_void_p), ("h_w", ctypes.c_void_p)]


class Plan(ctypes.Structure):
    _fields_ = [("G", ctypes.c_int), ("R", ctypes.c_int), ("P", ctypes.c_int), ("C", ctypes.c_int),
                ("NR", ctypes.c_int)]

    def as_dict(self):
        return dict(G=self.G, R=self.R, P=self.P, C=self.C, NR=self.NR)


class Opts(ctypes.Structure):
    _fields_ = [("tol_T", ctypes.c_double), ("tol_q", ctypes.c_double), ("max_iters", ctypes.c_int),
                ("check_every", ctypes.c_int), ("T_ref", ctypes.c_double), ("use_graph", ctypes.c_int),
                ("store_angular", ctypes.c_int), ("autotune_cache", ctypes.c_char_p)]


class Report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("eps_T", ctypes.c_double), ("eps_q", ctypes.c_double),
                ("seconds", ctypes.c_double), ("status", ctypes.c_int)]

    def as_dict(self):
        return dict(iters=self.iters, eps_T=self.eps_T, eps_q=self.eps_q, seconds=self.seconds,
                    status=STATUS_NAMES.get(self.status, str(self.status)))


_P = ctypes.c_void_p
_H = ctypes.c_void_p
_S = ctypes.c_int


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


bte_version = _sig("bte_version", ctypes.c_char_p, [])
bte_last_error = _sig("bte_last_error", ctypes.c_char_p, [])
bte_validate = _sig("bte_validate", _S, [ctypes.POINTER(Geometry), ctypes.POINTER(Bands),
                                         ctypes.POINTER(Quadrature)])
bte_quadrature_gl_mu = _sig("bte_quadrature_gl_mu", _S, [ctypes.c_int, _P, _P])
bte_quadrature_octant_gl = _sig("bte_quadrature_octant_gl", _S, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                                 _P, _P])
bte_create = _sig("bte_create", _S, [ctypes.POINTER(Geometry), ctypes.POINTER(Bands),
                                     ctypes.POINTER(Quadrature), ctypes.c_int, ctypes.POINTER(_H)])
bte_batch_create = _sig("bte_batch_create", _S, [ctypes.c_int, ctypes.POINTER(Geometry),
                                                 ctypes.POINTER(Bands), ctypes.POINTER(Quadrature),
                                                 ctypes.c_int, ctypes.POINTER(_H)])
bte_workspace_bytes = _sig("bte_workspace_bytes", _S, [_H, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)])
bte_bind_workspace = _sig("bte_bind_workspace", _S, [_H, _P, ctypes.c_size_t])
bte_set_tau = _sig("bte_set_tau", _S, [_H, _P])
bte_set_order = _sig("bte_set_order", _S, [_H, ctypes.c_int])
bte_set_plan = _sig("bte_set_plan", _S, [_H, ctypes.POINTER(Plan)])
bte_get_plan = _sig("bte_get_plan", _S, [_H, ctypes.POINTER(Plan)])
bte_autotune = _sig("bte_autotune", _S, [_H, _P, ctypes.c_int, _P, ctypes.POINTER(Plan)])
bte_solve = _sig("bte_solve", _S, [_H, _P, _P, _P, _P, _P, ctypes.POINTER(Opts), _P, ctypes.POINTER(Report)])
bte_solve_noalloc = _sig("bte_solve_noalloc", _S, [_H, _P, _P, _P, _P, _P, ctypes.POINTER(Opts), _P,
                                                   ctypes.POINTER(Report)])
bte_adjoint = _sig("bte_adjoint", _S, [_H, _P, _P, _P, ctypes.POINTER(Opts), _P, ctypes.POINTER(Report)])
bte_adjoint_dscale = _sig("bte_adjoint_dscale", _S, [_H, _P])
bte_time_sweep = _sig("bte_time_sweep", _S, [_H, ctypes.c_int, _P, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)])
bte_batch_solve = _sig("bte_batch_solve", _S, [_H, _P, _P, _P, ctypes.POINTER(Opts), _P, _P])
bte_batch_adjoint = _sig("bte_batch_adjoint", _S, [_H, _P, _P, _P, ctypes.POINTER(Opts), _P, _P])
bte_destroy = _sig("bte_destroy", _S, [_H])

EXPORTED = ["bte_version", "bte_last_error", "bte_validate", "bte_quadrature_gl_mu",
            "bte_quadrature_octant_gl", "bte_create", "bte_workspace_bytes", "bte_bind_workspace",
            "bte_set_tau", "bte_set_order", "bte_set_plan", "bte_get_plan",
            "bte_autotune", "bte_solve", "bte_solve_noalloc", "bte_adjoint", "bte_adjoint_dscale", "bte_time_sweep", "bte_batch_create",
            "bte_batch_solve", "bte_batch_adjoint", "bte_destroy"]


class BTEError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def last_error() -> str:
    return bte_last_error().decode()


def _check(st, allow=()):
    if st != BTE_OK and st not in allow:
        raise BTEError(st, last_error())
    return st


def _c(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class _HostProblem:
    """Keeps the host arrays of a problem alive while the C structs point at them."""

    def __init__(self, p):
        self.mask = _c(p.mask, np.uint8)
        self.fbc = _c(p.face_bc, np.uint8).reshape(-1)
        self.bck = _c(p.bc_kind, np.int32)
        self.bcT = _c(p.bc_T, np.float64)
        self.v = _c(p.v, np.float64)
        self.tau = _c(p.tau, np.float64)
        self.C = _c(p.C, np.float64)
        self.s = _c(p.s, np.float64).reshape(-1)
        self.w = _c(p.w, np.float64)
        g = Geometry()
        g.dim = p.dim
        for d in range(3):
            g.n[d] = int(p.n[d])
            g.h[d] = float(p.h[d])
        g.h_mask = self.mask.ctypes.data
        g.h_face_bc = self.fbc.ctypes.data
        g.n_bc = int(self.bck.size)
        g.h_bc_kind = self.bck.ctypes.data
        g.h_bc_T = self.bcT.ctypes.data
        self.geom = g
        b = Bands()
        b.n_bands = int(self.v.size)
        b.h_v, b.h_tau, b.h_C = self.v.ctypes.data, self.tau.ctypes.data, self.C.ctypes.data
        self.bands = b
        q = Quadrature()
        q.n_dirs = int(self.w.size)
        q.h_s, q.h_w = self.s.ctypes.data, self.w.ctypes.data
        self.quad = q


def validate(p) -> None:
    """Host-only validation of a problem (raises BTEError)."""
    hp = _HostProblem(p)
    _check(bte_validate(ctypes.byref(hp.geom), ctypes.byref(hp.bands), ctypes.byref(hp.quad)))


def quadrature_gl_mu(n_mu: int):
    s = np.zeros(3 * n_mu)
    w = np.zeros(n_mu)
    _check(bte_quadrature_gl_mu(n_mu, s.ctypes.data, w.ctypes.data))
    return s.reshape(n_mu, 3), w


def quadrature_octant_gl(n_theta: int, n_phi: int, polar_axis: int = 0):
    M = 8 * n_theta * n_phi
    s = np.zeros(3 * M)
    w = np.zeros(M)
    _check(bte_quadrature_octant_gl(n_theta, n_phi, polar_axis, s.ctypes.data, w.ctypes.data))
    return s.reshape(M, 3), w


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_opts(tol=1e-10, tol_q=None, max_iters=100000, check_every=8, use_graph=True, store_state=False,
              T_ref=0.0, autotune_cache=None):
    """bte_opts; store_state sets store_angular (keep the angular field for the adjoint)."""
    o = Opts()
    o.tol_T = float(tol)
    o.tol_q = float(tol if tol_q is None else tol_q)
    o.max_iters = int(max_iters)
    o.check_every = int(check_every)
    o.T_ref = float(T_ref)
    o.use_graph = 1 if use_graph else 0
    o.store_angular = 1 if store_state else 0
    o.autotune_cache = None if autotune_cache is None else os.fsencode(autotune_cache)
    return o


class _Workspace:
    """bte_workspace_bytes / bte_bind_workspace for a handle owner."""

    def workspace_bytes(self, with_adjoint: bool = False) -> int:
        n = ctypes.c_size_t()
        _check(bte_workspace_bytes(self._h, 1 if with_adjoint else 0, ctypes.byref(n)))
        return int(n.value)

    def bind_workspace(self, ws) -> None:
        """Carve every device array from ws (a uint8 device tensor, kept alive
        here), or go back to the library's own memory with ws = None."""
        if ws is None:
            _check(bte_bind_workspace(self._h, None, 0))
        else:
            _check(bte_bind_workspace(self._h, ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()))
        self._ws = ws


class Solver(_Workspace):
    """One problem on the current HIP device (see bte_create).

    ``generation`` counts the solves and tau changes made through this object;
    the autograd binding uses it to tell whether the stored state is still the
    one its forward pass left."""

    def __init__(self, p, precision: str = "fp64", T_ref: Optional[float] = None, plan: Optional[dict] = None):
        self.problem = p
        self._hp = _HostProblem(p)
        self.prec = PREC_FP32 if precision == "fp32" else PREC_FP64
        self.T_ref = float(p.T_ref if T_ref is None else T_ref)
        self.generation = 0
        self._ws = None
        h = _H()
        _check(bte_create(ctypes.byref(self._hp.geom), ctypes.byref(self._hp.bands),
                          ctypes.byref(self._hp.quad), self.prec, ctypes.byref(h)))
        self._h = h
        if plan:
            self.set_plan(**plan)

    def close(self):
        if getattr(self, "_h", None):
            bte_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_plan(self, G=0, R=0, P=0, C=0, NR=0):
        pl = Plan(G, R, P, C, NR)
        _check(bte_set_plan(self._h, ctypes.byref(pl)))

    def set_order(self, order: int):
        """Face reconstruction: 1 first-order upwind, 2 the second-order face
        values by deferred correction (bte_set_order)."""
        self.generation += 1
        _check(bte_set_order(self._h, int(order)))

    def plan(self) -> dict:
        pl = Plan()
        _check(bte_get_plan(self._h, ctypes.byref(pl)))
        return pl.as_dict()

    def set_tau(self, tau):
        t = _c(tau, np.float64)
        self.generation += 1
        _check(bte_set_tau(self._h, t.ctypes.data))

    def autotune(self, Q=None, n_iters=5, stream=None) -> dict:
        pl = Plan()
        _check(bte_autotune(self._h, _ptr(Q), int(n_iters), _stream(stream), ctypes.byref(pl)))
        return pl.as_dict()

    def solve(self, Q, T_init=None, T_out=None, q_out=None, stream=None, allow_not_converged=False,
              tau=None, **opt):
        """Q: float64 device tensor [ncell]; tau: relaxation times for this solve
        (None keeps the current ones). Returns (T, q, report dict)."""
        import torch
        p = self.problem
        dev = Q.device
        T = T_out if T_out is not None else torch.empty(p.ncell, dtype=torch.float64, device=dev)
        q = q_out if q_out is not None else torch.empty(p.ncell * p.dim, dtype=torch.float64, device=dev)
        opt.setdefault("T_ref", self.T_ref)
        o = make_opts(**opt)
        rep = Report()
        t = None if tau is None else _c(tau, np.float64)
        self.generation += 1
        st = bte_solve(self._h, None if t is None else t.ctypes.data, _ptr(Q), _ptr(T_init), _ptr(T), _ptr(q),
                       ctypes.byref(o), _stream(stream), ctypes.byref(rep))
        allow = (BTE_ERR_NOT_CONVERGED,) if (allow_not_converged or o.tol_T <= 0 or o.tol_q <= 0) else ()
        _check(st, allow)
        return T, q.view(p.ncell, p.dim), rep.as_dict()

    def solve_noalloc(self, Q, T_out, q_out=None, T_init=None, stream=None, allow_not_converged=False,
                      tau=None, **opt):
        """bte_solve_noalloc: as solve, with the handle's arrays in the library's
        static device workspace; the outputs are caller tensors (nothing is
        allocated here either). Returns the report dict."""
        opt.setdefault("T_ref", self.T_ref)
        o = make_opts(**opt)
        rep = Report()
        t = None if tau is None else _c(tau, np.float64)
        self.generation += 1
        st = bte_solve_noalloc(self._h, None if t is None else t.ctypes.data, _ptr(Q), _ptr(T_init), _ptr(T_out),
                               _ptr(q_out), ctypes.byref(o), _stream(stream), ctypes.byref(rep))
        allow = (BTE_ERR_NOT_CONVERGED,) if (allow_not_converged or o.tol_T <= 0 or o.tol_q <= 0) else ()
        _check(st, allow)
        return rep.as_dict()

    def adjoint(self, dJdT, stream=None, allow_not_converged=False, **opt):
        """dJdT: float64 device tensor [ncell]. Returns (dJ/dtau [B] numpy, dJ/dQ tensor, report)."""
        import torch
        p = self.problem
        dq = torch.empty(p.ncell, dtype=torch.float64, device=dJdT.device)
        dtau = np.zeros(p.B)
        o = make_opts(**opt)
        rep = Report()
        st = bte_adjoint(self._h, _ptr(dJdT), dtau.ctypes.data, _ptr(dq), ctypes.byref(o),
                         _stream(stream), ctypes.byref(rep))
        allow = (BTE_ERR_NOT_CONVERGED,) if (allow_not_converged or o.tol_T <= 0) else ()
        _check(st, allow)
        return dtau, dq, rep.as_dict()

    def adjoint_dscale(self) -> float:
        """dJ/ds of the last adjoint for a common factor s on every cell size
        (L dJ/dL when all lengths scale with L)."""
        out = np.zeros(1)
        _check(bte_adjoint_dscale(self._h, out.ctypes.data))
        return float(out[0])

    def sweep_kernel_name(self) -> str:
        """Name of the forward sweep kernel the current plan launches (as a
        profiler reports it), for matching counter summaries."""
        pl = self.plan()
        t = "float" if self.prec == PREC_FP32 else "double"
        if self.problem.dim == 3 and pl["NR"] >= 1:
            return f"sweep2d_kernel<{t}, 1, {pl['NR']}, {pl['P']}, 1, 0, true>"
        if self.problem.dim == 3:
            return f"sweep_kernel<{t}, {pl['G']}, 1, 0, true>"
        return f"sweep2d_kernel<{t}, {pl['G']}, {pl['NR']}, {pl['P']}, 1, 0>"

    def time_sweep(self, n_launches=20, stream=None):
        ms = ctypes.c_double()
        upd = ctypes.c_double()
        _check(bte_time_sweep(self._h, int(n_launches), _stream(stream), ctypes.byref(ms), ctypes.byref(upd)))
        return ms.value, upd.value


class BatchSolver(_Workspace):
    """Many problems of one dimension, band table and quadrature (bte_batch_create)."""

    def __init__(self, problems: Sequence, precision: str = "fp32", T_ref: float = 300.0,
                 plan: Optional[dict] = None):
        self.problems = list(problems)
        self._hps = [_HostProblem(p) for p in self.problems]
        geoms = (Geometry * len(self._hps))(*[hp.geom for hp in self._hps])
        self._geoms = geoms
        self.prec = PREC_FP32 if precision == "fp32" else PREC_FP64
        self.T_ref = float(T_ref)
        self._ws = None
        h = _H()
        _check(bte_batch_create(len(self._hps), geoms, ctypes.byref(self._hps[0].bands),
                                ctypes.byref(self._hps[0].quad), self.prec, ctypes.byref(h)))
        self._h = h
        if plan:
            pl = Plan(plan.get("G", 0), plan.get("R", 0), plan.get("P", 0), plan.get("C", 0), plan.get("NR", 0))
            _check(bte_set_plan(self._h, ctypes.byref(pl)))

    def close(self):
        if getattr(self, "_h", None):
            bte_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def plan(self) -> dict:
        pl = Plan()
        _check(bte_get_plan(self._h, ctypes.byref(pl)))
        return pl.as_dict()

    def autotune(self, n_iters=5, stream=None) -> dict:
        """bte_autotune on the whole batch (zero source in the timing runs)."""
        pl = Plan()
        _check(bte_autotune(self._h, None, int(n_iters), _stream(stream), ctypes.byref(pl)))
        return pl.as_dict()

    def solve(self, Qs, stream=None, **opt):
        import torch
        n = len(self.problems)
        Ts = [torch.empty(p.ncell, dtype=torch.float64, device=Qs[0].device) for p in self.problems]
        qs = [torch.empty(p.ncell * p.dim, dtype=torch.float64, device=Qs[0].device) for p in self.problems]
        aQ = (ctypes.c_void_p * n)(*[q.data_ptr() for q in Qs])
        aT = (ctypes.c_void_p * n)(*[t.data_ptr() for t in Ts])
        aq = (ctypes.c_void_p * n)(*[t.data_ptr() for t in qs])
        reps = (Report * n)()
        opt.setdefault("T_ref", self.T_ref)
        o = make_opts(**opt)
        st = bte_batch_solve(self._h, aQ, aT, aq, ctypes.byref(o), _stream(stream), reps)
        _check(st, (BTE_ERR_NOT_CONVERGED,))
        return Ts, [q.view(p.ncell, p.dim) for q, p in zip(qs, self.problems)], [r.as_dict() for r in reps]

    def adjoint(self, dJdTs, stream=None, **opt):
        import torch
        n = len(self.problems)
        B = self.problems[0].B
        dqs = [torch.empty(p.ncell, dtype=torch.float64, device=dJdTs[0].device) for p in self.problems]
        dtau = np.zeros(n * B)
        ag = (ctypes.c_void_p * n)(*[g.data_ptr() for g in dJdTs])
        aq = (ctypes.c_void_p * n)(*[t.data_ptr() for t in dqs])
        reps = (Report * n)()
        o = make_opts(**opt)
        st = bte_batch_adjoint(self._h, ag, dtau.ctypes.data, aq, ctypes.byref(o), _stream(stream), reps)
        _check(st, (BTE_ERR_NOT_CONVERGED,))
        return dtau.reshape(n, B), dqs, [r.as_dict() for r in reps]

    def adjoint_dscale(self) -> np.ndarray:
        """dJ/ds of the last batched adjoint, per instance (common factor s on
        every cell size of that instance)."""
        out = np.zeros(len(self.problems))
        _check(bte_adjoint_dscale(self._h, out.ctypes.data))
        return out


from .autograd import BTESolve  # noqa: E402,F401
