"""FP64 CPU oracle for the phonon-BTE source-iteration solver.

TEST INFRASTRUCTURE ONLY: the reference that the HIP library is checked
against. Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import or run anything here. It shares no code with the
library (``paper_2503_23657_amd``) and does not import it.

Contents:
  * ``bte_oracle.c`` -- plain C FP64 solver in the paper's variables and order
    (see its header for the equations it follows); ``solve()`` wraps it.
  * ``unrolled.py``  -- plain PyTorch-CPU FP64 source iteration, unrolled, used
    for reverse-mode gradients through the iteration (small sizes only).
  * ``dense.py``     -- brute-force assembly of the full discrete linear system
    for tiny grids (direct solve and complex-step gradients).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bte_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_lib = None
_lock = threading.Lock()

STATUS = {0: "converged", 1: "invalid", 3: "not_converged", 4: "nonfinite"}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            lib.oracle_solve.restype = ctypes.c_int
            lib.oracle_solve.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, P, P,
                                         ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, P,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, P, P, P, P, P, ctypes.c_int]
            lib.oracle_count_bfaces.restype = ctypes.c_long
            lib.oracle_count_bfaces.argtypes = [ctypes.c_int, P, P]
            lib.oracle_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def solve(p, *, Q=None, tau=None, T_init=None, max_iters=100000, tol=1e-10, tol_q=None,
          threads=0, want_e=False, want_eb=False, order=1):
    """Run the oracle on a ``bte_inputs.Problem``. ``order`` 2 takes the
    paper's second-order face values (Green-Gauss gradients, deferred
    correction) instead of first-order upwind faces.

    Returns a dict with T (absolute, K, [ncell]), q ([ncell, dim], W/m^2),
    status, iters, eps_T, eps_q and optionally e ([B, M, ncell], absolute) and
    eb ([B, n_boundary_faces]). ``tol <= 0`` runs exactly ``max_iters`` sweeps.
    """
    lib = _load()
    n = np.ascontiguousarray(np.array(p.n, dtype=np.int32))
    h = np.ascontiguousarray(np.array(p.h, dtype=np.float64))
    mask = np.ascontiguousarray(p.mask, dtype=np.uint8)
    fbc = np.ascontiguousarray(p.face_bc, dtype=np.uint8).reshape(-1)
    bck = np.ascontiguousarray(p.bc_kind, dtype=np.int32)
    bcT = np.ascontiguousarray(p.bc_T, dtype=np.float64)
    v = np.ascontiguousarray(p.v, dtype=np.float64)
    tt = np.ascontiguousarray(p.tau if tau is None else tau, dtype=np.float64)
    C = np.ascontiguousarray(p.C, dtype=np.float64)
    s = np.ascontiguousarray(p.s, dtype=np.float64).reshape(-1)
    w = np.ascontiguousarray(p.w, dtype=np.float64)
    QQ = np.ascontiguousarray(p.Q if Q is None else Q, dtype=np.float64)
    Ti = None if T_init is None else np.ascontiguousarray(T_init, dtype=np.float64)
    ncell = p.ncell
    T = np.zeros(ncell)
    q = np.zeros(ncell * p.dim)
    nbf = int(lib.oracle_count_bfaces(p.dim, _ptr(n), _ptr(mask)))
    e = np.zeros(p.B * p.M * ncell) if want_e else None
    eb = np.zeros(p.B * max(nbf, 1)) if want_eb else None
    info = np.zeros(4)
    tq = tol if tol_q is None else tol_q
    st = lib.oracle_solve(p.dim, _ptr(n), _ptr(h), _ptr(mask), _ptr(fbc), len(bck), _ptr(bck),
                          _ptr(bcT), p.B, _ptr(v), _ptr(tt), _ptr(C), p.M, _ptr(s), _ptr(w),
                          _ptr(QQ), _ptr(Ti), float(p.T_ref), int(max_iters), float(tol),
                          float(tq), int(threads), _ptr(T), _ptr(q), _ptr(e), _ptr(eb),
                          _ptr(info), int(order))
    if st == 1:
        raise ValueError("oracle: invalid input")
    out = dict(T=T, q=q.reshape(ncell, p.dim), status=STATUS.get(st, str(st)),
               iters=int(info[0]), eps_T=float(info[1]), eps_q=float(info[2]),
               n_bfaces=int(info[3]))
    if want_e:
        out["e"] = e.reshape(p.B, p.M, ncell)
    if want_eb:
        out["eb"] = eb.reshape(p.B, max(nbf, 1))[:, :nbf]
    return out
