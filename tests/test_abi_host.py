"""Host-only checks of the C ABI (no device call): the library loads, exports
every entry point that include/bte.h declares, validates inputs, and its
quadrature helpers agree with library Gauss-Legendre rules."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import bte_inputs as bi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "bte.h")).read()
    return sorted(set(re.findall(r"^\s*(?:bte_status|const char\*)\s+(bte_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    import paper_2503_23657_amd as bte
    names = _declared()
    assert len(names) >= 15
    lib = ctypes.CDLL(bte.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(bte.EXPORTED)


def test_version_and_error_string():
    import paper_2503_23657_amd as bte
    assert bte.bte_version().startswith(b"bte-")
    with pytest.raises(bte.BTEError):
        bte.validate(bi.square_2d(8).replace(v=-np.ones(15)))
    assert "v[0]" in bte.last_error()


def _bad_cases():
    p = bi.square_2d(8, n_bands=3, n_theta=2, n_phi=1)
    yield "tau", p.replace(tau=np.array([1e-12, 0.0, 1e-11]))
    yield "C", p.replace(C=np.array([1.0, -1.0, 1.0]))
    yield "nan v", p.replace(v=np.array([1.0, np.nan, 1.0]))
    w = p.w.copy()
    w[0] *= 1.01
    yield "weights", p.replace(w=w)
    s = p.s.copy()
    s[0] *= 1.001
    yield "unit", p.replace(s=s)
    # not closed under reflection: drop the mirror of one direction
    keep = np.ones(p.M, bool)
    keep[0] = False
    w2 = p.w[keep] * (4 * math.pi / p.w[keep].sum())
    yield "reflection", p.replace(s=p.s[keep], w=w2)
    yield "empty mask", p.replace(mask=np.zeros_like(p.mask))
    yield "adiabatic only", p.replace(bc_kind=np.array([1], dtype=np.int32))
    yield "specular only", p.replace(bc_kind=np.array([2], dtype=np.int32))
    yield "bc kind", p.replace(bc_kind=np.array([3], dtype=np.int32))
    fb = p.face_bc.copy()
    fb[fb == 0] = 7
    yield "bc id range", p.replace(face_bc=fb)
    yield "dim", p.replace(dim=4)
    yield "unused axis", p.replace(n=(8, 8, 2))


@pytest.mark.parametrize("name,p", list(_bad_cases()), ids=[n for n, _ in _bad_cases()])
def test_validation_rejects(name, p):
    import paper_2503_23657_amd as bte
    with pytest.raises(bte.BTEError) as ei:
        bte.validate(p)
    assert ei.value.status == bte.BTE_ERR_INVALID


def test_validation_accepts_workloads():
    import paper_2503_23657_amd as bte
    for p in (bi.film_1d(), bi.square_2d(16), bi.finfet_3d(scale=8, n_bands=2),
              bi.random_box_2d(9, 7, seed=0), bi.random_box_3d(5, 4, 6, seed=0),
              bi.random_box_2d(9, 7, seed=0, kinds=(0, 2)), bi.finfet_3d_mixed(scale=8, n_bands=2)):
        bte.validate(p)


@pytest.mark.parametrize("n", [1, 2, 7, 32, 64])
def test_library_gl_mu_matches_numpy(n):
    import paper_2503_23657_amd as bte
    s, w = bte.quadrature_gl_mu(n)
    s2, w2 = bi.quad_gl_mu(n)
    assert np.abs(s - s2).max() < 1e-14
    assert np.abs(w - w2).max() < 1e-13
    assert abs(w.sum() - 4 * math.pi) < 1e-12


@pytest.mark.parametrize("nt,npp,ax", [(1, 1, 0), (4, 4, 0), (8, 2, 2), (4, 2, 2), (3, 5, 1)])
def test_library_octant_gl_matches_numpy(nt, npp, ax):
    import paper_2503_23657_amd as bte
    s, w = bte.quadrature_octant_gl(nt, npp, ax)
    s2, w2 = bi.quad_octant_gl(nt, npp, ax)
    assert np.abs(s - s2).max() < 1e-14
    assert np.abs(w - w2).max() < 1e-14


def test_quadrature_helper_rejects_bad_args():
    import paper_2503_23657_amd as bte
    with pytest.raises(bte.BTEError):
        bte.quadrature_octant_gl(0, 2, 0)
    with pytest.raises(bte.BTEError):
        bte.quadrature_octant_gl(2, 2, 3)


def test_calls_reject_a_null_handle():
    """Entry points that take a handle refuse NULL before any device call."""
    import paper_2503_23657_amd as bte
    n = ctypes.c_size_t(123)
    assert bte.bte_workspace_bytes(None, 0, ctypes.byref(n)) == bte.BTE_ERR_INVALID
    assert bte.bte_bind_workspace(None, None, 0) == bte.BTE_ERR_INVALID
    o = bte.make_opts()
    assert bte.bte_solve(None, None, None, None, None, None, ctypes.byref(o), None, None) == bte.BTE_ERR_INVALID
    assert bte.bte_set_tau(None, None) == bte.BTE_ERR_INVALID
    assert bte.bte_autotune(None, None, 1, None, None) == bte.BTE_ERR_INVALID
    assert bte.bte_destroy(None) == bte.BTE_OK


def test_options_struct_layout():
    """The binding's bte_opts mirrors include/bte.h field by field (two doubles,
    two ints, T_ref, two ints, the cache path)."""
    import paper_2503_23657_amd as bte
    names = [f[0] for f in bte.Opts._fields_]
    assert names == ["tol_T", "tol_q", "max_iters", "check_every", "T_ref", "use_graph", "store_angular",
                     "autotune_cache"]
    txt = open(os.path.join(ROOT, "include", "bte.h")).read()
    body = txt[txt.index("typedef struct {\n  double tol_T;"):]
    body = body[:body.index("} bte_opts;")]
    decl = re.findall(r"^\s*(?:const\s+)?\w+\*?\s+(\w+);", body, re.M)
    assert decl == names
    assert bte.Opts.T_ref.offset == 24 and ctypes.sizeof(bte.Opts) == 48
