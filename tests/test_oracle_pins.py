"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms,
limits, invariants, symmetries, or an independent brute-force assembly of the
discrete equations. Together they are meant to catch a dropped term, a wrong
sign or index, or a transposed operand anywhere in the oracle.
"""
import math

import numpy as np
import pytest

import bte_inputs as bi
import oracle
from oracle import dense

FOUR_PI = 4.0 * math.pi


# ---------------------------------------------------------------- P1 quadrature
@pytest.mark.parametrize("n_mu", [2, 8, 32])
def test_quadrature_gl_mu_moments(n_mu):
    s, w = bi.quad_gl_mu(n_mu)
    assert abs(w.sum() - FOUR_PI) < 1e-13
    assert abs((w * s[:, 0]).sum()) < 1e-13
    assert abs((w * s[:, 0] ** 2).sum() - FOUR_PI / 3) < 1e-13
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)
    # closed under mu -> -mu
    assert np.allclose(np.sort(s[:, 0]), np.sort(-s[:, 0]), atol=1e-15)


@pytest.mark.parametrize("nt,nph,axis", [(4, 4, 0), (8, 2, 2), (4, 2, 2), (2, 1, 2)])
def test_quadrature_octant_moments(nt, nph, axis):
    s, w = bi.quad_octant_gl(nt, nph, axis)
    assert s.shape == (8 * nt * nph, 3)
    assert abs(w.sum() - FOUR_PI) < 1e-12
    assert np.all(w > 0)
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-14)
    assert np.abs((w[:, None] * s).sum(0)).max() < 1e-12
    second = (w[:, None, None] * s[:, :, None] * s[:, None, :]).sum(0)
    off = second - np.diag(np.diag(second))
    assert np.abs(off).max() < 1e-12
    # the product rule's second moments approach 4 pi / 3 as the rule refines
    tol = {2: 0.2, 4: 2e-2, 8: 2e-2}[nt]
    assert np.abs(np.diag(second) - FOUR_PI / 3).max() < tol * FOUR_PI / 3
    # closed under each axis reflection
    for d in range(3):
        r = s.copy()
        r[:, d] *= -1
        for a in range(s.shape[0]):
            k = np.argmin(np.linalg.norm(s - r[a], axis=1))
            assert np.linalg.norm(s[k] - r[a]) < 1e-14 and abs(w[k] - w[a]) < 1e-15


# ------------------------------------------------------ P2 single-sweep closed form
def test_single_sweep_geometric_series():
    """One sweep from a uniform T0 with a hot left wall: for mu > 0 the energy
    relaxes as e_i - e0 = (e_wall - e0) r^(i+1), r = alpha/(1/tau + alpha),
    alpha = v mu / h; directions with mu < 0 see the right wall at T0 and stay
    at e0 exactly."""
    p = bi.film_1d(n_cells=40, L=20e-9, Kn=0.5, T_h=301.0, T_c=300.0, n_mu=8)
    r = oracle.solve(p, max_iters=1, tol=0.0, want_e=True)
    e = r["e"][0]
    C, v, tau, h = p.C[0], p.v[0], p.tau[0], p.h[0]
    e0 = C * 300.0 / FOUR_PI
    de_w = C * 1.0 / FOUR_PI
    i = np.arange(p.ncell)
    for a in range(p.M):
        mu = p.s[a, 0]
        if mu > 0:
            alpha = v * mu / h
            rr = alpha / (1.0 / tau + alpha)
            expect = e0 + de_w * rr ** (i + 1)
        else:
            expect = np.full(p.ncell, e0)
        assert np.abs(e[a] - expect).max() <= 1e-13 * e0
    # and T after one sweep is the weighted sum of those closed forms
    Texp = np.zeros(p.ncell)
    for a in range(p.M):
        mu = p.s[a, 0]
        rr = (v * mu / h) / (1.0 / tau + v * mu / h) if mu > 0 else 0.0
        Texp += p.w[a] * (300.0 + (rr ** (i + 1) if mu > 0 else 0.0))
    Texp /= FOUR_PI
    assert np.abs(r["T"] - Texp).max() < 1e-12


def test_single_sweep_constant_source():
    """Constant source, both walls at T0, one sweep: for mu > 0,
    e_i - e0 = Qs tau (1 - r^(i+1)) with Qs = Q/(4 pi) (gray band)."""
    n = 30
    p = bi.film_1d(n_cells=n, L=15e-9, Kn=0.3, T_h=300.0, T_c=300.0, n_mu=4,
                   Q=np.full(n, 3e18))
    r = oracle.solve(p, max_iters=1, tol=0.0, want_e=True)
    C, v, tau, h = p.C[0], p.v[0], p.tau[0], p.h[0]
    Qs = 3e18 / FOUR_PI
    i = np.arange(n)
    e0 = C * 300.0 / FOUR_PI
    for a in range(p.M):
        mu = p.s[a, 0]
        alpha = v * abs(mu) / h
        rr = alpha / (1.0 / tau + alpha)
        k = i if mu > 0 else (n - 1 - i)
        expect = e0 + Qs * tau * (1.0 - rr ** (k + 1))
        assert np.abs(r["e"][0, a] - expect).max() <= 1e-12 * abs(Qs * tau)


# ------------------------------------------------------------- P3 brute force
@pytest.mark.parametrize("seed,kinds", [(0, (0, 1)), (1, (0, 0)), (2, (0, 1))])
def test_fixed_point_matches_dense_2d(seed, kinds):
    p = bi.random_box_2d(5, 4, seed=seed, n_bands=3, n_theta=1, n_phi=1, kinds=kinds)
    Td = dense.solve_dense(p)
    r = oracle.solve(p, tol=0.0, max_iters=6000)
    act = p.mask > 0
    scale = np.abs(Td[act] - p.T_ref).max()
    assert np.abs(r["T"][act] - Td[act]).max() < 1e-11 * scale


def test_fixed_point_matches_dense_3d():
    p = bi.random_box_3d(4, 3, 5, seed=5, n_bands=2, n_theta=1, n_phi=1)
    Td = dense.solve_dense(p)
    r = oracle.solve(p, tol=0.0, max_iters=6000)
    act = p.mask > 0
    scale = np.abs(Td[act] - p.T_ref).max()
    assert scale > 1e-6
    assert np.abs(r["T"][act] - Td[act]).max() < 1e-10 * scale


def test_fixed_point_matches_dense_1d_nongray():
    base = bi.film_1d(n_cells=12, L=12e-9, n_mu=6, T_h=302.0, T_c=299.0)
    v, tau, C = bi.band_table_synthetic(4)
    p = base.replace(v=v, tau=tau * 0.01, C=C, Q=np.linspace(0, 1e18, 12))
    Td = dense.solve_dense(p)
    r = oracle.solve(p, tol=0.0, max_iters=3000)
    assert np.abs(r["T"] - Td).max() < 1e-11 * np.abs(Td - 300).max()


# --------------------------------------------------------------- P4 ballistic
def test_ballistic_limit():
    p = bi.film_1d(n_cells=50, Kn=1e6, n_mu=32, T_h=301.0, T_c=299.0)
    r = oracle.solve(p, tol=1e-13, max_iters=200)
    assert np.abs(r["T"] - 300.0).max() < 1e-5
    mu = p.s[:, 0]
    half = float((p.w * np.where(mu > 0, mu, 0.0)).sum())
    q_ball = p.C[0] * p.v[0] * 2.0 * half / FOUR_PI
    assert np.abs(r["q"][:, 0] / q_ball - 1.0).max() < 1e-5


# --------------------------------------------------------------- P5 diffusive
def test_diffusive_interior_is_linear_fourier():
    """Gray film at Kn = 0.01: e_a = C/(4 pi) (T - v tau mu_a T') with T linear
    solves the upwind equations exactly, so the converged interior is linear in
    x and carries q = -(C v^2 tau sum w mu^2 /(4 pi)) dT/dx."""
    n, L = 400, 100e-9
    p = bi.film_1d(n_cells=n, L=L, Kn=0.01, n_mu=16, T_h=301.0, T_c=299.0)
    x = (np.arange(n) + 0.5) / n
    r = oracle.solve(p, T_init=301.0 - 2.0 * x, tol=1e-14, tol_q=1e-14, max_iters=200000)
    T = r["T"]
    lo, hi = n // 4, 3 * n // 4
    d2 = T[lo + 1:hi + 1] - 2 * T[lo:hi] + T[lo - 1:hi - 1]
    slope = (T[hi] - T[lo]) / ((hi - lo) * p.h[0])
    assert np.abs(d2).max() < 1e-9 * abs(slope * p.h[0])
    k = p.C[0] * p.v[0] ** 2 * p.tau[0] * float((p.w * p.s[:, 0] ** 2).sum()) / FOUR_PI
    q = r["q"][lo:hi, 0]
    assert np.abs(q / (-k * slope) - 1.0).max() < 1e-8


# ------------------------------------------------------ P7 energy conservation
def _face_flux_divergence(p, r):
    """Discrete divergence of the band/direction-summed upwind face fluxes of the
    oracle's final angular field, per active cell (W/m^3)."""
    e = r["e"]
    eb = r.get("eb")
    n0, n1, n2 = p.n
    act = np.flatnonzero(p.mask)
    # boundary faces in the oracle's order: active cells ascending, faces ascending
    slot = {}
    for c in act:
        for f in range(2 * p.dim):
            if _nb(p, c, f) < 0:
                slot[(c, f)] = len(slot)
    div = np.zeros(p.ncell)
    for c in act:
        tot = 0.0
        for f in range(2 * p.dim):
            d = f // 2
            sn = p.s[:, d] if f % 2 else -p.s[:, d]
            nb = _nb(p, c, f)
            flux = 0.0
            for b in range(p.B):
                if nb >= 0:
                    eface = np.where(sn > 0, e[b, :, c], e[b, :, nb])
                elif p.bc_kind[p.face_bc[c, f]] == 2:
                    # specular: incoming along s carries the outgoing e along its mirror
                    eface = np.where(sn > 0, e[b, :, c], e[b, _mirror_index(p, d), c])
                else:
                    eface = np.where(sn > 0, e[b, :, c], eb[b, slot[(c, f)]])
                flux += p.v[b] * float((p.w * sn * eface).sum())
            tot += flux / p.h[d]
        div[c] = tot
    return div


def _mirror_index(p, d):
    """mir[a] = index of the direction s_a with its axis-d component negated,
    found by a nearest-vector search."""
    r = p.s.copy()
    r[:, d] *= -1
    mir = np.array([int(np.argmin(np.linalg.norm(p.s - r[a], axis=1))) for a in range(p.M)])
    assert np.abs(p.s[mir] - r).max() < 1e-14
    return mir


def _nb(p, c, f):
    n0, n1, n2 = p.n
    idx = [c % n0, (c // n0) % n1, c // (n0 * n1)]
    d = f // 2
    idx[d] += 1 if f % 2 else -1
    if idx[d] < 0 or idx[d] >= p.n[d]:
        return -1
    nb = idx[0] + n0 * (idx[1] + n1 * idx[2])
    return nb if p.mask[nb] else -1


def test_energy_balance_per_cell_with_diffuse_walls():
    """At the fixed point, the discrete divergence of the total heat flux equals
    the heat source in every cell (summing the per-ordinate balances over bands
    and directions, the scattering terms cancel by the T_L definition and the
    source shares sum to Q), and a diffuse wall carries no net flux."""
    p = bi.random_box_2d(6, 5, seed=3, n_bands=3, n_theta=2, n_phi=1, kinds=(0, 1))
    r = oracle.solve(p, tol=0.0, max_iters=4000, want_e=True, want_eb=True)
    div = _face_flux_divergence(p, r)
    act = p.mask > 0
    Qmax = np.abs(p.Q).max()
    assert np.abs(div[act] - p.Q[act]).max() < 1e-9 * Qmax
    # net flux through the diffuse faces vanishes face by face
    e, eb = r["e"], r["eb"]
    k = 0
    for c in np.flatnonzero(p.mask):
        for f in range(4):
            if _nb(p, c, f) >= 0:
                continue
            if p.bc_kind[p.face_bc[c, f]] == 1:
                d = f // 2
                sn = p.s[:, d] if f % 2 else -p.s[:, d]
                net = sum(p.v[b] * float((p.w * sn * np.where(sn > 0, e[b, :, c], eb[b, k])).sum())
                          for b in range(p.B))
                out = sum(p.v[b] * float((p.w * np.maximum(sn, 0) * e[b, :, c]).sum())
                          for b in range(p.B))
                assert abs(net) < 1e-10 * abs(out) + 1e-20
            k += 1


def test_1d_face_flux_uniform_without_source():
    p = bi.film_1d(n_cells=60, L=30e-9, Kn=1.0, n_mu=16)
    r = oracle.solve(p, tol=1e-14, max_iters=2000, want_e=True, want_eb=True)
    div = _face_flux_divergence(p, r)
    q_scale = np.abs(r["q"]).max()
    assert np.abs(div).max() * p.h[0] < 1e-10 * q_scale


def test_global_energy_balance_3d():
    p = bi.finfet_3d(scale=16, n_bands=2, n_theta=1, n_phi=1)
    r = oracle.solve(p, tol=0.0, max_iters=3000, want_e=True, want_eb=True)
    div = _face_flux_divergence(p, r)
    vol = p.h[0] * p.h[1] * p.h[2]
    assert abs(div.sum() * vol - p.Q.sum() * vol) < 1e-9 * p.Q.sum() * vol


# ------------------------------------------------------------ P8 symmetry
def test_film_antisymmetry():
    p = bi.film_1d()
    r = oracle.solve(p, tol=1e-13)
    dT = r["T"] - 300.0
    assert np.abs(dT + dT[::-1]).max() < 1e-12 * np.abs(dT).max()


def test_square_d4_symmetry():
    p = bi.square_2d(16, L=0.2e-6, n_bands=3, n_theta=2, n_phi=2, centered=True)
    r = oracle.solve(p, tol=1e-13, max_iters=5000)
    T = r["T"].reshape(16, 16) - 300.0
    sc = np.abs(T).max()
    for U in (T[:, ::-1], T[::-1, :], T.T, T[::-1, ::-1].T):
        assert np.abs(T - U).max() < 1e-12 * sc


# ---------------------------------------------- P12 equilibrium and linearity
def test_equilibrium_is_exact():
    p = bi.random_box_2d(6, 5, seed=4, n_bands=3, n_theta=2, n_phi=1, kinds=(0, 1),
                         T_walls=(307.0, 307.0), Q0=0.0)
    r = oracle.solve(p, T_init=np.full(p.ncell, 300.0), tol=0.0, max_iters=3000)
    act = p.mask > 0
    assert np.abs(r["T"][act] - 307.0).max() < 1e-10


def test_linearity_and_superposition():
    p = bi.square_2d(12, L=0.1e-6, n_bands=3, n_theta=2, n_phi=1)
    Q1 = p.Q
    Q2 = np.roll(p.Q, 17)
    r1 = oracle.solve(p, Q=Q1, tol=1e-14, max_iters=3000)["T"] - 300
    r2 = oracle.solve(p, Q=Q2, tol=1e-14, max_iters=3000)["T"] - 300
    r3 = oracle.solve(p, Q=2.5 * Q1 - Q2, tol=1e-14, max_iters=3000)["T"] - 300
    sc = np.abs(r3).max()
    assert np.abs(r3 - (2.5 * r1 - r2)).max() < 1e-11 * sc


def test_thread_count_does_not_change_result():
    p = bi.square_2d(16, L=0.3e-6, n_bands=3, n_theta=2, n_phi=1)
    a = oracle.solve(p, tol=0.0, max_iters=7, threads=1)
    b = oracle.solve(p, tol=0.0, max_iters=7, threads=4)
    assert np.array_equal(a["T"], b["T"]) and np.array_equal(a["q"], b["q"])


# ------------------------------------------------------ P13 specular walls
def _wall_box(dim, n, rule, mask, Q, n_bands=3, seed_quad=None):
    """Box problem with bc 0 isothermal at 305 K, bc 1 diffuse, bc 2 specular
    (Eq. 7); cell size 2 nm."""
    v, tau, C = bi.band_table_synthetic(n_bands)
    if dim == 1:
        s, w = bi.quad_gl_mu(8)
    elif dim == 2:
        s, w = bi.quad_octant_gl(2, 1, polar_axis=2)
    else:
        s, w = bi.quad_octant_gl(1, 1, polar_axis=0)
    fbc = bi.face_bc_from_mask(n, dim, mask, rule)
    return bi.Problem("wall_box", dim, tuple(n), (2e-9, 2e-9, 2e-9), mask, fbc,
                      np.array([bi.BC_ISOTHERMAL, bi.BC_DIFFUSE, bi.BC_SPECULAR], dtype=np.int32),
                      np.array([305.0, 300.0, 300.0]), v, tau, C, s, w, Q * mask, 300.0)


def _mirror_pair(dim, n, d, b, seed):
    """Problem A: a box whose -b edge is isothermal, whose +d edge is a specular
    wall and whose other boundary faces (holes included) are diffuse. Problem B:
    A and its mirror image across the +d edge, side by side, with no specular
    face at all. By symmetry, B's fixed point restricted to A's half solves A's
    discrete equations, with the mirror plane in the role of A's specular wall
    (method of images)."""
    rng = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0])
    m = np.ones(shape, dtype=np.uint8)
    if dim >= 2:
        hole = [int(rng.integers(1, n[a] - 1)) if n[a] > 2 else 0 for a in range(3)]
        m[hole[2], hole[1], hole[0]] = 0
    Q = 1e18 * rng.uniform(0.0, 1.0, size=shape)
    ax = 2 - d
    mB = np.concatenate([m, np.flip(m, ax)], axis=ax)
    QB = np.concatenate([Q, np.flip(Q, ax)], axis=ax)
    nB = list(n)
    nB[d] *= 2

    def rule_a(i, j, k, f):
        ijk = (i, j, k)
        if f == 2 * b and ijk[b] == 0:
            return 0
        if f == 2 * d + 1 and ijk[d] == n[d] - 1:
            return 2
        return 1

    def rule_b(i, j, k, f):
        ijk = (i, j, k)
        if f == 2 * b and ijk[b] == 0:
            return 0
        if b == d and f == 2 * b + 1 and ijk[b] == nB[b] - 1:
            return 0
        return 1

    pa = _wall_box(dim, n, rule_a, m.reshape(-1), Q.reshape(-1))
    pb = _wall_box(dim, nB, rule_b, mB.reshape(-1), QB.reshape(-1))
    return pa, pb, ax


@pytest.mark.parametrize("dim,n,d,b", [(1, (10, 1, 1), 0, 0), (2, (6, 5, 1), 0, 1),
                                       (2, (5, 6, 1), 1, 0), (3, (4, 3, 3), 2, 0)])
def test_specular_wall_is_a_mirror_plane(dim, n, d, b):
    pa, pb, ax = _mirror_pair(dim, n, d, b, seed=11 + d)
    assert np.all(pb.face_bc[pb.face_bc != bi.NO_BC] != 2)
    ra = oracle.solve(pa, tol=0.0, max_iters=6000)
    rb = oracle.solve(pb, tol=0.0, max_iters=6000)
    shape = (n[2], n[1], n[0])
    Ta = ra["T"].reshape(shape)
    Tb = np.take(rb["T"].reshape(pb.n[2], pb.n[1], pb.n[0]), np.arange(n[d]), axis=ax)
    act = pa.mask.reshape(shape) > 0
    scale = np.abs(Ta[act] - 300.0).max()
    assert scale > 1e-3
    assert np.abs(Ta[act] - Tb[act]).max() < 1e-9 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_specular_fixed_point_matches_dense(dim):
    if dim == 2:
        p = bi.random_box_2d(5, 4, seed=7, n_bands=3, n_theta=1, n_phi=1, kinds=(0, 2))
    else:
        p = bi.random_box_3d(3, 3, 4, seed=8, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 2))
    Td = dense.solve_dense(p)
    r = oracle.solve(p, tol=0.0, max_iters=6000)
    act = p.mask > 0
    scale = np.abs(Td[act] - p.T_ref).max()
    assert scale > 1e-6
    assert np.abs(r["T"][act] - Td[act]).max() < 1e-10 * scale


def test_energy_balance_per_cell_with_specular_walls():
    """With the incoming face value of a specular face taken as the outgoing e
    along the mirror direction, the fixed point balances energy in every cell,
    and the heat generated leaves through the isothermal faces only."""
    p = bi.random_box_2d(6, 5, seed=9, n_bands=3, n_theta=2, n_phi=1, kinds=(0, 2))
    r = oracle.solve(p, tol=0.0, max_iters=6000, want_e=True, want_eb=True)
    div = _face_flux_divergence(p, r)
    act = p.mask > 0
    Qmax = np.abs(p.Q).max()
    assert np.abs(div[act] - p.Q[act]).max() < 1e-9 * Qmax


def test_specular_side_walls_reduce_to_the_film():
    """A 2D strip with isothermal -x / +x walls, specular -y / +y walls and a
    source that varies in x only has the 1D film's solution (same bands and
    directions, only s_x transporting) in every row: the mirror directions carry
    the same s_x, so the y fluxes cancel at the walls."""
    nx, ny = 12, 3
    v, tau, C = bi.band_table_synthetic(3)
    s, w = bi.quad_octant_gl(2, 2, polar_axis=2)
    qx = 1e18 * np.linspace(0.2, 1.0, nx)
    m2 = np.ones(nx * ny, dtype=np.uint8)
    fbc2 = bi.face_bc_from_mask((nx, ny, 1), 2, m2, lambda i, j, k, f: {0: 0, 1: 1}.get(f, 2))
    p2 = bi.Problem("strip", 2, (nx, ny, 1), (2e-9, 2e-9, 2e-9), m2, fbc2,
                    np.array([0, 0, 2], dtype=np.int32), np.array([305.0, 300.0, 300.0]),
                    v, tau, C, s, w, np.tile(qx, ny), 300.0)
    m1 = np.ones(nx, dtype=np.uint8)
    fbc1 = bi.face_bc_from_mask((nx, 1, 1), 1, m1, lambda i, j, k, f: f)
    p1 = bi.Problem("film", 1, (nx, 1, 1), (2e-9, 2e-9, 2e-9), m1, fbc1,
                    np.array([0, 0], dtype=np.int32), np.array([305.0, 300.0]),
                    v, tau, C, s, w, qx, 300.0)
    r2 = oracle.solve(p2, tol=0.0, max_iters=6000)
    r1 = oracle.solve(p1, tol=0.0, max_iters=6000)
    T2 = r2["T"].reshape(ny, nx)
    scale = np.abs(r1["T"] - 300.0).max()
    for j in range(ny):
        assert np.abs(T2[j] - r1["T"]).max() < 1e-10 * scale


def test_specular_needs_mirror_directions():
    p = bi.random_box_2d(5, 4, seed=7, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 2))
    a = 0.1
    rot = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    with pytest.raises(ValueError):
        oracle.solve(p.replace(s=p.s @ rot.T), tol=0.0, max_iters=2)


# ------------------------------------------------ P14 stored oracle values
def test_film_matches_stored_values():
    """The oracle's converged film profile against the values stored by
    tests/golden/make_golden.py: a change to the oracle's arithmetic shows up
    here and has to be justified by the passage it follows."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "film_1d_kn1.txt")
    stored = np.loadtxt(path, comments="#")
    r = oracle.solve(bi.film_1d(), tol=1e-12, max_iters=100000)
    assert stored.shape == r["T"].shape
    assert np.abs(r["T"] - stored).max() < 1e-12
    # the profile is antisymmetric about 300 K and has temperature jumps at the walls
    assert abs(stored[0] - 301.0) > 0.1 and abs(stored[-1] - 299.0) > 0.1


# ------------------------------------- P15 semi-analytic gray film (Kn = 1)
def _gray_slab_theta(tau0, n):
    """Nondimensional temperature theta = (T - T_c)/(T_h - T_c) of a gray slab of
    optical thickness tau0 between black walls, in radiative (here: phonon)
    equilibrium: theta(t) = E2(t)/2 + (1/2) int_0^tau0 theta(t') E1(|t - t'|) dt',
    the continuous limit of the film problem. Nystrom with piecewise-constant
    theta and the E1 kernel integrated exactly over each cell (E2 differences)."""
    from scipy.special import expn
    edges = np.linspace(0.0, tau0, n + 1)
    a, b = edges[:-1], edges[1:]
    tc = 0.5 * (a + b)
    t = tc[:, None]
    e2 = lambda x: expn(2, np.maximum(x, 0.0))  # noqa: E731
    W = np.where(b[None, :] <= t, e2(t - b[None, :]) - e2(t - a[None, :]),
                 np.where(a[None, :] >= t, e2(a[None, :] - t) - e2(b[None, :] - t),
                          2.0 - e2(t - a[None, :]) - e2(b[None, :] - t)))
    theta = np.linalg.solve(np.eye(n) - 0.5 * W, 0.5 * e2(tc))
    return tc / tau0, theta


def test_film_matches_gray_slab_integral_equation():
    """Results, "1D cross-plane phonon transport": the Kn = 1 gray film against
    the semi-analytic solution of the slab's integral equation. The first-order
    upwind oracle agrees to 1e-3 of the imposed difference at 200 cells and 32
    directions, and its RMS error falls under spatial refinement."""
    xs, th = _gray_slab_theta(1.0, 4000)
    err = {}
    for n, n_mu in ((200, 32), (200, 64), (400, 64)):
        p = bi.film_1d(n_cells=n, Kn=1.0, n_mu=n_mu)
        r = oracle.solve(p, tol=1e-13, max_iters=100000)
        x = (np.arange(n) + 0.5) / n
        d = (r["T"] - 299.0) / 2.0 - np.interp(x, xs, th)
        err[(n, n_mu)] = (np.abs(d).max(), np.sqrt(np.mean(d * d)))
    assert err[(200, 32)][0] < 1e-3
    assert err[(400, 64)][1] < 0.6 * err[(200, 64)][1]


# ------------------------------------------ P16 heat flux along y and z (Eq. 4)
def _film_along(axis_perm, n_cells, v, tau, C, s, w, Qline, T_lo=305.0, T_hi=300.0):
    """1D film whose transport axis carries the component axis_perm[0] of the
    given directions: s' = s[:, axis_perm], same weights, isothermal walls."""
    m1 = np.ones(n_cells, dtype=np.uint8)
    fbc1 = bi.face_bc_from_mask((n_cells, 1, 1), 1, m1, lambda i, j, k, f: f)
    return bi.Problem("film", 1, (n_cells, 1, 1), (2e-9, 2e-9, 2e-9), m1, fbc1,
                      np.array([0, 0], dtype=np.int32), np.array([T_lo, T_hi]),
                      v, tau, C, np.ascontiguousarray(s[:, list(axis_perm)]), w, Qline, 300.0)


def test_flux_along_y_matches_film():
    """Methods, "Phonon BTE" (Eq. 4): a 2D strip with isothermal -y / +y walls,
    specular -x / +x walls and a source varying in y only carries the 1D film's
    solution along y in every column: T equal, q_y equal to the film's q_x
    (the film transports the y components of the same directions) and q_x zero,
    since each direction and its x mirror carry the same energy."""
    nx, ny = 3, 12
    v, tau, C = bi.band_table_synthetic(3)
    s, w = bi.quad_octant_gl(2, 2, polar_axis=2)
    qy = 1e18 * np.linspace(0.2, 1.0, ny)
    m2 = np.ones(nx * ny, dtype=np.uint8)
    fbc2 = bi.face_bc_from_mask((nx, ny, 1), 2, m2, lambda i, j, k, f: {2: 0, 3: 1}.get(f, 2))
    p2 = bi.Problem("strip_y", 2, (nx, ny, 1), (2e-9, 2e-9, 2e-9), m2, fbc2,
                    np.array([0, 0, 2], dtype=np.int32), np.array([305.0, 300.0, 300.0]),
                    v, tau, C, s, w, np.repeat(qy, nx), 300.0)
    p1 = _film_along((1, 0, 2), ny, v, tau, C, s, w, qy)
    r2 = oracle.solve(p2, tol=0.0, max_iters=6000)
    r1 = oracle.solve(p1, tol=0.0, max_iters=6000)
    T2 = r2["T"].reshape(ny, nx)
    q2 = r2["q"].reshape(ny, nx, 2)
    tsc = np.abs(r1["T"] - 300.0).max()
    qsc = np.abs(r1["q"][:, 0]).max()
    assert qsc > 0
    for i in range(nx):
        assert np.abs(T2[:, i] - r1["T"]).max() < 1e-10 * tsc
        assert np.abs(q2[:, i, 1] - r1["q"][:, 0]).max() < 1e-10 * qsc
    assert np.abs(q2[:, :, 0]).max() < 1e-12 * qsc


def test_flux_along_z_matches_film():
    """Eq. 4 along z: a 3D column with specular x and y walls, isothermal -z / +z
    walls and a source varying in z only reduces to the film along z: q_z equals
    the film's q_x, q_x and q_y vanish."""
    nx, ny, nz = 2, 3, 10
    v, tau, C = bi.band_table_synthetic(2)
    s, w = bi.quad_octant_gl(2, 1, polar_axis=0)
    qz = 1e18 * np.linspace(1.0, 0.3, nz)
    m3 = np.ones(nx * ny * nz, dtype=np.uint8)
    fbc3 = bi.face_bc_from_mask((nx, ny, nz), 3, m3, lambda i, j, k, f: {4: 0, 5: 1}.get(f, 2))
    p3 = bi.Problem("column_z", 3, (nx, ny, nz), (2e-9, 2e-9, 2e-9), m3, fbc3,
                    np.array([0, 0, 2], dtype=np.int32), np.array([305.0, 300.0, 300.0]),
                    v, tau, C, s, w, np.repeat(qz, nx * ny), 300.0)
    p1 = _film_along((2, 0, 1), nz, v, tau, C, s, w, qz)
    r3 = oracle.solve(p3, tol=0.0, max_iters=6000)
    r1 = oracle.solve(p1, tol=0.0, max_iters=6000)
    T3 = r3["T"].reshape(nz, ny * nx)
    q3 = r3["q"].reshape(nz, ny * nx, 3)
    tsc = np.abs(r1["T"] - 300.0).max()
    qsc = np.abs(r1["q"][:, 0]).max()
    for c in range(nx * ny):
        assert np.abs(T3[:, c] - r1["T"]).max() < 1e-10 * tsc
        assert np.abs(q3[:, c, 2] - r1["q"][:, 0]).max() < 1e-10 * qsc
    assert np.abs(q3[:, :, :2]).max() < 1e-12 * qsc


def test_flux_transposes_on_centred_square():
    """With the hot spot at the centre and a quadrature closed under x <-> y,
    the fixed point is symmetric under the transpose of the square, so the flux
    along y at (i, j) is the flux along x at (j, i) (Eq. 4)."""
    p = bi.square_2d(16, L=0.2e-6, n_bands=3, n_theta=2, n_phi=2, centered=True)
    r = oracle.solve(p, tol=1e-13, max_iters=5000)
    q = r["q"].reshape(16, 16, 2)
    sc = np.abs(q).max()
    assert sc > 0
    assert np.abs(q[:, :, 1] - q[:, :, 0].T).max() < 1e-12 * sc
    # and the flux points away from the hot spot on either side of it
    assert q[8, 12, 0] > 0 and q[8, 3, 0] < 0


# ------------------------------------------ P17 convergence residuals (Eq. 22)
@pytest.mark.parametrize("n_it", [1, 5, 12])
def test_residuals_follow_eq22(n_it):
    """Methods, "Iterative matrix formulation and solution scheme" (Eq. 22, with
    the deviational normalisation): the eps_T and eps_q reported after n + 1
    iterations equal the RMS change of T and of |q| between the fields returned
    after n and n + 1 iterations, over the active cells, divided by the largest
    |T - T_ref| and the largest |q| of the newer fields."""
    p = bi.random_box_2d(7, 6, seed=5, n_bands=3, n_theta=2, n_phi=1, kinds=(0, 1))
    a = oracle.solve(p, tol=0.0, max_iters=n_it)
    b = oracle.solve(p, tol=0.0, max_iters=n_it + 1)
    act = p.mask > 0
    dT = (b["T"] - a["T"])[act]
    eT = math.sqrt(float(np.mean(dT * dT))) / float(np.abs(b["T"][act] - p.T_ref).max())
    qa = np.linalg.norm(a["q"][act], axis=1)
    qb = np.linalg.norm(b["q"][act], axis=1)
    eq = math.sqrt(float(np.mean((qb - qa) ** 2))) / float(qb.max())
    assert b["iters"] == n_it + 1
    assert abs(b["eps_T"] - eT) <= 1e-12 * eT
    assert abs(b["eps_q"] - eq) <= 1e-12 * eq


def test_residual_stop_rule():
    """The solve stops at the first iteration whose eps_T and eps_q are both
    below the target (Eq. 22): one iteration fewer leaves one of them above."""
    p = bi.random_box_2d(7, 6, seed=5, n_bands=3, n_theta=2, n_phi=1, kinds=(0, 1))
    r = oracle.solve(p, tol=1e-6, max_iters=5000)
    assert r["status"] == "converged" and r["eps_T"] < 1e-6 and r["eps_q"] < 1e-6
    prev = oracle.solve(p, tol=0.0, max_iters=r["iters"] - 1)
    assert prev["eps_T"] >= 1e-6 or prev["eps_q"] >= 1e-6


# ------------------------- P18 second-order faces by deferred correction
@pytest.mark.parametrize("case", ["diffuse_2d", "specular_2d", "box_3d", "film_nongray"])
def test_second_order_fixed_point_matches_dense(case):
    """Methods, "Spatial discretization" and Eq. rhs_b: the oracle's
    deferred-correction iteration (second-order face values of e^n on the
    right-hand side, first-order A) converges to the solution of the
    second-order discrete equations assembled directly."""
    if case == "diffuse_2d":
        p = bi.random_box_2d(6, 5, seed=7, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 1))
    elif case == "specular_2d":
        p = bi.random_box_2d(5, 6, seed=8, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 2))
    elif case == "box_3d":
        p = bi.random_box_3d(3, 4, 4, seed=8, n_bands=2, n_theta=1, n_phi=1, kinds=(0, 1))
    else:
        base = bi.film_1d(n_cells=14, L=20e-9, n_mu=6)
        v, tau, C = bi.band_table_synthetic(3)
        p = base.replace(v=v, tau=tau * 0.05, C=C, Q=np.linspace(0, 1e18, 14))
    Td = dense.solve_dense(p, order=2)
    T1 = dense.solve_dense(p, order=1)
    r = oracle.solve(p, tol=0.0, max_iters=6000, order=2)
    act = p.mask > 0
    scale = np.abs(Td[act] - p.T_ref).max()
    assert np.abs(r["T"][act] - Td[act]).max() < 1e-10 * scale
    # the second-order solution is a different one
    assert np.abs(T1[act] - Td[act]).max() > 1e-6 * scale


def _film_theta(n, n_mu, order):
    p = bi.film_1d(n_cells=n, Kn=1.0, n_mu=n_mu)
    r = oracle.solve(p, tol=1e-12, max_iters=5000, order=order)
    assert r["status"] == "converged"
    return (r["T"] - 299.0) / 2.0


def test_second_order_film_order_of_accuracy():
    """Results, "1D cross-plane phonon transport" (the paper's grid study at
    50, 100 and 200 cells, observed orders 1.8 and 1.9): the second-order
    film's RMS error against the 3200-cell solution of the same discrete
    directions falls at an observed order of about 2, the first-order one's at
    about 1."""
    xf = (np.arange(3200) + 0.5) / 3200
    orders = {}
    for order in (1, 2):
        fine = _film_theta(3200, 64, order)
        err = []
        for n in (50, 100, 200):
            x = (np.arange(n) + 0.5) / n
            d = _film_theta(n, 64, order) - np.interp(x, xf, fine)
            err.append(math.sqrt(float(np.mean(d * d))))
        orders[order] = [math.log2(err[i] / err[i + 1]) for i in range(2)]
    assert all(1.75 < o < 2.3 for o in orders[2]), orders
    assert all(0.85 < o < 1.2 for o in orders[1]), orders


def test_second_order_film_matches_gray_slab_integral_equation():
    """With enough directions that the angular error stays small, the
    second-order film at 200 cells is within 3e-5 of the imposed difference of
    the semi-analytic slab solution, ten times closer than first order."""
    xs, th = _gray_slab_theta(1.0, 8000)
    x = (np.arange(200) + 0.5) / 200
    e2 = np.abs(_film_theta(200, 256, 2) - np.interp(x, xs, th))
    e1 = np.abs(_film_theta(200, 256, 1) - np.interp(x, xs, th))
    assert math.sqrt(float(np.mean(e2 * e2))) < 3e-5
    assert math.sqrt(float(np.mean(e2 * e2))) < 0.1 * math.sqrt(float(np.mean(e1 * e1)))


def test_second_order_square_d4_symmetry():
    p = bi.square_2d(12, L=0.1e-6, n_bands=3, n_theta=2, n_phi=2, centered=True)
    r = oracle.solve(p, tol=1e-12, max_iters=5000, order=2)
    T = r["T"].reshape(12, 12) - 300.0
    sc = np.abs(T).max()
    for U in (T[:, ::-1], T[::-1, :], T.T):
        assert np.abs(T - U).max() < 1e-11 * sc
