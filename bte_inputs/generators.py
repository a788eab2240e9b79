"""Seeded input recipes (geometry, bands, quadrature, sources, probes, batches).

Everything here is an *input* to the solver: values that the paper takes from
meshes, DFT band data or user choices, replaced by seeded synthetic stand-ins
of the same shape. No function here performs a transport sweep, a temperature
update or any other step of the solution method.

Array conventions (shared by the oracle and the HIP library):
  * cells are indexed c = i + n0*(j + n1*k), x fastest; arrays of cell data
    have shape (n2, n1, n0) when reshaped;
  * faces of a cell are numbered 0..5 = -x, +x, -y, +y, -z, +z;
  * face_bc[c, f] holds the boundary-condition id of face f of cell c when that
    face is a boundary (domain edge or inactive neighbour), else NO_BC;
  * quadrature directions s[a] are unit vectors (x, y, z), weights w[a] sum to
    4*pi.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BC_ISOTHERMAL = 0
BC_DIFFUSE = 1
BC_SPECULAR = 2
NO_BC = 255

FOUR_PI = 4.0 * math.pi

__all__ = [
    "BC_ISOTHERMAL", "BC_DIFFUSE", "BC_SPECULAR", "NO_BC", "Problem",
    "band_table_synthetic", "band_table_gray", "quad_gl_mu", "quad_octant_gl",
    "face_bc_from_mask", "gaussian_source", "film_1d", "square_2d", "finfet_3d", "finfet_3d_mixed",
    "adjoint_case", "batch_instances", "scattering_mfp", "random_box_2d", "random_box_3d", "multi_hole_2d",
    "staircase_3d",
]


@dataclasses.dataclass
class Problem:
    """One steady BTE problem: geometry + boundary table + bands + quadrature + source."""
    name: str
    dim: int
    n: tuple            # cells per axis (unused axes = 1)
    h: tuple            # cell size per axis, metres
    mask: np.ndarray    # uint8 [ncell], 1 = active
    face_bc: np.ndarray  # uint8 [ncell, 6]
    bc_kind: np.ndarray  # int32 [n_bc]
    bc_T: np.ndarray     # float64 [n_bc], wall temperature (isothermal walls), K
    v: np.ndarray        # float64 [B], m/s
    tau: np.ndarray      # float64 [B], s
    C: np.ndarray        # float64 [B], J m^-3 K^-1
    s: np.ndarray        # float64 [M, 3]
    w: np.ndarray        # float64 [M]
    Q: np.ndarray        # float64 [ncell], W/m^3
    T_ref: float = 300.0

    @property
    def ncell(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def n_active(self) -> int:
        return int(self.mask.sum())

    @property
    def B(self) -> int:
        return int(self.v.shape[0])

    @property
    def M(self) -> int:
        return int(self.w.shape[0])

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------------------
# Band tables
# ----------------------------------------------------------------------------
def band_table_synthetic(n_bands: int = 15, C_total: float = 1.66e6):
    """Silicon-like synthetic band table (stand-in for DFT-derived bands).

    v_b linear 1e3 -> 8e3 m/s, tau_b log-spaced 1e-12 -> 1e-9 s, and
    C_b proportional to omega_b^2 with omega_b at the centre of equidistant
    wave-vector bands (Debye-like), normalised so that sum C_b = C_total.
    """
    b = np.arange(n_bands, dtype=np.float64)
    last = max(n_bands - 1, 1)
    v = 1000.0 + (7000.0 / last) * b
    tau = 1e-12 * 10.0 ** (3.0 * b / last)
    C = (b + 0.5) ** 2
    C = C / C.sum() * C_total
    return v, tau, C


def band_table_gray(v: float, tau: float, C: float = 1.66e6):
    return (np.array([v], dtype=np.float64), np.array([tau], dtype=np.float64),
            np.array([C], dtype=np.float64))


def scattering_mfp(v, tau, C) -> float:
    """Scattering-weighted mean free path sum(C v) / sum(C / tau) (input recipe)."""
    v, tau, C = (np.asarray(x, dtype=np.float64) for x in (v, tau, C))
    return float((C * v).sum() / (C / tau).sum())


# ----------------------------------------------------------------------------
# Angular quadrature tables
# ----------------------------------------------------------------------------
def quad_gl_mu(n_mu: int):
    """Gauss-Legendre in mu = cos(theta) on [-1, 1], azimuth integrated out.

    Direction a has s = (mu_a, sqrt(1 - mu_a^2), 0) and weight 2*pi*g_a; only the
    x component transports in a 1D slab. The weights sum to 4*pi exactly in exact
    arithmetic.
    """
    mu, g = np.polynomial.legendre.leggauss(n_mu)
    s = np.zeros((n_mu, 3))
    s[:, 0] = mu
    s[:, 1] = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    w = 2.0 * math.pi * g
    return s, w


def quad_octant_gl(n_theta: int, n_phi: int, polar_axis: int = 0, renormalize: bool = True):
    """Octant product Gauss-Legendre quadrature (paper Eq. 14, Methods: angle
    discretization).

    Per octant, theta in (0, pi/2) and phi in (0, pi/2) each take an n-point
    Gauss-Legendre rule; the weight of direction (theta, phi) is
    beta_theta * beta_phi * sin(theta). The eight octants are the mirror images.
    With polar_axis = 0 the direction is (cos t, sin t cos p, sin t sin p) as in
    the paper; polar_axis = 2 puts the polar axis along z:
    (sin t cos p, sin t sin p, cos t). The product rule integrates sin(theta) only
    approximately; with renormalize=True the weights are scaled so they sum to
    4*pi exactly, which keeps a uniform equilibrium a fixed point.
    Returns M = 8*n_theta*n_phi directions.
    """
    xt, gt = np.polynomial.legendre.leggauss(n_theta)
    xp, gp = np.polynomial.legendre.leggauss(n_phi)
    th = (xt + 1.0) * (math.pi / 4.0)
    bt = gt * (math.pi / 4.0)
    ph = (xp + 1.0) * (math.pi / 4.0)
    bp = gp * (math.pi / 4.0)
    dirs: List[np.ndarray] = []
    wts: List[float] = []
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                for it in range(n_theta):
                    for ip in range(n_phi):
                        t, p = th[it], ph[ip]
                        a = math.cos(t)
                        b_ = math.sin(t) * math.cos(p)
                        c = math.sin(t) * math.sin(p)
                        if polar_axis == 0:
                            vec = (sx * a, sy * b_, sz * c)
                        elif polar_axis == 2:
                            vec = (sx * b_, sy * c, sz * a)
                        elif polar_axis == 1:
                            vec = (sx * c, sy * a, sz * b_)
                        else:
                            raise ValueError("polar_axis must be 0, 1 or 2")
                        dirs.append(np.array(vec))
                        wts.append(bt[it] * bp[ip] * math.sin(t))
    s = np.array(dirs, dtype=np.float64)
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    w = np.array(wts, dtype=np.float64)
    if renormalize:
        w *= FOUR_PI / w.sum()
    return s, w


# ----------------------------------------------------------------------------
# Geometry helpers
# ----------------------------------------------------------------------------
def _offsets(dim):
    return [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)][: 2 * dim]


def face_bc_from_mask(n, dim, mask, rule):
    """Boundary table: face_bc[c, f] = rule(i, j, k, f) for every boundary face f
    of every active cell (domain edge or inactive neighbour), NO_BC elsewhere."""
    n0, n1, n2 = n
    m = mask.reshape(n2, n1, n0).astype(bool)
    fbc = np.full((n2, n1, n0, 6), NO_BC, dtype=np.uint8)
    kk, jj, ii = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    for f, (dx, dy, dz) in enumerate(_offsets(dim)):
        ni, nj, nk = ii + dx, jj + dy, kk + dz
        inside = (ni >= 0) & (ni < n0) & (nj >= 0) & (nj < n1) & (nk >= 0) & (nk < n2)
        nb_active = np.zeros_like(m)
        nb_active[inside] = m[nk[inside], nj[inside], ni[inside]]
        bnd = m & ~nb_active
        if bnd.any():
            ids = np.vectorize(lambda i, j, k: rule(int(i), int(j), int(k), f), otypes=[np.int64])(
                ii[bnd], jj[bnd], kk[bnd])
            fbc[..., f][bnd] = ids.astype(np.uint8)
    return fbc.reshape(n0 * n1 * n2, 6)


def gaussian_source(n, h, Q0, center, sigma):
    """Q = Q0 exp(-|x - x0|^2 / (2 sigma^2)) at cell centres of a 2D grid."""
    n0, n1, n2 = n
    x = (np.arange(n0) + 0.5) * h[0]
    y = (np.arange(n1) + 0.5) * h[1]
    X, Y = np.meshgrid(x, y, indexing="xy")
    r2 = (X - center[0]) ** 2 + (Y - center[1]) ** 2
    Q = Q0 * np.exp(-r2 / (2.0 * sigma * sigma))
    return np.broadcast_to(Q, (n2, n1, n0)).reshape(-1).astype(np.float64).copy()


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------
def film_1d(n_cells=200, L=100e-9, Kn=1.0, v=6000.0, C=1.66e6, T_h=301.0, T_c=299.0,
            n_mu=32, T_ref=300.0, Q=None):
    """1D gray cross-plane film (paper Results: 1D cross-plane phonon transport).

    Kn = v*tau/L (the mean free path over the film thickness). The -x wall is
    isothermal at T_h (bc 0), the +x wall isothermal at T_c (bc 1).
    """
    tau = Kn * L / v
    h = L / n_cells
    n = (n_cells, 1, 1)
    mask = np.ones(n_cells, dtype=np.uint8)
    fbc = face_bc_from_mask(n, 1, mask, lambda i, j, k, f: 0 if f == 0 else 1)
    s, w = quad_gl_mu(n_mu)
    vv, tt, CC = band_table_gray(v, tau, C)
    QQ = np.zeros(n_cells) if Q is None else np.asarray(Q, dtype=np.float64)
    return Problem("film_1d", 1, n, (h, h, h), mask, fbc,
                   np.array([BC_ISOTHERMAL, BC_ISOTHERMAL], dtype=np.int32),
                   np.array([T_h, T_c]), vv, tt, CC, s, w, QQ, T_ref)


def square_2d(n_cells=256, L=1e-6, n_bands=15, n_theta=8, n_phi=2, Q0=1e19, seed=1,
              centered=False, T_wall=300.0, T_ref=300.0, bands=None, quad=None,
              center=None, sigma=None):
    """2D nongray square with a Gaussian hot spot and isothermal edges.

    sigma = L/16; the centre is drawn from U[0.25L, 0.75L]^2 with `seed`, or is
    the square's centre when `centered`. Quadrature: z-polar octant product with
    n_theta polar nodes per hemisphere and n_phi azimuthal nodes per quadrant.
    """
    n = (n_cells, n_cells, 1)
    hh = L / n_cells
    mask = np.ones(n_cells * n_cells, dtype=np.uint8)
    fbc = face_bc_from_mask(n, 2, mask, lambda i, j, k, f: 0)
    v, tau, C = band_table_synthetic(n_bands) if bands is None else bands
    s, w = quad_octant_gl(n_theta, n_phi, polar_axis=2) if quad is None else quad
    if center is None:
        if centered:
            center = (0.5 * L, 0.5 * L)
        else:
            rng = np.random.default_rng(seed)
            center = tuple(rng.uniform(0.25 * L, 0.75 * L, size=2))
    sig = L / 16.0 if sigma is None else sigma
    Q = gaussian_source(n, (hh, hh, hh), Q0, center, sig)
    p = Problem("square_2d", 2, n, (hh, hh, hh), mask, fbc,
                np.array([BC_ISOTHERMAL], dtype=np.int32), np.array([T_wall]),
                np.asarray(v, float), np.asarray(tau, float), np.asarray(C, float),
                np.asarray(s, float), np.asarray(w, float), Q, T_ref)
    p.center, p.sigma, p.Q0 = center, sig, Q0  # type: ignore[attr-defined]
    return p


def random_box_2d(nx, ny, seed, n_bands=3, n_theta=2, n_phi=1, hole=True, kinds=(0, 1),
                  T_walls=(305.0, 300.0), dx=2e-9, Q0=1e18):
    """Small 2D test geometry: rectangle with an optional inactive hole, the
    bottom edge isothermal (bc 0) and every other boundary face of bc kind
    kinds[1] (bc 1). Used for brute-force and parity tests."""
    rng = np.random.default_rng(seed)
    n = (nx, ny, 1)
    m = np.ones((1, ny, nx), dtype=np.uint8)
    if hole and nx >= 4 and ny >= 4:
        hx = int(rng.integers(1, nx - 2))
        hy = int(rng.integers(1, ny - 2))
        m[0, hy:hy + 2, hx:hx + 1] = 0
    mask = m.reshape(-1)
    fbc = face_bc_from_mask(n, 2, mask, lambda i, j, k, f: 0 if (f == 2 and j == 0) else 1)
    v, tau, C = band_table_synthetic(n_bands)
    s, w = quad_octant_gl(n_theta, n_phi, polar_axis=2)
    Q = Q0 * rng.uniform(0.0, 1.0, size=nx * ny) * mask
    return Problem("random_box_2d", 2, n, (dx, dx, dx), mask, fbc,
                   np.array([BC_ISOTHERMAL, kinds[1]], dtype=np.int32),
                   np.array(T_walls, dtype=np.float64), v, tau, C, s, w, Q, 300.0)


def multi_hole_2d(nx, ny, seed, n_holes=8, **kw):
    """random_box_2d without its hole but with several seeded inactive blocks,
    so that holes fall inside a lane's rows, across lanes and next to strip
    boundaries of the 2D sweep layouts."""
    p = random_box_2d(nx, ny, seed, hole=False, **kw)
    rng = np.random.default_rng(seed + 100)
    m = p.mask.reshape(ny, nx).copy()
    for _ in range(n_holes):
        hx, hy = int(rng.integers(1, nx - 3)), int(rng.integers(1, ny - 4))
        m[hy:hy + int(rng.integers(1, 4)), hx:hx + int(rng.integers(1, 3))] = 0
    mask = m.reshape(-1).astype(np.uint8)
    fbc = face_bc_from_mask(p.n, 2, mask, lambda i, j, k, f: 0 if (f == 2 and j == 0) else 1)
    return p.replace(name="multi_hole_2d", mask=mask, face_bc=fbc, Q=p.Q * mask)


def random_box_3d(nx, ny, nz, seed, n_bands=2, n_theta=1, n_phi=1, hole=True, kinds=(0, 1),
                  T_walls=(305.0, 300.0), dx=2e-9, Q0=1e18):
    """Small 3D test geometry: box with an optional inactive notch, the bottom
    (-z at k = 0) isothermal (bc 0) and every other boundary face bc 1 of kind
    kinds[1]."""
    rng = np.random.default_rng(seed)
    n = (nx, ny, nz)
    m = np.ones((nz, ny, nx), dtype=np.uint8)
    if hole and min(nx, ny, nz) >= 3:
        m[nz - 1, int(rng.integers(0, ny)), int(rng.integers(0, nx))] = 0
        m[int(rng.integers(1, nz - 1)), int(rng.integers(1, ny - 1)), int(rng.integers(1, nx - 1))] = 0
    mask = m.reshape(-1)
    fbc = face_bc_from_mask(n, 3, mask, lambda i, j, k, f: 0 if (f == 4 and k == 0) else 1)
    v, tau, C = band_table_synthetic(n_bands)
    s, w = quad_octant_gl(n_theta, n_phi, polar_axis=0)
    Q = Q0 * rng.uniform(0.0, 1.0, size=nx * ny * nz) * mask
    return Problem("random_box_3d", 3, n, (dx, dx, dx), mask, fbc,
                   np.array([BC_ISOTHERMAL, kinds[1]], dtype=np.int32),
                   np.array(T_walls, dtype=np.float64), v, tau, C, s, w, Q, 300.0)


def staircase_3d(kind=1, nx=24, ny=20, nz=12, seed=8, n_bands=2, n_theta=1, n_phi=1):
    """3D staircase: the block of 8 columns x in [8k, 8k + 8) holds the planes
    z in [4k - 1, 4k + 4], so neighbouring blocks share one or two planes and
    the planes in use differ from block to block. Bottom face of every step
    isothermal (bc 0), every other boundary face bc 1 of the given kind."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    for k in range((nx + 7) // 8):
        m[max(0, 4 * k - 1):min(nz, 4 * k + 5), :, 8 * k:8 * k + 8] = 1
    mask = m.reshape(-1)
    base = random_box_3d(nx, ny, nz, seed=seed, n_bands=n_bands, n_theta=n_theta, n_phi=n_phi, hole=False,
                         kinds=(0, kind))
    fbc = face_bc_from_mask((nx, ny, nz), 3, mask, lambda i, j, k, f: 0 if f == 4 else 1)
    return base.replace(name="staircase_3d", mask=mask, face_bc=fbc, Q=base.Q * mask)


def finfet_3d(scale=1, seed=2, n_bands=15, n_theta=4, n_phi=4, Q0=1e19, T_ref=300.0,
              bands=None, quad=None):
    """3D FinFET-like voxel domain (stand-in for the paper's long-base FinFET).

    Full size (scale=1): mask 96(x) x 96(y) x 120(z), cell 2 nm; substrate
    z in [0, 92) plus a 16 x 64 x 28 fin box on top at a seeded (x0, y0);
    heat source Q0 in the fin's top 8 layers; bottom face isothermal 300 K
    (bc 0); every other boundary face diffusely reflecting (bc 1).
    `scale` divides every length in cells (scale=4 gives 24 x 24 x 30).
    Quadrature: octant product, 4 theta x 4 phi per octant (128 directions).
    """
    rng = np.random.default_rng(seed)
    x0 = int(rng.integers(0, 81))
    y0 = int(rng.integers(0, 33))
    nx, ny, nz = 96 // scale, 96 // scale, 120 // scale
    sub = 92 // scale
    fw, fl, fh = 16 // scale, 64 // scale, 28 // scale
    x0, y0 = x0 // scale, y0 // scale
    top = 8 // scale if scale <= 8 else 1
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[:sub] = 1
    m[sub:sub + fh, y0:y0 + fl, x0:x0 + fw] = 1
    n = (nx, ny, nz)
    mask = m.reshape(-1)
    fbc = face_bc_from_mask(n, 3, mask, lambda i, j, k, f: 0 if (f == 4 and k == 0) else 1)
    hh = 2e-9 * scale
    v, tau, C = band_table_synthetic(n_bands) if bands is None else bands
    s, w = quad_octant_gl(n_theta, n_phi, polar_axis=0) if quad is None else quad
    Qa = np.zeros((nz, ny, nx))
    zt0 = sub + fh - top
    Qa[zt0:sub + fh, y0:y0 + fl, x0:x0 + fw] = Q0
    Q = (Qa.reshape(-1) * mask).astype(np.float64)
    return Problem("finfet_3d", 3, n, (hh, hh, hh), mask, fbc,
                   np.array([BC_ISOTHERMAL, BC_DIFFUSE], dtype=np.int32),
                   np.array([300.0, 300.0]), np.asarray(v, float), np.asarray(tau, float),
                   np.asarray(C, float), np.asarray(s, float), np.asarray(w, float), Q, T_ref)


def finfet_3d_mixed(scale=1, **kw):
    """finfet_3d with the wall mix of the paper's short-base FinFET case
    (Results, FinFET with specular and diffuse walls): isothermal 300 K at the
    substrate bottom (bc 0) and on the top face of the fin (bc 3), diffusely
    reflecting fin side walls (bc 1), specularly reflecting base surfaces
    (bc 2: the substrate's sides and its top around the fin)."""
    p = finfet_3d(scale=scale, **kw)
    nz = p.n[2]
    sub = 92 // scale
    fh = 28 // scale
    fin_top = sub + fh - 1

    def rule(i, j, k, f):
        if f == 4 and k == 0:
            return 0
        if f == 5 and k == fin_top:
            return 3
        return 1 if k >= sub else 2

    assert fin_top < nz
    fbc = face_bc_from_mask(p.n, 3, p.mask, rule)
    return p.replace(name="finfet_3d_mixed", face_bc=fbc,
                     bc_kind=np.array([BC_ISOTHERMAL, BC_DIFFUSE, BC_SPECULAR, BC_ISOTHERMAL], dtype=np.int32),
                     bc_T=np.array([300.0, 300.0, 300.0, 300.0]))


def adjoint_case(base: Problem, seed_truth=3, seed_probe=4, seed_fd=5, n_probes=64, rim=4,
                 n_fd_tau=5, n_fd_Q=15, fd_radius=8):
    """Inverse-problem inputs on a 2D square: ground-truth tau* and source Q*,
    probe cells, and the parameters checked by finite differences.

    tau*_b = tau_b exp(0.25 z_b), z ~ N(0, 1); Q* = 1.5 Q0 Gaussian whose centre
    is shifted by U[-L/16, L/16]^2 from the base problem's centre. Probes are
    distinct cells at least `rim` cells from the edge. Finite-difference
    parameters: n_fd_tau band indices and n_fd_Q cells within fd_radius cells of
    a probe.
    """
    n0, n1, _ = base.n
    L = n0 * base.h[0]
    rng = np.random.default_rng(seed_truth)
    z = rng.standard_normal(base.B)
    tau_true = base.tau * np.exp(0.25 * z)
    shift = rng.uniform(-L / 16, L / 16, size=2)
    center = (base.center[0] + shift[0], base.center[1] + shift[1])
    Q0 = float(base.Q0)
    Q_true = gaussian_source(base.n, base.h, 1.5 * Q0, center, L / 16.0)
    rng = np.random.default_rng(seed_probe)
    ii, jj = np.meshgrid(np.arange(rim, n0 - rim), np.arange(rim, n1 - rim), indexing="xy")
    cand = (ii + n0 * jj).reshape(-1)
    probes = np.sort(rng.choice(cand, size=min(n_probes, cand.size), replace=False)).astype(np.int64)
    rng = np.random.default_rng(seed_fd)
    fd_tau = np.sort(rng.choice(base.B, size=min(n_fd_tau, base.B), replace=False)).astype(np.int64)
    pi_, pj_ = probes % n0, probes // n0
    near = []
    for c in range(n0 * n1):
        i, j = c % n0, c // n0
        if np.any((np.abs(pi_ - i) <= fd_radius) & (np.abs(pj_ - j) <= fd_radius)):
            near.append(c)
    near = np.array(near, dtype=np.int64)
    fd_Q = np.sort(rng.choice(near, size=min(n_fd_Q, near.size), replace=False)).astype(np.int64)
    return dict(tau_true=tau_true, Q_true=Q_true, probes=probes, fd_tau=fd_tau, fd_Q=fd_Q)


def batch_instances(n_inst=256, seed=6, nx_range=(32, 192), ny_range=(32, 160),
                    Kn_range=(0.01, 10.0), n_bands=15, n_theta=4, n_phi=2, Q0=1e19):
    """Many uneven 2D nongray instances (seeded grid sizes and Knudsen numbers).

    nx ~ U{nx_range}, ny ~ U{ny_range}, Kn ~ logU(Kn_range); the film length is
    L_x = Lambda_s / Kn with Lambda_s the band table's scattering-weighted mean
    free path; square cells h = L_x / nx; Gaussian hot spot sigma = L_x/16 at a
    seeded centre; isothermal edges at 300 K. 15 bands x 64 directions
    (z-polar, 4 theta per hemisphere x 2 phi per quadrant).
    """
    rng = np.random.default_rng(seed)
    v, tau, C = band_table_synthetic(n_bands)
    s, w = quad_octant_gl(n_theta, n_phi, polar_axis=2)
    lam = scattering_mfp(v, tau, C)
    out = []
    for _ in range(n_inst):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        ny = int(rng.integers(ny_range[0], ny_range[1] + 1))
        Kn = float(np.exp(rng.uniform(np.log(Kn_range[0]), np.log(Kn_range[1]))))
        cx, cy = rng.uniform(0.25, 0.75, size=2)
        Lx = lam / Kn
        hh = Lx / nx
        n = (nx, ny, 1)
        mask = np.ones(nx * ny, dtype=np.uint8)
        fbc = face_bc_from_mask(n, 2, mask, lambda i, j, k, f: 0)
        Q = gaussian_source(n, (hh, hh, hh), Q0, (cx * Lx, cy * ny * hh), Lx / 16.0)
        p = Problem(f"batch_{len(out)}", 2, n, (hh, hh, hh), mask, fbc,
                    np.array([BC_ISOTHERMAL], dtype=np.int32), np.array([300.0]),
                    v, tau, C, s, w, Q, 300.0)
        p.Kn = Kn  # type: ignore[attr-defined]
        out.append(p)
    return out


def problem_signature(p: Optional[Problem]) -> str:
    if p is None:
        return "none"
    return f"{p.name}:dim{p.dim}:n{p.n}:B{p.B}:M{p.M}:active{p.n_active}"
