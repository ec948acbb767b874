"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds no arithmetic of the transport method itself: it only
lays down point clouds (jittered lattices, Poisson-disk samples), support
radii, material regions and the closed-form problem data (manufactured
solutions and their sources, beams, Gaussian sources) that define each
workload.  Both the oracle and the HIP path receive exactly these arrays.

Point placement follows the paper's Results section: a uniform lattice
whose points are perturbed by up to 0.2 times the spacing in each
dimension, independently per point and dimension.  The asteroid problem
(Sec. 5.4) grades its spacing with the distance to the shell and to the
source; its points are the jittered leaves of a quadtree refined to that
spacing.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence

import numpy as np

SEED_BASE = 20080220


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def jittered_lattice(counts: Sequence[int], lo: Sequence[float], hi: Sequence[float],
                     jitter: float, seed: int) -> tuple[np.ndarray, float]:
    """Cell-centred lattice with ``counts[a]`` points along axis ``a``.

    Point ``(i+1/2)*dx`` along each axis, moved by ``gamma*dx`` with
    ``gamma ~ U[-jitter, jitter]`` drawn per point and per axis.  Returns
    ``(x[N][d], dx_nominal)`` where ``dx_nominal`` is the spacing of axis 0.
    Points are ordered with axis 0 fastest.
    """
    d = len(counts)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    dxs = (hi - lo) / np.asarray(counts, dtype=np.float64)
    axes = [lo[a] + (np.arange(counts[a]) + 0.5) * dxs[a] for a in range(d)]
    grids = np.meshgrid(*axes, indexing="ij")
    # axis 0 fastest
    x = np.stack([g.transpose(*reversed(range(d))).reshape(-1) for g in grids], axis=1)
    if jitter > 0.0:
        g = rng(seed).uniform(-jitter, jitter, size=x.shape)
        x = x + g * dxs[None, :]
    return np.ascontiguousarray(x, dtype=np.float64), float(dxs[0])


def poisson_disk(lo: Sequence[float], hi: Sequence[float], r: float, seed: int,
                 k: int = 30) -> np.ndarray:
    """Maximal Poisson-disk sample of the 2D box by Bridson's algorithm (2007).

    Every pair of points is at least ``r`` apart; candidates are drawn in the
    annulus ``[r, 2r]`` around active points, ``k`` tries each.
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    g = rng(seed)
    cs = r / math.sqrt(2.0)
    nx = int(math.ceil((hi[0] - lo[0]) / cs))
    ny = int(math.ceil((hi[1] - lo[1]) / cs))
    grid = -np.ones((nx, ny), dtype=np.int64)
    pts: list[tuple[float, float]] = []

    def cell_of(p):
        return (min(nx - 1, int((p[0] - lo[0]) / cs)), min(ny - 1, int((p[1] - lo[1]) / cs)))

    def ok(p):
        if not (lo[0] <= p[0] < hi[0] and lo[1] <= p[1] < hi[1]):
            return False
        ci, cj = cell_of(p)
        for a in range(max(0, ci - 2), min(nx, ci + 3)):
            for b in range(max(0, cj - 2), min(ny, cj + 3)):
                q = grid[a, b]
                if q >= 0:
                    dx = pts[q][0] - p[0]
                    dy = pts[q][1] - p[1]
                    if dx * dx + dy * dy < r * r:
                        return False
        return True

    p0 = (lo[0] + g.uniform() * (hi[0] - lo[0]), lo[1] + g.uniform() * (hi[1] - lo[1]))
    pts.append(p0)
    grid[cell_of(p0)] = 0
    active = [0]
    while active:
        ai = int(g.integers(len(active)))
        base = pts[active[ai]]
        placed = False
        for _ in range(k):
            rad = r * (1.0 + g.uniform())
            th = 2.0 * math.pi * g.uniform()
            p = (base[0] + rad * math.cos(th), base[1] + rad * math.sin(th))
            if ok(p):
                pts.append(p)
                grid[cell_of(p)] = len(pts) - 1
                active.append(len(pts) - 1)
                placed = True
                break
        if not placed:
            active[ai] = active[-1]
            active.pop()
    return np.asarray(pts, dtype=np.float64)


# ---------------------------------------------------------------------------
# Closed-form problem data
# ---------------------------------------------------------------------------

def mms_sin_psi(x: np.ndarray, omega: np.ndarray, t: float) -> np.ndarray:
    """Manufactured angular flux psi = sin(pi x) sin(pi y) (1 + mu/2) e^{-t}, mu = Omega_x.

    Returns ``[N][M]``.  Vanishes on the boundary of the unit square, so the
    inflow data is zero.
    """
    s = np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])
    return (s[:, None] * (1.0 + 0.5 * omega[None, :, 0])) * math.exp(-t)


def mms_sin_source(x: np.ndarray, omega: np.ndarray, t: float, sigma_t: float,
                   sigma_s: float) -> np.ndarray:
    """Source q that makes ``mms_sin_psi`` solve the continuous transport equation.

    q = d_t psi + Omega . grad psi + sigma_t psi - sigma_s/(4 pi) phi with
    phi = 4 pi sin(pi x) sin(pi y) e^{-t} (the mu term integrates to zero).
    """
    sx, sy = np.sin(np.pi * x[:, 0]), np.sin(np.pi * x[:, 1])
    cx, cy = np.cos(np.pi * x[:, 0]), np.cos(np.pi * x[:, 1])
    s = sx * sy
    gx, gy = np.pi * cx * sy, np.pi * sx * cy
    mu = omega[None, :, 0]
    ang = 1.0 + 0.5 * mu
    odg = omega[None, :, 0] * gx[:, None] + omega[None, :, 1] * gy[:, None]
    e = math.exp(-t)
    q = (-s[:, None] * ang + odg * ang + sigma_t * s[:, None] * ang - sigma_s * s[:, None]) * e
    return q


def mms_sin_phi(x: np.ndarray, t: float) -> np.ndarray:
    return 4.0 * np.pi * np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * math.exp(-t)


# The manufactured problems of the paper's results section (Sec. 5.1), on
# [-1, 1]^d.  Both solutions are isotropic, so phi = 4 pi psi and the
# scattering term cancels sigma_s psi:  q = (1/c) d_t psi + Omega.grad psi + sigma_a psi.

def mms_cos_psi(x: np.ndarray, t: float) -> np.ndarray:
    """psi = 1 + (1/(2 pi)) prod_alpha cos(pi (x_alpha + t)), per point ``[N]``."""
    return 1.0 + np.prod(np.cos(np.pi * (x + t)), axis=1) / (2.0 * np.pi)


def mms_cos_sigma_a(x: np.ndarray) -> np.ndarray:
    """sigma_a = 1 + (2/3) prod_alpha cos(3 x_alpha)."""
    return 1.0 + (2.0 / 3.0) * np.prod(np.cos(3.0 * x), axis=1)


def mms_cos_sigma_s(x: np.ndarray) -> np.ndarray:
    """sigma_s = 1 + (3/4) prod_alpha sin(2 x_alpha)."""
    return 1.0 + 0.75 * np.prod(np.sin(2.0 * x), axis=1)


# The opacities above as material fields (a, b, k, phase, material): material
# 1 absorbs (sigma_t = 1), material 2 scatters (sigma_t = sigma_s = 1) and
# material 0 is void; sin(2x) = cos(2x - pi/2).
MMS_COS_FIELDS = ((1.0, 2.0 / 3.0, 3.0, 0.0, 1), (1.0, 0.75, 2.0, -0.5 * math.pi, 2))
MMS_COS_SIGMA_T = (0.0, 1.0, 1.0)
MMS_COS_SIGMA_S = (0.0, 0.0, 1.0)


def mms_cos_source(x: np.ndarray, omega: np.ndarray, t: float, inv_c: float) -> np.ndarray:
    """Source ``[N][M]`` of the sinusoidal manufactured problem at time t."""
    d = x.shape[1]
    c = np.cos(np.pi * (x + t))
    s = np.sin(np.pi * (x + t))
    grad = np.empty_like(x)
    for b in range(d):
        others = np.prod(np.delete(c, b, axis=1), axis=1) if d > 1 else 1.0
        grad[:, b] = -0.5 * s[:, b] * others          # (1/(2 pi)) * (-pi sin) * prod of the others
    dpsi_dt = grad.sum(axis=1)
    psi = mms_cos_psi(x, t)
    odg = grad @ omega[:, :d].T
    return inv_c * dpsi_dt[:, None] + odg + (mms_cos_sigma_a(x) * psi)[:, None]


def mms_wave_psi(x: np.ndarray, t: float) -> np.ndarray:
    """psi = 1 + exp(-10 (|x| - t)^2) / (t^2 + 6), per point ``[N]``."""
    r = np.sqrt(np.sum(x * x, axis=1))
    return 1.0 + np.exp(-10.0 * (r - t) ** 2) / (t * t + 6.0)


MMS_WAVE_SIGMA_A, MMS_WAVE_SIGMA_S = 0.5, 2.0


def mms_wave_source(x: np.ndarray, omega: np.ndarray, t: float, inv_c: float) -> np.ndarray:
    """Source ``[N][M]`` of the outgoing-wave manufactured problem (constant opacities)."""
    d = x.shape[1]
    r = np.sqrt(np.sum(x * x, axis=1))
    e = np.exp(-10.0 * (r - t) ** 2)
    den = t * t + 6.0
    dr = -20.0 * (r - t) * e / den                   # d psi / d r
    rs = np.where(r > 0.0, r, 1.0)
    grad = np.where(r[:, None] > 0.0, dr[:, None] * x / rs[:, None], 0.0)
    dpsi_dt = -2.0 * t * e / (den * den) + 20.0 * (r - t) * e / den
    odg = grad @ omega[:, :d].T
    return inv_c * dpsi_dt[:, None] + odg + (MMS_WAVE_SIGMA_A * mms_wave_psi(x, t))[:, None]


def gaussian_source(x: np.ndarray, center: Sequence[float], s: float) -> np.ndarray:
    """Isotropic per-steradian source of unit total emission: a Gaussian of std ``s``."""
    d = x.shape[1]
    r2 = np.sum((x - np.asarray(center)[None, :]) ** 2, axis=1)
    norm = (2.0 * np.pi) ** (d / 2.0) * s ** d * 4.0 * np.pi
    return np.exp(-r2 / (2.0 * s * s)) / norm


def absorber_psi(x: np.ndarray, mu: float, sigma_t: float) -> np.ndarray:
    """Plane-wave solution exp(-sigma_t x / mu) of Omega.grad psi + sigma_t psi = 0 (mu = Omega_x > 0)."""
    return np.exp(-sigma_t * x[:, 0] / mu)


# ---------------------------------------------------------------------------
# Workload definitions
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    lo: tuple
    hi: tuple
    counts: Optional[tuple]          # lattice counts, or None for Poisson-disk
    jitter: float
    radius_factor: float             # support radius R = factor * dx_nominal
    rk_order: int
    n_ord: int                       # ordinates
    ord_kind: str                    # "product" | "beam-dense"
    sigma_t: tuple                   # per material
    sigma_s: tuple
    regions: tuple                   # ((lo), (hi), mat) boxes, last match wins
    steps: int                       # 0 => steady
    dt: float
    c: float
    source: str                      # "uniform" | "mms-sin" | "gaussian" | "none"
    inflow: str                      # "vacuum" | "beam"
    seed: int
    pd_radius: float = 0.0           # Poisson-disk spacing when counts is None
    fields: tuple = ()               # smooth material fields (a, b, k, phase, material)
    t0: float = 0.0                  # time of the initial state (steady problems: time of the solution)
    velocity: float = 0.0            # points move with the cellular flow of this amplitude (0: fixed)

    @property
    def inv_c_dt(self) -> float:
        return 0.0 if self.steps == 0 else 1.0 / (self.c * self.dt)


def config(k: int, scale: Optional[int] = None) -> Workload:
    """The five workloads (k = 1..5).  ``scale`` replaces the lattice count per
    axis, for the small and mid-size parity variants of the same problem."""
    if k == 1:
        n = scale or 32
        return Workload("2d-lattice-steady-q1", 2, (0.0, 0.0), (1.0, 1.0), (n, n), 0.2, 2.0, 1,
                        16, "product", (1.0,), (0.5,), (), 0, 0.0, 1.0, "uniform", "vacuum",
                        SEED_BASE + 1)
    if k == 2:
        n = scale or 128
        return Workload("2d-mms-be20", 2, (0.0, 0.0), (1.0, 1.0), (n, n), 0.2, 2.0, 1,
                        64, "product", (1.0,), (0.5,), (), 20, 1e-2, 1.0, "mms-sin", "vacuum",
                        SEED_BASE + 2)
    if k == 3:
        n = scale or 40
        return Workload("3d-gauss-steady", 3, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (n, n, n), 0.2, 2.5, 2,
                        96, "product", (1.0,), (0.9,), (), 0, 0.0, 1.0, "gaussian", "vacuum",
                        SEED_BASE + 3)
    if k == 4:
        return Workload("2d-beam-void-opaque", 2, (0.0, 0.0), (2.0, 1.0), None, 0.0, 2.0, 1,
                        256, "beam-dense", (1e-4, 100.0), (0.0, 99.0),
                        (((1.0, 0.0), (2.0, 1.0), 1),), 10, 0.05, 1.0, "none", "beam",
                        SEED_BASE + 4, pd_radius=0.00438)
    if k == 8:
        # workload 2 with points that move every step (the cellular flow below),
        # so that cells, integration and assembly are redone inside the time loop
        n = scale or 128
        return Workload("2d-mms-be20-moving", 2, (0.0, 0.0), (1.0, 1.0), (n, n), 0.2, 2.0, 1,
                        64, "product", (1.0,), (0.5,), (), 20, 1e-2, 1.0, "mms-sin", "vacuum",
                        SEED_BASE + 8, velocity=0.25)
    if k == 6:
        # Sec. 5.1 sinusoidal manufactured problem: uniform lattice on [-1, 1]^2,
        # varying opacities as material fields, steady (solution at t = 0)
        n = scale or 128
        return Workload("2d-paper-mms-cos", 2, (-1.0, -1.0), (1.0, 1.0), (n, n), 0.0, 2.0, 1, 16, "product",
                        MMS_COS_SIGMA_T, MMS_COS_SIGMA_S, (), 0, 0.0, 1.0, "paper-cos", "paper-cos",
                        SEED_BASE + 6, fields=MMS_COS_FIELDS)
    if k == 7:
        # Sec. 5.1 outgoing-wave manufactured problem, steady (solution at t = 0.5)
        n = scale or 128
        return Workload("2d-paper-mms-wave", 2, (-1.0, -1.0), (1.0, 1.0), (n, n), 0.0, 2.0, 1, 16, "product",
                        (MMS_WAVE_SIGMA_A + MMS_WAVE_SIGMA_S,), (MMS_WAVE_SIGMA_S,), (), 0, 0.0, 1.0,
                        "paper-wave", "paper-wave", SEED_BASE + 7, t0=0.5)
    raise ValueError(k)


def paper_mms_psi(w: Workload, x: np.ndarray, t: float) -> np.ndarray:
    """The isotropic manufactured solution of a Sec. 5.1 workload at time t, per point."""
    if w.source == "paper-cos":
        return mms_cos_psi(x, t)
    if w.source == "paper-wave":
        return mms_wave_psi(x, t)
    raise ValueError(w.source)


# ---------------------------------------------------------------------------
# Asteroid problem (Sec. 5.4 and its appendix), 2D: an absorbing shell around
# the origin lit by a small source in a thin background.  Lengths are scaled
# by ``scale`` from the paper's (asteroid radius 35, source 70 from the
# surface); the shell stays 20 mean free paths thick.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Asteroid:
    radius: float            # outer radius of the asteroid
    thickness: float         # shell thickness
    sigma_shell: float
    sigma_back: float
    src: tuple               # source centre
    src_radius: float        # radius of the small disk that stands in for the point source
    strength: float          # emission per unit length of the source (isotropic)
    lo: tuple
    hi: tuple


def asteroid(scale: float = 0.1) -> Asteroid:
    R = 35.0 * scale
    sig = 10.0 / scale                      # keeps 20 mean free paths in 2.0 * scale
    return Asteroid(R, 2.0 * scale, sig, 0.001 / scale, (-(R + 70.0 * scale), 0.0), 1.0 * scale, 1.0,
                    (-(R + 75.0 * scale), -(R + 5.0 * scale)), (R + 5.0 * scale, R + 5.0 * scale))


def asteroid_source(a: Asteroid, x: np.ndarray, m: int) -> np.ndarray:
    """Isotropic per-steradian source ``[N][M]``: the strength spread uniformly over the source disk."""
    inside = np.sum((x - np.asarray(a.src)) ** 2, axis=1) <= a.src_radius ** 2
    q = np.where(inside, a.strength / (4.0 * np.pi * np.pi * a.src_radius ** 2), 0.0)
    return np.repeat(q[:, None], m, axis=1)


def chord_in_circle(src: np.ndarray, xe: np.ndarray, radius: float) -> np.ndarray:
    """Length of the segment src -> xe (per point) inside the circle |x| <= radius, from the
    intercepts s = (-l1 +- sqrt(l1^2 - l0 l2)) / l2 of the parametric line x = src + (xe - src) s."""
    d = xe - src[None, :]
    l0 = src @ src - radius * radius
    l1 = d @ src
    l2 = np.sum(d * d, axis=1)
    disc = l1 * l1 - l0 * l2
    ok = (disc > 0.0) & (l2 > 0.0)
    sq = np.sqrt(np.where(ok, disc, 0.0))
    l2s = np.where(l2 > 0.0, l2, 1.0)
    s0 = np.clip((-l1 - sq) / l2s, 0.0, 1.0)
    s1 = np.clip((-l1 + sq) / l2s, 0.0, 1.0)
    return np.where(ok, (s1 - s0) * np.sqrt(l2), 0.0)


def asteroid_optical_depth(a: Asteroid, x: np.ndarray, extra: float = 0.0) -> np.ndarray:
    """omega = integral of sigma_a from the source centre to each point (straight ray), with a
    uniform absorption ``extra`` added everywhere (a backward-Euler step from zero radiation adds
    1/(c dt) to sigma_a)."""
    src = np.asarray(a.src, dtype=np.float64)
    r = np.sqrt(np.sum((x - src[None, :]) ** 2, axis=1))
    in_shell = chord_in_circle(src, x, a.radius) - chord_in_circle(src, x, a.radius - a.thickness)
    return a.sigma_back * (r - in_shell) + a.sigma_shell * in_shell + extra * r


def asteroid_phi_paper(a: Asteroid, x: np.ndarray) -> np.ndarray:
    """The appendix's scalar flux (1/r) [exp(-omega) - omega E1(omega)] of a unit line source."""
    from scipy.special import exp1
    r = np.sqrt(np.sum((x - np.asarray(a.src)[None, :]) ** 2, axis=1))
    om = asteroid_optical_depth(a, x)
    e1 = np.where(om > 0.0, exp1(np.maximum(om, 1e-300)), 0.0)
    return (np.exp(-om) - om * e1) / r


def asteroid_phi_ordinates(a: Asteroid, x: np.ndarray, xi: np.ndarray, wp: np.ndarray,
                           extra: float = 0.0) -> np.ndarray:
    """Scalar flux of a line source of the asteroid's strength seen through polar levels with cosines
    xi and weights wp (folded: 2 wp each) and a continuum of azimuths: along the in-plane ray of length
    r the path is r / sin(theta), so phi = S / (4 pi r) sum_p 2 wp_p exp(-omega / st_p) / st_p, with
    the optical depth omega of ``asteroid_optical_depth`` (``extra`` as there)."""
    r = np.sqrt(np.sum((x - np.asarray(a.src)[None, :]) ** 2, axis=1))
    om = asteroid_optical_depth(a, x, extra)
    st = np.sqrt(1.0 - np.asarray(xi) ** 2)
    tot = sum(2.0 * w * np.exp(-om / t) / t for w, t in zip(wp, st))
    return a.strength / (4.0 * np.pi * r) * tot


def asteroid_points(a: Asteroid, spacing: float, seed: int = SEED_BASE + 9, jitter: float = 0.2):
    """Jittered lattice of the given spacing over the asteroid domain; returns (x, R, dx) with R = 2 dx."""
    counts = [max(2, int(round((h - l) / spacing))) for l, h in zip(a.lo, a.hi)]
    x, dx = jittered_lattice(counts, a.lo, a.hi, jitter, seed)
    return x, np.full(x.shape[0], 2.0 * dx), dx


def asteroid_spacing(a: Asteroid, x: np.ndarray, coarsen: float = 1.0) -> np.ndarray:
    """Target point spacing h(x) of Sec. 5.4, in the paper's units times the workload's scale s:
    0.2 s on the shell's inner surface, 0.1 s on its outer surface (linear across the shell), 0.1 s at
    the source, 1.0 s halfway (35 s) between the source and the asteroid.  Away from the shell and from
    the source h grows linearly with the distance, from those surface values to 1.0 s at 35 s, and
    is capped at 1.0 s; inside the shell's inner radius it grows inward at the same rate.  h is the
    smaller of the shell's and the source's ramps, times ``coarsen``."""
    s = a.radius / 35.0
    slope = 0.9 / 35.0
    r = np.sqrt(np.sum(x * x, axis=1))
    R, t = a.radius, a.thickness
    h_out = 0.1 * s + slope * np.maximum(r - R, 0.0)
    h_shell = 0.1 * s + 0.1 * s * (R - r) / t
    h_in = 0.2 * s + slope * np.maximum(R - t - r, 0.0)
    h = np.where(r >= R, h_out, np.where(r >= R - t, h_shell, h_in))
    d_src = np.sqrt(np.sum((x - np.asarray(a.src)[None, :]) ** 2, axis=1))
    h = np.minimum(h, 0.1 * s + slope * d_src)
    return coarsen * np.minimum(h, 1.0 * s)


def morton_order(x: np.ndarray, lo: Sequence[float], hi: Sequence[float], bits: int = 16) -> np.ndarray:
    """Permutation that sorts 2D points along the Z (Morton) curve of a 2^bits grid over the box."""
    lo = np.asarray(lo, dtype=np.float64)
    ext = np.asarray(hi, dtype=np.float64) - lo
    q = np.clip(((x - lo[None, :]) / ext[None, :] * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    key = np.zeros(x.shape[0], dtype=np.int64)
    for b in range(bits):
        key |= ((q[:, 0] >> b) & 1) << (2 * b)
        key |= ((q[:, 1] >> b) & 1) << (2 * b + 1)
    return np.argsort(key, kind="stable")


def asteroid_graded_points(a: Asteroid, coarsen: float = 1.0, seed: int = SEED_BASE + 10, jitter: float = 0.2):
    """Points at the graded spacing of Sec. 5.4 (``asteroid_spacing``): the leaves of a quadtree over
    the domain, split while a leaf's size exceeds sqrt(2) h at its centre (so each leaf is within a
    factor sqrt(2) of h there), one point per leaf at its centre moved by U[-jitter, jitter] times the
    leaf's sides, in Morton order of the leaves.  Root cells are the near-square cells of the
    coarsest spacing, ceil(extent / hmax) per axis.  A leaf on the domain's edge is also split while
    a leaf touching its inner face (the face opposite that edge) is finer: with the support radius
    R = 2 L of every point (L = sqrt(area), the leaf size and local spacing), a coarse edge row beside
    a finer row inside would leave the edge covered by the supports of one row of points only, where
    the linear RK moment matrix is nearly singular.  Returns (x, R, L); the SUPG length is L."""
    lo = np.asarray(a.lo, dtype=np.float64)
    hi = np.asarray(a.hi, dtype=np.float64)
    ext = hi - lo
    hmax = coarsen * a.radius / 35.0
    nroot = np.maximum(1, np.ceil(ext / hmax - 1e-9).astype(np.int64))
    root = ext / nroot
    ii, jj = np.meshgrid(np.arange(nroot[0]), np.arange(nroot[1]), indexing="ij")
    corner = lo[None, :] + np.stack([ii.ravel(), jj.ravel()], axis=1) * root[None, :]
    sz = np.repeat(root[None, :], corner.shape[0], axis=0)

    def children(c, s):
        h = 0.5 * s
        return (np.concatenate([c, c + h * [1.0, 0.0], c + h * [0.0, 1.0], c + h]), np.tile(h, (4, 1)))

    c_l, s_l = [], []
    while corner.shape[0]:
        L = np.sqrt(sz[:, 0] * sz[:, 1])
        split = L > math.sqrt(2.0) * asteroid_spacing(a, corner + 0.5 * sz, coarsen)
        c_l.append(corner[~split])
        s_l.append(sz[~split])
        corner, sz = children(corner[split], sz[split])
    corner, sz = np.concatenate(c_l), np.concatenate(s_l)
    tol = 1e-9 * float(ext.max())
    from scipy.spatial import cKDTree
    while True:
        cen = corner + 0.5 * sz
        L = np.sqrt(sz[:, 0] * sz[:, 1])
        at_lo = corner - lo[None, :] < tol
        at_hi = hi[None, :] - (corner + sz) < tol
        edge = np.nonzero(np.any(at_lo | at_hi, axis=1))[0]
        # leaves touching an edge leaf: centres within (s_i + s_j) / 2 along both axes, which for
        # touching leaves of at most twice the size is within 1.5 leaf diagonals
        near = cKDTree(cen).query_ball_point(cen[edge], 1.5 * 1.01 * np.sqrt(np.sum(sz[edge] ** 2, axis=1)))
        split = np.zeros(corner.shape[0], dtype=bool)
        for i, js in zip(edge, near):
            js = np.asarray(js, dtype=np.int64)
            gap = np.abs(cen[js] - cen[i]) - 0.5 * (sz[js] + sz[i])
            js = js[np.all(gap <= tol, axis=1) & (L[js] < L[i] * (1.0 - 1e-9))]
            for ax in range(2):
                d = cen[js, ax] - cen[i, ax]
                inner = (d > 0.0) if at_lo[i, ax] else (d < 0.0) if at_hi[i, ax] else np.zeros(js.size, bool)
                # across the inner face: the centres are (s_i + s_j) / 2 apart along this axis
                inner &= np.abs(np.abs(d) - 0.5 * (sz[js, ax] + sz[i, ax])) <= tol
                split[i] |= bool(inner.any())
        if not split.any():
            break
        c2, s2 = children(corner[split], sz[split])
        corner, sz = np.concatenate([corner[~split], c2]), np.concatenate([sz[~split], s2])
    cen = corner + 0.5 * sz
    order = morton_order(cen, lo, hi)
    cen, sz = cen[order], sz[order]
    L = np.sqrt(sz[:, 0] * sz[:, 1])
    g = rng(seed).uniform(-jitter, jitter, size=cen.shape)
    x = np.ascontiguousarray(cen + g * sz, dtype=np.float64)
    return x, 2.0 * L, L


def asteroid_step_inv_c_dt(a: Asteroid) -> float:
    """1/(c dt) of the asteroid's single backward-Euler step (Sec. 5.4: one step long enough for the
    radiation to cross the domain): c dt is 100 times the domain's diagonal."""
    return 1.0 / (100.0 * float(np.linalg.norm(np.subtract(a.hi, a.lo))))


def asteroid_materials(a: Asteroid):
    """Shells ((centre, r_in, r_out, material),), sigma_t and sigma_s per material (no scattering)."""
    return ((((0.0, 0.0), a.radius - a.thickness, a.radius, 1),), (a.sigma_back, a.sigma_shell), (0.0, 0.0))


def asteroid_lit_region(a: Asteroid, x: np.ndarray, near: float) -> np.ndarray:
    """Points in the background between the source and the asteroid, inside the cone of rays that
    hit it and at least ``near`` from the source: where the refined ordinates resolve the flux."""
    src = np.asarray(a.src)
    d = np.linalg.norm(src)
    v = x - src[None, :]
    r = np.linalg.norm(v, axis=1)
    ang = np.abs(np.arctan2(v[:, 1], v[:, 0]))
    return (r >= near) & (ang <= math.asin(a.radius / d)) & (np.linalg.norm(x, axis=1) > a.radius + 2 * a.thickness) \
        & (x[:, 0] < 0.0)


def cellular_flow(x: np.ndarray, amplitude: float) -> np.ndarray:
    """Divergence-free velocity U (sin(pi x) cos(pi y), -cos(pi x) sin(pi y)) on the unit square.

    Its normal component vanishes on the boundary, so points stay inside and
    their density stays uniform while the lattice shears."""
    u = np.empty_like(x)
    u[:, 0] = amplitude * np.sin(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])
    u[:, 1] = -amplitude * np.cos(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])
    return u


def advect_points(w: Workload, x: np.ndarray, dt: float) -> np.ndarray:
    """Positions after one step of the workload's point motion (explicit Euler)."""
    return x + dt * cellular_flow(x, w.velocity)


def points_for(w: Workload) -> tuple[np.ndarray, float]:
    if w.counts is not None:
        return jittered_lattice(w.counts, w.lo, w.hi, w.jitter, w.seed)
    x = poisson_disk(w.lo, w.hi, w.pd_radius, w.seed)
    area = float(np.prod(np.asarray(w.hi) - np.asarray(w.lo)))
    return x, math.sqrt(area / x.shape[0])


def radii_for(w: Workload, x: np.ndarray, dx: float) -> np.ndarray:
    return np.full(x.shape[0], w.radius_factor * dx, dtype=np.float64)


def source_values(w: Workload, x: np.ndarray, omega: np.ndarray, t: float) -> np.ndarray:
    """Per-steradian source point values q_m(x_i) as ``[N][M]``."""
    m = omega.shape[0]
    if w.source == "uniform":
        return np.ones((x.shape[0], m))
    if w.source == "mms-sin":
        return mms_sin_source(x, omega, t, w.sigma_t[0], w.sigma_s[0])
    if w.source == "gaussian":
        g = gaussian_source(x, (0.5,) * w.dim, 0.05)
        return np.repeat(g[:, None], m, axis=1)
    if w.source == "none":
        return np.zeros((x.shape[0], m))
    if w.source in ("paper-cos", "paper-wave"):
        fn = mms_cos_source if w.source == "paper-cos" else mms_wave_source
        return fn(x, omega, t, 1.0 / w.c if w.steps > 0 else 0.0)
    raise ValueError(w.source)


def initial_psi(w: Workload, x: np.ndarray, omega: np.ndarray) -> np.ndarray:
    if w.source == "mms-sin":
        return mms_sin_psi(x, omega, 0.0)
    if w.source in ("paper-cos", "paper-wave"):
        return np.repeat(paper_mms_psi(w, x, w.t0)[:, None], omega.shape[0], axis=1)
    return np.zeros((x.shape[0], omega.shape[0]))


def inflow_values(w: Workload, y: np.ndarray, omega: np.ndarray, t: Optional[float] = None) -> np.ndarray:
    """Incoming angular flux psi_b at boundary points ``y[nb][d]`` for each ordinate: ``[nb][M]``.

    Beam: psi_b = 1 on the face x = 0 where |y - 1/2| < 0.05, for ordinates
    within 10 degrees of +x; 0 elsewhere.  Manufactured problems: the
    solution itself at time t (default: the workload's t0).
    """
    nb, m = y.shape[0], omega.shape[0]
    if w.inflow == "vacuum":
        return np.zeros((nb, m))
    if w.inflow in ("paper-cos", "paper-wave"):
        return np.repeat(paper_mms_psi(w, y, w.t0 if t is None else t)[:, None], m, axis=1)
    if w.inflow == "beam":
        on = (np.abs(y[:, 0] - w.lo[0]) < 1e-12) & (np.abs(y[:, 1] - 0.5) < 0.05)
        ang = np.arctan2(omega[:, 1], omega[:, 0])
        win = (np.abs(ang) <= math.radians(10.0) + 1e-12) & (omega[:, 0] > 0)
        return (on[:, None] & win[None, :]).astype(np.float64)
    raise ValueError(w.inflow)


# ---------------------------------------------------------------------------
# Request stream (many independent steady problems arriving over time)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class RequestSpec:
    rid: int
    arrival: float           # seconds after the start of the stream
    side: int                # lattice points per axis (N = side^2)
    n_ord: int
    sigma_t: float
    sigma_s: float
    seed: int


def request_stream(count: int, seed: int = SEED_BASE + 5, rate: float = 50.0, n_min: int = 1024,
                   n_max: int = 65536, ordinates=(16, 32, 64, 128), sigma_range=(0.1, 100.0),
                   c_max: float = 0.95) -> list:
    """Independent 2D steady problems with Poisson arrivals: point count
    log-uniform in [n_min, n_max] (rounded to a square lattice), ordinate count
    uniform over ``ordinates``, sigma_t log-uniform, scattering ratio uniform in
    [0, c_max].  One seed for the whole stream."""
    g = rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += g.exponential(1.0 / rate)
        n = math.exp(g.uniform(math.log(n_min), math.log(n_max)))
        side = max(2, int(round(math.sqrt(n))))
        m = int(ordinates[int(g.integers(len(ordinates)))])
        st = math.exp(g.uniform(math.log(sigma_range[0]), math.log(sigma_range[1])))
        c = g.uniform(0.0, c_max)
        out.append(RequestSpec(k, t, side, m, st, c * st, int(seed * 1000 + k)))
    return out


def request_problem(r: RequestSpec):
    """Points, radii (R = 2 dx) and the uniform per-steradian source of one request."""
    x, dx = jittered_lattice((r.side, r.side), (0.0, 0.0), (1.0, 1.0), 0.2, r.seed)
    R = np.full(x.shape[0], 2.0 * dx)
    return x, R, dx
