"""Seeded synthetic inputs for the KFBI workloads.

This module only *generates inputs*: boundary samples of the test domains,
manufactured exact solutions (and the right-hand sides they imply), and seeded
densities.  It holds none of the method's arithmetic (no spline, no jump, no
correction, no fast solve, no interpolation, no Krylov step), so both the CPU
oracle and the HIP path may draw their inputs from it.

Workloads follow the paper's numerical-results section: a Dirichlet problem
for ``Lap u - kappa u = f`` (eq. of the modified Helmholtz problem, Sec. 2) on
a curved domain inside the box ``[-1.2, 1.2]^2`` (Example 1), with ``f`` and
``g`` taken from a closed-form solution.  The concrete domains (circle r=0.8,
star ``0.6 + 0.15 sin 5 theta``, random stars) and solutions are the
benchmark configurations this library is measured on.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BOX_LO = -1.2
BOX_HI = 1.2


# --------------------------------------------------------------------------
# boundary curves (counter-clockwise, first sample at theta = 0)
# --------------------------------------------------------------------------

def circle_points(m: int, r: float = 0.8) -> np.ndarray:
    """``m`` equally spaced points on the circle of radius ``r``, CCW, theta_0 = 0."""
    th = 2.0 * np.pi * np.arange(m) / m
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def _star_speed(theta, r0, a, k):
    r = r0 + a * np.sin(k * theta)
    dr = a * k * np.cos(k * theta)
    return np.sqrt(r * r + dr * dr)


def star_points(m: int, r0: float = 0.6, a: float = 0.15, k: int = 5,
                n_grid: int = 1 << 16) -> np.ndarray:
    """``m`` points of equal arc length on ``r(theta) = r0 + a sin(k theta)``.

    The speed ``|X'(theta)|`` is smooth and periodic, so its Fourier series
    gives the arc length in closed form; it is evaluated on a fine uniform
    grid by one inverse FFT, and each target length is inverted on its grid
    cell with the cubic Hermite interpolant of (arc length, speed), solved by
    Newton's method.  The first point sits at ``theta = 0``.
    """
    th = 2.0 * np.pi * np.arange(n_grid) / n_grid
    sp = _star_speed(th, r0, a, k)
    c = np.fft.rfft(sp) / n_grid              # speed = c0 + 2 Re sum_j c_j e^{ij theta}
    c0 = c[0].real
    d = np.zeros(n_grid // 2 + 1, dtype=complex)
    j = np.arange(1, n_grid // 2)
    d[1:n_grid // 2] = c[1:n_grid // 2] / (1j * j)
    osc = np.fft.irfft(d, n=n_grid) * n_grid   # 2 Re sum_j d_j e^{ij theta}
    s_g = c0 * th + osc - osc[0]
    perim = 2.0 * np.pi * c0
    s_g = np.append(s_g, perim)
    sp_g = np.append(sp, sp[0])
    dth = 2.0 * np.pi / n_grid
    target = perim * np.arange(m) / m
    cell = np.clip(np.searchsorted(s_g, target, side="right") - 1, 0, n_grid - 1)
    sa, sb = s_g[cell], s_g[cell + 1]
    da, db = sp_g[cell] * dth, sp_g[cell + 1] * dth
    u = (target - sa) / (sb - sa)
    for _ in range(6):
        # Hermite cubic on the cell and its derivative in u
        h00, h10, h01, h11 = (2 * u ** 3 - 3 * u ** 2 + 1, u ** 3 - 2 * u ** 2 + u, -2 * u ** 3 + 3 * u ** 2,
                              u ** 3 - u ** 2)
        H = h00 * sa + h10 * da + h01 * sb + h11 * db
        dH = (6 * u ** 2 - 6 * u) * sa + (3 * u ** 2 - 4 * u + 1) * da + (-6 * u ** 2 + 6 * u) * sb + \
             (3 * u ** 2 - 2 * u) * db
        u = u - (H - target) / dH
    t = (cell + u) * dth
    t[0] = 0.0
    r = r0 + a * np.sin(k * t)
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)


def circle_normals(xy: np.ndarray) -> np.ndarray:
    """Exact outward unit normals of a circle centred at the origin at points ``xy``."""
    return xy / np.hypot(xy[:, 0], xy[:, 1])[:, None]


def star_normals(xy: np.ndarray, r0: float = 0.6, a: float = 0.15, k: int = 5) -> np.ndarray:
    """Exact outward unit normals of ``r(theta) = r0 + a sin(k theta)`` at its points ``xy``:
    the tangent ``X'(theta)`` turned clockwise."""
    t = np.arctan2(xy[:, 1], xy[:, 0])
    r = r0 + a * np.sin(k * t)
    dr = a * k * np.cos(k * t)
    tx, ty = dr * np.cos(t) - r * np.sin(t), dr * np.sin(t) + r * np.cos(t)
    sp = np.hypot(tx, ty)
    return np.stack([ty / sp, -tx / sp], axis=1)


def star_perimeter(r0: float, a: float, k: int, n: int = 8192) -> float:
    th = 2.0 * np.pi * np.arange(n) / n
    return float(np.mean(_star_speed(th, r0, a, k)) * 2.0 * np.pi)


def star_min_radius_of_curvature(r0: float, a: float, k: int, n: int = 20000) -> float:
    th = 2.0 * np.pi * np.arange(n) / n
    r = r0 + a * np.sin(k * th)
    r1 = a * k * np.cos(k * th)
    r2 = -a * k * k * np.sin(k * th)
    curv = np.abs(r * r + 2 * r1 * r1 - r * r2) / (r * r + r1 * r1) ** 1.5
    return float(1.0 / np.max(curv))


# --------------------------------------------------------------------------
# manufactured solutions: u, and Lap u (so f = Lap u - kappa u)
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Manufactured:
    """A closed-form solution ``u`` with its Laplacian and gradient."""
    name: str
    u: callable
    lap: callable
    grad: callable = None       # (x, y) -> (u_x, u_y)

    def f(self, x, y, kappa):
        """Right-hand side of ``Lap u - kappa u = f``."""
        return self.lap(x, y) - kappa * self.u(x, y)


EXP_SIN = Manufactured(
    "exp(x) sin(y)",
    lambda x, y: np.exp(x) * np.sin(y),
    lambda x, y: np.zeros_like(np.asarray(x, dtype=float) + np.asarray(y, dtype=float)),
    lambda x, y: (np.exp(x) * np.sin(y), np.exp(x) * np.cos(y)),
)

PAPER_EX1 = Manufactured(
    "exp(x) cos(y) + exp(y) sin(x)",
    lambda x, y: np.exp(x) * np.cos(y) + np.exp(y) * np.sin(x),
    lambda x, y: np.zeros_like(np.asarray(x, dtype=float) + np.asarray(y, dtype=float)),
)

SIN_COS_X2 = Manufactured(
    "sin(pi x) cos(pi y) + x^2",
    lambda x, y: np.sin(np.pi * x) * np.cos(np.pi * y) + x * x,
    lambda x, y: -2.0 * np.pi ** 2 * np.sin(np.pi * x) * np.cos(np.pi * y) + 2.0,
    lambda x, y: (np.pi * np.cos(np.pi * x) * np.cos(np.pi * y) + 2.0 * x,
                  -np.pi * np.sin(np.pi * x) * np.sin(np.pi * y)),
)


@dataclasses.dataclass(frozen=True)
class Manufactured3:
    """A closed-form solution ``u(x, y, z)`` with its Laplacian."""
    name: str
    u: callable
    lap: callable

    def f(self, x, y, z, kappa):
        return self.lap(x, y, z) - kappa * self.u(x, y, z)


EXP_XYZ = Manufactured3(
    "exp(x+y+z)",
    lambda x, y, z: np.exp(x + y + z),
    lambda x, y, z: 3.0 * np.exp(x + y + z),
)


def random_manufactured(rng: np.random.Generator, xp=np) -> Manufactured:
    """``u = A sin(w1 x + a) cos(w2 y + b) + B (x^2 - y^2)`` with seeded parameters.

    ``xp`` is the array module the closed forms are evaluated with (numpy, or
    torch for inputs generated directly in device memory).
    """
    A, B = rng.uniform(-1.0, 1.0, size=2)
    w1, w2 = rng.uniform(0.5, np.pi, size=2)
    al, be = rng.uniform(0.0, 2.0 * np.pi, size=2)
    return Manufactured(
        f"{A:.3f} sin({w1:.3f}x+{al:.3f}) cos({w2:.3f}y+{be:.3f}) + {B:.3f}(x^2-y^2)",
        lambda x, y: A * xp.sin(w1 * x + al) * xp.cos(w2 * y + be) + B * (x * x - y * y),
        lambda x, y: -(w1 * w1 + w2 * w2) * A * xp.sin(w1 * x + al) * xp.cos(w2 * y + be),
        lambda x, y: (A * w1 * xp.cos(w1 * x + al) * xp.cos(w2 * y + be) + 2.0 * B * x,
                      -A * w2 * xp.sin(w1 * x + al) * xp.sin(w2 * y + be) - 2.0 * B * y),
    )


# --------------------------------------------------------------------------
# densities for the stand-alone operator apply
# --------------------------------------------------------------------------

def smooth_density(m: int, seed: int = 1234, kmax: int = 8) -> np.ndarray:
    """``phi_m = sum_{k<=kmax} a_k cos(k th_m) + b_k sin(k th_m)``, ``a,b ~ N(0,1)/(1+k^2)``."""
    rng = np.random.default_rng(seed)
    th = 2.0 * np.pi * np.arange(m) / m
    phi = np.zeros(m)
    for k in range(kmax + 1):
        a, b = rng.standard_normal(2) / (1.0 + k * k)
        phi += a * np.cos(k * th) + b * np.sin(k * th)
    return phi


# --------------------------------------------------------------------------
# problem bundles
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    """Everything a Dirichlet solve needs, in plain host arrays.

    ``xy``: (M, 2) boundary samples (CCW).  ``n``: intervals per axis.
    ``f_grid``: (n+1, n+1) right-hand side sampled at every node, indexed
    ``[j, i]`` (row j is the grid line ``y = lo + j h``, i runs along x).
    ``f_gamma`` and ``g``: f and the Dirichlet data at the boundary samples.
    """
    name: str
    xy: np.ndarray
    n: int
    kappa: float
    lo: float
    hi: float
    f_grid: np.ndarray
    f_gamma: np.ndarray
    g: np.ndarray
    exact: Manufactured

    @property
    def h(self):
        return (self.hi - self.lo) / self.n

    def node_coords(self):
        k = np.arange(self.n + 1)
        return self.lo + k * self.h


def make_problem(name, xy, n, kappa, sol: Manufactured, lo=BOX_LO, hi=BOX_HI) -> Problem:
    h = (hi - lo) / n
    c = lo + np.arange(n + 1) * h
    X, Y = np.meshgrid(c, c, indexing="xy")       # X[j, i] = x_i, Y[j, i] = y_j
    f_grid = sol.f(X, Y, kappa)
    f_gamma = sol.f(xy[:, 0], xy[:, 1], kappa)
    g = sol.u(xy[:, 0], xy[:, 1])
    return Problem(name, xy, n, kappa, lo, hi, np.ascontiguousarray(f_grid, dtype=np.float64),
                   np.asarray(f_gamma, dtype=np.float64), np.asarray(g, dtype=np.float64), sol)


def circle_problem(n=64, m=128, kappa=0.0, sol=EXP_SIN, r=0.8) -> Problem:
    """Interior Dirichlet problem on the circle of radius ``r`` (``e^x sin y`` by default)."""
    return make_problem(f"circle r={r} n={n} m={m} kappa={kappa}", circle_points(m, r), n, kappa, sol)


def star_problem(n=512, m=None, kappa=1.0, sol=SIN_COS_X2, r0=0.6, a=0.15, k=5) -> Problem:
    """Modified Helmholtz problem on the star ``r0 + a sin(k theta)``, ``m = n/2`` samples by default."""
    if m is None:
        m = n // 2
    return make_problem(f"star {r0}+{a}sin({k}t) n={n} m={m} kappa={kappa}",
                        star_points(m, r0, a, k), n, kappa, sol)


@dataclasses.dataclass
class NeumannProblem:
    """Everything a Neumann solve needs: as ``Problem`` with ``g_n = d_n u`` (exact
    outward normals) in place of the Dirichlet data; ``g`` is the exact trace, for
    checking the solution on Gamma."""
    name: str
    xy: np.ndarray
    n: int
    kappa: float
    lo: float
    hi: float
    f_grid: np.ndarray
    f_gamma: np.ndarray
    g_n: np.ndarray
    g: np.ndarray
    exact: Manufactured

    @property
    def h(self):
        return (self.hi - self.lo) / self.n


def make_neumann_problem(name, xy, normals, n, kappa, sol: Manufactured, lo=BOX_LO, hi=BOX_HI) -> NeumannProblem:
    p = make_problem(name, xy, n, kappa, sol, lo, hi)
    gx, gy = sol.grad(xy[:, 0], xy[:, 1])
    g_n = np.asarray(gx * normals[:, 0] + gy * normals[:, 1], dtype=np.float64)
    return NeumannProblem(name, p.xy, n, kappa, lo, hi, p.f_grid, p.f_gamma, g_n, p.g, sol)


def circle_neumann_problem(n=64, m=128, kappa=1.0, sol=EXP_SIN, r=0.8) -> NeumannProblem:
    """Interior Neumann problem on the circle of radius ``r``."""
    xy = circle_points(m, r)
    return make_neumann_problem(f"neumann circle r={r} n={n} m={m} kappa={kappa}", xy, circle_normals(xy),
                                n, kappa, sol)


def star_neumann_problem(n=512, m=None, kappa=1.0, sol=SIN_COS_X2, r0=0.6, a=0.15, k=5) -> NeumannProblem:
    """Modified Helmholtz Neumann problem on the star ``r0 + a sin(k theta)``, ``m = n/2`` by default."""
    if m is None:
        m = n // 2
    xy = star_points(m, r0, a, k)
    return make_neumann_problem(f"neumann star {r0}+{a}sin({k}t) n={n} m={m} kappa={kappa}", xy,
                                star_normals(xy, r0, a, k), n, kappa, sol)


# --------------------------------------------------------------------------
# Gray-Scott reaction-diffusion (Example 3): disk r = 1.8 in the box (-2, 2)^2
# --------------------------------------------------------------------------

GS_LO, GS_HI, GS_RADIUS = -2.0, 2.0, 1.8


@dataclasses.dataclass(frozen=True)
class GrayScottParams:
    """``u_t = eps1 Lap u + (gamma (1-u) - u v^2) / eps0``,
    ``v_t = eps2 Lap v + (u v^2 - (gamma + kill) v) / eps0`` (the paper's
    removal rate, called kappa there, is ``kill`` here)."""
    gamma: float = 0.024
    kill: float = 0.06
    eps0: float = 0.01
    eps1: float = 0.008
    eps2: float = 0.004


def gray_scott_initial(x, y):
    """Initial ``(u, v)``: ``v = sin^2(4 pi x) sin^2(4 pi y) / 4`` on ``[-1/4, 1/4]^2``, else 0;
    ``u = 1 - 2 v``."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    box = (np.abs(x) <= 0.25) & (np.abs(y) <= 0.25)
    v = np.where(box, 0.25 * np.sin(4 * np.pi * x) ** 2 * np.sin(4 * np.pi * y) ** 2, 0.0)
    return 1.0 - 2.0 * v, v


def gray_scott_samples(n: int) -> np.ndarray:
    """Boundary samples of the disk for an ``n x n`` grid on the box: ``M = 64 ceil(P / (128 h))``,
    about two grid spacings apart."""
    h = (GS_HI - GS_LO) / n
    m = 64 * int(math.ceil(2.0 * np.pi * GS_RADIUS / (128.0 * h)))
    return circle_points(m, GS_RADIUS)


@dataclasses.dataclass
class RequestSpec:
    """Domain and data of one serving request, before any grid array exists."""
    name: str
    n: int
    kappa: float
    xy: np.ndarray
    sol: Manufactured           # numpy closed forms
    sol_torch: Manufactured     # the same closed forms over torch tensors
    min_radius: float = float("inf")   # smallest radius of curvature of the boundary

    @property
    def under_resolved(self) -> bool:
        """Boundary features finer than three grid spacings (served, but flagged)."""
        return self.min_radius < 3.0 * (BOX_HI - BOX_LO) / self.n


def serving_spec(seed: int, n: int) -> RequestSpec:
    """One request of the mixed serving stream: a random star, kappa and solution."""
    def draw(xp):
        rng = np.random.default_rng(seed)
        a = rng.uniform(0.05, 0.2)
        k = int(rng.integers(3, 9))
        kappa = rng.uniform(0.0, 10.0)
        return a, k, kappa, random_manufactured(rng, xp)
    a, k, kappa, sol = draw(np)
    try:
        import torch
        sol_t = draw(torch)[3]
    except ImportError:                        # CPU-only environments
        sol_t = None
    # samples about two grid spacings apart along the boundary, in multiples of 64
    h = (BOX_HI - BOX_LO) / n
    per = star_perimeter(0.6, a, k)
    m = 64 * int(math.ceil(per / (128 * h)))
    return RequestSpec(f"req{seed} star a={a:.3f} k={k} n={n} m={m} kappa={kappa:.3f}", n, kappa,
                       star_points(m, 0.6, a, k), sol, sol_t, star_min_radius_of_curvature(0.6, a, k))


def serving_request(seed: int, n: int):
    """One request of the mixed serving stream as a full host-side Problem."""
    sp = serving_spec(seed, n)
    return make_problem(sp.name, sp.xy, n, sp.kappa, sp.sol)


def serving_stream(n_requests: int, seed: int = 2404, qps: float = 100.0,
                   sizes=(256, 512, 1024, 2048), weights=(0.4, 0.3, 0.2, 0.1)):
    """Seeded request stream: Poisson arrival times, grid sizes and per-request seeds."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    arrivals = np.cumsum(gaps)
    ns = rng.choice(np.asarray(sizes), size=n_requests, p=np.asarray(weights))
    seeds = rng.integers(0, 2 ** 31 - 1, size=n_requests)
    return [(float(t), int(n), int(s)) for t, n, s in zip(arrivals, ns, seeds)]


# --------------------------------------------------------------------------
# 3D: the ellipsoid workload
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Problem3:
    """A Dirichlet problem on the ellipsoid ``x^2/a^2 + y^2/b^2 + z^2/c^2 < 1``.

    ``f_grid`` is sampled at every node of the ``(n+1)^3`` grid, indexed
    ``[k, j, i]`` (k along z, j along y, i along x).  The boundary data live at
    the control points, which the discretisation chooses (the grid-line /
    surface intersections): ``boundary_data(points)`` samples them there.
    """
    name: str
    axes: tuple
    n: int
    kappa: float
    lo: float
    hi: float
    f_grid: np.ndarray
    exact: Manufactured3

    @property
    def h(self):
        return (self.hi - self.lo) / self.n

    def node_coords(self):
        return self.lo + np.arange(self.n + 1) * self.h

    def boundary_data(self, pts):
        """``(f_gamma, g)`` at the points ``pts`` (shape (M, 3))."""
        x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
        return (np.asarray(self.exact.f(x, y, z, self.kappa), dtype=np.float64),
                np.asarray(self.exact.u(x, y, z), dtype=np.float64))

    def exact_grid(self):
        c = self.node_coords()
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        return self.exact.u(X, Y, Z)


def ellipsoid_problem(n=64, axes=(0.9, 0.7, 0.5), kappa=0.0, sol=EXP_XYZ, lo=BOX_LO, hi=BOX_HI) -> Problem3:
    """Interior Dirichlet problem on the ellipsoid with semi-axes ``axes`` (``e^{x+y+z}`` by default)."""
    h = (hi - lo) / n
    c = lo + np.arange(n + 1) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    f_grid = np.ascontiguousarray(sol.f(X, Y, Z, kappa), dtype=np.float64)
    return Problem3(f"ellipsoid {axes} n={n} kappa={kappa}", tuple(float(a) for a in axes), n, kappa, lo, hi,
                    f_grid, sol)


def smooth_density3(pts: np.ndarray, seed: int = 1234) -> np.ndarray:
    """A smooth seeded density at the points ``pts``: a random combination of
    low-order trigonometric functions of the position."""
    rng = np.random.default_rng(seed)
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    out = np.zeros(len(pts))
    for k in range(1, 4):
        a = rng.standard_normal(6) / (1.0 + k * k)
        out += (a[0] * np.cos(k * x) + a[1] * np.sin(k * y) + a[2] * np.cos(k * z)
                + a[3] * np.sin(k * (x + y)) + a[4] * np.cos(k * (y - z)) + a[5] * np.sin(k * (x - z)))
    return out
