"""Plain FP64 CPU oracle of the KFBI hot path in three dimensions.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, the package's smoke check and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; the only common module is the seeded input generator ``synth``.

The method is the one of the two-dimensional oracle (``kfbi_oracle``), Sec. 2
and Alg. 1-5 of Tan, Huang & Ying (arXiv 2404.15249), on a cube with the
7-point Laplacian.  The paper gives no three-dimensional scheme for the
Poisson problem, so these readings are taken (reading R-19):

* Omega is the ellipsoid ``F(p) = x^2/a^2 + y^2/b^2 + z^2/c^2 - 1 < 0``; a node
  is inside iff ``F`` evaluated there is negative (no snapping: a node exactly
  on the surface is outside, and then no edge needs a crossing at it).
* The control points are all intersections of grid edges with the surface
  (``M = Q``), found by the quadratic formula on each sign-changing edge, in a
  fixed order: x-edges, then y-edges, then z-edges; lines ordered by their
  other two node indices (slowest last: for x-lines z then y), and along a line
  by node index.  The density lives at these points.
* Surface derivatives of the density at a control point come from a weighted
  least-squares quadratic in the tangent-plane coordinates ``(u, v)`` of the
  other control points within ``2.5 h`` (the 12 nearest if fewer), weights
  ``1 / (1 + (d/h)^2)``, with the constant term fixed at the point's own value.
* Jumps: ``[v] = Phi``, ``[d_n v] = Psi``, ``[Lap v - kappa v] = [F]`` with the
  shape operator ``S`` (second fundamental form, positive on the convex
  ellipsoid with the outward normal) in place of the curvature:
  ``[v_ab] = Phi_ab + Psi S_ab``, ``[v_an] = Psi_a - S_ab Phi_b``,
  ``[v_nn] = [F] + kappa Phi - [v_11] - [v_22]``.
* Correction: the second-order Taylor expansion of the jump along each grid
  edge through its crossing, as in two dimensions.
* Interpolation: the 7-point cross around the nearest node plus the three
  diagonal nodes toward the point in the xy, xz and yz planes; the quadratic
  through the ten (jump-corrected) values is evaluated at the point.
* Fast solve: DST-I on all three axes (eigenvalues ``l_k + l_l + l_m - kappa``).
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy import fft as sfft

from .kfbi_oracle import GeometryError, gmres

FIT_RADIUS = 2.5      # neighbourhood of the surface fit, in h
FIT_MIN = 12          # at least this many neighbours


def level(p, axes):
    """``F(p) = x^2/a^2 + y^2/b^2 + z^2/c^2 - 1`` (negative inside), evaluated left to right."""
    a, b, c = axes
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    return x * x / (a * a) + y * y / (b * b) + z * z / (c * c) - 1.0


@dataclasses.dataclass
class Plan3:
    n: int
    lo: float
    hi: float
    h: float
    axes: tuple
    inside: np.ndarray      # (n+1)^3 bool, [k, j, i]
    q_pos: np.ndarray       # (Q, 3) crossings = control points
    q_axis: np.ndarray      # (Q,) axis of the crossed edge (0 x, 1 y, 2 z)
    normal: np.ndarray      # (Q, 3) outward unit normal
    t1: np.ndarray          # (Q, 3) tangent basis
    t2: np.ndarray
    shape: np.ndarray       # (Q, 2, 2) second fundamental form in (t1, t2)
    nbr: list               # per point: indices of the fit neighbours
    fit: list               # per point: (5, K) weights of (Phi_u, Phi_v, Phi_uu, Phi_uv, Phi_vv)
    irr: list               # irregular nodes (i, j, k), lexicographic in (k, j, i)
    arms: list              # per irregular node: [(q, d)] with d = xi(neighbour) - xi(q)

    @property
    def M(self):
        return len(self.q_pos)

    def coord(self, k):
        return self.lo + k * self.h


def _frame(p, axes):
    """Outward normal, tangent basis and second fundamental form of the ellipsoid at ``p``."""
    a, b, c = axes
    g = np.array([2.0 * p[0] / (a * a), 2.0 * p[1] / (b * b), 2.0 * p[2] / (c * c)])
    gn = np.linalg.norm(g)
    n = g / gn
    e = np.zeros(3)
    e[int(np.argmin(np.abs(n)))] = 1.0
    t1 = np.cross(e, n)
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    hess = np.diag([2.0 / (a * a), 2.0 / (b * b), 2.0 / (c * c)])
    T = np.stack([t1, t2])
    S = T @ hess @ T.T / gn
    return n, t1, t2, S


def build_plan(n: int, lo: float, hi: float, axes) -> Plan3:
    """Classification, crossings, fit weights and the irregular-node arm table."""
    axes = tuple(float(v) for v in axes)
    h = (hi - lo) / n
    c = lo + np.arange(n + 1) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    inside = level(P, axes) < 0.0
    if inside[0].any() or inside[-1].any() or inside[:, 0].any() or inside[:, -1].any() \
            or inside[:, :, 0].any() or inside[:, :, -1].any():
        raise GeometryError("the surface reaches the box")
    # crossings, axis by axis; along each axis the sign-changing edges are taken
    # in the order (slower other axis, faster other axis, position on the line)
    q_pos, q_axis, q_of_edge = [], [], {}
    for ax in range(3):
        A = axes[ax]
        others = [o for o in range(3) if o != ax]
        # view the [k, j, i] array as [t_hi, t_lo, s] (s runs along ax)
        perm = [2 - others[1], 2 - others[0], 2 - ax]
        ins = np.transpose(inside, perm)
        chg = ins[:, :, 1:] != ins[:, :, :-1]
        for t_hi, t_lo, s in zip(*np.nonzero(chg)):
            t_hi, t_lo, s = int(t_hi), int(t_lo), int(s)
            idx_a = [0, 0, 0]
            idx_a[ax] = s
            idx_a[others[0]] = t_lo
            idx_a[others[1]] = t_hi
            # the root of F = 0 along the line: xi^2 / A^2 = 1 - (other terms)
            p0 = c[t_lo] / axes[others[0]]
            p1 = c[t_hi] / axes[others[1]]
            rest = 1.0 - p0 * p0 - p1 * p1
            root = A * np.sqrt(max(rest, 0.0))
            sa, sb = c[s], c[s + 1]
            xi = root if sa + sb > 0.0 else -root
            xi = min(max(xi, sa), sb)
            pos = [0.0, 0.0, 0.0]
            pos[ax] = xi
            pos[others[0]] = c[t_lo]
            pos[others[1]] = c[t_hi]
            q_of_edge[(ax, tuple(idx_a))] = len(q_pos)
            q_pos.append(pos)
            q_axis.append(ax)
    q_pos = np.array(q_pos, dtype=np.float64).reshape(-1, 3)
    q_axis = np.array(q_axis, dtype=np.int64)
    Q = len(q_pos)
    normal = np.empty((Q, 3))
    t1 = np.empty((Q, 3))
    t2 = np.empty((Q, 3))
    shape = np.empty((Q, 2, 2))
    for m in range(Q):
        normal[m], t1[m], t2[m], shape[m] = _frame(q_pos[m], axes)
    # weighted least-squares fit of the density around each point
    nbr, fit = [], []
    for m in range(Q):
        dx = q_pos[:, 0] - q_pos[m, 0]
        dy = q_pos[:, 1] - q_pos[m, 1]
        dz = q_pos[:, 2] - q_pos[m, 2]
        d = np.sqrt(dx * dx + dy * dy + dz * dz)
        d[m] = np.inf
        near = np.nonzero(d <= FIT_RADIUS * h)[0]
        if len(near) < FIT_MIN:
            near = np.argsort(d, kind="stable")[:FIT_MIN]
        near = np.sort(near)
        rel = q_pos[near] - q_pos[m]
        u = rel @ t1[m] / h
        v = rel @ t2[m] / h
        A = np.stack([u, v, 0.5 * u * u, u * v, 0.5 * v * v], axis=1)
        w = 1.0 / (1.0 + (d[near] / h) ** 2)
        G = A.T @ (w[:, None] * A)
        W = np.linalg.solve(G, A.T * w[None, :])
        scale = np.array([1.0 / h, 1.0 / h, 1.0 / (h * h), 1.0 / (h * h), 1.0 / (h * h)])
        nbr.append(near)
        fit.append(W * scale[:, None])
    # irregular nodes and their arms
    core = inside[1:n, 1:n, 1:n]
    flag = np.zeros_like(core)
    for ax in range(3):
        for step in (-1, 1):
            sl = [slice(1, n)] * 3
            sl[2 - ax] = slice(1 + step, n + step)
            flag |= inside[tuple(sl)] != core
    irr, arms = [], []
    for k, j, i in zip(*np.nonzero(flag)):
        i, j, k = int(i) + 1, int(j) + 1, int(k) + 1
        here = inside[k, j, i]
        lst = []
        for ax in range(3):
            for step in (-1, 1):
                nb = [i, j, k]
                nb[ax] += step
                if inside[nb[2], nb[1], nb[0]] == here:
                    continue
                low = [i, j, k] if step > 0 else nb
                q = q_of_edge[(ax, tuple(low))]
                d = c[nb[ax]] - q_pos[q, ax]
                lst.append((q, d))
        irr.append((i, j, k))
        arms.append(lst)
    return Plan3(n, lo, hi, h, axes, inside, q_pos, q_axis, normal, t1, t2, shape, nbr, fit, irr, arms)


def surface_derivs(plan: Plan3, phi):
    """``(Phi_u, Phi_v, Phi_uu, Phi_uv, Phi_vv)`` at every control point, shape (M, 5)."""
    phi = np.asarray(phi, dtype=np.float64)
    out = np.empty((plan.M, 5))
    for m in range(plan.M):
        out[m] = plan.fit[m] @ (phi[plan.nbr[m]] - phi[m])
    return out


def cartesian_jumps3(n, t1, t2, S, Phi, dPhi, Psi, dPsi, Fjump, kappa):
    """``([v], [v_x], [v_y], [v_z], [v_xx], [v_yy], [v_zz], [v_xy], [v_xz], [v_yz])``.

    ``dPhi = (Phi_u, Phi_v, Phi_uu, Phi_uv, Phi_vv)`` in the tangent basis,
    ``dPsi = (Psi_u, Psi_v)``, ``S`` the second fundamental form.  The
    tangential block of the Hessian jump is ``Phi_ab + Psi S_ab``, the mixed
    entries ``Psi_a - S_ab Phi_b``, the normal-normal entry closes the trace
    with ``[Lap v] = [F] + kappa Phi``; the Cartesian jumps are the rotation back.
    """
    g = dPhi[..., 0:1] * t1 + dPhi[..., 1:2] * t2 + Psi[..., None] * n
    h11 = dPhi[..., 2] + Psi * S[..., 0, 0]
    h12 = dPhi[..., 3] + Psi * S[..., 0, 1]
    h22 = dPhi[..., 4] + Psi * S[..., 1, 1]
    h1n = dPsi[..., 0] - (S[..., 0, 0] * dPhi[..., 0] + S[..., 0, 1] * dPhi[..., 1])
    h2n = dPsi[..., 1] - (S[..., 1, 0] * dPhi[..., 0] + S[..., 1, 1] * dPhi[..., 1])
    hnn = Fjump + kappa * Phi - h11 - h22

    def outer(a, b):
        return a[..., :, None] * b[..., None, :]

    H = (h11[..., None, None] * outer(t1, t1) + h22[..., None, None] * outer(t2, t2)
         + h12[..., None, None] * (outer(t1, t2) + outer(t2, t1))
         + h1n[..., None, None] * (outer(t1, n) + outer(n, t1))
         + h2n[..., None, None] * (outer(t2, n) + outer(n, t2))
         + hnn[..., None, None] * outer(n, n))
    return np.stack([Phi, g[..., 0], g[..., 1], g[..., 2], H[..., 0, 0], H[..., 1, 1], H[..., 2, 2],
                     H[..., 0, 1], H[..., 0, 2], H[..., 1, 2]], axis=-1)


def jumps(plan: Plan3, phi, f_gamma, kappa):
    """Cartesian jumps at every control point for ``[v] = phi``, ``[F] = f_gamma`` (Dirichlet: ``Psi = 0``)."""
    phi = np.asarray(phi, dtype=np.float64)
    d = surface_derivs(plan, phi)
    Fj = np.zeros(plan.M) if f_gamma is None else np.asarray(f_gamma, dtype=np.float64)
    zero = np.zeros(plan.M)
    return cartesian_jumps3(plan.normal, plan.t1, plan.t2, plan.shape, phi, d, zero, np.zeros((plan.M, 2)),
                            Fj, kappa)


def correction(plan: Plan3, jq: np.ndarray) -> np.ndarray:
    """Correction of the 7-point right-hand side at every irregular node (as in 2D, three axes)."""
    out = np.zeros(len(plan.irr))
    h2 = plan.h * plan.h
    for r, ((i, j, k), arms) in enumerate(zip(plan.irr, plan.arms)):
        s = 1.0 if plan.inside[k, j, i] else -1.0
        acc = 0.0
        for q, d in arms:
            ax = plan.q_axis[q]
            J = jq[q, 0] + d * jq[q, 1 + ax] + 0.5 * d * d * jq[q, 4 + ax]
            acc -= s * J / h2
        out[r] = acc
    return out


def dst_solve3(rhs: np.ndarray, h: float, kappa: float) -> np.ndarray:
    """Solve ``(L_h - kappa) v = rhs`` for the 7-point Laplacian, ``v = 0`` on the cube.

    Eigenvectors are products of ``sin(pi i k / n)``, eigenvalues
    ``l_k + l_l + l_m - kappa`` with ``l_k = -(4/h^2) sin^2(pi k / (2n))``;
    scipy's unnormalised DST-I is twice the sine matrix, so the round trip
    scales by ``1 / (2n)^3``.  ``rhs`` has shape ``(n-1,)*3``.
    """
    n = rhs.shape[0] + 1
    k = np.arange(1, n)
    lam = -(4.0 / (h * h)) * np.sin(np.pi * k / (2.0 * n)) ** 2
    sym = lam[:, None, None] + lam[None, :, None] + lam[None, None, :] - kappa
    hat = sfft.dstn(rhs, type=1)
    return sfft.dstn(hat / sym, type=1) / (2.0 * n) ** 3


def stencil_nodes(plan: Plan3, z: np.ndarray):
    """The ten interpolation nodes (i, j, k) of each point: nearest node, its six
    neighbours, and the diagonal nodes toward the point in the xy, xz, yz planes."""
    h, lo = plan.h, plan.lo
    i0 = np.floor((z - lo) / h + 0.5).astype(np.int64)          # (M, 3)
    sg = np.where(z >= lo + i0 * h, 1, -1)
    offs = [np.array(o) for o in [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]]
    nodes = [i0 + o for o in offs]
    nodes.append(i0 + sg * np.array([1, 1, 0]))
    nodes.append(i0 + sg * np.array([1, 0, 1]))
    nodes.append(i0 + sg * np.array([0, 1, 1]))
    return np.stack(nodes, axis=1)                                # (M, 10, 3)


def interpolate(plan: Plan3, vgrid: np.ndarray, jz: np.ndarray) -> np.ndarray:
    """``v+`` at the control points: values at far-side stencil nodes moved to the
    Omega side with the Taylor expansion of the jumps at the point, then the
    quadratic through the ten values (a 10x10 system per point) evaluated there."""
    z = plan.q_pos
    st = stencil_nodes(plan, z)
    h = plan.h
    P = plan.lo + st * h                                          # (M, 10, 3)
    vals = vgrid[st[..., 2], st[..., 1], st[..., 0]]
    ins = plan.inside[st[..., 2], st[..., 1], st[..., 0]]
    D = P - z[:, None, :]
    J = jz[:, None, :]
    taylor = (J[..., 0] + D[..., 0] * J[..., 1] + D[..., 1] * J[..., 2] + D[..., 2] * J[..., 3]
              + 0.5 * (D[..., 0] ** 2 * J[..., 4] + D[..., 1] ** 2 * J[..., 5] + D[..., 2] ** 2 * J[..., 6])
              + D[..., 0] * D[..., 1] * J[..., 7] + D[..., 0] * D[..., 2] * J[..., 8]
              + D[..., 1] * D[..., 2] * J[..., 9])
    vals = np.where(ins, vals, vals + taylor)
    x, y, w = D[..., 0] / h, D[..., 1] / h, D[..., 2] / h
    A = np.stack([np.ones_like(x), x, y, w, x * x, y * y, w * w, x * y, x * w, y * w], axis=-1)
    coef = np.linalg.solve(A, vals[..., None])[..., 0]
    return coef[:, 0]


def interface_solve_with_jumps(plan: Plan3, jq, ftilde, kappa):
    """Correct, fast-solve and interpolate with given jumps at the control points."""
    n = plan.n
    rhs = np.array(ftilde[1:n, 1:n, 1:n], dtype=np.float64, copy=True)
    corr = correction(plan, jq)
    for (i, j, k), c in zip(plan.irr, corr):
        rhs[k - 1, j - 1, i - 1] += c
    v = np.zeros((n + 1, n + 1, n + 1))
    v[1:n, 1:n, 1:n] = dst_solve3(rhs, plan.h, kappa)
    return v, interpolate(plan, v, jq)


def interface_solve(plan: Plan3, phi, ftilde, f_gamma, kappa):
    jq = jumps(plan, phi, f_gamma, kappa)
    return interface_solve_with_jumps(plan, jq, ftilde, kappa)


def apply_KD(plan: Plan3, phi, kappa):
    """``K_D phi``: the interior limit of the double layer at the control points."""
    zero = np.zeros((plan.n + 1,) * 3)
    return interface_solve(plan, np.asarray(phi, dtype=np.float64), zero, None, kappa)[1]


def zero_extension(plan: Plan3, f_grid):
    ft = np.where(plan.inside, f_grid, 0.0)
    ft[0], ft[-1] = 0.0, 0.0
    ft[:, 0], ft[:, -1] = 0.0, 0.0
    ft[:, :, 0], ft[:, :, -1] = 0.0, 0.0
    return ft


@dataclasses.dataclass
class Solution3:
    u_grid: np.ndarray
    u_gamma: np.ndarray
    phi: np.ndarray
    iters: int
    relres: float
    plan: Plan3


def solve_bvp(plan: Plan3, kappa, f_grid, f_gamma, g, tol=1e-10, restart=50, max_iter=500):
    """``Lap u - kappa u = f`` in the ellipsoid, ``u = g`` at the control points."""
    ft = zero_extension(plan, f_grid)
    _, yf = interface_solve(plan, np.zeros(plan.M), ft, f_gamma, kappa)
    ghat = np.asarray(g, dtype=np.float64) - yf
    phi, it, rel = gmres(lambda p: apply_KD(plan, p, kappa), ghat, tol, restart, max_iter)
    v, ug = interface_solve(plan, phi, ft, f_gamma, kappa)
    return Solution3(np.where(plan.inside, v, 0.0), ug, phi, it, rel, plan)
