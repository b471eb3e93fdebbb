"""Plain FP64 CPU oracle of the kernel-free boundary integral (KFBI) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, the package's smoke check and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; the only common module is the seeded input generator ``synth``.

What it computes (Tan, Huang & Ying, "A GPU-accelerated Cartesian grid method
for PDEs on irregular domain", arXiv 2404.15249):

* Sec. 2: the Dirichlet problem ``Lap u - kappa u = f`` in Omega, ``u = g`` on
  Gamma, rewritten as the second-kind equation ``phi/2 + W phi + Y f = g``
  (eq. second_fredholm); ``K_D = I/2 + W`` is the interior limit of the
  double-layer potential.  Both potentials are evaluated through one interface
  problem on the box (eq. interface and the table under it):
  ``Lap v - kappa v = F`` off Gamma, ``[v] = Phi``, ``[d_n v] = 0``, ``v = 0`` on
  the box, with ``(F, Phi) = (0, phi)`` for ``W phi`` and ``(f~, 0)`` for ``Y f``.
* Alg. 1: jumps, correction of the 5-point system at irregular nodes (Alg. 2),
  fast solve (Alg. 4, here a DST-I on both axes: the same discrete system),
  interpolation to the boundary (Alg. 3).
* Alg. 5: restarted GMRES on ``K_D phi = g - (Y f)^+``; the Richardson
  iteration of Sec. 2.1 and BiCGSTAB, the alternatives Table 2 compares.
* The Neumann problem ``d_n u = g_n`` (Sec. 4 procedure, which extracts
  ``d_n u`` instead of ``u+``): the same interface problem with the density as
  the normal-derivative jump, ``K_N psi = d_n v+``, and GMRES on
  ``K_N psi = g_n - d_n (Y f)^+``.
* Sec. 5: the error norms and the relative-residual stopping rule.

The paper defers the discrete details to the first KFBI paper, which is not
part of it.  Where it is silent this oracle takes the following readings (the
same ones the HIP library takes):

R-03 ``n`` is the number of intervals per axis, ``h = (hi-lo)/n``, node
     ``k`` sits at ``lo + k*h``; unknowns are the ``(n-1)^2`` interior nodes.
R-06 Gamma, the density and ``f`` on Gamma are periodic cubic splines in the
     sample index ``t`` (knots at ``t = 0..M-1``).
R-07 Node classification by horizontal scan lines: a node closer than
     ``1e-10 h`` to a crossing lies on Gamma and counts as inside; otherwise
     it is inside iff an odd number of crossings lie left of it.
R-08 Each grid edge whose end nodes differ must hold exactly one crossing and
     no edge may be crossed twice; the curve keeps ``2h`` from the box.
R-09 Jumps: ``[v_tau] = Phi_s``, ``[v_n] = Psi``, ``[v_tautau] = Phi_ss + c Psi``,
     ``[v_taun] = Psi_s - c Phi_s``, ``[v_nn] = [F] + kappa Phi - [v_tautau]``
     (``n`` outward, ``c`` the curvature, positive on convex CCW curves).
R-10 Correction from the second-order Taylor expansion of the jump along the
     grid edge through the crossing.
R-11 The six-point interpolation stencil is the 5-point cross around the
     nearest node plus the diagonal node on the side of the boundary point.
R-13 GMRES(50), modified Gram-Schmidt, Givens rotations, ``phi_0 = 0``.
R-20 Neumann problem: ``[v] = 0``, ``[d_n v] = psi``; ``d_n v+`` is the gradient
     of the six-point quadratic at the sample along the spline's outward
     normal; ``kappa > 0``.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy import fft as sfft
from scipy import linalg as sla

SNAP = 1e-10          # R-07: relative (to h) on-curve tolerance


# ==========================================================================
# periodic cubic spline in the sample index (R-06)
# ==========================================================================

def spline_second_derivs(y: np.ndarray) -> np.ndarray:
    """Second derivatives of the periodic cubic spline through ``y`` at ``t = 0..M-1``.

    Continuity of the first derivative at every knot gives the circulant system
    ``s[m-1] + 4 s[m] + s[m+1] = 6 (y[m+1] - 2 y[m] + y[m-1])``.
    """
    y = np.asarray(y, dtype=np.float64)
    m = y.shape[0]
    if m < 3:
        raise ValueError("need at least 3 boundary samples")
    col = np.zeros(m)
    col[0] = 4.0
    col[1] += 1.0
    col[-1] += 1.0
    rhs = 6.0 * (np.roll(y, -1, axis=0) - 2.0 * y + np.roll(y, 1, axis=0))
    if y.ndim == 1:
        return np.real(sla.solve_circulant(col, rhs))
    return np.stack([np.real(sla.solve_circulant(col, rhs[:, k])) for k in range(y.shape[1])], axis=1)


def spline_eval(y: np.ndarray, s2: np.ndarray, t: np.ndarray):
    """Value and first two ``t``-derivatives of the periodic spline at parameters ``t``.

    On segment ``[m, m+1]`` with ``u = t - m``:
    ``S = (1-u) y0 + u y1 + ((1-u)^3 - (1-u)) s0/6 + (u^3 - u) s1/6``.
    """
    y = np.asarray(y, dtype=np.float64)
    m = y.shape[0]
    t = np.asarray(t, dtype=np.float64)
    fl = np.floor(t)
    u = t - fl
    i0 = fl.astype(np.int64) % m
    i1 = (i0 + 1) % m
    y0, y1, s0, s1 = y[i0], y[i1], s2[i0], s2[i1]
    if y.ndim == 2:
        u = u[..., None]
    w = 1.0 - u
    val = w * y0 + u * y1 + (w ** 3 - w) * s0 / 6.0 + (u ** 3 - u) * s1 / 6.0
    d1 = (y1 - y0) - (3.0 * w * w - 1.0) * s0 / 6.0 + (3.0 * u * u - 1.0) * s1 / 6.0
    d2 = w * s0 + u * s1
    return val, d1, d2


# ==========================================================================
# grid-line crossings of the spline curve
# ==========================================================================

def _segment_poly(y0, y1, s0, s1):
    """Power-basis coefficients (A, B, C, D) of one spline segment in ``u``."""
    return y0, y1 - y0 - s0 / 3.0 - s1 / 6.0, s0 / 2.0, (s1 - s0) / 6.0


def _crossings_of_component(vals: np.ndarray, s2: np.ndarray, levels: np.ndarray):
    """All parameters ``t`` where one coordinate of the curve equals a level.

    Each segment ``[m, m+1)`` is split at the zeros of its derivative into
    monotone pieces; a level reached on a piece is found by bisection.  A piece
    owns the levels in its half-open value range (start included), so a
    crossing exactly at a knot is counted once, by the segment starting there.
    Returns ``(t, level_index)``.
    """
    m = vals.shape[0]
    out_t, out_l = [], []
    for seg in range(m):
        y0, y1 = vals[seg], vals[(seg + 1) % m]
        s0, s1 = s2[seg], s2[(seg + 1) % m]
        A, B, C, D = _segment_poly(y0, y1, s0, s1)
        poly = lambda u: A + u * (B + u * (C + u * D))
        # zeros of B + 2 C u + 3 D u^2 inside (0, 1)
        crit = []
        qa, qb, qc = 3.0 * D, 2.0 * C, B
        if qa != 0.0:
            disc = qb * qb - 4.0 * qa * qc
            if disc >= 0.0:
                sq = np.sqrt(disc)
                crit = [(-qb - sq) / (2 * qa), (-qb + sq) / (2 * qa)]
        elif qb != 0.0:
            crit = [-qc / qb]
        crit = sorted(c for c in crit if 0.0 < c < 1.0)
        knots = [0.0] + crit + [1.0]
        fv = [y0] + [poly(c) for c in crit] + [y1]
        for a, b, fa, fb in zip(knots[:-1], knots[1:], fv[:-1], fv[1:]):
            if fb > fa:
                sel = np.nonzero((levels >= fa) & (levels < fb))[0]
            elif fb < fa:
                sel = np.nonzero((levels <= fa) & (levels > fb))[0]
            else:
                continue
            for li in sel:
                c = levels[li]
                if c == fa:
                    u = a
                else:
                    lo_, hi_ = a, b
                    up = fb > fa
                    for _ in range(80):
                        mid = 0.5 * (lo_ + hi_)
                        if mid <= lo_ or mid >= hi_:
                            break
                        fm = poly(mid)
                        if (fm < c) == up:
                            lo_ = mid
                        else:
                            hi_ = mid
                    u = 0.5 * (lo_ + hi_)
                out_t.append(seg + u)
                out_l.append(li)
    return np.asarray(out_t, dtype=np.float64), np.asarray(out_l, dtype=np.int64)


# ==========================================================================
# geometry plan (Alg. 1 steps 1-3; Sec. 3.1 irregular nodes; Sec. 4 Procedure 1)
# ==========================================================================

class GeometryError(ValueError):
    pass


@dataclasses.dataclass
class Plan:
    n: int
    lo: float
    hi: float
    h: float
    xy: np.ndarray            # (M, 2) samples
    sxy: np.ndarray           # (M, 2) spline second derivatives
    inside: np.ndarray        # (n+1, n+1) bool, [j, i]
    # intersections: one per grid edge whose end nodes differ
    q_axis: np.ndarray        # 0: edge along x (on line y = y_j), 1: edge along y
    q_t: np.ndarray           # spline parameter
    q_xy: np.ndarray          # (Q, 2) position
    q_nodes: np.ndarray       # (Q, 2, 2) the two end nodes (i, j), lower one first
    # irregular nodes and their arms
    irr: np.ndarray           # (I, 2) node (i, j)
    arms: list                # per irregular node: list of (q index, d) with d = xi(other) - xi(q)

    @property
    def M(self):
        return self.xy.shape[0]

    def coord(self, k):
        return self.lo + np.asarray(k) * self.h


def build_plan(xy: np.ndarray, n: int, lo: float, hi: float) -> Plan:
    """Classification, intersections and irregular nodes of the curve through ``xy``."""
    xy = np.asarray(xy, dtype=np.float64)
    h = (hi - lo) / n
    eps = SNAP * h
    sxy = spline_second_derivs(xy)
    grid = lo + np.arange(n + 1) * h

    # crossings with horizontal lines y = y_j (x varies) and vertical lines x = x_i
    th, lh = _crossings_of_component(xy[:, 1], sxy[:, 1], grid)
    tv, lv = _crossings_of_component(xy[:, 0], sxy[:, 0], grid)
    xh = spline_eval(xy[:, 0], sxy[:, 0], th)[0]       # x of crossings on y = y_j
    yv = spline_eval(xy[:, 1], sxy[:, 1], tv)[0]       # y of crossings on x = x_i

    margin_lo, margin_hi = lo + 2.0 * h, hi - 2.0 * h
    allc = np.concatenate([xh, yv, xy[:, 0], xy[:, 1]])
    if np.any(allc < margin_lo) or np.any(allc > margin_hi):
        raise GeometryError("curve within 2h of the box boundary")
    if len(th) == 0:
        raise GeometryError("curve crosses no grid line")

    # R-07: classification along horizontal lines
    inside = np.zeros((n + 1, n + 1), dtype=bool)
    hl = [np.sort(xh[lh == j]) for j in range(n + 1)]
    vl = [np.sort(yv[lv == i]) for i in range(n + 1)]
    for j in range(n + 1):
        xc = hl[j]
        if len(xc) == 0:
            continue
        if len(xc) % 2:
            raise GeometryError("odd number of crossings on a grid line")
        cnt = np.searchsorted(xc, grid, side="left")
        near = np.min(np.abs(grid[:, None] - xc[None, :]), axis=1) <= eps
        inside[j] = near | (cnt % 2 == 1)

    q_axis, q_t, q_xy, q_nodes = [], [], [], []
    # R-08: every edge whose end nodes differ holds exactly one crossing; no
    # edge holds a crossing strictly inside while its end nodes agree.
    for ax, (tt, ll, pos) in enumerate(((th, lh, xh), (tv, lv, yv))):
        for line in range(n + 1):
            sel = ll == line
            ps, ts = pos[sel], tt[sel]
            cls = inside[line, :] if ax == 0 else inside[:, line]
            differ = np.nonzero(cls[:-1] != cls[1:])[0]
            a, b = grid[differ], grid[differ + 1]
            hit = (ps[None, :] >= a[:, None] - eps) & (ps[None, :] <= b[:, None] + eps)
            cnt = hit.sum(axis=1)
            if np.any(cnt != 1):
                e = differ[np.nonzero(cnt != 1)[0][0]]
                raise GeometryError(f"edge {e} on line {line} (axis {ax}) holds "
                                    f"{cnt[np.nonzero(cnt != 1)[0][0]]} crossings")
            for r, e in enumerate(differ):
                k = np.nonzero(hit[r])[0][0]
                q_axis.append(ax)
                q_t.append(ts[k])
                if ax == 0:
                    q_xy.append((ps[k], grid[line]))
                    q_nodes.append(((e, line), (e + 1, line)))
                else:
                    q_xy.append((grid[line], ps[k]))
                    q_nodes.append(((line, e), (line, e + 1)))
            # crossings strictly inside an edge whose end nodes agree
            ec = np.clip(np.floor((ps - lo) / h).astype(np.int64), 0, n - 1)
            for c_e, c_p in zip(ec, ps):
                for e in (c_e - 1, c_e, c_e + 1):
                    if 0 <= e < n and cls[e] == cls[e + 1] and grid[e] + eps < c_p < grid[e + 1] - eps:
                        raise GeometryError(f"edge {e} on line {line} (axis {ax}) crossed twice")

    q_axis = np.asarray(q_axis, dtype=np.int64)
    q_t = np.asarray(q_t, dtype=np.float64)
    q_xy = np.asarray(q_xy, dtype=np.float64).reshape(-1, 2)
    q_nodes = np.asarray(q_nodes, dtype=np.int64).reshape(-1, 2, 2)

    # irregular nodes: a 4-neighbour on the other side of Gamma (Sec. 3.1)
    arms = {}
    for k in range(len(q_t)):
        ax = q_axis[k]
        pa, pb = q_nodes[k]
        for me, other in ((pa, pb), (pb, pa)):
            d = grid[other[ax]] - q_xy[k, ax]
            arms.setdefault((int(me[0]), int(me[1])), []).append((k, d))
    keys = sorted(arms.keys(), key=lambda p: (p[1], p[0]))
    irr = np.asarray(keys, dtype=np.int64).reshape(-1, 2)
    return Plan(n, lo, hi, h, xy, sxy, inside, q_axis, q_t, q_xy, q_nodes, irr,
                [arms[k] for k in keys])


# ==========================================================================
# jumps (Sec. 2.2 interface problem; reading R-09)
# ==========================================================================

def local_geometry(plan: Plan, t):
    """Unit tangent, outward normal, curvature, speed and ``X'.X''`` at parameters ``t``."""
    _, d1, d2 = spline_eval(plan.xy, plan.sxy, t)
    sig = np.hypot(d1[..., 0], d1[..., 1])
    T = d1 / sig[..., None]
    nrm = np.stack([T[..., 1], -T[..., 0]], axis=-1)           # outward for a CCW curve
    curv = (d1[..., 0] * d2[..., 1] - d1[..., 1] * d2[..., 0]) / sig ** 3
    xdx = d1[..., 0] * d2[..., 0] + d1[..., 1] * d2[..., 1]
    return T, nrm, curv, sig, xdx


def cartesian_jumps(T, nrm, curv, Phi, Phi_s, Phi_ss, Psi, Psi_s, Fjump, kappa):
    """``([v], [v_x], [v_y], [v_xx], [v_xy], [v_yy])`` from the interface data.

    ``[v] = Phi``, ``[d_n v] = Psi`` and ``[Lap v - kappa v] = [F]`` along a curve
    with unit tangent ``T``, outward normal ``n`` and curvature ``c``:
    differentiating ``[v]`` and ``[d_n v]`` along arc length gives the tangential
    derivatives, the PDE gives the normal-normal one, and the Cartesian
    gradient and Hessian follow by rotating back.
    """
    v_t = Phi_s
    v_n = Psi
    v_tt = Phi_ss + curv * Psi
    v_tn = Psi_s - curv * Phi_s
    v_nn = Fjump + kappa * Phi - v_tt
    tx, ty = T[..., 0], T[..., 1]
    nx, ny = nrm[..., 0], nrm[..., 1]
    gx = v_t * tx + v_n * nx
    gy = v_t * ty + v_n * ny
    hxx = v_tt * tx * tx + 2.0 * v_tn * tx * nx + v_nn * nx * nx
    hxy = v_tt * tx * ty + v_tn * (tx * ny + nx * ty) + v_nn * nx * ny
    hyy = v_tt * ty * ty + 2.0 * v_tn * ty * ny + v_nn * ny * ny
    return np.stack([np.broadcast_to(Phi, gx.shape), gx, gy, hxx, hxy, hyy], axis=-1)


def jumps_at(plan: Plan, t, phi, f_gamma, kappa, psi=None):
    """Cartesian jumps at curve parameters ``t`` for ``[v] = phi``, ``[d_n v] = psi``, ``[F] = f_gamma``.

    The densities and ``f_gamma`` are sampled at the knots and interpolated by
    the periodic spline; ``None`` stands for zero.  Arc-length derivatives:
    ``Y_s = Y'/sig``, ``Y_ss = Y''/sig^2 - Y' (X'.X'')/sig^4``.  The Dirichlet
    operator has ``psi = 0``; the Neumann operator has ``phi = 0`` (R-20).
    """
    T, nrm, curv, sig, xdx = local_geometry(plan, t)
    zero = np.zeros(np.shape(np.asarray(t, dtype=np.float64)))

    def along(y):
        if y is None:
            return zero, zero, zero
        Y, Y1, Y2 = spline_eval(y, spline_second_derivs(y), t)
        return Y, Y1 / sig, Y2 / sig ** 2 - Y1 * xdx / sig ** 4

    P, Phi_s, Phi_ss = along(phi)
    Psi, Psi_s, _ = along(psi)
    Fj = along(f_gamma)[0]
    return cartesian_jumps(T, nrm, curv, P, Phi_s, Phi_ss, Psi, Psi_s, Fj, kappa)


# ==========================================================================
# correction (Alg. 2)
# ==========================================================================

def correction(plan: Plan, jq: np.ndarray) -> np.ndarray:
    """Correction of the 5-point right-hand side at every irregular node.

    For the arm from node ``a`` to its neighbour ``b`` across Gamma at crossing
    ``q`` (axis ``xi``, ``d = xi(b) - xi(q)``), the jump ``w+ - w-`` continued to
    ``b`` is ``J = [v] + d [v_xi] + d^2 [v_xixi] / 2``; the stencil at ``a``
    then needs ``-s_a J / h^2`` added to its right-hand side (``s_a = +1`` in
    Omega, ``-1`` outside).  Returns one value per irregular node.
    """
    out = np.zeros(len(plan.irr))
    h2 = plan.h * plan.h
    for r, ((i, j), arms) in enumerate(zip(plan.irr, plan.arms)):
        s = 1.0 if plan.inside[j, i] else -1.0
        acc = 0.0
        for k, d in arms:
            ax = plan.q_axis[k]
            J = jq[k, 0] + d * jq[k, 1 + ax] + 0.5 * d * d * jq[k, 3 + 2 * ax]
            acc -= s * J / h2
        out[r] = acc
    return out


# ==========================================================================
# fast solver (Alg. 4; reading R-12: DST-I along both axes)
# ==========================================================================

def dst_solve(rhs: np.ndarray, h: float, kappa: float) -> np.ndarray:
    """Solve ``(L_h - kappa) v = rhs`` on the interior nodes, ``v = 0`` on the box.

    ``L_h`` is the 5-point Laplacian.  Its eigenvectors are ``sin(pi i k / n)``
    with eigenvalues ``-(4/h^2) sin^2(pi k / (2n))``; scipy's unnormalised
    DST-I equals twice the sine matrix, so one forward and one inverse
    transform on both axes scale by ``1/(2n)^2``.
    ``rhs`` has shape ``(n-1, n-1)`` (``[j, i]``).
    """
    n = rhs.shape[0] + 1
    k = np.arange(1, n)
    lam = -(4.0 / (h * h)) * np.sin(np.pi * k / (2.0 * n)) ** 2
    sym = lam[:, None] + lam[None, :] - kappa
    hat = sfft.dst(sfft.dst(rhs, type=1, axis=0), type=1, axis=1)
    return sfft.dst(sfft.dst(hat / sym, type=1, axis=0), type=1, axis=1) / (2.0 * n) ** 2


# ==========================================================================
# interpolation (Alg. 3; reading R-11)
# ==========================================================================

def stencils(plan: Plan, z: np.ndarray):
    """Nearest node and the six stencil nodes (i, j) for boundary points ``z``."""
    h, lo = plan.h, plan.lo
    i0 = np.floor((z[:, 0] - lo) / h + 0.5).astype(np.int64)
    j0 = np.floor((z[:, 1] - lo) / h + 0.5).astype(np.int64)
    sx = np.where(z[:, 0] >= lo + i0 * h, 1, -1)
    sy = np.where(z[:, 1] >= lo + j0 * h, 1, -1)
    offs = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    nodes = [np.stack([i0 + a, j0 + b], axis=1) for a, b in offs]
    nodes.append(np.stack([i0 + sx, j0 + sy], axis=1))
    return np.stack(nodes, axis=1)            # (M, 6, 2)


def local_quadratics(plan: Plan, vgrid: np.ndarray, z: np.ndarray, jz: np.ndarray) -> np.ndarray:
    """Coefficients of the six-point quadratic of the Omega-side solution at each point ``z``.

    Stencil values on the far side of Gamma are moved to the Omega side with
    the Taylor expansion of the jumps at ``z``; the quadratic
    ``c0 + c1 xi + c2 eta + c3 xi^2 + c4 xi eta + c5 eta^2`` in the scaled
    offsets ``xi = (x - z_x)/h``, ``eta = (y - z_y)/h`` through the six values
    is found from a 6x6 linear system per point (Alg. 3).  ``vgrid`` is the
    full ``(n+1, n+1)`` grid (zero on the box).  Returns ``(len(z), 6)``.
    """
    st = stencils(plan, z)
    h = plan.h
    out = np.empty((len(z), 6))
    for m in range(len(z)):
        A = np.empty((6, 6))
        rhs = np.empty(6)
        for k in range(6):
            i, j = st[m, k]
            px, py = plan.coord(i), plan.coord(j)
            val = vgrid[j, i]
            if not plan.inside[j, i]:
                dx, dy = px - z[m, 0], py - z[m, 1]
                J = jz[m]
                val = val + J[0] + dx * J[1] + dy * J[2] + 0.5 * (dx * dx * J[3] + 2 * dx * dy * J[4] + dy * dy * J[5])
            xi, eta = (px - z[m, 0]) / h, (py - z[m, 1]) / h
            A[k] = [1.0, xi, eta, xi * xi, xi * eta, eta * eta]
            rhs[k] = val
        out[m] = np.linalg.solve(A, rhs)
    return out


def interpolate(plan: Plan, vgrid: np.ndarray, z: np.ndarray, jz: np.ndarray) -> np.ndarray:
    """One-sided limit ``v+`` at the boundary points ``z``: the local quadratic at ``z``."""
    return local_quadratics(plan, vgrid, z, jz)[:, 0]


def normal_derivative(plan: Plan, coef: np.ndarray, nrm: np.ndarray) -> np.ndarray:
    """``d_n v+`` at the points of ``coef`` (from ``local_quadratics``): the gradient of
    the local quadratic at its centre, ``(c1, c2)/h``, along the unit normals ``nrm``
    (Alg. 3 extracts the value and its derivatives from the same system)."""
    return (coef[:, 1] * nrm[:, 0] + coef[:, 2] * nrm[:, 1]) / plan.h


# ==========================================================================
# one interface solve (Alg. 1 steps 4-6) and the boundary operator
# ==========================================================================

def grid_solve_with_jumps(plan: Plan, jq, ftilde, kappa):
    """Correct and fast-solve with given jumps at the crossings (Alg. 1 steps 4-5).

    ``ftilde`` is the ``(n+1, n+1)`` base right-hand side (``F``; zero on the
    box).  Returns the full grid solution.
    """
    n = plan.n
    rhs = np.array(ftilde[1:n, 1:n], dtype=np.float64, copy=True)
    corr = correction(plan, jq)
    for (i, j), c in zip(plan.irr, corr):
        rhs[j - 1, i - 1] += c
    v = np.zeros((n + 1, n + 1))
    v[1:n, 1:n] = dst_solve(rhs, plan.h, kappa)
    return v


def interface_solve_with_jumps(plan: Plan, jq, jz, ftilde, kappa):
    """Correct, fast-solve and interpolate with given jumps at crossings and at the samples.

    Returns the full grid solution and ``v+`` at the samples.
    """
    v = grid_solve_with_jumps(plan, jq, ftilde, kappa)
    return v, interpolate(plan, v, plan.xy, jz)


def interface_solve(plan: Plan, phi, ftilde, f_gamma, kappa):
    """Solve the interface problem with ``[v] = phi`` and ``F = ftilde`` (jump ``f_gamma``)."""
    jq = jumps_at(plan, plan.q_t, phi, f_gamma, kappa)
    jz = jumps_at(plan, np.arange(plan.M, dtype=np.float64), phi, f_gamma, kappa)
    return interface_solve_with_jumps(plan, jq, jz, ftilde, kappa)


def apply_KD(plan: Plan, phi, kappa):
    """``K_D phi = (I/2 + W) phi`` at the samples: the interior limit of the double layer."""
    zero = np.zeros((plan.n + 1, plan.n + 1))
    return interface_solve(plan, np.asarray(phi, dtype=np.float64), zero, None, kappa)[1]


def zero_extension(plan: Plan, f_grid):
    """``f~``: ``f`` at nodes in Omega, zero elsewhere and on the box."""
    ft = np.where(plan.inside, f_grid, 0.0)
    ft[0, :] = ft[-1, :] = 0.0
    ft[:, 0] = ft[:, -1] = 0.0
    return ft


# ==========================================================================
# GMRES with restarts (Alg. 5; reading R-13)
# ==========================================================================

def gmres(apply, b, tol=1e-10, restart=50, max_iter=500, x0=None):
    """Restarted GMRES with modified Gram-Schmidt and Givens rotations.

    Stops when ``||b - A x|| / ||b - A x0|| < tol``.  Returns ``(x, iters, relres)``
    with the true relative residual at exit.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x) if x0 is not None else b.copy()
    r0 = np.linalg.norm(r)
    if r0 == 0.0:
        return x, 0, 0.0
    it = 0
    while it < max_iter:
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, len(b)))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for j in range(restart):
            w = apply(V[j])
            it += 1
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                       # previous rotations
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k_used = j + 1
            if abs(g[j + 1]) / r0 < tol or it >= max_iter:
                break
        y = sla.solve_triangular(H[:k_used, :k_used], g[:k_used])
        x = x + V[:k_used].T @ y
        r = b - apply(x)
        rel = np.linalg.norm(r) / r0
        if rel < tol:
            return x, it, rel
    return x, it, np.linalg.norm(b - apply(x)) / r0


# ==========================================================================
# the other outer iterations of Table 2: Richardson (Sec. 2.1) and BiCGSTAB
# ==========================================================================

def richardson(apply, b, gamma=1.0, tol=1e-10, max_iter=500, x0=None):
    """The Richardson iteration of Sec. 2.1: ``x <- x + gamma (b - A x)``.

    Stops when ``||b - A x|| / ||b - A x0|| < tol`` (the residual of the current
    iterate, which the next update needs anyway).  Returns ``(x, iters, relres)``;
    ``iters`` counts the updates made (each costs one apply).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x)
    r0 = np.linalg.norm(r)
    if r0 == 0.0:
        return x, 0, 0.0
    it = 0
    rel = 1.0
    while it < max_iter:
        x = x + gamma * r
        it += 1
        r = b - apply(x)
        rel = np.linalg.norm(r) / r0
        if rel < tol:
            break
    return x, it, rel


def bicgstab(apply, b, tol=1e-10, max_iter=500, x0=None):
    """Unpreconditioned BiCGSTAB (van der Vorst, 1992), shadow residual ``r^ = r_0``.

    Per iteration: ``v = A p``, ``alpha = rho / (r^ . v)``, ``s = r - alpha v``;
    ``t = A s``, ``omega = (t . s) / (t . t)``, ``x += alpha p + omega s``,
    ``r = s - omega t``, ``rho' = r^ . r``, ``p = r + (rho'/rho)(alpha/omega)(p - omega v)``.
    Stops when the updated residual satisfies ``||r|| / ||r_0|| < tol``, or when
    ``||s|| / ||r_0|| < tol`` half way (then ``x += alpha p`` only).  Returns
    ``(x, iters, relres)`` with ``relres`` the true relative residual at exit and
    ``iters`` the iterations begun (two applies each, one if it stopped half way).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x)
    r0 = np.linalg.norm(r)
    if r0 == 0.0:
        return x, 0, 0.0
    rhat = r.copy()
    rho = float(rhat @ r)
    p = r.copy()
    it = 0
    while it < max_iter:
        it += 1
        v = apply(p)
        alpha = rho / float(rhat @ v)
        s = r - alpha * v
        if np.linalg.norm(s) / r0 < tol:
            x = x + alpha * p
            break
        t = apply(s)
        omega = float(t @ s) / float(t @ t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        if np.linalg.norm(r) / r0 < tol:
            break
        rho_new = float(rhat @ r)
        p = r + (rho_new / rho) * (alpha / omega) * (p - omega * v)
        rho = rho_new
    return x, it, np.linalg.norm(b - apply(x)) / r0


# ==========================================================================
# the Dirichlet boundary value problem (Sec. 2.1)
# ==========================================================================

@dataclasses.dataclass
class Solution:
    u_grid: np.ndarray        # (n+1, n+1), zero outside Omega
    u_gamma: np.ndarray       # u+ at the samples
    phi: np.ndarray
    iters: int
    relres: float
    plan: Plan


def solve_bvp(xy, n, lo, hi, kappa, f_grid, f_gamma, g, tol=1e-10, restart=50, max_iter=500,
              method="gmres", relax=1.0):
    """Solve ``Lap u - kappa u = f`` in Omega, ``u = g`` on Gamma by the KFBI method.

    ``g^ = g - (Y f)^+``; GMRES (or ``method`` = ``"bicgstab"``, or
    ``"richardson"`` with ``gamma = relax``: Table 2's alternatives) solves
    ``K_D phi = g^``; the final interface solve with ``[v] = phi`` and ``F = f~``
    gives ``u = W phi + Y f`` on the grid.
    """
    plan = build_plan(xy, n, lo, hi)
    ft = zero_extension(plan, f_grid)
    zeros_m = np.zeros(plan.M)
    _, yf = interface_solve(plan, zeros_m, ft, f_gamma, kappa)
    ghat = np.asarray(g, dtype=np.float64) - yf
    A = lambda p: apply_KD(plan, p, kappa)
    if method == "gmres":
        phi, it, rel = gmres(A, ghat, tol, restart, max_iter)
    elif method == "bicgstab":
        phi, it, rel = bicgstab(A, ghat, tol, max_iter)
    elif method == "richardson":
        phi, it, rel = richardson(A, ghat, relax, tol, max_iter)
    else:
        raise ValueError(f"unknown method {method!r}")
    v, ug = interface_solve(plan, phi, ft, f_gamma, kappa)
    u = np.where(plan.inside, v, 0.0)
    return Solution(u, ug, phi, it, rel, plan)


def error_norms(plan: Plan, u_grid, exact):
    """Max norm and scaled l2 norm of the error over grid nodes in Omega (Sec. 5)."""
    c = plan.coord(np.arange(plan.n + 1))
    X, Y = np.meshgrid(c, c, indexing="xy")
    e = (u_grid - exact(X, Y))[plan.inside]
    return float(np.max(np.abs(e))), float(np.sqrt(np.mean(e * e)))


# ==========================================================================
# the Neumann boundary value problem (Sec. 2 interface problem with a
# normal-derivative jump; Sec. 4 procedure: extract d_n u for Neumann; R-20)
# ==========================================================================

def sample_normals(plan: Plan) -> np.ndarray:
    """Unit outward normals of the spline curve at the samples."""
    return local_geometry(plan, np.arange(plan.M, dtype=np.float64))[1]


def interface_solve_neumann(plan: Plan, psi, ftilde, f_gamma, kappa):
    """Solve the interface problem with ``[v] = 0``, ``[d_n v] = psi`` and ``F = ftilde``.

    ``psi`` (samples, or ``None`` for zero) and ``f_gamma`` (``[F]`` at the
    samples, or ``None``) are splined.  Returns the full grid solution and
    ``v+`` and ``d_n v+`` at the samples.
    """
    t_z = np.arange(plan.M, dtype=np.float64)
    jq = jumps_at(plan, plan.q_t, None, f_gamma, kappa, psi=psi)
    jz = jumps_at(plan, t_z, None, f_gamma, kappa, psi=psi)
    v = grid_solve_with_jumps(plan, jq, ftilde, kappa)
    coef = local_quadratics(plan, v, plan.xy, jz)
    return v, coef[:, 0], normal_derivative(plan, coef, sample_normals(plan))


def apply_KN(plan: Plan, psi, kappa):
    """``K_N psi = d_n v+`` at the samples for ``[v] = 0``, ``[d_n v] = psi``, ``F = 0``.

    ``v`` is a single-layer potential of the box Green's function (up to the
    sign convention of the density), so ``K_N psi = psi/2 - K' psi`` with
    ``K'`` the adjoint double-layer operator: a second-kind operator.
    """
    zero = np.zeros((plan.n + 1, plan.n + 1))
    return interface_solve_neumann(plan, np.asarray(psi, dtype=np.float64), zero, None, kappa)[2]


@dataclasses.dataclass
class NeumannSolution:
    u_grid: np.ndarray        # (n+1, n+1), zero outside Omega
    u_gamma: np.ndarray       # u+ at the samples (the Dirichlet trace, an output here)
    dn_gamma: np.ndarray      # d_n u+ at the samples (reproduces g_N to the GMRES tolerance)
    psi: np.ndarray
    iters: int
    relres: float
    plan: Plan


def solve_neumann(xy, n, lo, hi, kappa, f_grid, f_gamma, g_n, tol=1e-10, restart=50, max_iter=500):
    """Solve ``Lap u - kappa u = f`` in Omega, ``d_n u = g_n`` on Gamma (``kappa > 0``).

    ``u = v_psi + Y f`` with ``v_psi`` the interface solution for ``[v] = 0``,
    ``[d_n v] = psi``; the boundary condition gives the second-kind equation
    ``K_N psi = g_n - d_n (Y f)^+``, solved by GMRES; the final interface solve
    with ``[d_n v] = psi`` and ``F = f~`` gives ``u`` on the grid.  For
    ``kappa = 0`` the interior problem loses uniqueness (constants), so it is
    rejected.
    """
    return solve_neumann_on(build_plan(xy, n, lo, hi), kappa, f_grid, f_gamma, g_n, tol, restart, max_iter)


def solve_neumann_on(plan: Plan, kappa, f_grid, f_gamma, g_n, tol=1e-10, restart=50, max_iter=500, psi0=None):
    """``solve_neumann`` on a built plan, from the initial density ``psi0`` (``None``: zero)."""
    if not kappa > 0.0:
        raise ValueError("the Neumann problem needs kappa > 0")
    ft = zero_extension(plan, f_grid)
    _, _, dyf = interface_solve_neumann(plan, None, ft, f_gamma, kappa)
    ghat = np.asarray(g_n, dtype=np.float64) - dyf
    psi, it, rel = gmres(lambda p: apply_KN(plan, p, kappa), ghat, tol, restart, max_iter, x0=psi0)
    v, ug, dn = interface_solve_neumann(plan, psi, ft, f_gamma, kappa)
    u = np.where(plan.inside, v, 0.0)
    return NeumannSolution(u, ug, dn, psi, it, rel, plan)
