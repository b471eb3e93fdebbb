"""Pins of the Neumann part of the FP64 oracle (the interface problem with the
density as the normal-derivative jump, the normal derivative from the six-point
quadratic, the operator K_N and the Neumann boundary value problem), each
against something other than the oracle itself:

* exactness on piecewise quadratics (the extraction is exact there);
* a manufactured interface problem with ``[v] = 0`` and ``[d_n v] = Psi != 0``
  built from a level-set function, converging at second order (any dropped or
  mis-signed Psi term in the jumps costs an order);
* Green's second identity on both sides of Gamma, which ties K_N to the
  already pinned K_D: ``<K_D phi, psi> + <phi, K_N psi> = <phi, psi>`` on Gamma;
* manufactured Neumann problems converging at second order.
"""
import numpy as np
import pytest

import synth
from oracle import kfbi_oracle as O

LO, HI = synth.BOX_LO, synth.BOX_HI
L = HI - LO


def _quad(x, y):
    v = 0.3 + 1.1 * x - 0.6 * y + 0.9 * x * x - 0.8 * x * y + 0.45 * y * y
    return np.stack([v, 1.1 + 1.8 * x - 0.8 * y, -0.6 - 0.8 * x + 0.9 * y,
                     1.8 + 0 * x, -0.8 + 0 * x, 0.9 + 0 * x], axis=-1)


@pytest.mark.parametrize("domain", ["circle", "star"])
@pytest.mark.parametrize("kappa", [0.0, 3.0])
def test_normal_derivative_exact_on_piecewise_quadratics(domain, kappa):
    """v+ = q (quadratic), v- = 0, exact jumps: the extracted d_n v+ is grad q . n."""
    n = 64 if domain == "circle" else 128
    xy = synth.circle_points(128, 0.8) if domain == "circle" else synth.star_points(160)
    plan = O.build_plan(xy, n, LO, HI)
    c = plan.coord(np.arange(n + 1))
    X, Y = np.meshgrid(c, c, indexing="xy")
    Q = _quad(X, Y)
    F = Q[..., 3] + Q[..., 5] - kappa * Q[..., 0]
    jq = _quad(plan.q_xy[:, 0], plan.q_xy[:, 1])
    jz = _quad(plan.xy[:, 0], plan.xy[:, 1])
    v = O.grid_solve_with_jumps(plan, jq, O.zero_extension(plan, F), kappa)
    nrm = O.sample_normals(plan)
    coef = O.local_quadratics(plan, v, plan.xy, jz)
    dn = O.normal_derivative(plan, coef, nrm)
    assert np.max(np.abs(dn - (jz[:, 1] * nrm[:, 0] + jz[:, 2] * nrm[:, 1]))) < 1e-9
    assert np.max(np.abs(coef[:, 0] - jz[:, 0])) < 1e-11
    if domain == "circle":          # the spline normal is the circle's to spline accuracy
        assert np.max(np.abs(nrm - synth.circle_normals(plan.xy))) < 1e-6


# --------------------------------------------------------------------------
# a manufactured interface problem with a normal-derivative jump
# --------------------------------------------------------------------------
# Ellipse rho = x^2/a^2 + y^2/b^2 - 1 = 0, sampled at uniform angle (uneven
# speed).  Outside v = B (zero on the box); inside v = B + rho A, so [v] = 0 and
# [d_n v] = A |grad rho| on Gamma; F = Lap v - kappa v on each side.

EA, EB = 0.87, 0.53


def _B(x, y):
    k = np.pi / L
    cx, cy, sx, sy = np.cos(k * x), np.cos(k * y), np.sin(k * x), np.sin(k * y)
    v = cx * cy * (1 + 0.3 * x)
    gx = cy * (-k * sx * (1 + 0.3 * x) + 0.3 * cx)
    gy = -k * sy * cx * (1 + 0.3 * x)
    lap = cy * (-k * k * cx * (1 + 0.3 * x) - 0.6 * k * sx) - k * k * v
    return v, gx, gy, lap


def _A(x, y):
    return 0.5 + 0.4 * x - 0.3 * y * y, 0.4 + 0 * x, -0.6 * y, -0.6 + 0 * x


def _rho(x, y):
    return x * x / EA ** 2 + y * y / EB ** 2 - 1.0, 2 * x / EA ** 2, 2 * y / EB ** 2, 2 / EA ** 2 + 2 / EB ** 2


def _inside(x, y):
    b, bx, by, bl = _B(x, y)
    a, ax, ay, al = _A(x, y)
    r, rx, ry, rl = _rho(x, y)
    return b + r * a, bx + rx * a + r * ax, by + ry * a + r * ay, bl + a * rl + 2 * (rx * ax + ry * ay) + r * al


def test_manufactured_interface_problem_with_normal_jump_is_second_order():
    kappa = 1.3
    eg, ev, ed = [], [], []
    for n in (64, 128, 256):
        m = 4 * n
        th = 2 * np.pi * np.arange(m) / m
        xy = np.stack([EA * np.cos(th), EB * np.sin(th)], 1)
        plan = O.build_plan(xy, n, LO, HI)
        c = plan.coord(np.arange(n + 1))
        X, Y = np.meshgrid(c, c, indexing="xy")
        vin, _, _, lin = _inside(X, Y)
        vout, _, _, lout = _B(X, Y)
        ft = np.where(plan.inside, lin - kappa * vin, lout - kappa * vout)
        ft[0, :] = ft[-1, :] = ft[:, 0] = ft[:, -1] = 0.0
        zx, zy = xy[:, 0], xy[:, 1]
        zin, zinx, ziny, zinl = _inside(zx, zy)
        zb, zbx, zby, zbl = _B(zx, zy)
        _, rx, ry, _ = _rho(zx, zy)
        psi = _A(zx, zy)[0] * np.hypot(rx, ry)
        fj = (zinl - kappa * zin) - (zbl - kappa * zb)
        v, vp, dn = O.interface_solve_neumann(plan, psi, ft, fj, kappa)
        exact = np.where(plan.inside, vin, vout)
        nrm = O.sample_normals(plan)
        eg.append(np.max(np.abs(v - exact)))
        ev.append(np.max(np.abs(vp - zb)))
        ed.append(np.max(np.abs(dn - (zinx * nrm[:, 0] + ziny * nrm[:, 1]))))
    for e in (eg, ev, ed):
        assert e[0] / e[1] > 3.3 and e[1] / e[2] > 3.3, (eg, ev, ed)
    assert eg[-1] < 2e-5 and ed[-1] < 2e-4, (eg, ed)


# --------------------------------------------------------------------------
# Green's second identity: K_N against the pinned K_D
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kappa", [0.0, 2.0])
def test_green_identity_ties_KN_to_KD(kappa):
    """With a = v_phi ([a] = phi, [d_n a] = 0) and b = v_psi ([b] = 0, [d_n b] = psi),
    Green's second identity on Omega and on B \\ Omega (both vanish on the box)
    gives <a+, psi> + <phi, d_n b+> = <phi, psi> on Gamma.  The defect of the
    discrete operators is their truncation error."""
    defects = []
    for n in (128, 512):
        m = 2 * n
        plan = O.build_plan(synth.circle_points(m, 0.8), n, LO, HI)
        phi, psi = synth.smooth_density(m, 11), synth.smooth_density(m, 22)
        kd, kn = O.apply_KD(plan, phi, kappa), O.apply_KN(plan, psi, kappa)
        sig = O.local_geometry(plan, np.arange(m, dtype=np.float64))[3]   # ds = |X'| dt
        ip = lambda a, b: float(np.sum(a * b * sig))
        scale = np.sqrt(ip(phi, phi) * ip(psi, psi))
        assert abs(ip(phi, kn)) > 0.02 * scale                # K_N psi is not trivially small
        defects.append(abs(ip(kd, psi) + ip(phi, kn) - ip(phi, psi)) / scale)
    assert defects[1] < 5e-7 and defects[0] / defects[1] > 8.0, defects


# --------------------------------------------------------------------------
# the Neumann boundary value problem
# --------------------------------------------------------------------------

def _neumann_errors(p):
    s = O.solve_neumann(p.xy, p.n, p.lo, p.hi, p.kappa, p.f_grid, p.f_gamma, p.g_n, tol=1e-10)
    c = p.lo + np.arange(p.n + 1) * p.h
    X, Y = np.meshgrid(c, c, indexing="xy")
    e = float(np.max(np.abs(s.u_grid - p.exact.u(X, Y))[s.plan.inside]))
    return s, e


def test_neumann_circle_second_order():
    errs = []
    for n in (32, 64, 128, 256):
        p = synth.circle_neumann_problem(n=n, m=2 * n, kappa=1.0)
        s, e = _neumann_errors(p)
        assert s.relres < 1e-10
        assert np.max(np.abs(s.dn_gamma - p.g_n)) < 1e-8      # the boundary condition holds
        assert np.max(np.abs(s.u_gamma - p.g)) < 4.0 * e + 1e-12
        errs.append(e)
    # the local order varies with how the circle meets the grid; over three
    # halvings the error falls well beyond first order (8x) towards 64x
    assert errs[-1] < 2e-5 and errs[0] / errs[-1] > 40.0, errs


def test_neumann_star_modified_helmholtz():
    errs = []
    for n in (256, 512):
        p = synth.star_neumann_problem(n=n, kappa=1.0)
        s, e = _neumann_errors(p)
        assert s.relres < 1e-10 and s.iters < 40
        errs.append(e)
    assert errs[-1] < 4e-4 and errs[0] / errs[1] > 4.0, errs


def test_neumann_needs_positive_kappa():
    p = synth.circle_neumann_problem(n=32, m=64, kappa=1.0)
    with pytest.raises(ValueError):
        O.solve_neumann(p.xy, p.n, p.lo, p.hi, 0.0, p.f_grid, p.f_gamma, p.g_n)
