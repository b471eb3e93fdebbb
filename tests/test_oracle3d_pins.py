"""Pins of the three-dimensional oracle against what the mathematics fixes.

* the 3D fast solve equals a dense direct solve of the 7-point system;
* the plan's crossing and irregular-node counts equal the brute-force counts
  of the ellipsoid (0.9, 0.7, 0.5) at 64^3 (Q = 6394, I_r = 7352), every
  crossing lies on the surface inside its grid edge;
* Cartesian jumps assembled from the surface data of a quadratic field are
  that field's value, gradient and Hessian;
* the weighted surface fit converges at the expected orders;
* correction + fast solve + interpolation reproduce a piecewise quadratic
  exactly (the 7-point stencil, the Taylor correction and the quadratic fit are
  all exact for quadratics);
* the full Dirichlet solve converges at second order.
"""
import numpy as np
import pytest

import synth
from oracle import kfbi_oracle3d as O3

LO, HI = synth.BOX_LO, synth.BOX_HI
AXES = (0.9, 0.7, 0.5)


def seven_point_matrix(n, h, kappa):
    m = n - 1
    N = m ** 3
    A = np.zeros((N, N))
    idx = lambda i, j, k: (k * m + j) * m + i
    for k in range(m):
        for j in range(m):
            for i in range(m):
                r = idx(i, j, k)
                A[r, r] = -6.0 / (h * h) - kappa
                for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    a, b, c = i + di, j + dj, k + dk
                    if 0 <= a < m and 0 <= b < m and 0 <= c < m:
                        A[r, idx(a, b, c)] = 1.0 / (h * h)
    return A


@pytest.mark.parametrize("kappa", [0.0, 3.0])
def test_dst_solve3_equals_dense_direct_solve(kappa):
    n, h = 6, 0.4
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal((n - 1,) * 3)
    A = seven_point_matrix(n, h, kappa)
    ref = np.linalg.solve(A, rhs.reshape(-1)).reshape(rhs.shape)
    got = O3.dst_solve3(rhs, h, kappa)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.fixture(scope="module")
def plan64():
    return O3.build_plan(64, LO, HI, AXES)


@pytest.fixture(scope="module")
def plan16():
    return O3.build_plan(16, LO, HI, AXES)


def test_plan_counts_match_brute_force(plan64):
    assert plan64.M == 6394
    assert len(plan64.irr) == 7352


def test_crossings_lie_on_the_surface_inside_their_edges(plan64):
    p = plan64
    F = O3.level(p.q_pos, AXES)
    assert np.max(np.abs(F)) < 1e-12
    h = p.h
    for ax in range(3):
        sel = p.q_axis == ax
        t = (p.q_pos[sel, ax] - LO) / h
        other = [(p.q_pos[sel, o] - LO) / h for o in range(3) if o != ax]
        for o in other:                                  # on grid lines in the other two axes
            assert np.max(np.abs(o - np.round(o))) < 1e-9
        assert np.all(t > -1e-9) and np.all(t < p.n + 1e-9)


def surface_data_of_quadratic(p, c0, g0, B, kappa):
    """Phi = q on the surface, Psi = d_n q, their tangential derivatives, [F] = Lap q - kappa q,
    for q(x) = c0 + g0.x + x.B.x / 2 (B symmetric), from the definitions."""
    X = p.q_pos
    q = c0 + X @ g0 + 0.5 * np.einsum("mi,ij,mj->m", X, B, X)
    grad = g0[None, :] + X @ B
    t = np.stack([p.t1, p.t2], axis=1)                    # (M, 2, 3)
    n = p.normal
    dq_t = np.einsum("mai,mi->ma", t, grad)               # t_a . grad q
    dq_n = np.einsum("mi,mi->m", n, grad)
    tBt = np.einsum("mai,ij,mbj->mab", t, B, t)
    tBn = np.einsum("mai,ij,mj->ma", t, B, n)
    S = p.shape
    Phi_ab = tBt - S * dq_n[:, None, None]                # covariant Hessian of q on the surface
    Psi_a = tBn + np.einsum("mab,mb->ma", S, dq_t)        # tangential derivative of d_n q
    dPhi = np.stack([dq_t[:, 0], dq_t[:, 1], Phi_ab[:, 0, 0], Phi_ab[:, 0, 1], Phi_ab[:, 1, 1]], axis=1)
    Fj = np.trace(B) - kappa * q
    return q, grad, dPhi, dq_n, Psi_a, Fj


def random_quadratic(seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((3, 3))
    return rng.standard_normal(), rng.standard_normal(3), B + B.T


@pytest.mark.parametrize("kappa", [0.0, 2.5])
def test_cartesian_jumps_of_a_quadratic_are_its_derivatives(plan16, kappa):
    p = plan16
    c0, g0, B = random_quadratic(11)
    q, grad, dPhi, Psi, dPsi, Fj = surface_data_of_quadratic(p, c0, g0, B, kappa)
    J = O3.cartesian_jumps3(p.normal, p.t1, p.t2, p.shape, q, dPhi, Psi, dPsi, Fj, kappa)
    ref = np.stack([q, grad[:, 0], grad[:, 1], grad[:, 2], np.full_like(q, B[0, 0]), np.full_like(q, B[1, 1]),
                    np.full_like(q, B[2, 2]), np.full_like(q, B[0, 1]), np.full_like(q, B[0, 2]),
                    np.full_like(q, B[1, 2])], axis=1)
    assert np.max(np.abs(J - ref)) < 1e-11


def test_surface_fit_converges():
    c0, g0, B = random_quadratic(4)
    errs = []
    for n in (16, 32, 64):
        p = O3.build_plan(n, LO, HI, AXES)
        q, grad, dPhi, *_ = surface_data_of_quadratic(p, c0, g0, B, 0.0)
        got = O3.surface_derivs(p, q)
        errs.append((np.max(np.abs(got[:, :2] - dPhi[:, :2])), np.max(np.abs(got[:, 2:] - dPhi[:, 2:]))))
    (g16, h16), (g32, h32), (g64, h64) = errs
    assert g32 < g16 / 3.0 and g64 < g32 / 3.0          # gradient O(h^2)
    assert h32 < h16 / 1.6 and h64 < h32 / 1.6          # Hessian O(h)


@pytest.mark.parametrize("kappa", [0.0, 2.0])
def test_piecewise_quadratic_is_reproduced_exactly(plan16, kappa):
    """v = q in Omega, 0 outside: with the exact jumps of q at the crossings the
    corrected 7-point system has exactly that grid function as its solution."""
    p = plan16
    c0, g0, B = random_quadratic(7)
    q, grad, *_ = surface_data_of_quadratic(p, c0, g0, B, kappa)
    jq = np.stack([q, grad[:, 0], grad[:, 1], grad[:, 2], np.full_like(q, B[0, 0]), np.full_like(q, B[1, 1]),
                   np.full_like(q, B[2, 2]), np.full_like(q, B[0, 1]), np.full_like(q, B[0, 2]),
                   np.full_like(q, B[1, 2])], axis=1)
    c = LO + np.arange(p.n + 1) * p.h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    qg = c0 + P @ g0 + 0.5 * np.einsum("...i,ij,...j->...", P, B, P)
    F = np.where(p.inside, np.trace(B) - kappa * qg, 0.0)
    v, vz = O3.interface_solve_with_jumps(p, jq, F, kappa)
    ref = np.where(p.inside, qg, 0.0)
    assert np.max(np.abs(v - ref)) < 1e-11 * max(1.0, np.max(np.abs(qg)))
    assert np.max(np.abs(vz - q)) < 1e-11 * max(1.0, np.max(np.abs(q)))


@pytest.mark.slow
def test_dirichlet_solve_converges_at_second_order():
    errs = []
    for n in (16, 32):
        pr = synth.ellipsoid_problem(n=n)
        plan = O3.build_plan(n, LO, HI, AXES)
        fg, g = pr.boundary_data(plan.q_pos)
        sol = O3.solve_bvp(plan, pr.kappa, pr.f_grid, fg, g, tol=1e-12)
        e = np.max(np.abs(sol.u_grid - pr.exact_grid())[plan.inside])
        errs.append(e)
    assert errs[1] < errs[0] / 3.0, errs
    assert errs[1] < 5e-3, errs                        # |u| reaches e^2.1 on the ellipsoid


def test_stored_128_solution_is_the_manufactured_one_to_second_order():
    """The stored 128^3 oracle solve (tests/golden/make_ellipsoid128.py) is
    pinned to the mathematics, not to the oracle: its trace and its sampled
    node values are e^(x+y+z) up to the discretisation error at that grid
    (the 64^3 error quartered, about 6e-5), its residual is below the stored
    tolerance, and the sampled nodes lie in Omega."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ellipsoid128_oracle.npz")
    ref = np.load(path)
    n = int(ref["n"])
    assert n == 128 and tuple(ref["axes"]) == AXES
    assert float(ref["relres"]) < float(ref["tol"])
    h = (HI - LO) / n
    node = ref["node"]
    i, j, k = node % (n + 1), (node // (n + 1)) % (n + 1), node // (n + 1) ** 2
    x, y, z = LO + i * h, LO + j * h, LO + k * h
    assert np.all(x * x / AXES[0] ** 2 + y * y / AXES[1] ** 2 + z * z / AXES[2] ** 2 < 1.0)
    e_node = np.max(np.abs(ref["u_node"] - np.exp(x + y + z)))
    plan = O3.build_plan(n, LO, HI, AXES)
    q = plan.q_pos
    e_gam = np.max(np.abs(ref["u_gamma"] - np.exp(q[:, 0] + q[:, 1] + q[:, 2])))
    assert len(ref["u_gamma"]) == len(q)
    assert e_node < 2e-4 and e_gam < 2e-4, (e_node, e_gam)
