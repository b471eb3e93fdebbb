"""Pins of the Gray-Scott oracle (Example 3, Strang splitting) against closed
forms that do not come from the oracle:

* the reaction step is the classical fourth-order Runge-Kutta method (its
  order, and the steady state (1, 0) kept exactly);
* with the reaction off, a Neumann eigenmode of the disk, J_m(alpha r) cos(m t)
  with J_m'(alpha R) = 0, decays by the Crank-Nicolson factor
  ((1 - a)/(1 + a))^steps, a = eps alpha^2 dt / 2, to the spatial error, and not
  by the exact or the backward-Euler factor;
* with v = 0 the u-equation is linear (rate gamma/eps0) and commutes with the
  diffusion, so a Strang step multiplies u - 1 = c J_0(alpha r) by the CN factor
  times the square of the RK4 factor of a half step: this pins the order of the
  sub-steps and their lengths;
* the uniform state (u, v) = (1, 0) solves the whole system (zero reaction,
  zero Laplacian, zero normal derivative), so the scheme must keep it to
  rounding, and the Crank-Nicolson step is linear and keeps constants, so it
  must commute with adding a constant to the state;
* the maximum principle: Example 3's data has 0 <= v and u <= 1, and for
  u <= 1 the u-reaction gamma (1 - u) - u v^2 <= gamma (1 - u) never pushes u
  above 1, so u must stay at most 1 over the run.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.special import jnp_zeros, jv

import synth
from oracle import gray_scott as G
from oracle import kfbi_oracle as O

R = synth.GS_RADIUS


@pytest.fixture(scope="module")
def plan128():
    return O.build_plan(synth.gray_scott_samples(128), 128, synth.GS_LO, synth.GS_HI)


def test_reaction_step_is_fourth_order_and_keeps_the_steady_state():
    P = synth.GrayScottParams()
    u0, v0 = 0.6, 0.25
    ref = lambda dt: solve_ivp(lambda t, y: G.reaction_rates(y[0], y[1], P), (0, dt), [u0, v0],
                               rtol=1e-13, atol=1e-15, method="DOP853").y[:, -1]
    errs = []
    for dt in (0.02, 0.01, 0.005):
        u, v = G.reaction_step(u0, v0, dt, P)
        errs.append(np.hypot(*(np.array([u, v]) - ref(dt))))
    # local error O(dt^5): halving dt gains about 32
    assert errs[0] / errs[1] > 20 and errs[1] / errs[2] > 20, errs
    u, v = G.reaction_step(np.ones(3), np.zeros(3), 0.3, P)
    assert np.all(u == 1.0) and np.all(v == 0.0)


@pytest.mark.parametrize("gamma,kill", [(0.05, 0.01), (0.03, 0.02)])
def test_reaction_rates_vanish_at_the_steady_states(gamma, kill):
    """Besides (1, 0), the steady states solve u v = gamma + kill and
    (gamma + kill) v^2 - gamma v + gamma (gamma + kill) = 0 (both rates zero);
    the uv^2 terms cancel in the sum of the rates."""
    P = synth.GrayScottParams(gamma=gamma, kill=kill)
    s = gamma + kill
    disc = gamma * gamma - 4.0 * gamma * s * s
    assert disc > 0
    for v in ((gamma + np.sqrt(disc)) / (2 * s), (gamma - np.sqrt(disc)) / (2 * s)):
        a, b = G.reaction_rates(s / v, v, P)
        assert abs(a) < 1e-12 and abs(b) < 1e-12, (a, b)
    a, b = G.reaction_rates(1.0, 0.0, P)
    assert a == 0.0 and b == 0.0
    a, b = G.reaction_rates(0.3, 0.6, P)
    assert a > 0 or b > 0                                  # not trivially zero
    assert abs((a + b) - (gamma * 0.7 - s * 0.6) / P.eps0) < 1e-12


def _grid(plan):
    c = plan.coord(np.arange(plan.n + 1))
    return np.meshgrid(c, c, indexing="xy")


@pytest.mark.parametrize("m,eps", [(0, 0.5), (1, 2.0)])
def test_diffusion_eigenmode_decays_by_the_crank_nicolson_factor(plan128, m, eps):
    al = jnp_zeros(m, 1)[0] / R
    mode = lambda x, y: jv(m, al * np.hypot(x, y)) * np.cos(m * np.arctan2(y, x))
    P = synth.GrayScottParams(eps1=eps, eps2=eps / 2)
    dt, steps = 0.4, 2
    st = G.initial_state(plan128, lambda x, y: (mode(x, y), 0 * x))
    st = G.run(plan128, st, dt, steps, P, tol=1e-12, reaction=False)
    a = eps * al * al * dt / 2
    X, Y = _grid(plan128)
    ins = plan128.inside
    err = lambda f: np.max(np.abs(st.u - f * mode(X, Y))[ins])
    cn, ex, be = ((1 - a) / (1 + a)) ** steps, np.exp(-2 * a * steps), (1 / (1 + 2 * a)) ** steps
    assert err(cn) < 5e-4, err(cn)
    assert err(ex) > 10 * err(cn) and err(be) > 10 * err(cn), (err(cn), err(ex), err(be))
    assert np.max(np.abs(st.u_gamma - cn * mode(plan128.xy[:, 0], plan128.xy[:, 1]))) < 5e-4


def test_strang_step_with_a_linear_reaction(plan128):
    eps, dt, steps = 0.5, 0.4, 2
    P = synth.GrayScottParams(eps1=eps, eps2=eps / 2)
    al = jnp_zeros(0, 1)[0] / R
    mode = lambda x, y: jv(0, al * np.hypot(x, y))
    st = G.initial_state(plan128, lambda x, y: (1 + 0.5 * mode(x, y), 0 * x))
    st = G.run(plan128, st, dt, steps, P, tol=1e-12)
    z = -(P.gamma / P.eps0) * dt / 2
    rk = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24          # RK4 on y' = lambda y, one half step
    a = eps * al * al * dt / 2
    cn = (1 - a) / (1 + a)
    X, Y = _grid(plan128)
    ins = plan128.inside
    err = lambda f: np.max(np.abs(st.u - 1 - 0.5 * f ** steps * mode(X, Y))[ins])
    assert np.all(st.v == 0.0)
    assert err(cn * rk * rk) < 1e-3, err(cn * rk * rk)
    zx, zy = plan128.xy[:, 0], plan128.xy[:, 1]
    assert np.max(np.abs(st.u_gamma - 1 - 0.5 * (cn * rk * rk) ** steps * mode(zx, zy))) < 1e-3
    # whole steps of reaction on both sides, or no reaction, are far off
    assert err(cn * rk ** 4) > 5 * err(cn * rk * rk) and err(cn) > 5 * err(cn * rk * rk)


def test_gray_scott_state_stays_bounded_and_symmetric(plan128):
    """The Example 3 data at 128^2, two steps of dt = 1/8: v stays in [0, 1], and the
    state keeps the symmetry of the data and the disk under x -> -x."""
    P = synth.GrayScottParams()
    st = G.initial_state(plan128, synth.gray_scott_initial)
    st = G.run(plan128, st, 0.125, 2, P, tol=1e-10)
    ins = plan128.inside
    assert np.all(st.v[ins] >= -1e-12) and np.all(st.v[ins] <= 1.0)
    assert np.max(np.abs(st.v - st.v[:, ::-1])) < 1e-8
    assert np.max(np.abs(st.u - st.u[:, ::-1])) < 1e-8


def test_uniform_steady_state_is_kept_exactly(plan128):
    """(1, 0) at Example 3's parameters, 128^2, dt = 1/8, T = 1 (kappa h^2 about 2
    for u): every value stays 1 (u) and 0 (v) to rounding, on the grid and at
    the samples."""
    P = synth.GrayScottParams()
    st = G.initial_state(plan128, lambda x, y: (np.ones_like(x), np.zeros_like(x)))
    st = G.run(plan128, st, 0.125, 8, P, tol=1e-10)
    ins = plan128.inside
    assert np.max(np.abs(st.u[ins] - 1.0)) < 1e-12, np.max(np.abs(st.u[ins] - 1.0))
    assert np.max(np.abs(st.u_gamma - 1.0)) < 1e-12
    assert np.max(np.abs(st.v[ins])) < 1e-12 and np.max(np.abs(st.v_gamma)) < 1e-12
    assert np.all(st.u[~ins] == 0.0)


def test_diffusion_step_commutes_with_adding_a_constant(plan128):
    """D(w + a) = D(w) + a on the grid in Omega and at the samples, for a smooth
    non-constant w (a Neumann eigenmode plus a tilt) and a = 0.7."""
    al = jnp_zeros(2, 1)[0] / R
    X, Y = _grid(plan128)
    w = lambda x, y: jv(2, al * np.hypot(x, y)) * np.cos(2 * np.arctan2(y, x)) + 0.1 * x
    ins = plan128.inside
    wg, wz = np.where(ins, w(X, Y), 0.0), w(plan128.xy[:, 0], plan128.xy[:, 1])
    a = 0.7
    g0, z0, _, _ = G.diffusion_step(plan128, wg, wz, 0.05, 0.25, tol=1e-13)
    g1, z1, _, _ = G.diffusion_step(plan128, np.where(ins, wg + a, 0.0), wz + a, 0.05, 0.25, tol=1e-13)
    assert np.max(np.abs(g1 - a - g0)[ins]) < 1e-10, np.max(np.abs(g1 - a - g0)[ins])
    assert np.max(np.abs(z1 - a - z0)) < 1e-10
    # the step did something (not the identity, not a constant)
    assert np.max(np.abs(g0 - wg)[ins]) > 1e-3


def test_example3_keeps_u_at_most_one_over_unit_time(plan128):
    """Example 3's data and parameters at 128^2, 8 steps of dt = 1/8 (T = 1),
    GMRES tol 1e-8: u <= 1 + 1e-8 and v >= -1e-12 everywhere, on the grid and
    at the samples."""
    P = synth.GrayScottParams()
    st = G.initial_state(plan128, synth.gray_scott_initial)
    st = G.run(plan128, st, 0.125, 8, P, tol=1e-8)
    ins = plan128.inside
    assert st.u[ins].max() <= 1.0 + 1e-8, st.u[ins].max()
    assert st.u_gamma.max() <= 1.0 + 1e-8, st.u_gamma.max()
    assert st.v[ins].min() >= -1e-12 and st.v_gamma.min() >= -1e-12
    # the pattern evolved (not a frozen state)
    assert st.u[ins].min() < 0.5 and st.v[ins].max() > 0.2
