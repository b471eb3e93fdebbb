"""Plain FP64 CPU oracle of the Gray-Scott time stepping (Example 3).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, the package's smoke check and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library.

What it computes (Tan, Huang & Ying, arXiv 2404.15249, Example 3): the
Gray-Scott system

    u_t = eps1 Lap u + (gamma (1 - u) - u v^2) / eps0
    v_t = eps2 Lap v + (u v^2 - (gamma + kill) v) / eps0

in Omega with ``d_n u = d_n v = 0`` on Gamma, advanced by second-order Strang
splitting.  The paper names the splitting and nothing else; the readings here
(R-21, the same as the HIP library's):

* one step is ``R(dt/2) D(dt) R(dt/2)``: reaction half steps around a full
  diffusion step;
* ``R``: the pointwise reaction ODE, one classical Runge-Kutta step of size
  ``dt/2``, at every grid node in Omega and at every boundary sample (the
  state keeps its trace on Gamma, which the diffusion solve needs as ``[F]``);
* ``D``: Crank-Nicolson for ``w_t = eps Lap w``, written as
  ``w_new = 2 z - w`` with ``z`` the backward-Euler half step
  ``(I - (dt/2) eps Lap) z = w``, i.e. the Neumann problem
  ``Lap z - kappa z = -kappa w``, ``d_n z = 0``, ``kappa = 2 / (eps dt)``
  (Sec. 2 interface problem with the normal-derivative jump as the density);
  GMRES starts from the previous step's density of the same species;
* the half step is solved for the deviation from a constant: with ``c`` the
  mean of the trace of ``w`` at the samples, ``z = c + z'`` and ``z'`` solves
  ``Lap z' - kappa z' = -kappa (w - c)``, ``d_n z' = 0``.  A constant solves
  the Neumann problem exactly, so this is the same ``z``; but the volume
  potential's zero extension (the Sec. 2.2 table) now jumps across Gamma by
  ``kappa (w - c)`` instead of ``kappa w``.  At Example 3's ``kappa h^2`` of
  about 2 the exterior boundary layer of that jump is narrower than a cell,
  and solving for ``z`` itself moved the uniform state ``u = 1`` near Gamma to
  1.24 within eight steps at 128^2;
* grid nodes outside Omega hold zero.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import kfbi_oracle as O


def reaction_rates(u, v, P):
    """Right-hand sides of the reaction ODE at ``(u, v)``."""
    uvv = u * v * v
    return (P.gamma * (1.0 - u) - uvv) / P.eps0, (uvv - (P.gamma + P.kill) * v) / P.eps0


def reaction_step(u, v, dt, P):
    """One classical fourth-order Runge-Kutta step of size ``dt`` of the reaction ODE."""
    a1, b1 = reaction_rates(u, v, P)
    a2, b2 = reaction_rates(u + 0.5 * dt * a1, v + 0.5 * dt * b1, P)
    a3, b3 = reaction_rates(u + 0.5 * dt * a2, v + 0.5 * dt * b2, P)
    a4, b4 = reaction_rates(u + dt * a3, v + dt * b3, P)
    return (u + dt / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4),
            v + dt / 6.0 * (b1 + 2.0 * b2 + 2.0 * b3 + b4))


def diffusion_step(plan, w_grid, w_gamma, eps, dt, psi0=None, tol=1e-10):
    """Crank-Nicolson step of ``w_t = eps Lap w`` with ``d_n w = 0``.

    The half step is solved as ``c + z'`` with ``c`` the trace's mean (module
    docstring).  Returns the new grid (zero outside Omega), the new trace at the
    samples, the Neumann density of the ``z'`` solve and its GMRES iterations.
    """
    kappa = 2.0 / (eps * dt)
    c = np.mean(w_gamma)
    f_grid = np.where(plan.inside, -kappa * (w_grid - c), 0.0)
    sol = O.solve_neumann_on(plan, kappa, f_grid, -kappa * (w_gamma - c), np.zeros(plan.M), tol=tol, psi0=psi0)
    new_grid = np.where(plan.inside, 2.0 * (c + sol.u_grid) - w_grid, 0.0)
    return new_grid, 2.0 * (c + sol.u_gamma) - w_gamma, sol.psi, sol.iters


@dataclasses.dataclass
class GSState:
    u: np.ndarray             # (n+1, n+1), zero outside Omega
    v: np.ndarray
    u_gamma: np.ndarray       # M: trace at the samples
    v_gamma: np.ndarray
    psi_u: np.ndarray         # M: last Neumann densities (the next solves' initial guesses)
    psi_v: np.ndarray
    iters: int = 0            # GMRES iterations so far (both species)


def initial_state(plan, init):
    """The state from ``init(x, y) -> (u, v)`` at the grid nodes in Omega and at the samples."""
    c = plan.coord(np.arange(plan.n + 1))
    X, Y = np.meshgrid(c, c, indexing="xy")
    u, v = init(X, Y)
    ug, vg = init(plan.xy[:, 0], plan.xy[:, 1])
    zero = np.zeros(plan.M)
    return GSState(np.where(plan.inside, u, 0.0), np.where(plan.inside, v, 0.0), ug, vg, zero, zero.copy())


def strang_step(plan, st: GSState, dt, P, tol=1e-10, reaction=True):
    """One step ``R(dt/2) D(dt) R(dt/2)``; ``reaction=False`` leaves only the diffusion step."""
    u, v, ug, vg = st.u, st.v, st.u_gamma, st.v_gamma
    if reaction:
        u, v = reaction_step(u, v, 0.5 * dt, P)
        ug, vg = reaction_step(ug, vg, 0.5 * dt, P)
    u, ug, pu, iu = diffusion_step(plan, np.where(plan.inside, u, 0.0), ug, P.eps1, dt, st.psi_u, tol)
    v, vg, pv, iv = diffusion_step(plan, np.where(plan.inside, v, 0.0), vg, P.eps2, dt, st.psi_v, tol)
    if reaction:
        u, v = reaction_step(u, v, 0.5 * dt, P)
        ug, vg = reaction_step(ug, vg, 0.5 * dt, P)
    return GSState(np.where(plan.inside, u, 0.0), np.where(plan.inside, v, 0.0), ug, vg, pu, pv,
                   st.iters + iu + iv)


def run(plan, st: GSState, dt, steps, P, tol=1e-10, reaction=True):
    for _ in range(steps):
        st = strang_step(plan, st, dt, P, tol, reaction)
    return st
