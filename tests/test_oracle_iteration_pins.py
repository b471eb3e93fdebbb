"""Pins of the oracle's Richardson iteration (Sec. 2.1) and BiCGSTAB (Table 2's
alternatives to GMRES): the Richardson iterate in closed form, its divergence
past the convergent range of gamma, BiCGSTAB's iterates against SciPy's
implementation of the same method, and both against a dense LU solve of the
assembled K_D."""
import numpy as np
import pytest
from scipy.sparse.linalg import bicgstab as scipy_bicgstab

import synth
from oracle import kfbi_oracle as O

LO, HI = synth.BOX_LO, synth.BOX_HI


def _matrix(n=12, seed=3):
    rng = np.random.default_rng(seed)
    return np.eye(n) * 0.75 + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n), rng.standard_normal(n)


@pytest.mark.parametrize("gamma,k", [(1.0, 5), (0.6, 9)])
def test_richardson_iterate_in_closed_form(gamma, k):
    """From x0 = 0, k updates give x_k = sum_{j<k} (I - gamma A)^j gamma b."""
    A, b = _matrix()
    x, it, _ = O.richardson(lambda v: A @ v, b, gamma, tol=0.0, max_iter=k)
    G = np.eye(len(b)) - gamma * A
    ref = sum(np.linalg.matrix_power(G, j) @ (gamma * b) for j in range(k))
    assert it == k
    assert np.max(np.abs(x - ref)) < 1e-13 * np.max(np.abs(ref)) * 10


def test_richardson_diverges_outside_the_contraction_range():
    """With eigenvalues of A in [0.5, 1], gamma = 3 makes |1 - gamma lambda| > 1."""
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    A = Q @ np.diag(np.linspace(0.5, 1.0, 10)) @ Q.T
    b = rng.standard_normal(10)
    _, _, rel_bad = O.richardson(lambda v: A @ v, b, 3.0, tol=0.0, max_iter=30)
    x, _, rel_ok = O.richardson(lambda v: A @ v, b, 1.0, tol=1e-12, max_iter=200)
    assert rel_bad > 1e3 and rel_ok < 1e-12
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-10)


def test_bicgstab_iterates_match_scipy():
    A, b = _matrix(16, 5)
    mine = []
    for k in range(1, 5):
        x, it, _ = O.bicgstab(lambda v: A @ v, b, tol=0.0, max_iter=k)
        assert it == k
        mine.append(x)
    theirs = []
    scipy_bicgstab(A, b, rtol=0.0, atol=0.0, maxiter=4, callback=lambda xk: theirs.append(xk.copy()))
    assert len(theirs) == 4
    for a, c in zip(mine, theirs):
        assert np.max(np.abs(a - c)) < 1e-12 * np.max(np.abs(c))


def test_bicgstab_and_richardson_on_KD_match_a_dense_solve():
    """The 128x128 K_D of the circle (r = 0.8, Laplace) assembled column by column."""
    p = synth.circle_problem(n=64, m=128)
    plan = O.build_plan(p.xy, p.n, LO, HI)
    K = np.stack([O.apply_KD(plan, e, 0.0) for e in np.eye(plan.M)], axis=1)
    b = synth.smooth_density(plan.M, 7)
    ref = np.linalg.solve(K, b)
    A = lambda v: O.apply_KD(plan, v, 0.0)
    x1, it1, rel1 = O.bicgstab(A, b, tol=1e-13)
    x2, it2, rel2 = O.richardson(A, b, 1.0, tol=1e-13, max_iter=400)
    for x, rel in ((x1, rel1), (x2, rel2)):
        assert rel < 1e-12
        assert np.max(np.abs(x - ref)) < 1e-10 * np.max(np.abs(ref))
    # Table 2's ordering on this operator: GMRES needs the fewest applies
    _, itg, _ = O.gmres(A, b, tol=1e-13)
    assert itg < 2 * it1 and itg < it2


@pytest.mark.parametrize("method", ["bicgstab", "richardson"])
def test_solve_bvp_with_each_method_gives_the_gmres_solution(method):
    p = synth.make_problem("circle r=1", synth.circle_points(128, 1.0), 256, 0.0, synth.PAPER_EX1)
    ref = O.solve_bvp(p.xy, p.n, p.lo, p.hi, 0.0, p.f_grid, p.f_gamma, p.g, tol=1e-12)
    s = O.solve_bvp(p.xy, p.n, p.lo, p.hi, 0.0, p.f_grid, p.f_gamma, p.g, tol=1e-12, method=method)
    assert s.relres < 1e-12
    assert np.max(np.abs(s.u_grid - ref.u_grid)) < 1e-9
