"""NaN and Inf in the caller's data, through the C ABI: every call that meets
one returns KFBI_ERR_NONFINITE (-6) and writes none of its outputs (they keep
a sentinel value), and the same problem handle then solves clean data as
before.  A NaN outside Omega in f is ignored, as the header states.
"""
import ctypes as ct
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

NONFINITE = -6
SENTINEL = 7.25


@pytest.fixture(scope="module")
def K():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_15249_amd import kfbi
    return kfbi


@pytest.fixture(scope="module")
def ctx(K):
    return K.Context(0)


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def filled(shape):
    import torch
    if isinstance(shape, int):
        shape = (shape,)
    return torch.full(tuple(shape), SENTINEL, dtype=torch.float64, device="cuda:0")


def untouched(*ts):
    import torch
    torch.cuda.synchronize()
    return all(bool((t == SENTINEL).all()) for t in ts)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def P(t):
    return ct.c_void_p(t.data_ptr())


def with_bad(a, k, value=np.nan):
    b = np.array(a, dtype=np.float64, copy=True)
    b.flat[k] = value
    return b


@pytest.fixture(scope="module")
def circle(K, ctx):
    p = synth.circle_problem(n=64, m=128, kappa=1.0)
    return p, K.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-12)


def call_solve(K, ctx, prob, f, fg, g, phi):
    n1 = prob.n + 1
    u, ug = filled((n1, n1)), filled(prob.M)
    it, rel = ct.c_int(-1), ct.c_double(-1.0)
    with ctx:
        st = K._lib.kfbi_solve(prob._h, P(f), P(fg), P(g), P(u), P(ug), P(phi), ct.byref(it), ct.byref(rel))
    return st, u, ug


@pytest.mark.parametrize("where", ["g", "f_gamma", "f_inside", "phi0"])
def test_solve_reports_nonfinite_and_writes_nothing(K, ctx, circle, where):
    p, prob = circle
    f, fg, g = p.f_grid, p.f_gamma, p.g
    phi0 = np.zeros(prob.M)
    mask = prob.mask()
    if where == "g":
        g = with_bad(g, 17)
    elif where == "f_gamma":
        fg = with_bad(fg, 3, np.inf)
    elif where == "f_inside":
        j, i = np.argwhere(mask)[len(np.argwhere(mask)) // 2]
        f = with_bad(f, j * (p.n + 1) + i)
    else:
        phi0 = with_bad(phi0, 5)
    note(f"kfbi_solve with a non-finite value in {where}")
    phi = dev(phi0)
    phi_before = phi.clone()
    st, u, ug = call_solve(K, ctx, prob, dev(f), dev(fg), dev(g), phi)
    assert st == NONFINITE, st
    assert untouched(u, ug)
    assert np.array_equal(phi.cpu().numpy(), phi_before.cpu().numpy(), equal_nan=True)
    # the handle still solves clean data
    st, u, ug = call_solve(K, ctx, prob, dev(p.f_grid), dev(p.f_gamma), dev(p.g), dev(np.zeros(prob.M)))
    assert st == 0, st


def test_nan_outside_omega_in_f_is_ignored(K, ctx, circle):
    p, prob = circle
    mask = prob.mask()
    j, i = np.argwhere(~mask)[0]
    f = with_bad(p.f_grid, j * (p.n + 1) + i)
    st, u, ug = call_solve(K, ctx, prob, dev(f), dev(p.f_gamma), dev(p.g), dev(np.zeros(prob.M)))
    assert st == 0, st
    st2, u2, ug2 = call_solve(K, ctx, prob, dev(p.f_grid), dev(p.f_gamma), dev(p.g), dev(np.zeros(prob.M)))
    assert st2 == 0 and np.array_equal(u.cpu().numpy(), u2.cpu().numpy())


def test_apply_reports_nonfinite_and_writes_nothing(K, ctx, circle):
    p, prob = circle
    phi = synth.smooth_density(prob.M, 1234)
    for fn in ("kfbi_apply", "kfbi_apply_neumann"):
        out = filled(prob.M)
        bad, good = dev(with_bad(phi, 40)), dev(phi)       # kept alive across the calls
        with ctx:
            st = getattr(K._lib, fn)(prob._h, P(bad), P(out))
        assert st == NONFINITE, (fn, st)
        assert untouched(out), fn
        with ctx:
            st = getattr(K._lib, fn)(prob._h, P(good), P(out))
        assert st == 0 and np.all(np.isfinite(out.cpu().numpy())), fn


@pytest.mark.parametrize("method", ["kfbi_gmres", "kfbi_bicgstab", "kfbi_richardson"])
def test_outer_iterations_report_nonfinite(K, ctx, circle, method):
    p, prob = circle
    rhs = dev(with_bad(p.g, 60, -np.inf))
    x = filled(prob.M)
    x0 = x.clone()
    it, ap, rel = ct.c_int(), ct.c_int(), ct.c_double()
    with ctx:
        if method == "kfbi_richardson":
            st = K._lib.kfbi_richardson(prob._h, P(rhs), P(x), 1.0, 1e-10, 50, ct.byref(it), ct.byref(rel))
        else:
            st = getattr(K._lib, method)(prob._h, P(rhs), P(x), 1e-10, 50, ct.byref(it), ct.byref(ap),
                                         ct.byref(rel))
    note(f"{method}: status {st}")
    assert st == NONFINITE, st
    assert untouched(x) and bool((x == x0).all())


def test_neumann_solve_reports_nonfinite(K, ctx):
    p = synth.circle_neumann_problem(n=64, m=128, kappa=1.0)
    prob = K.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-12)
    n1 = p.n + 1
    u, ug, dn = filled((n1, n1)), filled(prob.M), filled(prob.M)
    psi = filled(prob.M)
    it, rel = ct.c_int(), ct.c_double()
    f, fg, gn = dev(p.f_grid), dev(p.f_gamma), dev(with_bad(p.g_n, 9))
    with ctx:
        st = K._lib.kfbi_solve_neumann(prob._h, P(f), P(fg), P(gn), P(u), P(ug), P(dn), P(psi), ct.byref(it),
                                       ct.byref(rel))
    assert st == NONFINITE, st
    assert untouched(u, ug, dn, psi)


def test_surface_problem_reports_nonfinite(K, ctx):
    prob = K.Problem3(ctx, 64, (0.9, 0.7, 0.5))
    pts, _ = prob.points()
    phi = synth.smooth_density3(pts, 1234)
    out = filled(prob.M)
    bad = dev(with_bad(phi, 100))
    with ctx:
        st = K._lib.kfbi3_apply(prob._h, P(bad), P(out))
    assert st == NONFINITE and untouched(out)
    p3 = synth.ellipsoid_problem(64)
    fg, g = p3.boundary_data(pts)
    n1 = 65
    u, ug, ph = filled((n1, n1, n1)), filled(prob.M), filled(prob.M)
    it, rel = ct.c_int(), ct.c_double()
    f3, fg3, g3 = dev(p3.f_grid), dev(fg), dev(with_bad(g, 1))
    with ctx:
        st = K._lib.kfbi3_solve(prob._h, P(f3), P(fg3), P(g3), P(u), P(ug), P(ph), ct.byref(it), ct.byref(rel))
    assert st == NONFINITE and untouched(u, ug, ph)


def test_batch_slot_with_nan_stops_and_others_converge(K, ctx):
    good = synth.star_problem(n=256, kappa=1.0)
    bad = synth.circle_problem(n=128, m=256, kappa=3.0)
    batch = K.Batch(ctx, max_slots=4, m_max=1024)
    pg = K.Problem(ctx, good.xy, good.n, good.kappa, tol=1e-12)
    pb = K.Problem(ctx, bad.xy, bad.n, bad.kappa, tol=1e-12)
    sg = batch.admit(pg, dev(good.f_grid), dev(good.f_gamma), dev(good.g))
    sb = batch.admit(pb, dev(bad.f_grid), dev(bad.f_gamma), dev(with_bad(bad.g, 0)))
    state = None
    for _ in range(100):
        batch.step(8)
        state, it, rel = batch.poll()
        if state[sg] != 0 and state[sb] != 0:
            break
    note(f"batch states: good {state[sg]}, NaN request {state[sb]}")
    assert state[sb] == -3 and state[sg] == 1
    with pytest.raises(K.NonfiniteError):
        batch.finish(sb)
    u, ug, phi, _ = batch.finish(sg)
    u1, ug1, phi1, _, _, conv = pg.solve(dev(good.f_grid), dev(good.f_gamma), dev(good.g))
    assert conv
    ref = u1.cpu().numpy()
    assert np.max(np.abs(u.cpu().numpy() - ref)) <= 1e-11 * np.max(np.abs(ref))
    info_live = ct.c_int()
    K._lib.kfbi_batch_info(batch._h, ct.byref(info_live), None)
    assert info_live.value == 0
    batch.close()
