"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Tolerances: the FP64 path must match the oracle to relative 1e-10 end to end;
a single K_D apply or fast solve to 1e-12 relative to the largest output
(different summation orders only).  Integer and index work (classification,
crossing sets, irregular nodes) must match exactly.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import kfbi_oracle as O

pytestmark = pytest.mark.gpu

LO, HI = synth.BOX_LO, synth.BOX_HI


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


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


CASES = {
    "circle64": lambda: synth.circle_problem(n=64, m=128),
    "circle128_k3": lambda: synth.circle_problem(n=128, m=200, kappa=3.0),
    "star256": lambda: synth.star_problem(n=256, kappa=1.0),
    "star512": lambda: synth.star_problem(n=512, kappa=1.0),
}


# --------------------------------------------------------------------------- plan

@pytest.mark.parametrize("name", list(CASES))
def test_plan_matches_oracle(K, ctx, name):
    p = CASES[name]()
    note(f"plan parity {name}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    plan = O.build_plan(p.xy, p.n, LO, HI)
    assert np.array_equal(prob.mask(), plan.inside)
    axis, nodes, t, xy = prob.crossings()
    assert prob.Q == len(plan.q_t) and prob.I == len(plan.irr)
    key = lambda ax, nd: (int(ax), *map(int, nd))
    mine = {key(a, nd): (tt, pp) for a, nd, tt, pp in zip(axis, nodes, t, xy)}
    theirs = {key(a, nd.reshape(-1)): (tt, pp) for a, nd, tt, pp in zip(plan.q_axis, plan.q_nodes, plan.q_t, plan.q_xy)}
    assert mine.keys() == theirs.keys()
    for k in mine:
        assert abs(mine[k][0] - theirs[k][0]) < 1e-12
        assert np.max(np.abs(mine[k][1] - theirs[k][1])) < 1e-13
    ij = prob.irregular()
    assert sorted(map(tuple, ij)) == sorted(map(tuple, plan.irr))


def test_geometry_errors(K, ctx):
    with pytest.raises(K.GeometryError):
        K.Problem(ctx, synth.circle_points(64, 1.15), 64, 0.0)
    with pytest.raises(K.KfbiError):
        K.Problem(ctx, synth.circle_points(64, 0.8), 100, 0.0)          # not a power of two


# --------------------------------------------------------------------------- steps

@pytest.mark.parametrize("name", ["circle64", "star512"])
def test_correction_matches_oracle(K, ctx, name):
    p = CASES[name]()
    note(f"correction parity {name}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    plan = O.build_plan(p.xy, p.n, LO, HI)
    phi = synth.smooth_density(plan.M, 1234)
    for fg in (None, p.f_gamma):
        ref = O.correction(plan, O.jumps_at(plan, plan.q_t, phi, fg, p.kappa))
        got = host(prob.correct(dev(phi), None if fg is None else dev(fg)))
        order = {tuple(x): k for k, x in enumerate(map(tuple, plan.irr))}
        perm = [order[tuple(x)] for x in prob.irregular()]
        assert relerr(got, ref[perm]) < 1e-12


@pytest.mark.parametrize("n,kappa", [(64, 0.0), (128, 1.0), (512, 100.0), (1024, 1.0)])
def test_fast_solve_matches_oracle(K, ctx, n, kappa):
    note(f"fast solve n={n} kappa={kappa}")
    prob = K.Problem(ctx, synth.circle_points(2 * n, 0.8), n, kappa)
    rng = np.random.default_rng(n)
    rhs = rng.standard_normal((n + 1, n + 1))
    rhs[n // 3, n // 5] = 50.0
    got = host(prob.fast_solve(dev(rhs)))
    ref = np.zeros_like(rhs)
    ref[1:n, 1:n] = O.dst_solve(rhs[1:n, 1:n], (HI - LO) / n, kappa)
    assert relerr(got, ref) < 1e-12


def _quad(x, y):
    v = 0.3 + 1.1 * x - 0.6 * y + 0.9 * x * x - 0.8 * x * y + 0.45 * y * y
    return np.stack([v, 1.1 + 1.8 * x - 0.8 * y, -0.6 - 0.8 * x + 0.9 * y,
                     1.8 + 0 * x, -0.8 + 0 * x, 0.9 + 0 * x], axis=-1)


@pytest.mark.parametrize("name", ["circle64", "star256"])
def test_quadratic_exactness_on_gpu(K, ctx, name):
    p = CASES[name]()
    note(f"quadratic exactness {name}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    mask = prob.mask()
    axis, nodes, t, qxy = prob.crossings()
    c = LO + np.arange(p.n + 1) * (HI - LO) / p.n
    X, Y = np.meshgrid(c, c, indexing="xy")
    Q = _quad(X, Y)
    F = np.where(mask, Q[..., 3] + Q[..., 5] - p.kappa * Q[..., 0], 0.0)
    vg, vz = prob.interface_solve_jumps(dev(_quad(qxy[:, 0], qxy[:, 1])), dev(_quad(p.xy[:, 0], p.xy[:, 1])), dev(F))
    expect = np.where(mask, Q[..., 0], 0.0)
    expect[0, :] = expect[-1, :] = expect[:, 0] = expect[:, -1] = 0.0
    assert np.max(np.abs(host(vg) - expect)) < 1e-11
    assert np.max(np.abs(host(vz) - _quad(p.xy[:, 0], p.xy[:, 1])[:, 0])) < 1e-11


# --------------------------------------------------------------------------- the operator

@pytest.mark.parametrize("name", list(CASES))
def test_apply_matches_oracle(K, ctx, name):
    p = CASES[name]()
    note(f"K_D apply parity {name}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    plan = O.build_plan(p.xy, p.n, LO, HI)
    for seed in (1234, 99):
        phi = synth.smooth_density(plan.M, seed)
        got = host(prob.apply(dev(phi)))
        ref = O.apply_KD(plan, phi, p.kappa)
        assert relerr(got, ref) < 1e-12, seed


def test_apply_sparse_equals_dense_path(K, ctx):
    p = CASES["star256"]()
    note("sparse vs dense apply star256")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    phi = dev(synth.smooth_density(prob.M, 5))
    a = host(prob.apply(phi))
    _, b = prob.interface_solve(phi, dev(np.zeros((p.n + 1, p.n + 1))))
    assert relerr(a, host(b)) < 1e-12


@pytest.mark.parametrize("name", ["circle64", "star512"])
def test_KD_one_is_one(K, ctx, name):
    p = CASES[name]()
    note(f"K_D(1)=1 {name}")
    prob = K.Problem(ctx, p.xy, p.n, 0.0)
    out = host(prob.apply(dev(np.ones(prob.M))))
    assert np.max(np.abs(out - 1.0)) < 1e-12


# --------------------------------------------------------------------------- solve

@pytest.mark.parametrize("name", ["circle64", "star256"])
def test_solve_matches_oracle(K, ctx, name):
    p = CASES[name]()
    note(f"solve parity {name}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-13)
    u, ug, phi, it, rel, conv = prob.solve(dev(p.f_grid), dev(p.f_gamma), dev(p.g))
    ref = O.solve_bvp(p.xy, p.n, LO, HI, p.kappa, p.f_grid, p.f_gamma, p.g, tol=1e-13)
    assert conv and rel < 1e-13
    assert relerr(host(phi), ref.phi) < 1e-10
    assert relerr(host(u), ref.u_grid) < 1e-10
    assert relerr(host(ug), ref.u_gamma) < 1e-10
    assert abs(it - ref.iters) <= 2


@pytest.mark.parametrize("name", ["circle64", "star512"])
def test_gmres_with_corrections_in_the_emit_launch(K, ctx, name):
    """Outside timing mode each GMRES step's emit launch also makes the next
    apply's corrections from its own window of the next input; with timing on
    they come from a separate correction launch.  Both runs, across a restart
    (60 steps with restart 50), give the same iterate."""
    p = CASES[name]()
    note(f"fused corrections {name}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    rhs = dev(p.g)
    prob.set_timing(False)
    a, it_a, *_ = prob.gmres(rhs, tol=0.0, max_iter=60)
    prob.set_timing(True)
    b, it_b, *_ = prob.gmres(rhs, tol=0.0, max_iter=60)
    prob.set_timing(False)
    assert it_a == it_b == 60
    assert relerr(host(a), host(b)) < 1e-13


@pytest.mark.parametrize("name", ["circle64", "star512"])
def test_gmres_from_a_nonzero_guess_matches_oracle(K, ctx, name):
    """GMRES warm-started from a smooth density (the first step is then a
    residual apply) against the oracle's GMRES from the same guess, and the
    count of K_D applications: Arnoldi steps plus one residual apply per cycle
    end, plus the initial residual apply only for a nonzero guess."""
    p = CASES[name]()
    note(f"warm-started GMRES {name}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    plan = O.build_plan(p.xy, p.n, LO, HI)
    x0 = synth.smooth_density(prob.M, 99)
    rhs = p.g
    phi, it, ap, rel, conv = prob.gmres(dev(rhs), phi0=dev(x0), tol=1e-12)
    ref, rit, rrel = O.gmres(lambda v: O.apply_KD(plan, v, p.kappa), rhs, tol=1e-13, x0=x0)
    note(f"  gpu {it} iterations / {ap} applies ({rel:.2e}), oracle {rit} ({rrel:.2e})")
    assert conv and abs(it - rit) <= 2
    assert relerr(host(phi), ref) < 1e-10
    # fixed work: 60 steps with restart 50 cross one restart
    _, it0, ap0, _, _ = prob.gmres(dev(rhs), tol=0.0, max_iter=60)
    _, it1, ap1, _, _ = prob.gmres(dev(rhs), phi0=dev(x0), tol=0.0, max_iter=60)
    assert (it0, ap0) == (60, 62) and (it1, ap1) == (60, 63), (it0, ap0, it1, ap1)
    _, it2, ap2, _, _ = prob.gmres(dev(rhs), tol=0.0, max_iter=20)
    assert (it2, ap2) == (20, 21), (it2, ap2)


@pytest.mark.parametrize("eta", [0.0, 1.0])
def test_solve_with_and_without_the_second_gram_schmidt_pass(K, ctx, eta):
    """The second Gram-Schmidt pass, made on every step (eta = 1, by the
    committing workgroup) or never (eta = 0), gives the oracle's solution and
    iteration count, as the default threshold does."""
    p = CASES["star512"]()
    note(f"solve with reorth eta={eta}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-12)
    prob.set_reorth(eta)
    u, ug, phi, it, rel, conv = prob.solve(dev(p.f_grid), dev(p.f_gamma), dev(p.g))
    ref = O.solve_bvp(p.xy, p.n, LO, HI, p.kappa, p.f_grid, p.f_gamma, p.g, tol=1e-12)
    assert conv and rel < 1e-12 and abs(it - ref.iters) <= 1
    assert relerr(host(u), ref.u_grid) < 1e-10
    assert relerr(host(phi), ref.phi) < 1e-10
    with pytest.raises(K.KfbiError):
        prob.set_reorth(1.5)
