"""GPU parity of the Neumann problem (density = jump of the normal derivative,
d_n u+ extracted from the six-point quadratic) against the FP64 oracle, through
the C ABI: the K_N apply to relative 1e-12 (circle, star, and the 2048^2 star
grid of the benchmark), the full-grid interface solve with all three outputs,
the whole Neumann solve to relative 1e-10, Green's identity between the
library's K_D and K_N, and second-order convergence on the GPU.

Tolerance of a normal derivative: d_n v+ is a combination of six grid values
with weights of size 1/h, so the rounding of the grid solution (relative
~1e-14 of its largest value, from the different summation orders) reaches
d_n v+ multiplied by about 3/h; relative to the largest output the bar is
1e-12 max(1, n/256).  Values (v+, the grid) keep 1e-12."""
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


def dn_tol(n):
    return 1e-12 * max(1.0, n / 256.0)


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


CASES = {
    "circle64": lambda: synth.circle_neumann_problem(n=64, m=128, kappa=1.0),
    "circle128_k3": lambda: synth.circle_neumann_problem(n=128, m=200, kappa=3.0),
    "star512": lambda: synth.star_neumann_problem(n=512, kappa=1.0),
    "star2048": lambda: synth.star_neumann_problem(n=2048, kappa=1.0),
}

_plans = {}


def oracle_plan(name, p):
    if name not in _plans:
        _plans[name] = O.build_plan(p.xy, p.n, LO, HI)
    return _plans[name]


@pytest.mark.parametrize("name", list(CASES))
def test_apply_neumann_matches_oracle(K, ctx, name):
    p = CASES[name]()
    note(f"K_N apply parity {name}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    plan = oracle_plan(name, p)
    for seed in (1234, 99):
        psi = synth.smooth_density(plan.M, seed)
        got = host(prob.apply_neumann(dev(psi)))
        ref = O.apply_KN(plan, psi, p.kappa)
        assert relerr(got, ref) < dn_tol(p.n), seed


def test_apply_neumann_at_the_largest_grid(K, ctx):
    """4096^2 (the largest grid the library takes), 2048 samples."""
    p = synth.star_neumann_problem(n=4096, kappa=1.0)
    note("K_N apply parity star4096")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    plan = O.build_plan(p.xy, p.n, LO, HI)
    psi = synth.smooth_density(plan.M, 8)
    assert relerr(host(prob.apply_neumann(dev(psi))), O.apply_KN(plan, psi, p.kappa)) < dn_tol(p.n)


def test_apply_neumann_laplace(K, ctx):
    """The operator itself is defined for kappa = 0 as well."""
    p = CASES["circle64"]()
    note("K_N apply parity circle64 kappa=0")
    prob = K.Problem(ctx, p.xy, p.n, 0.0)
    plan = oracle_plan("circle64", p)
    psi = synth.smooth_density(plan.M, 5)
    assert relerr(host(prob.apply_neumann(dev(psi))), O.apply_KN(plan, psi, 0.0)) < dn_tol(p.n)


def test_apply_neumann_sparse_equals_dense_path(K, ctx):
    p = CASES["star512"]()
    note("K_N sparse vs dense star512")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    psi = dev(synth.smooth_density(prob.M, 5))
    a = host(prob.apply_neumann(psi))
    _, _, b = prob.interface_solve_neumann(psi, dev(np.zeros((p.n + 1, p.n + 1))))
    assert relerr(a, host(b)) < dn_tol(p.n)


@pytest.mark.parametrize("name", ["circle64", "star512"])
def test_interface_solve_neumann_matches_oracle(K, ctx, name):
    """psi, a right-hand side that is f inside and zero outside, and its jump:
    the grid, v+ and d_n v+."""
    p = CASES[name]()
    note(f"Neumann interface solve parity {name}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    plan = oracle_plan(name, p)
    psi = synth.smooth_density(plan.M, 31)
    ft = O.zero_extension(plan, p.f_grid)
    vg, vz, dn = prob.interface_solve_neumann(dev(psi), dev(ft), dev(p.f_gamma))
    rv, rz, rdn = O.interface_solve_neumann(plan, psi, ft, p.f_gamma, p.kappa)
    assert relerr(host(vg), rv) < 1e-12
    assert relerr(host(vz), rz) < 1e-12
    assert relerr(host(dn), rdn) < dn_tol(p.n)


def test_green_identity_of_the_library_operators(K, ctx):
    """<K_D phi, psi> + <phi, K_N psi> = <phi, psi> on Gamma up to truncation
    error, with both operators from the library on the 2048^2 star grid."""
    p = CASES["star2048"]()
    note("Green identity star2048")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    plan = oracle_plan("star2048", p)
    phi, psi = synth.smooth_density(plan.M, 11), synth.smooth_density(plan.M, 22)
    kd = host(prob.apply(dev(phi)))
    kn = host(prob.apply_neumann(dev(psi)))
    sig = O.local_geometry(plan, np.arange(plan.M, dtype=np.float64))[3]
    ip = lambda a, b: float(np.sum(a * b * sig))
    d = abs(ip(kd, psi) + ip(phi, kn) - ip(phi, psi)) / np.sqrt(ip(phi, phi) * ip(psi, psi))
    note(f"  relative defect {d:.2e}")
    assert d < 1e-5


@pytest.mark.parametrize("name", ["circle64", "star512", "star2048"])
def test_solve_neumann_matches_oracle(K, ctx, name):
    p = CASES[name]()
    note(f"Neumann solve parity {name}")
    tol = 1e-13 if p.n < 2048 else 1e-12
    prob = K.Problem(ctx, p.xy, p.n, p.kappa, tol=tol)
    u, ug, dn, psi, it, rel, conv = prob.solve_neumann(dev(p.f_grid), dev(p.f_gamma), dev(p.g_n))
    ref = O.solve_neumann(p.xy, p.n, LO, HI, p.kappa, p.f_grid, p.f_gamma, p.g_n, tol=tol)
    note(f"  iters gpu {it} ({rel:.2e}) oracle {ref.iters} ({ref.relres:.2e})")
    assert conv and rel < tol
    assert abs(it - ref.iters) <= 2
    assert relerr(host(psi), ref.psi) < 1e-10
    assert relerr(host(u), ref.u_grid) < 1e-10
    assert relerr(host(ug), ref.u_gamma) < 1e-10
    assert relerr(host(dn), ref.dn_gamma) < 1e-10


@pytest.mark.parametrize("name", ["circle64", "star512"])
def test_gmres_neumann_fused_and_separate_corrections_agree(K, ctx, name):
    """The emit launch's corrections of the next K_N input (outside timing mode)
    and the separate correction launch (timing mode) give the same iterate
    across a restart."""
    p = CASES[name]()
    note(f"Neumann fused corrections {name}")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    rhs = dev(p.g_n)
    prob.set_timing(False)
    a, it_a, *_ = prob.gmres_neumann(rhs, tol=0.0, max_iter=60)
    prob.set_timing(True)
    b, it_b, *_ = prob.gmres_neumann(rhs, tol=0.0, max_iter=60)
    prob.set_timing(False)
    assert it_a == it_b == 60
    assert relerr(host(a), host(b)) < 1e-13


def test_dirichlet_and_neumann_share_a_problem(K, ctx):
    """Both operators' GMRES graphs live side by side on one problem: solving
    Dirichlet, then Neumann, then Dirichlet again repeats the first result."""
    p = CASES["star512"]()
    note("Dirichlet / Neumann interleaved star512")
    prob = K.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-12)
    a = prob.solve(dev(p.f_grid), dev(p.f_gamma), dev(p.g))
    n1 = prob.solve_neumann(dev(p.f_grid), dev(p.f_gamma), dev(p.g_n))
    b = prob.solve(dev(p.f_grid), dev(p.f_gamma), dev(p.g))
    assert a[5] and n1[6] and b[5]
    assert np.array_equal(host(a[0]), host(b[0]))
    # the two solves describe the same u
    mask = prob.mask().astype(bool)
    assert np.max(np.abs(host(a[0]) - host(n1[0]))[mask]) < 1e-3


def test_solve_neumann_rejects_kappa_zero(K, ctx):
    p = synth.circle_neumann_problem(n=64, m=128, kappa=0.0)
    prob = K.Problem(ctx, p.xy, p.n, 0.0)
    with pytest.raises(K.KfbiError):
        prob.solve_neumann(dev(p.f_grid), dev(p.f_gamma), dev(p.g_n))


def test_neumann_second_order_on_the_gpu(K, ctx):
    errs = []
    for n in (128, 256, 512, 1024):
        p = synth.circle_neumann_problem(n=n, m=2 * n, kappa=1.0)
        prob = K.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-11)
        u, ug, dn, psi, it, rel, conv = prob.solve_neumann(dev(p.f_grid), dev(p.f_gamma), dev(p.g_n))
        assert conv
        c = LO + np.arange(n + 1) * p.h
        X, Y = np.meshgrid(c, c, indexing="xy")
        mask = prob.mask().astype(bool)
        errs.append(float(np.max(np.abs(host(u) - p.exact.u(X, Y))[mask])))
        note(f"  n={n}: iters {it}, Linf error {errs[-1]:.3e}, |d_n u - g_n| {np.max(np.abs(host(dn) - p.g_n)):.1e}")
    # second order: the least-squares slope of log error against log h over the
    # four grids, and the error over three doublings (64 for exact second order;
    # the local ratios move with how the circle meets each grid)
    slope = -np.polyfit(np.log2([128, 256, 512, 1024]), np.log2(errs), 1)[0]
    note(f"  fitted order {slope:.2f}, error ratio over three doublings {errs[0] / errs[-1]:.1f}")
    assert slope > 1.8, (slope, errs)
    assert errs[0] / errs[-1] > 40.0, errs
