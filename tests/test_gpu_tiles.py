"""Launch shapes: every valid shape of the sparse fast solve (sine modes per
workgroup) and of the column transforms gives the oracle's K_D apply and grid
solve (1e-12 relative: only the grouping of partial sums changes), and the
autotuner returns one of them."""
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


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("n", [64, 512, 2048])
def test_every_apply_shape_matches_oracle(K, ctx, n):
    p = synth.star_problem(n=n, kappa=1.0, m=max(64, n // 2))
    print(f"apply shapes {p.name}", flush=True)
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    plan = O.build_plan(p.xy, p.n, LO, HI)
    phi = synth.smooth_density(plan.M, 1234)
    ref = O.apply_KD(plan, phi, p.kappa)
    dst = prob.tiles()["dst_cols"]
    tried = 0
    for r in (1, 2, 4, 8, 16):
        try:
            prob.set_tiles(r, dst)
        except K.KfbiError:
            continue
        assert relerr(host(prob.apply(dev(phi))), ref) < 1e-12, r
        tried += 1
    assert tried >= 2

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_transform_tile_matches_oracle(K, ctx, precision):
    n = 256
    prob = K.Problem(ctx, synth.circle_points(2 * n, 0.8), n, 1.0, precision=precision, refine_steps=2)
    print(f"transform tiles n={n} {precision}", flush=True)
    rng = np.random.default_rng(3)
    rhs = rng.standard_normal((n + 1, n + 1))
    ref = np.zeros_like(rhs)
    ref[1:n, 1:n] = O.dst_solve(rhs[1:n, 1:n], (HI - LO) / n, 1.0)
    t = prob.tiles()
    tol = 1e-12 if precision == "fp64" else 1e-10
    tried = []
    for b in (4, 8, 16, 32, 64):
        try:
            prob.set_tiles(t["modes_per_group"], b)
        except K.KfbiError:
            continue
        assert relerr(host(prob.fast_solve(dev(rhs))), ref) < tol, b
        tried.append(b)
    # 16-byte pairs (FP64) also take the wide tiles of 32 and 64 columns
    assert tried == ([4, 8, 16, 32, 64] if precision == "fp64" else [4, 8, 16]), tried


@pytest.mark.parametrize("n", [64, 128])
def test_short_columns_fast_solve_matches_oracle(K, ctx, n):
    """Grids of 64 rows take the transform with one wavefront per column pair
    (128 the tiled one): both against the oracle's DST-I solve."""
    prob = K.Problem(ctx, synth.circle_points(2 * n, 0.8), n, 1.0)
    print(f"short columns n={n}", flush=True)
    rng = np.random.default_rng(n)
    rhs = rng.standard_normal((n + 1, n + 1))
    ref = np.zeros_like(rhs)
    ref[1:n, 1:n] = O.dst_solve(rhs[1:n, 1:n], (HI - LO) / n, 1.0)
    assert relerr(host(prob.fast_solve(dev(rhs))), ref) < 1e-12


def test_invalid_shapes_are_refused(K, ctx):
    p = synth.circle_problem(n=64, m=128)
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    t = prob.tiles()
    for bad in [(3, 8), (0, 8), (32, 8), (t["modes_per_group"], 2), (t["modes_per_group"], 12),
                (t["modes_per_group"], 128)]:
        with pytest.raises(K.KfbiError):
            prob.set_tiles(*bad)
    assert prob.tiles()["modes_per_group"] == t["modes_per_group"]


def test_autotune_picks_a_valid_shape_and_keeps_results(K, ctx):
    p = synth.star_problem(n=512, kappa=1.0)
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    phi = dev(synth.smooth_density(prob.M, 7))
    before = host(prob.apply(phi))
    t = prob.autotune(reps=3)
    print(f"autotune star512: {t}", flush=True)
    assert t["apply_us"] > 0 and t["grid_solve_us"] > 0
    prob.set_tiles(t["modes_per_group"], t["dst_cols"])   # the choice is itself valid
    assert relerr(host(prob.apply(phi)), before) < 1e-12
