"""FP32 grid solves with FP64 refinement, against the FP64 oracle (through the C ABI).

The dense grid solves (volume potential and final solution of a Dirichlet
solve, and the fast-solve step entry) run their column sine transforms in FP32
and correct them with FP64 residuals; everything else stays FP64.  The bar is
an L-infinity error of at most 1e-6 against the FP64 oracle on the same
discretisation, stated for every case.  Errors are printed so that each run
records them.
"""
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


def test_fast_solve_refinement_reaches_fp64(K, ctx):
    """Alg. 4 on a random right-hand side: each refinement step shrinks the error."""
    p = synth.circle_problem(n=256, m=256, kappa=1.0)
    rng = np.random.default_rng(7)
    rhs = np.zeros((p.n + 1, p.n + 1))
    rhs[1:-1, 1:-1] = rng.standard_normal((p.n - 1, p.n - 1))
    ref = O.dst_solve(rhs[1:-1, 1:-1], (HI - LO) / p.n, p.kappa)
    scale = np.max(np.abs(ref))
    errs = []
    for steps in (0, 1, 2):
        prob = K.Problem(ctx, p.xy, p.n, p.kappa, precision="fp32", refine_steps=steps)
        v = host(prob.fast_solve(dev(rhs)))
        err = float(np.max(np.abs(v[1:-1, 1:-1] - ref)) / scale)
        note(f"fast solve n=256 fp32, {steps} refine steps: relative Linf error {err:.3e}")
        errs.append(err)
    assert errs[0] < 1e-5
    assert errs[1] < 1e-9 and errs[1] < errs[0] * 1e-3
    assert errs[2] < 1e-12


def inside_linf(u, ref, mask):
    return float(np.max(np.abs(np.where(mask, u - ref, 0.0))))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("n", [2048, 4096])
@pytest.mark.parametrize("kappa", [0.0, 1.0, 100.0])
def test_circle_solve_fp32_refined_vs_oracle(K, ctx, n, kappa):
    """Circle r = 0.8, M = N (samples about 2h apart), u = e^x sin y: the
    FP32-refined solve and the FP64 solve against the oracle at the full sizes
    (L-infinity, absolute)."""
    p = synth.circle_problem(n=n, m=n, kappa=kappa)
    note(f"mixed-precision solve {p.name}")
    ref = O.solve_bvp(p.xy, p.n, LO, HI, p.kappa, p.f_grid, p.f_gamma, p.g, tol=1e-12)
    out = {}
    for prec in ("fp64", "fp32"):
        prob = K.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-12, precision=prec)
        mask = prob.mask()
        u, ug, phi, it, rel, conv = prob.solve(dev(p.f_grid), dev(p.f_gamma), dev(p.g))
        u, ug = host(u), host(ug)
        e_grid = inside_linf(u, ref.u_grid, mask)
        e_gam = float(np.max(np.abs(ug - ref.u_gamma)))
        c = LO + np.arange(n + 1) * ((HI - LO) / n)
        e_true = inside_linf(u, p.exact.u(*np.meshgrid(c, c)), mask)
        note(f"  {prec}: iters {it} relres {rel:.2e}  Linf vs oracle grid {e_grid:.3e} gamma {e_gam:.3e}"
             f"  Linf vs exact {e_true:.3e}")
        assert conv
        out[prec] = (e_grid, e_gam)
    assert max(out["fp32"]) <= 1e-6
    scale = max(np.max(np.abs(ref.u_grid)), 1.0)
    assert max(out["fp64"]) <= 1e-10 * scale
