"""kfbi_apply_noalloc through the C ABI: the K_D apply with the library's
static scratch array in place of the problem's workspace.  Its output equals
kfbi_apply's on two calls in a row (the second on a smaller problem, so
stale scratch from the first would show), it leaves the device's free memory
unchanged, it refuses a problem whose scratch exceeds the array, and a NaN in
the density leaves the output untouched.
"""
import ctypes as ct
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

UNSUPPORTED = -7


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


def P(t):
    return ct.c_void_p(t.data_ptr())


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def noalloc(K, ctx, prob, phi, out):
    with ctx:
        return K._lib.kfbi_apply_noalloc(prob._h, P(phi), P(out))


def test_noalloc_apply_matches_apply_on_two_calls(K, ctx):
    import torch
    cases = [synth.star_problem(n=2048, kappa=1.0), synth.circle_problem(n=256, m=512, kappa=3.0)]
    probs = [K.Problem(ctx, p.xy, p.n, p.kappa) for p in cases]
    phis = [dev(synth.smooth_density(q.M, 1234 + k)) for k, q in enumerate(probs)]
    refs = [q.apply(phi) for q, phi in zip(probs, phis)]
    outs = [torch.full((q.M,), 7.25, dtype=torch.float64, device="cuda:0") for q in probs]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    for q, phi, out, ref, p in zip(probs, phis, outs, refs, cases):     # large first, then small
        note(f"kfbi_apply_noalloc on {p.name} (M={q.M})")
        assert noalloc(K, ctx, q, phi, out) == 0
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        err = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        note(f"  relative difference from kfbi_apply {err:.2e}, bitwise equal {np.array_equal(a, b)}")
        assert err <= 1e-13
    assert torch.cuda.mem_get_info(0)[0] == free0          # nothing was allocated on the device
    # the large problem again after the small one
    outs[0].fill_(7.25)
    assert noalloc(K, ctx, probs[0], phis[0], outs[0]) == 0
    torch.cuda.synchronize()
    assert np.array_equal(outs[0].cpu().numpy(), refs[0].cpu().numpy())


def test_noalloc_apply_refuses_a_problem_beyond_its_scratch(K, ctx):
    import torch
    p = synth.circle_problem(n=4096, m=8192, kappa=1.0)
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    phi = dev(synth.smooth_density(prob.M, 5))
    out = torch.full((prob.M,), 7.25, dtype=torch.float64, device="cuda:0")
    assert noalloc(K, ctx, prob, phi, out) == UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((out == 7.25).all())


def test_noalloc_apply_leaves_out_untouched_on_nan(K, ctx):
    import torch
    p = synth.circle_problem(n=128, m=256, kappa=1.0)
    prob = K.Problem(ctx, p.xy, p.n, p.kappa)
    phi = synth.smooth_density(prob.M, 9)
    phi[17] = np.nan
    phi_d = dev(phi)
    out = torch.full((prob.M,), 7.25, dtype=torch.float64, device="cuda:0")
    assert noalloc(K, ctx, prob, phi_d, out) == 0
    torch.cuda.synchronize()
    assert bool((out == 7.25).all())
