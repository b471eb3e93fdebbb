"""GPU parity of the Gray-Scott time stepping (Example 3: disk r = 1.8 in
(-2, 2)^2, Strang splitting with Crank-Nicolson diffusion as Neumann solves)
against the FP64 oracle, through the C ABI: the whole state (grids and traces
of u and v, each relative to the species' largest value) to 1e-10 after T = 1 at 128^2 (8 steps) and after one step
at 1024^2 (dt = 1/64), the Crank-Nicolson decay of a disk eigenmode, the mirror
symmetry of the state, and the refusal of bad parameters."""
import sys

import numpy as np
import pytest
from scipy.special import jnp_zeros, jv

import synth
from oracle import gray_scott as G
from oracle import kfbi_oracle as O

pytestmark = pytest.mark.gpu

LO, HI = synth.GS_LO, synth.GS_HI
P = synth.GrayScottParams()


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


def gpu_initial(K, ctx, xy, n, init):
    """The initial state for the library: the closed form at the nodes of the
    library's own inside mask and at the samples."""
    mask = K.Problem(ctx, xy, n, 1.0, lo=LO, hi=HI).mask()
    c = LO + np.arange(n + 1) * (HI - LO) / n
    X, Y = np.meshgrid(c, c, indexing="xy")
    u, v = init(X, Y)
    ug, vg = init(xy[:, 0], xy[:, 1])
    return dev(np.where(mask, u, 0.0)), dev(np.where(mask, v, 0.0)), dev(ug), dev(vg)


def run_both(K, ctx, n, dt, steps, tol, params=P, init=synth.gray_scott_initial, reaction=True):
    xy = synth.gray_scott_samples(n)
    gs = K.GrayScott(ctx, xy, n, dt, params.gamma, params.kill, params.eps0, params.eps1, params.eps2,
                     lo=LO, hi=HI, tol=tol)
    gs.set_state(*gpu_initial(K, ctx, xy, n, init))
    gs.step(steps)
    got = [host(t) for t in gs.state()]
    info = gs.info()
    gs.close()
    plan = O.build_plan(xy, n, LO, HI)
    st = G.run(plan, G.initial_state(plan, init), dt, steps, params, tol=tol, reaction=reaction)
    return got, st, info, plan


@pytest.mark.parametrize("n,dt,steps", [(128, 0.125, 8), (1024, 1.0 / 64, 1)])
def test_gray_scott_matches_oracle(K, ctx, n, dt, steps):
    note(f"Gray-Scott parity n={n} dt={dt} steps={steps}")
    (u, v, ug, vg), st, info, plan = run_both(K, ctx, n, dt, steps, tol=1e-12)
    note(f"  GMRES iterations gpu {info['gmres_iters']} oracle {st.iters}")
    assert info["steps"] == steps
    assert abs(info["gmres_iters"] - st.iters) <= 2 * steps
    # each species against its largest value on the grid (v is ~0 on Gamma, far
    # from the initial patch, so a trace-relative measure would divide by ~0)
    su, sv = np.max(np.abs(st.u)), np.max(np.abs(st.v))
    note(f"  |v| on Gamma: gpu {np.max(np.abs(vg)):.1e} oracle {np.max(np.abs(st.v_gamma)):.1e}")
    assert np.max(np.abs(u - st.u)) / su < 1e-10
    assert np.max(np.abs(v - st.v)) / sv < 1e-10
    assert np.max(np.abs(ug - st.u_gamma)) / su < 1e-10
    assert np.max(np.abs(vg - st.v_gamma)) / sv < 1e-10
    assert np.all(u[~plan.inside] == 0.0) and np.all(v[~plan.inside] == 0.0)


def test_gray_scott_eigenmode_decay_on_the_gpu(K, ctx):
    """Reaction rates zero (gamma = kill = 0 and v = 0): a disk Neumann
    eigenmode decays by the Crank-Nicolson factor per step."""
    n, eps, dt, steps = 512, 0.5, 0.4, 2
    al = jnp_zeros(0, 1)[0] / synth.GS_RADIUS
    mode = lambda x, y: jv(0, al * np.hypot(x, y))
    params = synth.GrayScottParams(gamma=0.0, kill=0.0, eps1=eps, eps2=eps / 2)
    xy = synth.gray_scott_samples(n)
    gs = K.GrayScott(ctx, xy, n, dt, 0.0, 0.0, params.eps0, eps, eps / 2, lo=LO, hi=HI, tol=1e-12)
    gs.set_state(*gpu_initial(K, ctx, xy, n, lambda x, y: (mode(x, y), 0 * x)))
    gs.step(steps)
    u, v, ug, vg = [host(t) for t in gs.state()]
    gs.close()
    a = eps * al * al * dt / 2
    cn = ((1 - a) / (1 + a)) ** steps
    c = LO + np.arange(n + 1) * (HI - LO) / n
    X, Y = np.meshgrid(c, c, indexing="xy")
    mask = K.Problem(ctx, xy, n, 1.0, lo=LO, hi=HI).mask()
    e = float(np.max(np.abs(u - cn * mode(X, Y))[mask]))
    note(f"  eigenmode error vs CN factor {e:.2e} (CN {cn:.4f}, exact {np.exp(-2 * a * steps):.4f})")
    assert e < 5e-5
    assert np.max(np.abs(v)) == 0.0


def test_gray_scott_state_is_mirror_symmetric_at_1024(K, ctx):
    n, dt, steps = 1024, 1.0 / 64, 8
    xy = synth.gray_scott_samples(n)
    gs = K.GrayScott(ctx, xy, n, dt, lo=LO, hi=HI, tol=1e-10)
    gs.set_state(*gpu_initial(K, ctx, xy, n, synth.gray_scott_initial))
    gs.step(steps)
    u, v, ug, vg = [host(t) for t in gs.state()]
    note(f"  1024^2, 8 steps: {gs.info()}")
    gs.close()
    assert np.max(np.abs(u - u[:, ::-1])) < 1e-8 and np.max(np.abs(v - v[:, ::-1])) < 1e-8
    assert np.max(np.abs(u - u[::-1, :])) < 1e-8 and np.max(np.abs(u - u.T)) < 1e-8
    assert v.min() > -1e-12 and v.max() < 1.0


def test_gray_scott_zero_steps_keep_the_state(K, ctx):
    n = 128
    xy = synth.gray_scott_samples(n)
    gs = K.GrayScott(ctx, xy, n, 0.125, lo=LO, hi=HI)
    init = gpu_initial(K, ctx, xy, n, synth.gray_scott_initial)
    gs.set_state(*init)
    gs.step(0)
    out = gs.state()
    assert gs.info()["steps"] == 0
    for a, b in zip(out, init):
        assert np.array_equal(host(a), host(b))
    gs.close()


def test_gray_scott_rejects_bad_parameters(K, ctx):
    xy = synth.gray_scott_samples(128)
    for kw in ({"dt": 0.0}, {"dt": 0.1, "eps1": 0.0}, {"dt": 0.1, "eps0": -1.0}):
        with pytest.raises(K.KfbiError):
            K.GrayScott(ctx, xy, 128, lo=LO, hi=HI, **kw)
