"""Batched solves and the serving loop on the GPU, through the C ABI.

- Every problem of a mixed batch (64^2 to 512^2) matches its single-problem
  solve (relative 1e-11: the fast solve's partial sums are grouped
  differently) and the oracle (relative 1e-10; GMRES at 1e-12 on the GPU,
  1e-13 in the oracle).
- A problem's result is bitwise the same alone in a batch and in the mix.
- The memory budget refuses admissions that do not fit and accepts them once
  memory is freed.
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


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


MIX = [
    lambda: synth.circle_problem(n=64, m=128),
    lambda: synth.star_problem(n=256, kappa=1.0),
    lambda: synth.circle_problem(n=128, m=256, kappa=3.0),
    lambda: synth.star_problem(n=512, kappa=2.0),
    lambda: synth.serving_request(11, 256),
]


def note(msg):
    print(msg, flush=True)


def run_batch(K, ctx, problems, tol=1e-12, max_slots=8):
    note("batch: " + ", ".join(p.name for p in problems) + f" tol={tol}")
    batch = K.Batch(ctx, max_slots=max_slots, m_max=2048)
    slots, probs = [], []
    for p in problems:
        prob = K.Problem(ctx, p.xy, p.n, p.kappa, tol=tol)
        s = batch.admit(prob, dev(p.f_grid), dev(p.f_gamma), dev(p.g))
        assert s is not None
        slots.append(s)
        probs.append(prob)
    out = {}
    for _ in range(200):
        batch.step(8)
        st, it, rel = batch.poll()
        for s in slots:
            if s not in out and st[s] != 0:
                u, ug, phi, _ = batch.finish(s)
                out[s] = (host(u), host(ug), host(phi), int(st[s]), int(it[s]), float(rel[s]))
        if len(out) == len(slots):
            break
    batch.close()
    return [out[s] for s in slots]


def test_mixed_batch_matches_single_solves_and_oracle(K, ctx):
    problems = [f() for f in MIX]
    res = run_batch(K, ctx, problems)
    for p, (u, ug, phi, st, it, rel) in zip(problems, res):
        note(f"{p.name}: state {st} iters {it} relres {rel:.3e}")
        assert st == 1, (p.name, it, rel)
        prob = K.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-12)
        u1, ug1, phi1, it1, rel1, conv1 = prob.solve(dev(p.f_grid), dev(p.f_gamma), dev(p.g))
        note(f"  single: iters {it1} relres {rel1:.3e}")
        assert abs(it1 - it) <= 1, p.name
        assert relerr(phi, host(phi1)) < 1e-11, p.name
        assert relerr(u, host(u1)) < 1e-11, p.name
        ref = O.solve_bvp(p.xy, p.n, LO, HI, p.kappa, p.f_grid, p.f_gamma, p.g, tol=1e-13)
        assert relerr(u, ref.u_grid) < 1e-10, p.name
        assert relerr(ug, ref.u_gamma) < 1e-10, p.name


def test_alone_and_in_the_mix_are_bitwise_equal(K, ctx):
    problems = [f() for f in MIX]
    mixed = run_batch(K, ctx, problems, tol=1e-10)
    for k in (1, 3):
        alone = run_batch(K, ctx, [problems[k]], tol=1e-10)[0]
        for a, b in zip(alone[:3], mixed[k][:3]):
            assert np.array_equal(a, b), problems[k].name
        assert alone[4] == mixed[k][4]


def test_large_grids_in_a_batch(K, ctx):
    """The 2048^2 and 4096^2 grids (the largest a batch serves: four modes per
    workgroup at 4096^2) beside a small problem: each matches its single-problem
    solve, and the 4096^2 member is bitwise the same alone and in the mix."""
    problems = [synth.star_problem(n=4096, kappa=1.0), synth.circle_problem(n=2048, m=1024, kappa=1.0),
                synth.circle_problem(n=64, m=128)]
    mixed = run_batch(K, ctx, problems, tol=1e-10)
    for p, (u, ug, phi, st, it, rel) in zip(problems, mixed):
        note(f"{p.name}: state {st} iters {it} relres {rel:.3e}")
        assert st == 1, (p.name, it, rel)
        prob = K.Problem(ctx, p.xy, p.n, p.kappa, tol=1e-10)
        u1, ug1, phi1, it1, rel1, conv1 = prob.solve(dev(p.f_grid), dev(p.f_gamma), dev(p.g))
        note(f"  single: iters {it1} relres {rel1:.3e}")
        assert conv1 and abs(it1 - it) <= 1, p.name
        assert relerr(phi, host(phi1)) < 1e-9, p.name
        assert relerr(u, host(u1)) < 1e-9, p.name
        prob.close()
    alone = run_batch(K, ctx, [problems[0]], tol=1e-10)[0]
    for a, b in zip(alone[:3], mixed[0][:3]):
        assert np.array_equal(a, b)


def test_budget_admission(K, ctx):
    p1, p2 = synth.star_problem(n=256, kappa=1.0), synth.circle_problem(n=256, m=512)
    a = K.Problem(ctx, p1.xy, p1.n, p1.kappa)
    b = K.Problem(ctx, p2.xy, p2.n, p2.kappa)
    est = K.Batch.estimate_bytes(256, 512)
    assert a.device_bytes <= est and b.device_bytes <= est
    # room for either problem (with its batch partials) but not for both
    batch = K.Batch(ctx, max_slots=4, m_max=1024, hbm_budget=a.device_bytes + b.device_bytes)
    ins = [dev(p1.f_grid), dev(p1.f_gamma), dev(p1.g)]
    s1 = batch.admit(a, *ins)
    assert s1 is not None
    assert batch.admit(b, dev(p2.f_grid), dev(p2.f_gamma), dev(p2.g)) is None       # over budget now
    for _ in range(100):
        batch.step(8)
        st, _, _ = batch.poll()
        if st[s1] != 0:
            break
    batch.finish(s1)
    assert batch.admit(b, dev(p2.f_grid), dev(p2.f_gamma), dev(p2.g)) is not None  # fits after the finish
    batch.close()


def test_serving_loop_small_stream(K, ctx):
    """Eight requests through the continuous-batching loop: every one converges,
    the under-resolved flag is the one the geometry predicts, every result is
    bitwise the same when its request is served alone, and a seeded subsample
    is within the metric's L-infinity 1e-6 of the FP64 oracle."""
    note("serving loop: 8 requests n in {256, 512}, two preparation threads")
    from paper_2404_15249_amd.serving import GpuExecutor, Request, Scheduler, summarize
    sizes = [256, 512, 256, 256, 512, 256, 256, 512]
    reqs = [Request(i, 0.002 * i, int(n), 100 + i) for i, n in enumerate(sizes)]
    spec = lambda r: synth.serving_spec(r.seed, r.n)
    ex = GpuExecutor(ctx, max_slots=6, m_max=4096, budget_bytes=0, make_spec=spec, check_error=True)
    sch = Scheduler(ex, 4 << 30, 6, steps_per_poll=8, prepare_workers=2, keep_results=True)
    recs, span = sch.run(reqs)
    assert len(recs) == len(reqs) and not any(r.rejected for r in recs)
    recs = sorted(recs, key=lambda r: r.rid)
    for r in recs:
        note(f"  req {r.rid} n={r.n}: iters {r.iters} relres {r.relres:.2e} converged {r.converged} "
             f"under-resolved {r.result['under_resolved']} Linf err vs exact {r.result['linf_err']:.2e}")
    assert all(r.converged for r in recs)
    # the flag follows the geometry: smallest radius of curvature below 3h
    assert [r.result["under_resolved"] for r in recs] == [spec(q).under_resolved for q in reqs]
    assert sum(r.result["under_resolved"] for r in recs) == 1
    assert sch.peak_live >= 2                     # requests overlapped in the batch
    errs = [r.result["linf_err"] for r in recs if not r.result["under_resolved"]]
    assert max(errs) < 1e-3, errs                 # second-order discretisation error at these grids
    s = summarize(recs, span)
    assert s["p99_ms"] >= s["p50_ms"] > 0
    # each request served alone gives the same bits
    ex1 = GpuExecutor(ctx, max_slots=1, m_max=4096, budget_bytes=0, make_spec=spec, check_error=True)
    alone, _ = Scheduler(ex1, 4 << 30, 1, prepare_workers=0, keep_results=True).run(
        [Request(q.rid, 0.0, q.n, q.seed) for q in reqs])
    for a in alone:
        m = recs[a.rid]
        assert a.iters == m.iters, a.rid
        for key in ("u", "u_gamma", "phi"):
            assert np.array_equal(host(a.result[key]), host(m.result[key])), (a.rid, key)
    # a seeded subsample against the FP64 oracle, at the metric's bar
    pick = np.random.default_rng(2404).choice(len(reqs), size=3, replace=False)
    for k in sorted(int(i) for i in pick):
        p = synth.serving_request(reqs[k].seed, reqs[k].n)
        ref = O.solve_bvp(p.xy, p.n, LO, HI, p.kappa, p.f_grid, p.f_gamma, p.g, tol=1e-13)
        u, ug = host(recs[k].result["u"]), host(recs[k].result["u_gamma"])
        e_grid = float(np.max(np.abs(u - ref.u_grid)))
        e_gam = float(np.max(np.abs(ug - ref.u_gamma)))
        note(f"  req {k} n={p.n} vs oracle: Linf grid {e_grid:.2e}, trace {e_gam:.2e}")
        assert e_grid <= 1e-6 and e_gam <= 1e-6, (k, e_grid, e_gam)
