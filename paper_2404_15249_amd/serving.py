"""Continuous-batching server of Dirichlet solves on one GPU.

Requests (a domain, a grid size, data) arrive over time.  The scheduler keeps
a first-in-first-out queue and admits the head of the queue as soon as a batch
slot and enough device memory (the HBM budget, counted with each problem's
byte estimate) are free.  Admitted problems run their GMRES iterations inside
one shared batch (:class:`paper_2404_15249_amd.kfbi.Batch`): every launch
advances every live problem, so requests that arrive while others are running
join the next launches.  When a problem converges the scheduler runs its final
solve, frees its slot and memory, and records its latency (finish - arrival).

Host-side preparation of a request (the geometry plan and the device inputs)
runs in a small thread pool ahead of admission; the native calls release the
interpreter lock, so preparation overlaps the GPU work.

The scheduler only talks to an executor object (``estimate``, ``prepare``,
``admit``, ``step``, ``poll``, ``finish``, ``release``), so its host logic can be
exercised without a GPU.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float        # seconds after the start of the stream
    n: int                # grid intervals per axis
    seed: int             # seed of the request's domain and data


@dataclasses.dataclass
class Record:
    rid: int
    n: int
    arrival: float
    admitted: float
    finished: float
    iters: int
    relres: float
    converged: bool
    result: object = None
    rejected: str = ""           # why the request was refused before admission (e.g. its geometry)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def summarize(records, makespan: float) -> dict:
    """Throughput and latency over the solved requests (refused ones are counted apart)."""
    solved = [r for r in records if not r.rejected]
    lat = np.array([r.latency for r in solved]) if solved else np.zeros(1)
    return {
        "completed": len(solved),
        "rejected": len(records) - len(solved),
        "makespan_s": makespan,
        "solves_per_s": len(solved) / makespan if makespan > 0 else 0.0,
        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "mean_ms": 1e3 * float(lat.mean()),
        "converged": int(sum(r.converged for r in solved)),
        "mean_iters": float(np.mean([r.iters for r in solved])) if solved else 0.0,
    }


class Scheduler:
    """FIFO admission by slots and memory budget, continuous batching, latency records."""

    def __init__(self, executor, budget_bytes: int, max_slots: int, steps_per_poll: int = 8,
                 prepare_workers: int = 4, prepare_ahead: int = 4, keep_results: bool = False):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.steps_per_poll = int(steps_per_poll)
        self.prepare_workers = prepare_workers
        self.prepare_ahead = prepare_ahead
        self.keep_results = keep_results
        self.reserved = 0            # bytes of prepared + live requests
        self.peak_reserved = 0
        self.peak_live = 0

    def run(self, requests, clock=time.perf_counter, sleep=time.sleep, time_scale: float = 1.0):
        """Serve ``requests`` (sorted by arrival); returns ``(records, makespan)``.

        ``time_scale`` stretches the arrival times (1.0 = real time).
        """
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            if self.ex.estimate(r) > self.budget:
                raise ValueError(f"request {r.rid} can never fit the budget")
        pending = collections.deque()
        preparing = collections.deque()       # (request, bytes, future) in FIFO order
        live = {}                             # slot -> (request, bytes, handle, admitted time)
        records = []
        nxt = 0
        t0 = clock()
        pool = cf.ThreadPoolExecutor(max_workers=self.prepare_workers) if self.prepare_workers else None
        try:
            while len(records) < len(reqs):
                now = clock() - t0
                while nxt < len(reqs) and reqs[nxt].arrival * time_scale <= now:
                    pending.append(reqs[nxt])
                    nxt += 1
                # start preparing the queue head while memory and slots allow
                while pending and len(preparing) < self.prepare_ahead and \
                        len(preparing) + len(live) < self.max_slots:
                    nb = self.ex.estimate(pending[0])
                    if self.reserved + nb > self.budget:
                        break
                    r = pending.popleft()
                    self.reserved += nb
                    self.peak_reserved = max(self.peak_reserved, self.reserved)
                    fut = pool.submit(self.ex.prepare, r) if pool else _Done.call(self.ex.prepare, r)
                    preparing.append((r, nb, fut))
                # admit prepared requests in arrival order
                while preparing and preparing[0][2].done():
                    r, nb, fut = preparing.popleft()
                    try:
                        handle = fut.result()
                    except getattr(self.ex, "request_errors", ()) as e:   # e.g. an unsupported geometry
                        self.reserved -= nb
                        t = clock() - t0
                        records.append(Record(r.rid, r.n, r.arrival * time_scale, t, t, 0, float("nan"), False,
                                              None, rejected=str(e)))
                        continue
                    slot = self.ex.admit(handle)
                    if slot is None:                  # cannot happen while slots are counted here
                        raise RuntimeError("executor refused an admission the scheduler had room for")
                    live[slot] = (r, nb, handle, clock() - t0)
                    self.peak_live = max(self.peak_live, len(live))
                if live:
                    self.ex.step(self.steps_per_poll)
                    states = self.ex.poll()
                    for slot, (st, it, rel) in states.items():
                        if slot not in live or st == 0:
                            continue
                        r, nb, handle, t_adm = live.pop(slot)
                        res = self.ex.finish(slot, handle)
                        self.ex.release(handle)
                        self.reserved -= nb
                        records.append(Record(r.rid, r.n, r.arrival * time_scale, t_adm, clock() - t0, it, rel,
                                              st == 1, res if self.keep_results else None))
                elif preparing:
                    cf.wait([preparing[0][2]])
                elif nxt < len(reqs):
                    sleep(max(0.0, reqs[nxt].arrival * time_scale - (clock() - t0)))
        finally:
            if pool:
                pool.shutdown(wait=True)
        return records, clock() - t0


class _Done(cf.Future):
    """An already finished future (preparation without a thread pool)."""

    @classmethod
    def call(cls, fn, *args):
        f = cls()
        try:
            f.set_result(fn(*args))
        except Exception as e:       # delivered by result(), as from a pool
            f.set_exception(e)
        return f


class GpuExecutor:
    """Runs requests through one :class:`kfbi.Batch` on the GPU.

    Requests whose geometry the plan builder rejects are reported to the
    scheduler as refused (``request_errors``).

    ``make_spec(request)`` returns a ``synth.RequestSpec``-like object (``n``,
    ``kappa``, ``xy``, ``sol_torch``); the right-hand sides are evaluated
    directly in device memory.
    """

    def __init__(self, ctx, max_slots: int, m_max: int, budget_bytes: int, make_spec, tol: float = 1e-10,
                 restart: int = 50, check_error: bool = False, keep_ids=()):
        import torch
        from . import kfbi
        self.torch = torch
        self.kfbi = kfbi
        self.ctx = ctx
        self.batch = kfbi.Batch(ctx, max_slots=max_slots, m_max=m_max, hbm_budget=budget_bytes)
        self.make_spec = make_spec
        self.tol, self.restart = tol, restart
        self.check_error = check_error
        self.keep_ids = set(keep_ids)       # requests whose solution is copied to the host
        self._m_cache = {}
        self.request_errors = (kfbi.GeometryError,)

    def estimate(self, r) -> int:
        if r.rid not in self._m_cache:
            self._m_cache[r.rid] = self.make_spec(r)
        sp = self._m_cache[r.rid]
        return self.kfbi.Batch.estimate_bytes(sp.n, sp.xy.shape[0], self.restart)

    def prepare(self, r):
        torch = self.torch
        sp = self._m_cache.pop(r.rid, None) or self.make_spec(r)
        prob = self.kfbi.Problem(self.ctx, sp.xy, sp.n, sp.kappa, tol=self.tol, restart=self.restart)
        dev = f"cuda:{self.ctx.device}"
        h = (prob.hi - prob.lo) / sp.n
        c = prob.lo + torch.arange(sp.n + 1, device=dev, dtype=torch.float64) * h
        Y, X = torch.meshgrid(c, c, indexing="ij")
        f = sp.sol_torch.f(X, Y, sp.kappa).contiguous()
        zx = torch.as_tensor(sp.xy[:, 0], device=dev)
        zy = torch.as_tensor(sp.xy[:, 1], device=dev)
        fg = sp.sol_torch.f(zx, zy, sp.kappa).contiguous()
        g = sp.sol_torch.u(zx, zy).contiguous()
        torch.cuda.current_stream(self.ctx.device).synchronize()
        return {"prob": prob, "f": f, "fg": fg, "g": g, "spec": sp, "rid": r.rid}

    def admit(self, hd):
        return self.batch.admit(hd["prob"], hd["f"], hd["fg"], hd["g"])

    def step(self, k):
        self.batch.step(k)

    def poll(self):
        st, it, rel = self.batch.poll()
        return {s: (int(st[s]), int(it[s]), float(rel[s])) for s in range(len(st)) if st[s] != -2}

    def finish(self, slot, hd):
        try:
            u, ug, phi, prob = self.batch.finish(slot)
        except self.kfbi.NonfiniteError:              # a NaN or Inf in the request: released, nothing written
            return {"nonfinite": True, "under_resolved": bool(getattr(hd["spec"], "under_resolved", False))}
        if hd.get("rid") in self.keep_ids:
            return {"under_resolved": bool(getattr(hd["spec"], "under_resolved", False)),
                    "u_host": u.cpu().numpy(), "u_gamma_host": ug.cpu().numpy()}
        if not self.check_error:
            return {"under_resolved": bool(getattr(hd["spec"], "under_resolved", False))}
        torch = self.torch
        sp = hd["spec"]
        dev = u.device
        h = (prob.hi - prob.lo) / sp.n
        c = prob.lo + torch.arange(sp.n + 1, device=dev, dtype=torch.float64) * h
        Y, X = torch.meshgrid(c, c, indexing="ij")
        mask = torch.as_tensor(prob.mask(), device=dev)
        err = torch.where(mask, (u - sp.sol_torch.u(X, Y)).abs(), torch.zeros_like(u)).max()
        return {"linf_err": float(err), "u": u, "u_gamma": ug, "phi": phi,
                "under_resolved": bool(getattr(sp, "under_resolved", False))}

    def release(self, hd):
        hd["prob"].close()
