"""Autotuned launch shapes, cached across runs.

``kfbi_prob_autotune`` times the candidate shapes of one problem's kernels (the
sparse fast solve's sine modes per workgroup, the column transforms' tile
width) on the device and keeps the fastest.  Problems of the
same grid, precision and size class run fastest with the same shapes, so the
result is stored under a key of those and reused: a cache hit costs one
``kfbi_prob_set_tiles`` call instead of the timing runs.

The cache is a JSON file (``$KFBI_TILE_CACHE``, else
``~/.cache/paper_2404_15249_amd/tiles.json``), written atomically.
"""
from __future__ import annotations

import json
import os
import tempfile


def _pow2_ceil(v: int) -> int:
    p = 1
    while p < v:
        p *= 2
    return p


def default_path() -> str:
    return os.environ.get("KFBI_TILE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2404_15249_amd", "tiles.json")


class TileCache:
    def __init__(self, path: str | None = None, reps: int = 10, device_name: str | None = None):
        self.path = path or default_path()
        self.reps = reps
        self.device_name = device_name
        self.entries = {}
        self.hits = self.misses = 0
        try:
            with open(self.path) as f:
                data = json.load(f)
            if isinstance(data, dict):
                self.entries = data
        except (OSError, ValueError):
            self.entries = {}

    def key(self, prob) -> str:
        dev = self.device_name
        if dev is None:
            import torch
            dev = torch.cuda.get_device_name(prob.ctx.device)
        return f"{dev}|n={prob.n}|{prob.precision}|m<={_pow2_ceil(prob.M)}|i<={_pow2_ceil(max(prob.I, 1))}"

    def apply(self, prob) -> dict:
        """Give ``prob`` the cached shapes of its class, tuning (and storing) them on a miss."""
        from .kfbi import KfbiError
        k = self.key(prob)
        e = self.entries.get(k)
        if e is not None:
            try:
                prob.set_tiles(e["modes_per_group"], e["dst_cols"])
                self.hits += 1
                return dict(e)
            except (KfbiError, KeyError, TypeError):
                pass                                   # stale or foreign entry: tune again
        self.misses += 1
        t = prob.autotune(self.reps)
        self.entries[k] = t
        self.save()
        return dict(t)

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".tiles.", suffix=".json")
        try:
            with os.fdopen(fd, "w") as f:
                json.dump(self.entries, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except BaseException:
            if os.path.exists(tmp):
                os.unlink(tmp)
            raise
