"""Host logic of the launch-shape cache (no GPU): keys by size class, hits
reuse the stored shapes, misses tune once and persist."""
import json

from paper_2404_15249_amd.autotune import TileCache


class FakeCtx:
    device = 0


class FakeProb:
    def __init__(self, n=512, M=256, I=1900, precision="fp64", valid=True):
        self.ctx = FakeCtx()
        self.n, self.M, self.I, self.precision = n, M, I, precision
        self.valid = valid
        self.tuned = 0
        self.set = None

    def autotune(self, reps):
        self.tuned += 1
        return {"modes_per_group": 8, "modes_groups": 256, "dst_cols": 8, "apply_us": 12.5, "grid_solve_us": 40.0}

    def set_tiles(self, r, b):
        if not self.valid:
            from paper_2404_15249_amd.kfbi import KfbiError
            raise KfbiError(-1, "tile shape not valid for this problem")
        self.set = (r, b)


def test_miss_tunes_and_persists_then_hit_reuses(tmp_path):
    path = str(tmp_path / "tiles.json")
    c = TileCache(path, device_name="gfx950")
    p = FakeProb()
    t = c.apply(p)
    assert p.tuned == 1 and c.misses == 1 and t["modes_per_group"] == 8
    assert json.load(open(path))                      # written to disk
    c2 = TileCache(path, device_name="gfx950")       # a later run
    q = FakeProb(M=250, I=1950)                       # same size class
    c2.apply(q)
    assert q.tuned == 0 and q.set == (8, 8) and c2.hits == 1


def test_keys_separate_grid_precision_and_size_class(tmp_path):
    c = TileCache(str(tmp_path / "t.json"), device_name="gfx950")
    keys = {c.key(FakeProb()), c.key(FakeProb(n=1024)), c.key(FakeProb(precision="fp32")),
            c.key(FakeProb(M=600)), c.key(FakeProb(I=5000))}
    assert len(keys) == 5
    assert c.key(FakeProb(M=200)) == c.key(FakeProb(M=256))


def test_stale_entry_is_retuned(tmp_path):
    path = str(tmp_path / "t.json")
    c = TileCache(path, device_name="gfx950")
    c.apply(FakeProb())
    p = FakeProb(valid=False)
    TileCache(path, device_name="gfx950").apply(p)
    assert p.tuned == 1


def test_corrupt_file_starts_empty(tmp_path):
    path = tmp_path / "t.json"
    path.write_text("{not json")
    c = TileCache(str(path), device_name="gfx950")
    assert c.entries == {}
    c.apply(FakeProb())
    assert json.load(open(path))
