"""Host logic of the tuned-table generator (no GPU): the batch cap's choice
of slab depth, its parity gate, and the rewrite of table lines."""
import torch
import pytest

from paper_1812_03358_amd import ltm
from paper_1812_03358_amd.tuned import make_table as M


class FakePlan:
    """Stands in for ltm.Plan: an operator output that depends on the tiling
    only through a chosen perturbation, and a time per slab depth."""

    def __init__(self, ms_of_chunk, bad_chunk=None):
        self.ms_of_chunk = ms_of_chunk
        self.bad_chunk = bad_chunk
        self.tiling = None
        self.base = torch.linspace(1.0, 2.0, 64)

    def set_tiling(self, direction, camera, t):
        self.tiling = dict(t)

    def project(self, x, out=None):
        v = self.base.clone()
        if self.tiling is not None and self.tiling["chunk_mm"] == self.bad_chunk:
            v[0] += 1.0
        return v

    backproject = project


def tiling(**kw):
    t = dict(tile_u=2, tile_v=2, block_u=16, block_v=16, order=40, splits=4, brick_floats=8192,
             groups_per_cu=2, chunk_mm=40.0)
    t.update(kw)
    return t


@pytest.mark.parametrize("direction", [ltm.FORWARD, ltm.ADJOINT])
def test_batch_cap_keeps_the_fastest_depth(monkeypatch, direction):
    times = {40.0: 98.0, 20.0: 1.4, 10.0: 1.6}
    plan = FakePlan(times)
    monkeypatch.setattr(M, "time_direction", lambda p, d, x, y, out: p.ms_of_chunk[p.tiling["chunk_mm"]])
    t, ms = M.batch_capped(plan, direction, None, None, tiling())
    assert t["brick_floats"] == M.BATCH_BRICK_CAP and t["groups_per_cu"] == 0
    assert t["chunk_mm"] == 20.0 and ms == 1.4
    # everything but the cap and the depth is the searched tiling's
    assert {k: v for k, v in t.items() if k not in ("brick_floats", "groups_per_cu", "chunk_mm")} == \
        {k: v for k, v in tiling().items() if k not in ("brick_floats", "groups_per_cu", "chunk_mm")}


def test_batch_cap_within_the_cap_keeps_its_depth_unless_slower(monkeypatch):
    plan = FakePlan({32.0: 0.45, 16.0: 0.47, 8.0: 0.60})
    monkeypatch.setattr(M, "time_direction", lambda p, d, x, y, out: p.ms_of_chunk[p.tiling["chunk_mm"]])
    filed = tiling(brick_floats=4096, groups_per_cu=0, chunk_mm=32.0)
    t, _ = M.batch_capped(plan, ltm.FORWARD, None, None, filed)
    assert t == filed


def test_batch_cap_parity_gate(monkeypatch):
    plan = FakePlan({40.0: 1.0, 20.0: 0.5, 10.0: 0.7}, bad_chunk=20.0)
    monkeypatch.setattr(M, "time_direction", lambda p, d, x, y, out: p.ms_of_chunk[p.tiling["chunk_mm"]])
    with pytest.raises(RuntimeError, match="parity"):
        M.batch_capped(plan, ltm.ADJOINT, None, None, tiling())


def test_rewrite_replaces_only_the_capped_lines(tmp_path):
    path = tmp_path / "t.tsv"
    head = "# libltm tilings: key\ttile_u tile_v block_u block_v order splits brick_floats " \
           "groups_per_cu chunk_mm\tms default_ms"
    keep = "gfx950|A|k1\t2 2 16 16 2 4 4096 0 40\t0.30000 0.31000"
    old = "gfx950|AT|k1\t4 4 16 16 40 16 12288 2 40\t1.20000 1.40000"
    path.write_text("\n".join([head, keep, old]) + "\n")
    new = tiling(tile_u=4, tile_v=4, splits=16, brick_floats=6144, groups_per_cu=0, chunk_mm=20.0)
    M.rewrite(str(path), {"gfx950|AT|k1": (new, 1.25)})
    lines = path.read_text().splitlines()
    assert lines[:2] == [head, keep]
    assert lines[2] == "gfx950|AT|k1\t4 4 16 16 40 16 6144 0 20.0\t1.25000 1.40000"
    table = M.read_table(str(path))
    assert table["gfx950|AT|k1"] == new
