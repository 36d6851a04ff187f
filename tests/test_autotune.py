"""The autotuner's search and cache on the CPU (fake measurements)."""
import json

import pytest

from paper_1107_1525_amd.autotune import Autotuner, candidate_key

CANDS = [{"block_size": b, "sub_block": s, "encode_tile_loads": 0} for b in (4096, 65536) for s in (128, 1024)]


def test_picks_fastest_and_caches(tmp_path):
    calls = []
    times = {candidate_key(c): t for c, t in zip(CANDS, (3.0, 1.5, 2.0, 1.7))}

    def measure(c):
        calls.append(candidate_key(c))
        return times[candidate_key(c)]

    t = Autotuner(str(tmp_path / "tune.json"))
    best, table, cached = t.tune("gfx950|dev|256cu", "wl", CANDS, measure)
    assert best == CANDS[1] and not cached and len(table) == 4 and len(calls) == 4
    # a second tuning of the same device and workload takes the cache, measuring nothing
    best2, _, cached2 = t.tune("gfx950|dev|256cu", "wl", CANDS, measure)
    assert best2 == best and cached2 and len(calls) == 4
    # another device or workload is tuned anew
    t.tune("gfx942|dev|304cu", "wl", CANDS, measure)
    t.tune("gfx950|dev|256cu", "other", CANDS, measure)
    assert len(calls) == 12
    data = json.loads((tmp_path / "tune.json").read_text())
    assert set(data) == {"gfx950|dev|256cu", "gfx942|dev|304cu"}
    # force measures again
    t.tune("gfx950|dev|256cu", "wl", CANDS, measure, force=True)
    assert len(calls) == 16


def test_failed_candidates_are_never_chosen(tmp_path):
    def measure(c):
        if c["sub_block"] == 128:
            raise MemoryError("out of memory")
        return float(c["block_size"])

    best, table, _ = Autotuner(str(tmp_path / "t.json")).tune("d", "w", CANDS, measure)
    assert best == {"block_size": 4096, "sub_block": 1024, "encode_tile_loads": 0}
    assert sum("error" in r for r in table) == 2


def test_no_measurable_candidate_raises(tmp_path):
    def measure(c):
        raise RuntimeError("x")

    with pytest.raises(RuntimeError):
        Autotuner(str(tmp_path / "t.json")).tune("d", "w", CANDS, measure)
