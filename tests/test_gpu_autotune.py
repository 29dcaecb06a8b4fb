"""The autotuner's persistent result cache (eco_world_autotune_cached)."""
import json

import pytest

from gpu_util import need_gpu
from paper_2510_18221_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as e
    e.lib()
    return e


def test_cache_miss_tunes_and_appends_then_hits(eco, tmp_path):
    cache = tmp_path / "launch_cache.jsonl"
    cfg = wl.world_small(seed=0)
    w = eco.World(cfg)
    first = w.autotune(cache=str(cache))
    assert first["from_cache"] is False
    lines = [json.loads(l) for l in cache.read_text().splitlines()]
    assert len(lines) == 1
    key = lines[0]["key"]
    assert "D=104" in key and "H=32" in key and "A=5" in key and "live=2^8" in key and "gfx" in key
    assert (lines[0]["waves_per_block"], lines[0]["blocks_per_cu"], lines[0]["unroll"]) == \
        (first["waves_per_block"], first["blocks_per_cu"], first["unroll"])
    w.close()
    w = eco.World(cfg)
    second = w.autotune(cache=str(cache))
    assert second["from_cache"] is True
    assert {k: second[k] for k in ("waves_per_block", "blocks_per_cu", "unroll")} == \
        {k: first[k] for k in ("waves_per_block", "blocks_per_cu", "unroll")}
    assert w.get_launch() == {k: first[k] for k in ("waves_per_block", "blocks_per_cu", "unroll")}
    assert len(cache.read_text().splitlines()) == 1      # a hit writes nothing
    # a hand-written line for the same key (the last match wins) sets that shape
    with open(cache, "a") as f:
        f.write(json.dumps({"key": key, "waves_per_block": 2, "blocks_per_cu": 4, "unroll": 8}) + "\n")
    third = w.autotune(cache=str(cache))
    assert third["from_cache"] is True and (third["waves_per_block"], third["blocks_per_cu"], third["unroll"]) == \
        (2, 4, 8)
    w.step(2)   # the cached shape runs
    w.close()


def test_cache_keys_differ_by_policy_shape(eco, tmp_path):
    cache = tmp_path / "c.jsonl"
    a = eco.World(wl.world_small(seed=0))
    b = eco.World(wl.world_small(seed=0, wdtype=wl.BF16))
    assert a.autotune(cache=str(cache))["from_cache"] is False
    assert b.autotune(cache=str(cache))["from_cache"] is False
    keys = [json.loads(l)["key"] for l in cache.read_text().splitlines()]
    assert len(set(keys)) == 2 and "wdtype=0" in keys[0] and "wdtype=1" in keys[1]
    a.close()
    b.close()
