"""Autotuner search and cache logic (CPU: a synthetic cost function stands in for timing)."""
import json
import types

import pytest

torch = pytest.importorskip("torch")

from paper_2412_12734_amd import autotune as at
from paper_2412_12734_amd.render import Options


def synthetic_cost(o):
    # separable bowl with its minimum at tile 16x8, batch 16, batch_bwd 8, prefix 2048,
    # work-ordered tiles
    c = {(16, 16): 1.0, (16, 8): 0.5, (8, 8): 2.0}[(o.tile_w, o.tile_h)]
    c += {8: 0.3, 16: 0.0, 32: 0.2, 64: 0.9}[o.batch if o.batch else 16]
    c += {8: 0.0, 16: 0.4, 32: 1.5}[o.batch_bwd if o.batch_bwd else 8]
    c += {256: 0.6, 512: 0.1, 1024: 0.05, 2048: 0.0, -1: 3.0}[o.prefix_pairs_per_tile or 1024]
    c += {1: 0.0, -1: 0.2}[o.tile_order or 1]
    return c


def test_search_finds_the_separable_minimum():
    base = at.resolve_defaults(Options(), 8)
    assert (base.batch, base.batch_bwd, base.prefix_pairs_per_tile, base.tile_order) == \
        (16, 8, 1024, 1)
    best, cost, log = at.search(base, synthetic_cost)
    assert (best.tile_w, best.tile_h, best.batch, best.batch_bwd,
            best.prefix_pairs_per_tile, best.tile_order) == (16, 8, 16, 8, 2048, 1)
    assert cost == pytest.approx(0.5)
    # the base is measured first and no candidate twice
    assert log[0][0] == base.__dict__
    keys = [json.dumps(o, sort_keys=True) for o, _ in log]
    assert len(set(keys)) == len(keys)


def test_n16_defaults_and_search_space_use_batches_of_4(tmp_path):
    assert at.resolve_defaults(Options(), 16).batch == 4
    assert at.resolve_defaults(Options(), 16).batch_bwd == 4
    splats = types.SimpleNamespace(P=100, N=16, textures=torch.zeros(1))
    views = [types.SimpleNamespace(width=32, height=32)]
    seen = []

    def cost(o):
        seen.append((o.batch, o.batch_bwd))
        return 1.0

    at.autotune(splats, views, cost=cost)
    assert set(seen) == {(4, 4)}


def test_search_keeps_the_base_when_it_is_best():
    best, cost, log = at.search(Options(), lambda o: 0.0 if o == Options() else 1.0)
    assert best == Options() and cost == 0.0


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    splats = types.SimpleNamespace(P=1000, N=8, textures=torch.zeros(1, dtype=torch.bfloat16))
    views = [types.SimpleNamespace(width=64, height=48)]
    calls = []

    def cost(o):
        calls.append(o)
        return synthetic_cost(o)

    o1, rec1 = at.autotune(splats, views, cache_path=path, cost=cost)
    n = len(calls)
    assert n > 1 and rec1["ms"] <= rec1["default_ms"]
    o2, rec2 = at.autotune(splats, views, cache_path=path, cost=cost)
    assert len(calls) == n and o2 == o1  # served from the cache
    key = at.workload_key(8, True, 1000, [(64, 48)])
    assert key == "N8-bf16-P1024-64x48"
    assert key in json.load(open(path))
