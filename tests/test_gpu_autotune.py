"""GPU: tile autotuning and the tune cache.

The tuner times every compiled tile shape on one geometry, for one slice and
for stacks, and records the fastest of each; plans created afterwards use them,
plans that already exist keep theirs.
With FBP_TUNE_CACHE set, the choice is appended to a file, and the entries of the
file it names are applied when plans are created.  Every tile shape gives the
oracle's result (checked in the parity tests), so tuning only moves time, never
the tolerance.
"""
import numpy as np
import pytest
import torch

import paper_2109_02174_amd as fbp

pytestmark = pytest.mark.gpu


def test_autotune_picks_a_valid_shape_and_new_plans_use_it():
    g = fbp.Geometry(97, 141, 99, 1.0)          # a geometry no other test creates
    best = fbp.fbp_autotune(g)
    assert 0 <= best < fbp.fbp_num_tile_configs()
    assert fbp.fbp_plan_config(g) == best
    # re-tuning does not change an existing plan's shape (results stay reproducible)
    q = torch.randn(1, 97, 141, device="cuda")
    a = fbp.fbp_backproject(g, q).cpu().numpy()
    fbp.fbp_autotune(g)
    assert fbp.fbp_plan_config(g) == best
    assert np.array_equal(a, fbp.fbp_backproject(g, q).cpu().numpy())


def test_tune_cache_round_trip(tmp_path, monkeypatch):
    # tuning appends "arch K D N dt_bits angle_hash single_tile stack_tile filter weighting"
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FBP_TUNE_CACHE", str(cache))
    g = fbp.Geometry(61, 87, 57, 1.0)           # no plan of it exists yet
    best = fbp.fbp_autotune(g)
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1
    fields = lines[0].split()
    assert fields[0].startswith("gfx") and fields[1:4] == ["61", "87", "57"] and int(fields[6]) == best
    assert fields[8:] == ["0", "0"]
    # a cache file with other entries for the geometry is read when its plan is created
    plain = [c for c in range(fbp.fbp_num_tile_configs()) if "rotations" not in fbp.fbp_tile_config_name(c)]
    one = next(c for c in plain if c != best)
    stack = next(c for c in plain if c != int(fields[7]))
    cache2 = tmp_path / "tune2.txt"
    cache2.write_text(" ".join(fields[:6] + [str(one), str(stack)] + fields[8:]) + "\n")
    monkeypatch.setenv("FBP_TUNE_CACHE", str(cache2))
    assert fbp.fbp_plan_config(g) == one
    assert fbp.fbp_plan_stack_config(g) == stack
