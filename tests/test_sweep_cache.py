"""Host side of the sweep autotuner's cache (no GPU): the shape class a
choice is kept under, and the JSON file it is kept in."""

import json

from paper_1707_07803_amd import tnrsvd as binding


def shapes(d, n, r, batch=1):
    one = [(1 if i == 0 else r, n, n, 1 if i == d - 1 else r) for i in range(d)]
    return [one] * batch


def test_shape_class_separates_what_sets_the_ranks():
    base = binding.sweep_shape_class(shapes(50, 2, 10), 10, 10, 2, 0.0, 32, 0, "k_last")
    assert base == binding.sweep_shape_class(shapes(50, 2, 10), 10, 10, 2, 0.0, 32, 0, "k_last")
    others = [
        binding.sweep_shape_class(shapes(50, 2, 10, batch=20), 10, 10, 2, 0.0, 32, 0, "k_last"),
        binding.sweep_shape_class(shapes(50, 4, 10), 10, 10, 2, 0.0, 32, 0, "k_last"),
        binding.sweep_shape_class(shapes(50, 2, 40), 10, 10, 2, 0.0, 32, 0, "k_last"),
        binding.sweep_shape_class(shapes(50, 2, 10), 10, 12, 2, 0.0, 32, 0, "k_last"),
        binding.sweep_shape_class(shapes(50, 2, 10), 10, 10, 1, 0.0, 32, 0, "k_last"),
        binding.sweep_shape_class(shapes(50, 2, 10), 10, 10, 2, 1e-6, 32, 0, "k_last"),
        binding.sweep_shape_class(shapes(50, 2, 10), 10, 10, 2, 0.0, 64, 0, "k_last"),
        binding.sweep_shape_class(shapes(50, 2, 10), 10, 10, 2, 0.0, 32, 48, "k_last"),
        binding.sweep_shape_class(shapes(50, 2, 10), 10, 10, 2, 0.0, 32, 0, "k_first"),
    ]
    assert all(o != base for o in others)
    assert len(set(others)) == len(others)


def test_cache_file_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "sweeps.json")
    assert binding.read_sweep_cache(path) == {}
    binding.write_sweep_cache(path, "gfx950|f32|a", [257, 1])
    binding.write_sweep_cache(path, "gfx950|f64|a", [0, 0])
    binding.write_sweep_cache(path, "gfx950|f32|a", [129, 0])     # replaced
    assert binding.read_sweep_cache(path) == {"gfx950|f32|a": [129, 0], "gfx950|f64|a": [0, 0]}
    assert json.load(open(path)) == {"gfx950|f32|a": [129, 0], "gfx950|f64|a": [0, 0]}


def test_unreadable_cache_is_empty(tmp_path):
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert binding.read_sweep_cache(str(bad)) == {}
    odd = tmp_path / "odd.json"
    odd.write_text(json.dumps({"k": [1, 2, 3], "j": "x", "ok": [513, 1]}))
    assert binding.read_sweep_cache(str(odd)) == {"ok": [513, 1]}
