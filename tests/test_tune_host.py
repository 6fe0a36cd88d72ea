"""The autotuner's host logic without a GPU: size-class keys, the coordinate
search on synthetic costs, and the cache lookup."""
import json

import numpy as np

from paper_2507_00528_amd import nep, synth, tune


class _B:
    def __init__(self, n_atom, max_atoms, tilt=None):
        self.n_atom, self.max_atoms, self.tilt = n_atom, max_atoms, tilt


def test_size_class_separates_models_shapes_and_sizes():
    m = nep.Model.of(synth.SIZES_LARGE)
    k = tune.size_class(m, _B(87471, 512))
    assert k == "T2-R7x11-A5x11-l4.2.1-H50-cap64.32-orth-N2^16-small"
    assert tune.size_class(m, _B(27000, 27000)).endswith("N2^15-large")
    assert tune.size_class(m, _B(87471, 512, tilt=object())) != k
    assert tune.size_class(nep.Model.of(synth.SIZES_SMALL), _B(87471, 512)) != k
    assert tune.size_class(m, _B(0, 0)).endswith("N2^0-large")   # empty batch: max_atoms unknown


def test_search_finds_the_optimum_of_a_separable_cost():
    space = {"a": [0, 1, 2], "b": [10, 20, 30], "c": [5, 6]}
    want = {"a": 2, "b": 10, "c": 6}
    cost = lambda c: 1.0 + sum(abs(c[k] - want[k]) for k in c) * 0.1
    best, best_ms, base_ms, table = tune.search(cost, space)
    assert best == want
    assert best_ms == 1.0
    assert base_ms == cost({"a": 0, "b": 10, "c": 5})
    assert len(table) <= 1 + 2 * (2 + 2 + 1)          # each choice swept at most twice


def test_search_keeps_defaults_unless_the_gain_is_real_and_skips_refused_choices():
    space = {"a": [0, 1], "b": [0, 1]}
    cost = {(0, 0): 1.0, (1, 0): 0.995, (0, 1): None, (1, 1): 0.5}
    best, best_ms, _, _ = tune.search(lambda c: cost[(c["a"], c["b"])], space, min_gain=0.01)
    assert best == {"a": 0, "b": 0} and best_ms == 1.0   # 0.5% is noise; (0, 1) is refused


def test_cache_lookup_and_nondefault(tmp_path):
    m = nep.Model.of(synth.SIZES_LARGE)
    b = _B(87471, 512)
    p = tmp_path / "tuning.json"
    json.dump({tune.size_class(m, b): {"tuning": {"outer_blocks_w": 128}, "ms": 0.5}}, open(p, "w"))
    assert tune.lookup(m, b, path=str(p)) == {"outer_blocks_w": 128}
    assert tune.lookup(m, _B(1000, 100), path=str(p)) is None
    assert tune.nondefault(dict(tune.DEFAULTS, gather_lanes=8)) == {"gather_lanes": 8}


def test_tuning_struct_validates_keys():
    s = nep.tuning_struct({"outer_blocks_w": 96, "gather_lanes": 8})
    assert (s.outer_blocks_w, s.gather_lanes, s.persistent) == (96, 8, 0)
    try:
        nep.tuning_struct({"bogus": 1})
    except ValueError:
        pass
    else:
        raise AssertionError("unknown key accepted")
