"""Autotuner host logic: the coordinate search, the per-model file naming and
the validity of any committed tuned parameter file."""
import glob
import json
import math
import os

import pytest

from paper_1508_03619_amd import autotune as at


def test_coordinate_descent_finds_separable_optimum():
    space = {"a": [1, 2, 3, 4], "b": [10, 20, 30], "c": [0, 1]}
    target = {"a": 3, "b": 10, "c": 1}
    calls = []

    def score(p):
        calls.append(dict(p))
        return 1.0 + sum((p[k] - target[k]) ** 2 for k in p)

    best, s, nev = at.coordinate_descent(space, ["a", "b", "c"], {"a": 1, "b": 30, "c": 0}, score,
                                         passes=3, log=lambda m: None)
    assert best == target and s == pytest.approx(1.0)
    assert nev == len({tuple(sorted(c.items())) for c in calls})  # evaluations are cached


def test_coordinate_descent_ignores_noise_below_min_gain():
    space = {"a": [1, 2, 3]}
    best, _, _ = at.coordinate_descent(space, ["a"], {"a": 2}, lambda p: 1.0 - 0.001 * p["a"],
                                       passes=2, min_gain=0.01, log=lambda m: None)
    assert best == {"a": 2}


def test_coordinate_descent_scores_each_coordinate_on_its_own_items():
    """A two-argument score is asked per coordinate: a gain on the items a
    coordinate acts on counts in full, not diluted by items it leaves alone."""
    space = {"a": [1, 2], "b": [1, 2]}
    # a halves item 0's time only; b changes nothing
    def times(p):
        return [1.0 if p["a"] == 1 else 0.97, 1.0, 1.0, 1.0]
    acts = {"a": [0], "b": [0, 1, 2, 3], None: [0, 1, 2, 3]}

    def score(p, name):
        t = times(p)
        idx = acts[name]
        return math.exp(sum(math.log(t[i]) for i in idx) / len(idx))

    best, s, nev = at.coordinate_descent(space, ["a", "b"], {"a": 1, "b": 1}, score, passes=2,
                                         min_gain=0.02, log=lambda m: None)
    assert best == {"a": 2, "b": 1}  # 3 % on its own item; 0.76 % over all four
    assert s == pytest.approx(0.97 ** 0.25)
    assert nev == 3
    # the same gain scored over every item stays below min_gain
    best1, _, _ = at.coordinate_descent(space, ["a", "b"], {"a": 1, "b": 1},
                                        lambda p: score(p, None), passes=2, min_gain=0.02,
                                        log=lambda m: None)
    assert best1 == {"a": 1, "b": 1}


def test_affects_names_tuned_parameters():
    assert set(at.AFFECTS) <= set(at.SPACE)
    assert all(set(k) <= {"single", "batch"} for k in at.AFFECTS.values())
    # hub splitting is used by single searches and batches alike
    assert "hub_degree" not in at.AFFECTS and "chunk_edges" not in at.AFFECTS
    assert at.AFFECTS["batch_alpha"] == ("batch",) and at.AFFECTS["block"] == ("single",)


def test_space_covers_order_and_names_are_library_parameters():
    from paper_1508_03619_amd.gapbfs import PARAM_NAMES
    assert set(at.ORDER) == set(at.SPACE)
    assert set(at.SPACE) <= set(PARAM_NAMES)
    assert all(v % 64 == 0 for v in at.SPACE["chunk_edges"])
    assert set(at.SPACE["block"]) <= {256, 512, 1024}


def test_tuned_path_per_model():
    assert at.arch_key("gfx950:sramecc+:xnack-", 256) == "gfx950_256cu"
    assert at.tuned_path("gfx950", 256).endswith(os.path.join("tuned", "gfx950_256cu.json"))


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(at.TUNED_DIR, "*.json"))))
def test_committed_tuned_files_are_valid(path):
    from paper_1508_03619_amd.gapbfs import PARAM_NAMES
    params = at.read_tuned(path)
    assert set(params) <= set(PARAM_NAMES)
    for k, v in params.items():
        if k in at.SPACE:
            assert v in at.SPACE[k], (k, v)
    with open(path) as f:
        d = json.load(f)
    assert os.path.basename(path) == at.arch_key(d["device"]["arch"], d["device"]["compute_units"]) + ".json"
