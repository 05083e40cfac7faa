"""CPU checks of the autotuner's search (no GPU: the measurement is a synthetic
cost function).  Coordinate descent must try every value of every knob, end at
a coordinate-wise minimum, and find the global minimum of a separable cost;
small spaces are timed exhaustively."""
import itertools
import math

import pytest


@pytest.fixture(scope="module")
def AT():
    from paper_2210_04449_amd import autotune
    return autotune


def test_descent_finds_separable_minimum_and_tries_every_value(AT):
    space = AT.SPACE
    best_vals = {"blocks_per_cu": 4, "tile_texels": 32, "refill": 16, "stack_lds": 16, "bin_directions": 1, "loop": 3,
                 "bvh_width": 4}

    def cost(t):
        return 10.0 + sum((i + 1) * 0.1 * (t[k] != best_vals[k]) for i, k in enumerate(space))

    start = {k: v[0] for k, v in space.items()}
    best, ms, trials = AT.search(cost, start, space)
    assert best == best_vals and math.isclose(ms, 10.0)
    for k, vals in space.items():
        assert {t[k] for t, _ in trials} == set(vals), k
    # far fewer trials than the product of the space
    assert len(trials) < math.prod(len(v) for v in space.values()) // 4


def test_descent_result_is_a_coordinate_minimum(AT):
    space = {"a": (0, 1, 2, 3), "b": (0, 1, 2), "c": (0, 1)}

    def cost(t):  # coupled: the best b depends on a
        return (t["a"] - 2) ** 2 + (t["b"] - (t["a"] % 3)) ** 2 + 0.5 * t["c"] + 0.1 * t["a"] * t["b"] + 1.0

    best, ms, _ = AT.search(cost, {"a": 0, "b": 0, "c": 1}, space, exhaustive=False, min_gain=0.0)
    for k, vals in space.items():
        for v in vals:
            assert cost({**best, k: v}) >= ms - 1e-12, (k, v)


def test_small_space_is_exhaustive(AT):
    space = {"x": (0, 1), "y": (0, 1, 2)}
    seen = []

    def cost(t):
        seen.append(dict(t))
        return 5 - t["x"] - t["y"]

    best, ms, trials = AT.search(cost, {"x": 0, "y": 0}, space)
    assert best == {"x": 1, "y": 2} and ms == 2
    assert sorted(map(lambda t: (t["x"], t["y"]), seen)) == sorted(itertools.product((0, 1), (0, 1, 2)))
