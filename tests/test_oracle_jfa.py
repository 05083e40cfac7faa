"""Pins of the oracle's 3D jump flooding and coarse SDF (paper Sec. 2.1).

Jump flooding is an approximation of the nearest-seed transform, so it is
pinned by (i) the exact Euclidean distance transform (scipy's EDT and a brute
force over all seeds): flooding can never find a closer seed than the exact
one, and agrees with it almost everywhere; (ii) configurations where flooding
is provably exact (a single seed, a full plane of seeds); (iii) structural
invariants (seeds keep themselves, every answer is a seed, the tie rule).
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth.scenes import room_scene, tiny_scene

LO = np.zeros(3, np.float32)


def coords(idx, n):
    idx = np.asarray(idx)
    return np.stack([idx % n, (idx // n) % n, idx // (n * n)], -1)


def d2_of(seeds, n):
    p = coords(np.arange(n ** 3), n)
    s = coords(seeds, n)
    return ((p - s) ** 2).sum(-1)


def brute_nearest(seeds0, n):
    """Exact nearest seed (lowest index among equals) by brute force."""
    sidx = np.nonzero(seeds0 >= 0)[0]
    sc = coords(sidx, n)
    p = coords(np.arange(n ** 3), n)
    best = np.full(n ** 3, -1)
    bestd = np.full(n ** 3, np.iinfo(np.int64).max)
    for k in range(0, len(sidx), 256):
        d = ((p[:, None, :] - sc[None, k:k + 256, :]) ** 2).sum(-1)
        j = np.argmin(d, axis=1)  # first minimum = lowest index (sidx ascending)
        dj = d[np.arange(len(p)), j]
        upd = dj < bestd
        best[upd] = sidx[k + j[upd]]
        bestd[upd] = dj[upd]
    return best, bestd


@pytest.fixture(scope="module")
def tiny_flood():
    n = 32
    m = tiny_scene()
    s0 = oracle.voxelize(m.vertices, m.faces, LO, np.float32(1 / n), n)
    return n, s0, oracle.jfa(n, s0)


def test_seeds_keep_themselves_and_answers_are_seeds(tiny_flood):
    n, s0, s = tiny_flood
    occ = s0 >= 0
    assert np.array_equal(s[occ], s0[occ])
    assert np.all(s >= 0)
    assert np.all(s0[s] == s)


def test_never_closer_than_exact_and_rarely_worse(tiny_flood):
    n, s0, s = tiny_flood
    d2 = d2_of(s, n)
    best, bestd = brute_nearest(s0, n)
    # scipy's exact EDT agrees with the brute force (independent check of the latter)
    edt = ndimage.distance_transform_edt((s0 < 0).reshape(n, n, n))
    assert np.allclose(edt.ravel() ** 2, bestd)
    assert np.all(d2 >= bestd)
    err_rate = np.mean(d2 > bestd)
    # Rong & Tan report jump-flooding errors on a small fraction of pixels.
    assert err_rate < 0.02, err_rate
    # where the distance is exact, the tie rule picks the lowest seed index
    same = d2 == bestd
    assert np.mean(s[same] == best[same]) > 0.99


def test_room_error_rate():
    n = 64
    m = room_scene(1, n_prims=60)
    s0 = oracle.voxelize(m.vertices, m.faces, LO, np.float32(1 / n), n)
    s = oracle.jfa(n, s0)
    edt, ind = ndimage.distance_transform_edt((s0 < 0).reshape(n, n, n), return_indices=True)
    d2 = d2_of(s, n)
    assert np.all(d2 >= np.rint(edt.ravel() ** 2))
    assert np.mean(d2 > np.rint(edt.ravel() ** 2)) < 0.02


@pytest.mark.parametrize("n", [8, 16, 32])
def test_single_seed_exact(n):
    rng = np.random.default_rng(n)
    for _ in range(3):
        s0 = np.full(n ** 3, -1, np.int32)
        q = int(rng.integers(0, n ** 3))
        s0[q] = q
        s = oracle.jfa(n, s0)
        assert np.all(s == q)


def test_full_plane_exact():
    n, y0 = 32, 11
    s0 = np.full(n ** 3, -1, np.int32)
    p = coords(np.arange(n ** 3), n)
    on = p[:, 1] == y0
    s0[on] = np.nonzero(on)[0]
    s = oracle.jfa(n, s0)
    want = p[:, 0] + n * (y0 + n * p[:, 2])
    assert np.array_equal(s, want)


def test_tie_goes_to_lowest_index():
    # Two seeds mirrored about the plane x = 8 (n = 16): voxels on that plane are
    # equidistant and must take the lower linear index.
    n = 16
    a = 5 + n * (7 + n * 9)
    b = 11 + n * (7 + n * 9)
    s0 = np.full(n ** 3, -1, np.int32)
    s0[a], s0[b] = a, b
    s = oracle.jfa(n, s0)
    best, _ = brute_nearest(s0, n)
    assert np.array_equal(s, best)
    p = coords(np.arange(n ** 3), n)
    assert np.all(s[p[:, 0] == 8] == min(a, b))


def test_step_schedule_matters():
    # The passes must go n/2, n/4, ..., 1: stopping before step 1 leaves voxels
    # between seeds unresolved.  A pass with step 1 alone (no jumps) only
    # reaches direct neighbours.
    n = 16
    s0 = np.full(n ** 3, -1, np.int32)
    s0[0] = 0
    one = oracle.jfa_pass(n, 1, s0)
    assert (one >= 0).sum() == 8
    s = s0
    for k in (8, 4, 2):
        s = oracle.jfa_pass(n, k, s)
    assert np.any(s < 0)
    assert np.all(oracle.jfa_pass(n, 1, s) == 0)


def test_coarse_sdf_float32_definition(tiny_flood):
    n, s0, s = tiny_flood
    h = np.float32(1 / n)
    beta = np.float32(0.5) * h
    d2, c = oracle.coarse(n, s, h, beta)
    assert np.array_equal(d2, d2_of(s, n).astype(np.int32))
    # float32: h * sqrt(D2) - beta, each operation rounded once (numpy float32)
    want = (h * np.sqrt(d2.astype(np.float32))) - beta
    assert want.dtype == np.float32
    assert np.array_equal(c.view(np.int32), want.view(np.int32))
    # occupied voxels get exactly -beta: surfaces become negative (Sec. 2.1)
    assert np.all(c[s0 >= 0] == -beta)
    assert np.all(c[s0 < 0] > 0)
    # perfect squares are exact
    sq = d2 == 16
    assert np.all(c[sq] == np.float32(4) * h - beta)


def test_coarse_empty_grid():
    n = 8
    s = oracle.jfa(n, np.full(n ** 3, -1, np.int32))
    assert np.all(s == -1)
    d2, c = oracle.coarse(n, s, np.float32(1 / n), np.float32(0.01))
    assert np.all(d2 == np.iinfo(np.int32).max)
    assert np.all(np.isinf(c))


# ---------------------------------------------------- pass schedules ----
# The error-reducing variants of jump flooding (Rong & Tan): JFA+1 adds a pass
# with step 1, JFA+2 adds passes 2 and 1, 1+JFA runs a step-1 pass first.

def schedule(n, variant):
    base = [n >> i for i in range(1, int(np.log2(n)) + 1)]
    return {"jfa": base, "jfa+1": base + [1], "jfa+2": base + [2, 1], "1+jfa": [1] + base}[variant]


def test_schedule_driver_composes_passes(tiny_flood):
    n, s0, s = tiny_flood
    assert np.array_equal(oracle.jfa_steps(n, s0, schedule(n, "jfa")), s)
    # two passes by hand
    want = oracle.jfa_pass(n, 2, oracle.jfa_pass(n, 8, s0))
    assert np.array_equal(oracle.jfa_steps(n, s0, [8, 2]), want)
    assert np.array_equal(oracle.jfa_steps(n, s0, []), s0)


@pytest.mark.parametrize("variant", ["jfa+1", "jfa+2", "1+jfa"])
def test_variants_exact_on_single_seed_and_plane(variant):
    n = 16
    rng = np.random.default_rng(11)
    s0 = np.full(n ** 3, -1, np.int32)
    q = int(rng.integers(0, n ** 3))
    s0[q] = q
    assert np.all(oracle.jfa_steps(n, s0, schedule(n, variant)) == q)
    s0 = np.full(n ** 3, -1, np.int32)
    p = coords(np.arange(n ** 3), n)
    on = p[:, 2] == 5
    s0[on] = np.nonzero(on)[0]
    want = p[:, 0] + n * (p[:, 1] + n * 5)
    assert np.array_equal(oracle.jfa_steps(n, s0, schedule(n, variant)), want)


def test_variant_error_rates_room():
    """Extra passes never lengthen a voxel's distance (every pass keeps the
    voxel's own seed as a candidate), so JFA+1 and JFA+2 are pointwise between
    the exact transform and plain JFA; all variants stay >= exact."""
    n = 64
    m = room_scene(1, n_prims=60)
    s0 = oracle.voxelize(m.vertices, m.faces, LO, np.float32(1 / n), n)
    exact = np.rint(ndimage.distance_transform_edt((s0 < 0).reshape(n, n, n)).ravel() ** 2)
    d = {v: d2_of(oracle.jfa_steps(n, s0, schedule(n, v)), n) for v in ("jfa", "jfa+1", "jfa+2", "1+jfa")}
    rates = {v: float(np.mean(x > exact)) for v, x in d.items()}
    print("error rates (fraction of voxels farther than the exact EDT):", rates)
    for v, x in d.items():
        assert np.all(x >= exact), v
    assert np.all(d["jfa+1"] <= d["jfa"]) and np.all(d["jfa+2"] <= d["jfa"])
    assert rates["jfa+1"] <= rates["jfa"] and rates["jfa+2"] <= rates["jfa"]
    assert rates["jfa"] < 0.02
