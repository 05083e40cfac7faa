"""Pins of the oracle's selection (Sec. 2.2, Eq. (1) case split c <= d) and of
its random ray directions (Sec. 2.2: random points on a sphere).

The random bits are Philox4x64-10 (Salmon et al., SC'11); numpy ships an
independent implementation of the same generator, which pins the oracle's
round function, constants and key schedule.  Directions are pinned by the
sphere-point distribution itself (Archimedes: each coordinate of a uniform
point on the unit sphere is uniform on [-1, 1]).
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from synth.scenes import tiny_scene

LO = np.zeros(3, np.float32)


def morton_by_string(x, y, z, bits=10):
    """Morton code built by interleaving binary strings (z y x per level)."""
    s = ""
    for b in reversed(range(bits)):
        s += str((z >> b) & 1) + str((y >> b) & 1) + str((x >> b) & 1)
    return int(s, 2)


def test_threshold_closed_forms():
    h = np.float32(1 / 32)
    # (d + beta) / h = 2.5 -> K = 6 ;  3.5 -> 12 ; exactly 2 -> 4 (c <= d inclusive)
    assert oracle.select_threshold(h, np.float32(0.5) * h, np.float32(2) * h) == 6
    assert oracle.select_threshold(h, np.float32(0.5) * h, np.float32(3) * h) == 12
    assert oracle.select_threshold(h, np.float32(0), np.float32(2) * h) == 4


def test_plane_selects_band_and_morton_order():
    nc, nf, y0 = 16, 32, 6
    p = np.arange(nc ** 3)
    s0 = np.full(nc ** 3, -1, np.int32)
    on = (p // nc) % nc == y0
    s0[on] = p[on]
    s = oracle.jfa(nc, s0)
    h = np.float32(1 / nc)
    d2, c = oracle.coarse(nc, s, h, np.float32(0.5) * h)
    K = oracle.select_threshold(h, np.float32(0.5) * h, np.float32(2) * h)
    mask, queue = oracle.select(nc, d2, nf, K)
    j = np.arange(nf ** 3)
    fy = (j // nf) % nf
    # coarse layers |y - y0| <= floor(sqrt(6)) = 2 -> fine layers 2*(y0-2) .. 2*(y0+2)+1
    want = (fy >= 2 * (y0 - 2)) & (fy <= 2 * (y0 + 2) + 1)
    assert np.array_equal(mask.astype(bool), want)
    # equivalently: exactly the texels whose coarse value satisfies c <= d
    cz = c.reshape(nc, nc, nc)
    fz, fyy, fx = np.meshgrid(np.arange(nf), np.arange(nf), np.arange(nf), indexing="ij")
    cf = cz[fz // 2, fyy // 2, fx // 2].ravel()
    assert np.array_equal(mask.astype(bool), cf <= np.float32(2) * h)
    assert sorted(queue.tolist()) == np.nonzero(mask)[0].tolist()
    m = [morton_by_string(q % nf, (q // nf) % nf, q // (nf * nf)) for q in queue]
    assert all(a < b for a, b in zip(m, m[1:]))


def test_selection_monotone_in_d_and_children_counts():
    nc, nf = 32, 64
    mesh = tiny_scene()
    h = np.float32(1 / nc)
    s = oracle.jfa(nc, oracle.voxelize(mesh.vertices, mesh.faces, LO, h, nc))
    d2, _ = oracle.coarse(nc, s, h, np.float32(0.5) * h)
    prev = None
    for dv in (0.0, 1.0, 2.0, 3.0, 5.0):
        K = oracle.select_threshold(h, np.float32(0.5) * h, np.float32(dv) * h)
        mask, queue = oracle.select(nc, d2, nf, K)
        assert len(queue) == mask.sum() == 8 * (d2 <= K).sum()
        if prev is not None:
            assert np.all(mask >= prev)  # larger d traces more texels (Sec. 2.2)
        prev = mask


def test_philox_matches_numpy():
    rng = np.random.default_rng(11)
    for _ in range(25):
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        ctr = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr)
        want = bg.random_raw(4)
        # numpy advances the 256-bit counter by one before producing a block
        c1 = ctr.copy()
        c1[0] += np.uint64(1)
        if c1[0] == 0:
            c1[1] += np.uint64(1)
        got = oracle.philox4x64_10(c1, key)
        assert np.array_equal(got, np.asarray(want, np.uint64))


def test_philox_carry_counter():
    # counter word 0 at its maximum: numpy carries into word 1
    key = np.array([3, 5], np.uint64)
    ctr = np.array([2 ** 64 - 1, 7, 0, 0], np.uint64)
    want = np.random.Philox(key=key, counter=ctr).random_raw(4)
    got = oracle.philox4x64_10(np.array([0, 8, 0, 0], np.uint64), key)
    assert np.array_equal(got, np.asarray(want, np.uint64))


@pytest.fixture(scope="module")
def dirs():
    out = np.empty((20000, 3), np.float32)
    att = np.empty(20000, int)
    for i in range(20000):
        out[i], att[i] = oracle.direction(0, i // 16, 3, i % 16)
    return out, att


def test_direction_unit_length(dirs):
    d, att = dirs
    norm = np.linalg.norm(d.astype(np.float64), axis=1)
    assert np.all(np.abs(norm - 1) < 2 ** -21)
    # acceptance rate of a pair is pi/4: two or more attempts is rare
    assert np.mean(att > 0) < 0.01


def test_direction_uniform_on_sphere(dirs):
    d, _ = dirs
    d = d.astype(np.float64)
    for a in range(3):
        assert stats.kstest(d[:, a], stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3
    assert np.all(np.abs(d.mean(0)) < 0.03)
    cov = d.T @ d / len(d)
    assert np.allclose(cov, np.eye(3) / 3, atol=0.02)


def test_direction_depends_on_every_key_part():
    base, _ = oracle.direction(0, 10, 2, 3, 0)
    for args in [(1, 10, 2, 3, 0), (0, 11, 2, 3, 0), (0, 10, 3, 3, 0), (0, 10, 2, 4, 0), (0, 10, 2, 3, 1)]:
        other, _ = oracle.direction(*args)
        assert not np.array_equal(base, other)


def test_texel_origin_is_centre():
    for nf in (64, 256):
        h = np.float32(1) / np.float32(nf)
        for j in (0, 5, nf ** 3 - 1, 12345 % nf ** 3):
            o = oracle.texel_origin(nf, LO, h, j)
            want = (np.array([j % nf, (j // nf) % nf, j // nf ** 2]) + 0.5) / nf
            assert np.array_equal(o.astype(np.float64), want)
