"""Pins of the oracle's trilinear coarse sampling and of its selection on a
field given at the fine texels (the smoother reading of the coarse value c that
Sec. 2.2 compares with d; Sec. 2.1 notes the point-sampled coarse SDF is blocky).

* Against scipy's linear spline interpolation (``map_coordinates``, order 1) of
  the same samples at the same points: an independent implementation.
* An affine field in world coordinates, sampled at coarse voxel centres, is
  reproduced exactly at the fine texel centres inside the outermost coarse
  centres (linear interpolation is exact for linear functions; with dyadic
  coefficients no rounding occurs), and is held constant beyond them.
* A seed plane gives a coarse SDF that is piecewise linear with its kink at a
  sample, so the interpolated field and its selected band have closed forms
  that differ from point sampling by one fine layer on each side.
* Field selection equals point-sampled selection on the nearest-voxel field,
  and its queue is in Morton order.
"""
import numpy as np
from scipy import ndimage

import oracle
from synth.scenes import tiny_scene

LO = np.zeros(3, np.float32)


def morton_by_string(x, y, z, bits=10):
    s = ""
    for b in reversed(range(bits)):
        s += str((z >> b) & 1) + str((y >> b) & 1) + str((x >> b) & 1)
    return int(s, 2)


def fine_centres_in_coarse_units(nc, nf):
    """Fine texel centres expressed in coarse index units (voxel i's centre is at i)."""
    j = np.arange(nf)
    world = (j + 0.5) / nf                 # centre in the unit box
    return np.clip(world * nc - 0.5, 0, nc - 1)


def test_matches_scipy_linear_interpolation():
    rng = np.random.default_rng(5)
    for nc, nf in ((8, 8), (8, 16), (4, 32), (16, 64)):
        c = rng.uniform(-1, 2, nc ** 3).astype(np.float32)
        got = oracle.coarse_trilinear(nc, c, nf).astype(np.float64).reshape(nf, nf, nf)
        u = fine_centres_in_coarse_units(nc, nf)
        Z, Y, X = np.meshgrid(u, u, u, indexing="ij")
        want = ndimage.map_coordinates(c.astype(np.float64).reshape(nc, nc, nc), [Z.ravel(), Y.ravel(), X.ravel()],
                                       order=1, mode="nearest").reshape(nf, nf, nf)
        assert np.max(np.abs(got - want)) <= 4e-7 * 3, (nc, nf)
        if nc == nf:
            assert np.array_equal(got.ravel(), c.astype(np.float64))  # r = 1 is the identity


def test_affine_field_reproduced_exactly():
    nc, nf = 8, 32
    A = np.array([3.0, 5.0, -2.0]) * nc  # world-space gradient
    i = np.arange(nc) + 0.5
    Z, Y, X = np.meshgrid(i / nc, i / nc, i / nc, indexing="ij")
    c = (A[0] * X + A[1] * Y + A[2] * Z + 1.0).astype(np.float32).ravel()
    got = oracle.coarse_trilinear(nc, c, nf).astype(np.float64).reshape(nf, nf, nf)
    # world position of each fine centre, clamped to the span of the coarse centres
    p = np.clip((np.arange(nf) + 0.5) / nf, 0.5 / nc, 1 - 0.5 / nc)
    Zf, Yf, Xf = np.meshgrid(p, p, p, indexing="ij")
    want = A[0] * Xf + A[1] * Yf + A[2] * Zf + 1.0
    assert np.array_equal(got, want)


def test_infinite_corner_gives_infinity():
    nc, nf = 8, 16
    assert np.all(np.isinf(oracle.coarse_trilinear(nc, np.full(nc ** 3, np.inf, np.float32), nf)))
    c = np.ones(nc ** 3, np.float32)
    c[3 + nc * (3 + nc * 3)] = np.inf
    got = oracle.coarse_trilinear(nc, c, nf).reshape(nf, nf, nf)
    u = fine_centres_in_coarse_units(nc, nf)
    near = (np.floor(u) <= 3) & (np.minimum(np.floor(u) + 1, nc - 1) >= 3)  # cell corners include index 3
    Z, Y, X = np.meshgrid(near, near, near, indexing="ij")
    assert np.array_equal(np.isinf(got), Z & Y & X)
    assert np.all(got[~(Z & Y & X)] == 1.0)


def test_plane_band_closed_form():
    nc, nf, y0 = 16, 32, 6
    p = np.arange(nc ** 3)
    s0 = np.full(nc ** 3, -1, np.int32)
    on = (p // nc) % nc == y0
    s0[on] = p[on]
    h = np.float32(1 / nc)
    beta = np.float32(0.5) * h
    d2, c = oracle.coarse(nc, oracle.jfa(nc, s0), h, beta)
    cf = oracle.coarse_trilinear(nc, c, nf)
    j = np.arange(nf ** 3)
    fy = (j // nf) % nf
    u = np.clip(fy / 2 - 0.25, 0, nc - 1)  # fine layer centre in coarse units
    assert np.array_equal(cf.astype(np.float64), np.abs(u - y0) * float(h) - float(beta))
    d = np.float32(2.25) * h
    mask, queue = oracle.select_field(nf, cf, d)
    # |u - y0| <= (d + beta)/h = 2.75  ->  fine layers 2 y0 - 5 .. 2 y0 + 6
    assert np.array_equal(mask.astype(bool), (fy >= 2 * y0 - 5) & (fy <= 2 * y0 + 6))
    # point sampling: D^2 <= floor(2.75^2) = 7 -> coarse layers y0 +- 2 -> fine 2 y0 - 4 .. 2 y0 + 5
    pm, _ = oracle.select(nc, d2, nf, oracle.select_threshold(h, beta, d))
    assert np.array_equal(pm.astype(bool), (fy >= 2 * y0 - 4) & (fy <= 2 * y0 + 5))
    assert sorted(queue.tolist()) == np.nonzero(mask)[0].tolist()


def test_field_selection_equals_point_selection_on_nearest_field():
    nc, nf = 32, 64
    mesh = tiny_scene()
    h = np.float32(1 / nc)
    beta = np.float32(0.5) * h
    d2, c = oracle.coarse(nc, oracle.jfa(nc, oracle.voxelize(mesh.vertices, mesh.faces, LO, h, nc)), h, beta)
    j = np.arange(nf ** 3)
    x, y, z = j % nf, (j // nf) % nf, j // nf ** 2
    nearest = c[(x // 2) + nc * ((y // 2) + nc * (z // 2))]
    for dv in (0.0, 1.25, 2.25, 4.75):  # c = h sqrt(D^2) - beta never equals d for these
        d = np.float32(dv) * h
        m1, q1 = oracle.select_field(nf, nearest, d)
        m2, q2 = oracle.select(nc, d2, nf, oracle.select_threshold(h, beta, d))
        assert np.array_equal(m1, m2) and np.array_equal(q1, q2), dv
    m, q = oracle.select_field(nf, nearest, np.float32(2.25) * h)
    mk = [morton_by_string(t % nf, (t // nf) % nf, t // (nf * nf)) for t in q]
    assert all(a < b for a, b in zip(mk, mk[1:]))
    assert oracle.select_field(nf, nearest, np.float32(-np.inf))[1].size == 0
    assert oracle.select_field(nf, np.full(nf ** 3, np.inf, np.float32), np.float32(1e30))[1].size == 0


def test_trilinear_pipeline_selection_monotone_and_superset_on_curved_scene():
    nc, nf = 32, 64
    mesh = tiny_scene()
    h = np.float32(1 / nc)
    beta = np.float32(0.5) * h
    _, c = oracle.coarse(nc, oracle.jfa(nc, oracle.voxelize(mesh.vertices, mesh.faces, LO, h, nc)), h, beta)
    cf = oracle.coarse_trilinear(nc, c, nf)
    prev = None
    for dv in (0.0, 1.0, 2.0, 3.0):
        m, _ = oracle.select_field(nf, cf, np.float32(dv) * h)
        if prev is not None:
            assert np.all(m >= prev)
        prev = m
    # interpolation stays within the corner values: the field is finite and >= min(c)
    assert np.all(np.isfinite(cf)) and cf.min() >= c.min() and cf.max() <= c.max()
