"""Pins of the oracle's exact point-to-mesh distance (what the traced fine SDF
of Sec. 2.2 approaches from above).

* One triangle: the face, edge and vertex regions give the plane distance, the
  distance to the edge's line and the distance to the vertex, in closed form.
* An axis-aligned box mesh (12 triangles): the unsigned distance is the box's
  closed form, outside (|max(|p - c| - e, 0)|) and inside (the smallest
  margin to a face), over faces, edges and corners alike.
* A tessellated sphere: the distance of an outside point lies between its
  distances to the circumsphere and to the insphere.
* Points on the mesh are at distance 0, and the nearest-triangle index names a
  triangle at that distance.
"""
import math

import numpy as np
import pytest

import oracle
from synth.scenes import _unit_box, icosphere


def scene(v, f):
    return oracle.Scene(np.asarray(v, np.float32), np.asarray(f, np.int32))


def test_single_triangle_regions():
    sc = scene([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0, 1, 2]])
    cases = [
        ((0.2, 0.2, 0.5), 0.5),                      # face region
        ((0.2, 0.2, -0.25), 0.25),                   # face region, other side
        ((-1.0, -1.0, 0.0), math.sqrt(2.0)),         # vertex 0
        ((2.0, -0.5, 0.0), math.sqrt(1.0 + 0.25)),   # vertex 1
        ((0.5, -1.0, 0.3), math.sqrt(1.0 + 0.09)),   # edge 0-1
        ((1.0, 1.0, 0.0), 1.0 / math.sqrt(2.0)),     # hypotenuse 1-2
        ((-0.5, 0.5, 0.5), math.sqrt(0.5)),          # edge 2-0 (x = 0), above
    ]
    d, t = sc.point_distance([c[0] for c in cases])
    for (p, want), got in zip(cases, d):
        assert math.isclose(got, want, rel_tol=1e-12), (p, got, want)
    assert np.all(t == 0)


def box_udf(P, c, e):
    q = np.abs(P - c) - e
    outside = np.linalg.norm(np.maximum(q, 0), axis=1)
    inside = -np.max(q, axis=1)
    return np.where(np.all(q <= 0, axis=1), inside, outside)


def test_box_closed_form():
    v, f = _unit_box()
    c, e = np.array([0.5, 0.4, 0.6]), np.array([0.2, 0.1, 0.3])
    sc = scene(v * e + c, f)
    rng = np.random.default_rng(8)
    P = rng.uniform(-0.2, 1.2, (4000, 3))
    d, t = sc.point_distance(P)
    ve = (v * e + c).astype(np.float32).astype(np.float64)  # the mesh is stored from float32 vertices
    cf, ef = (ve.max(0) + ve.min(0)) / 2, (ve.max(0) - ve.min(0)) / 2
    assert np.max(np.abs(d - box_udf(P, cf, ef))) < 1e-12
    assert np.all((t >= 0) & (t < 12))


def test_sphere_bracket():
    R = 0.3
    m = icosphere(3, R, (0.5, 0.5, 0.5))
    sc = scene(m.vertices, m.faces)
    V = m.vertices.astype(np.float64)
    T = V[m.faces]
    n = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
    r_in = np.min(np.abs(np.einsum("ij,ij->i", n / np.linalg.norm(n, axis=1)[:, None], T[:, 0] - 0.5)))
    r_out = np.max(np.linalg.norm(V - 0.5, axis=1))
    rng = np.random.default_rng(9)
    dirs = rng.normal(size=(3000, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    rad = rng.uniform(0.35, 0.8, 3000)
    P = 0.5 + dirs * rad[:, None]
    d, _ = sc.point_distance(P)
    assert np.all(d >= rad - r_out - 1e-12) and np.all(d <= rad - r_in + 1e-12)


def test_points_on_mesh_and_nearest_triangle():
    m = icosphere(2, 0.3, (0.5, 0.5, 0.5))
    sc = scene(m.vertices, m.faces)
    T = m.vertices.astype(np.float32).astype(np.float64)[m.faces]
    rng = np.random.default_rng(10)
    b = rng.dirichlet(np.ones(3), size=len(T))
    P = np.einsum("tk,tkj->tj", b, T)
    d, t = sc.point_distance(P)
    assert np.max(d) < 1e-12
    # the reported triangle is at the reported distance
    Q = P + rng.normal(scale=0.05, size=P.shape)
    d, t = sc.point_distance(Q)
    for i in range(0, len(Q), 37):
        one = scene(T[t[i]], [[0, 1, 2]])
        assert one.point_distance(Q[i:i + 1])[0][0] == pytest.approx(d[i], rel=1e-12, abs=1e-15)
