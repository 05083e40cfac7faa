"""Exact-rational pins of the oracle's voxelization rule (Sec. 2.1: the scene is
rasterized along x, y and z; the rule used for the raster is stated in the
oracle's header) on the tiny workload (UV sphere of 320 triangles over a
ground quad, 32^3; also 64^3).

Every (triangle, axis, column) decision is re-evaluated here in Python's
``fractions.Fraction`` with a different construction from the oracle's int64
edge functions and integer floor division: the column centre's barycentric
coordinates in the projected triangle by Cramer's rule, "inside" when all
three are >= 0, the depth as the barycentric combination of the vertex
depths, its floor as the layer (a depth exactly on the far face goes to the
last layer; other depths outside [0, n) drop the voxel).  All columns whose
centre lies in the projected triangle's bounding box are evaluated; a centre
outside that box is outside the triangle.  The union over all decisions must
equal the oracle's occupancy exactly.

Snapping sensitivity: the same decisions from the unsnapped float32 vertex
positions (exact rationals of the floats) are counted where they differ from
the snapped ones; the count is reported and must stay a small fraction.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth.scenes import tiny_scene

LO = np.zeros(3, np.float32)


def snapped_coords(v, n):
    """Vertex coordinates in voxel units as exact rationals after the snap to 1/256 of a voxel (round half to
    even of (v - lo) / h * 256 in double precision: exact for h = 2^-k)."""
    h = np.float32(1.0 / n)
    X = np.rint((v.astype(np.float64) - LO.astype(np.float64)) / np.float64(h) * 256.0).astype(np.int64)
    return [[Fraction(int(x), 256) for x in row] for row in X]


def raw_coords(v, n):
    h = Fraction(float(np.float32(1.0 / n)))
    return [[(Fraction(float(x)) - Fraction(float(l))) / h for x, l in zip(row, LO)] for row in v]


def decisions(coords, faces, n):
    """{(tri, axis, i, j): layer or None} for every column centre in each projected triangle's bounding box."""
    out = {}
    half = Fraction(1, 2)
    for t, (a_, b_, c_) in enumerate(faces):
        A, B, C = coords[a_], coords[b_], coords[c_]
        for ax in range(3):
            e1, e2 = (ax + 1) % 3, (ax + 2) % 3
            p = [(A[e1], A[e2]), (B[e1], B[e2]), (C[e1], C[e2])]
            z = (A[ax], B[ax], C[ax])
            det = (p[1][0] - p[0][0]) * (p[2][1] - p[0][1]) - (p[2][0] - p[0][0]) * (p[1][1] - p[0][1])
            if det == 0:
                continue  # edge-on along this axis
            lo_i = max(0, int(np.floor(float(min(q[0] for q in p)) - 0.5)) - 1)
            hi_i = min(n - 1, int(np.ceil(float(max(q[0] for q in p)) - 0.5)) + 1)
            lo_j = max(0, int(np.floor(float(min(q[1] for q in p)) - 0.5)) - 1)
            hi_j = min(n - 1, int(np.ceil(float(max(q[1] for q in p)) - 0.5)) + 1)
            for i in range(lo_i, hi_i + 1):
                for j in range(lo_j, hi_j + 1):
                    cx, cy = i + half, j + half
                    # Cramer: c = p0 + l1 (p1 - p0) + l2 (p2 - p0)
                    rx, ry = cx - p[0][0], cy - p[0][1]
                    l1 = (rx * (p[2][1] - p[0][1]) - (p[2][0] - p[0][0]) * ry) / det
                    l2 = ((p[1][0] - p[0][0]) * ry - rx * (p[1][1] - p[0][1])) / det
                    l0 = 1 - l1 - l2
                    if l0 < 0 or l1 < 0 or l2 < 0:
                        out[(t, ax, i, j)] = None
                        continue
                    depth = l0 * z[0] + l1 * z[1] + l2 * z[2]
                    if depth == n:
                        layer = n - 1
                    else:
                        layer = depth.numerator // depth.denominator
                        if layer < 0 or layer >= n:
                            layer = None
                    out[(t, ax, i, j)] = layer
    return out


def occupancy(dec, n):
    occ = np.full(n ** 3, -1, np.int32)
    for (t, ax, i, j), layer in dec.items():
        if layer is None:
            continue
        q = [0, 0, 0]
        q[ax], q[(ax + 1) % 3], q[(ax + 2) % 3] = layer, i, j
        idx = q[0] + n * (q[1] + n * q[2])
        occ[idx] = idx
    return occ


@pytest.mark.parametrize("n", [32, 64])
def test_every_decision_exact_rational(n):
    m = tiny_scene()
    dec = decisions(snapped_coords(m.vertices, n), m.faces, n)
    want = occupancy(dec, n)
    got = oracle.voxelize(m.vertices, m.faces, LO, np.float32(1.0 / n), n)
    assert np.array_equal(got, want), int((got != want).sum())
    inside = sum(1 for v in dec.values() if v is not None)
    print(f"n={n}: {len(dec)} (triangle, axis, column) decisions, {inside} covered, "
          f"{int((want >= 0).sum())} voxels")
    assert inside > 1000


@pytest.mark.parametrize("n", [32, 64])
def test_snapping_sensitivity_count(n):
    m = tiny_scene()
    snap = decisions(snapped_coords(m.vertices, n), m.faces, n)
    raw = decisions(raw_coords(m.vertices, n), m.faces, n)
    keys = set(snap) | set(raw)
    flips = sum(1 for k in keys if snap.get(k) != raw.get(k))
    covered = sum(1 for v in snap.values() if v is not None)
    print(f"n={n}: {flips} of {len(keys)} decisions change without the 1/256-voxel snap ({covered} covered)")
    assert flips <= 0.005 * covered
