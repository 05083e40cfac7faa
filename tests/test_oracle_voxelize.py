"""Pins of the oracle's voxelizer (paper Sec. 2.1: orthographic projections along
x, y and z, depth culling off, the voxel under every fragment is marked).

The oracle's rule is an integer edge-function test on vertices snapped to 1/256
voxel.  These tests check it against things fixed independently of that code:
closed forms for axis-aligned quads and lattice-aligned triangles, a
floating-point ray cast along each axis through every column centre, and
invariances of the definition (triangle order, winding).
"""
import numpy as np
import pytest

import oracle
from synth.scenes import Mesh, ground_quad, icosphere, room_box, tiny_scene

LO = np.zeros(3, np.float32)


def occupied(seeds, n):
    idx = np.nonzero(seeds >= 0)[0]
    return np.stack([idx % n, (idx // n) % n, idx // (n * n)], 1)


@pytest.mark.parametrize("n", [32, 64])
def test_ground_quad_closed_form(n):
    # An axis-aligned quad at height y0 covering the whole floor occupies exactly
    # layer floor(y0 / h) in every column (the two triangles share the diagonal;
    # closed coverage leaves no hole along it).
    q = ground_quad(0.15)
    seeds = oracle.voxelize(q.vertices, q.faces, LO, np.float32(1.0 / n), n)
    occ = occupied(seeds, n)
    layer = int(np.floor(np.float64(np.float32(0.15)) * n))
    assert layer == {32: 4, 64: 9}[n]
    assert len(occ) == n * n
    assert np.all(occ[:, 1] == layer)
    assert np.all(seeds[seeds >= 0] == np.nonzero(seeds >= 0)[0])


def test_partial_quad_footprint():
    # Quad x in [a, b], z in [c, e] at height y0: a column is covered iff its
    # centre (i + 1/2) h lies in the closed interval, in both directions.
    n = 32
    h = 1.0 / n
    rng = np.random.default_rng(7)
    for _ in range(20):
        a, b = np.sort(rng.uniform(0, 1, 2))
        c, e = np.sort(rng.uniform(0, 1, 2))
        y0 = rng.uniform(0.05, 0.95)
        v = np.array([[a, y0, c], [b, y0, c], [b, y0, e], [a, y0, e]], np.float32)
        f = np.array([[0, 2, 1], [0, 3, 2]], np.int32)
        # keep the test away from snapping ties (1/256 voxel)
        centres = (np.arange(n) + 0.5) * h
        if min(np.abs(np.subtract.outer([a, b, c, e], centres)).min() * n * 256, 1e9) < 2:
            continue
        if abs(y0 * n - round(y0 * n)) * 256 < 2:
            continue
        seeds = oracle.voxelize(v, f, LO, np.float32(h), n)
        occ = occupied(seeds, n)
        xs = np.nonzero((centres >= v[0, 0]) & (centres <= v[1, 0]))[0]
        zs = np.nonzero((centres >= v[0, 2]) & (centres <= v[2, 2]))[0]
        want = {(x, int(np.floor(np.float64(v[0, 1]) * n)), z) for x in xs for z in zs}
        got = {tuple(map(int, p)) for p in occ}
        assert got == want


@pytest.mark.parametrize("m", [0, 1, 5, 11])
def test_lattice_triangle_count(m):
    # Right triangle with its three corners on column centres: the covered
    # columns are the lattice points (i, j), i, j >= 0, i + j <= m, whose number
    # is (m + 1)(m + 2) / 2 -- boundary points included (closed triangle).
    n = 32
    h = 1.0 / n
    z0 = 0.4
    if m == 0:
        # degenerate: all three corners on one centre -> zero area, skipped
        v = np.array([[0.5 * h, 0.5 * h, z0]] * 3, np.float32)
        seeds = oracle.voxelize(v, np.array([[0, 1, 2]], np.int32), LO, np.float32(h), n)
        assert (seeds >= 0).sum() == 0
        return
    v = np.array([[0.5 * h + 3 * h, 0.5 * h + 2 * h, z0],
                  [(m + 3.5) * h, 2.5 * h, z0],
                  [3.5 * h, (m + 2.5) * h, z0]], np.float32)
    seeds = oracle.voxelize(v, np.array([[0, 1, 2]], np.int32), LO, np.float32(h), n)
    occ = occupied(seeds, n)
    assert len(occ) == (m + 1) * (m + 2) // 2
    assert np.all(occ[:, 2] == int(np.floor(z0 * n)))
    assert np.all(occ[:, 0] - 3 + occ[:, 1] - 2 <= m)


def test_room_box_boundary_layers():
    # Walls on the six faces of the domain: the near faces land in layer 0, the
    # far faces (depth exactly n) in layer n - 1 -> the boundary shell.
    for n in (16, 32):
        v, f = room_box()
        seeds = oracle.voxelize(v.astype(np.float32), f.astype(np.int32), LO, np.float32(1.0 / n), n)
        occ = occupied(seeds, n)
        assert len(occ) == n ** 3 - (n - 2) ** 3
        assert np.all(np.any((occ == 0) | (occ == n - 1), axis=1))


def test_invariant_to_triangle_order_and_winding(tiny):
    n = 32
    h = np.float32(1.0 / n)
    v, f = tiny.mesh.vertices, tiny.mesh.faces
    base = oracle.voxelize(v, f, LO, h, n)
    rng = np.random.default_rng(3)
    f2 = f[rng.permutation(len(f))][:, ::-1].copy()
    assert np.array_equal(base, oracle.voxelize(v, f2, LO, h, n))


def test_rejects_vertices_outside_grown_domain():
    v = np.array([[0.1, 0.1, 0.1], [0.2, 0.1, 0.1], [0.1, 2.5, 0.1]], np.float32)
    with pytest.raises(ValueError):
        oracle.voxelize(v, np.array([[0, 1, 2]], np.int32), LO, np.float32(1 / 32), 32)


def _column_cast(v, f, n, axis):
    """Cast a line along ``axis`` through every column centre against every
    triangle in float64, from the unsnapped vertices.  Returns, per (triangle,
    column), the depth in voxels and the smallest signed distance (in voxels)
    of the column centre to the projected triangle's edges (>= 0 inside)."""
    e1, e2 = (axis + 1) % 3, (axis + 2) % 3
    P = v.astype(np.float64)[f] * n  # [nt, 3, 3] in voxel units
    A, B, Cc = P[:, 0], P[:, 1], P[:, 2]
    g = np.arange(n) + 0.5
    I, J = np.meshgrid(g, g, indexing="ij")  # column centre along e1, e2
    Q = np.stack([I.ravel(), J.ravel()], 1)  # [ncol, 2]

    def cross2(a, b):
        return a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]

    a2 = np.stack([A[:, e1], A[:, e2]], 1)
    b2 = np.stack([B[:, e1], B[:, e2]], 1)
    c2 = np.stack([Cc[:, e1], Cc[:, e2]], 1)
    area = cross2(b2 - a2, c2 - a2)  # [nt]
    ok = area != 0
    sgn = np.where(area < 0, -1.0, 1.0)
    dists = []
    bary = []
    for (p0, p1, opp) in ((b2, c2, 0), (c2, a2, 1), (a2, b2, 2)):
        ed = p1 - p0
        w = cross2(ed[:, None, :], Q[None, :, :] - p0[:, None, :]) * sgn[:, None]
        L = np.linalg.norm(ed, axis=1)[:, None]
        dists.append(w / np.where(L > 0, L, 1))
        bary.append(w / np.where(ok, np.abs(area), 1)[:, None])
    dmin = np.minimum(np.minimum(dists[0], dists[1]), dists[2])
    Z = np.stack([A[:, axis], B[:, axis], Cc[:, axis]], 1)
    depth = bary[0] * Z[:, 0:1] + bary[1] * Z[:, 1:2] + bary[2] * Z[:, 2:3]
    dmin[~ok] = -np.inf
    return depth, dmin, Q


def test_column_cast_completeness_and_soundness():
    # Every column centre strictly inside a triangle's projection (by 1% of a
    # voxel) must mark the voxel holding the cast depth (when that depth is at
    # least 1% of a voxel from a layer boundary); and every marked voxel must be
    # explained by some triangle/axis whose cast lands in it (within tolerance).
    n = 32
    mesh = tiny_scene()
    v, f = mesh.vertices, mesh.faces
    seeds = oracle.voxelize(v, f, LO, np.float32(1.0 / n), n)
    occ = np.zeros((n, n, n), bool)  # [z, y, x]
    occ.ravel()[np.nonzero(seeds >= 0)[0]] = True
    explained = np.zeros_like(occ)
    checked = 0
    for axis in range(3):
        e1, e2 = (axis + 1) % 3, (axis + 2) % 3
        depth, dmin, Q = _column_cast(v, f, n, axis)
        ci = np.floor(Q[:, 0]).astype(int)
        cj = np.floor(Q[:, 1]).astype(int)
        # completeness
        sure = (dmin > 0.01) & (depth >= 0) & (depth < n)
        frac = depth - np.floor(depth)
        sure &= (frac > 0.01) & (frac < 0.99)
        t_idx, c_idx = np.nonzero(sure)
        L = np.floor(depth[t_idx, c_idx]).astype(int)
        coord = np.zeros((len(L), 3), int)
        coord[:, axis] = L
        coord[:, e1] = ci[c_idx]
        coord[:, e2] = cj[c_idx]
        assert np.all(occ[coord[:, 2], coord[:, 1], coord[:, 0]])
        checked += len(L)
        # soundness support
        maybe = dmin > -0.01
        t_idx, c_idx = np.nonzero(maybe)
        dd = depth[t_idx, c_idx]
        for Ls in (np.floor(dd - 0.01), np.floor(dd + 0.01), np.floor(dd)):
            Ls = np.clip(Ls.astype(int), 0, n - 1)
            coord = np.zeros((len(Ls), 3), int)
            coord[:, axis] = Ls
            coord[:, e1] = ci[c_idx]
            coord[:, e2] = cj[c_idx]
            explained[coord[:, 2], coord[:, 1], coord[:, 0]] = True
    assert checked > 1000
    assert not np.any(occ & ~explained)


def test_sphere_occupancy_near_surface():
    # Every marked voxel's centre lies within half a voxel diagonal (plus the
    # 1/256 snapping) of the analytic sphere the icosphere approximates, widened
    # by the tessellation's sagitta.
    n = 32
    s = icosphere(2, 0.3, (0.5, 0.5, 0.5))
    seeds = oracle.voxelize(s.vertices, s.faces, LO, np.float32(1.0 / n), n)
    occ = occupied(seeds, n)
    centres = (occ + 0.5) / n
    r = np.linalg.norm(centres - 0.5, axis=1)
    v = s.vertices.astype(np.float64) - 0.5
    tri = v[s.faces]
    cen = tri.mean(1)
    nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    r_in = np.min(np.abs(np.einsum("ij,ij->i", cen, nrm)))
    slack = (np.sqrt(3) / 2 + 1 / 256) / n
    assert np.all(r <= 0.3 + slack)
    assert np.all(r >= r_in - slack)
