"""Pins of the oracle's world positions of rigid parts (two-level scenes).

* The identity transform leaves positions as they are; a part index of -1 too.
* A quarter turn about z with an integer translation maps (x, y, z) to
  (t0 - y, t1 + x, t2 + z) exactly (every product and sum is exact).
* A seeded rotation preserves distances within a part (rigid) to float32
  rounding, and matches the float64 product within a few ulps.
"""
import numpy as np

import oracle
from synth.scenes import DynamicScene, random_rotation, rigid_parts


def test_identity_and_unassigned():
    rng = np.random.default_rng(1)
    v = rng.uniform(-1, 1, (50, 3)).astype(np.float32)
    eye = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    part = np.zeros(50, np.int32)
    part[::3] = -1
    assert np.array_equal(oracle.instance_world(v, part, eye), v)
    rot = np.concatenate([random_rotation(rng), [[5.0], [6.0], [7.0]]], 1).reshape(1, 12).astype(np.float32)
    w = oracle.instance_world(v, part, rot)
    assert np.array_equal(w[::3], v[::3]) and not np.array_equal(w[1::3], v[1::3])


def test_quarter_turn_exact():
    v = np.array([[0.25, 0.5, -0.75], [1.0, -2.0, 3.0], [0.125, 0.0, 0.5]], np.float32)
    T = np.array([[0, -1, 0, 2, 1, 0, 0, -3, 0, 0, 1, 0.5]], np.float32)
    w = oracle.instance_world(v, np.zeros(3, np.int32), T)
    want = np.stack([2 - v[:, 1], -3 + v[:, 0], 0.5 + v[:, 2]], 1)
    assert np.array_equal(w, want)


def test_rigid_and_close_to_float64():
    v, f, offs, T = rigid_parts()
    part = np.full(len(v), -1, np.int32)
    for i in range(len(offs) - 1):
        part[np.unique(f[offs[i]:offs[i + 1]])] = i
    w = oracle.instance_world(v, part, T)
    Tm = T.astype(np.float64).reshape(-1, 3, 4)
    want = np.einsum("vab,vb->va", Tm[part][:, :, :3], v.astype(np.float64)) + Tm[part][:, :, 3]
    assert np.max(np.abs(w - want)) < 4e-7
    for i in range(1, len(offs) - 1):
        ids = np.unique(f[offs[i]:offs[i + 1]])[:40]
        dv = np.linalg.norm(v[ids][:, None] - v[ids][None], axis=-1)
        dw = np.linalg.norm(w[ids][:, None].astype(np.float64) - w[ids][None], axis=-1)
        assert np.max(np.abs(dv - dw)) < 1e-6


def test_dynamic_parts_reproduce_the_animated_mesh():
    d = DynamicScene(2, n_prims=24, detail="low")
    v, f, offs, moving = d.parts()
    part = np.full(len(v), -1, np.int32)
    for i in range(len(offs) - 1):
        part[np.unique(f[offs[i]:offs[i + 1]])] = i
    for frame in (0, 3, 7):
        w = oracle.instance_world(v, part, d.part_transforms(frame)).astype(np.float64)
        m = d.mesh(frame)
        # same multiset of triangles (the parts list static geometry first)
        key = lambda V, F: np.sort(np.round(V[F].reshape(len(F), 9), 5), axis=0)
        assert np.max(np.abs(key(w, f) - key(m.vertices.astype(np.float64), m.faces))) < 1e-4
