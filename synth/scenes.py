"""Seeded synthetic triangle scenes and workload descriptions.

This module only builds input meshes and parameter records.  It contains none
of the SDF method's arithmetic (no voxelization, flooding, ray generation or
tracing), so both the CPU oracle and the GPU path can take their inputs from
it without sharing any of the computation that is being checked.

Conventions
-----------
* Vertices are float32 ``[nv, 3]`` (x, y, z) in world units; faces are int32
  ``[nt, 3]`` vertex indices, counter-clockwise when seen from outside, so the
  geometric normal ``(v1 - v0) x (v2 - v0)`` points out of closed objects.
* The domain is the unit cube ``[0, 1]^3`` (``lo = 0``, side 1).
* Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64), so a
  scene is fully determined by its seed.

The workloads stand in for the paper's test scene (a furnished living room
rendered with one directional light), which is not available here; the sizes
follow the room-scale, tiny, dynamic, batched and differentiable cases the
method is exercised on.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PHI = (1.0 + math.sqrt(5.0)) / 2.0


@dataclass
class Mesh:
    vertices: np.ndarray  # float32 [nv, 3]
    faces: np.ndarray  # int32 [nt, 3]

    @property
    def nv(self) -> int:
        return int(self.vertices.shape[0])

    @property
    def nt(self) -> int:
        return int(self.faces.shape[0])


def _orient_outward(v: np.ndarray, f: np.ndarray, center: np.ndarray) -> np.ndarray:
    """Flip faces of a star-shaped mesh so their normals point away from ``center``."""
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    n = np.cross(b - a, c - a)
    out = ((a + b + c) / 3.0) - center
    flip = np.einsum("ij,ij->i", n, out) < 0
    f = f.copy()
    f[flip] = f[flip][:, [0, 2, 1]]
    return f


def icosahedron() -> tuple[np.ndarray, np.ndarray]:
    v = np.array(
        [
            [-1, PHI, 0], [1, PHI, 0], [-1, -PHI, 0], [1, -PHI, 0],
            [0, -1, PHI], [0, 1, PHI], [0, -1, -PHI], [0, 1, -PHI],
            [PHI, 0, -1], [PHI, 0, 1], [-PHI, 0, -1], [-PHI, 0, 1],
        ],
        dtype=np.float64,
    )
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int64,
    )
    return v, _orient_outward(v, f, np.zeros(3))


def _unit_icosphere(level: int) -> tuple[np.ndarray, np.ndarray]:
    """Icosahedron with each face split into 4, ``level`` times; unit radius."""
    v, f = icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            if key not in cache:
                p = (np.asarray(verts[i]) + np.asarray(verts[j])) * 0.5
                p /= np.linalg.norm(p)
                cache[key] = len(verts)
                verts.append(tuple(p))
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.array(nf, dtype=np.int64)
    v = np.array(verts, dtype=np.float64)
    return v, _orient_outward(v, f, np.zeros(3))


def _unit_geodesic(freq: int) -> tuple[np.ndarray, np.ndarray]:
    """Class-I geodesic sphere: every icosahedron face cut into ``freq**2`` triangles."""
    v0, f0 = icosahedron()
    key_to_idx: dict[tuple[int, int, int], int] = {}
    verts: list[np.ndarray] = []
    faces: list[list[int]] = []

    def vid(p: np.ndarray) -> int:
        q = p / np.linalg.norm(p)
        key = tuple(np.round(q * 1e9).astype(np.int64))
        if key not in key_to_idx:
            key_to_idx[key] = len(verts)
            verts.append(q)
        return key_to_idx[key]

    for a, b, c in f0:
        A, B, C = v0[a], v0[b], v0[c]
        grid: dict[tuple[int, int], int] = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                k = freq - i - j
                grid[(i, j)] = vid((i * A + j * B + k * C) / freq)
        for i in range(freq):
            for j in range(freq - i):
                faces.append([grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]])
                if i + j < freq - 1:
                    faces.append([grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]])
    v = np.array(verts, dtype=np.float64)
    f = np.array(faces, dtype=np.int64)
    return v, _orient_outward(v, f, np.zeros(3))


def _unit_box() -> tuple[np.ndarray, np.ndarray]:
    v = np.array([[x, y, z] for z in (-1, 1) for y in (-1, 1) for x in (-1, 1)], dtype=np.float64)
    # two triangles per face of the cube [-1, 1]^3
    quads = [[0, 1, 3, 2], [4, 6, 7, 5], [0, 4, 5, 1], [2, 3, 7, 6], [0, 2, 6, 4], [1, 5, 7, 3]]
    f = []
    for a, b, c, d in quads:
        f += [[a, b, c], [a, c, d]]
    f = np.array(f, dtype=np.int64)
    return v, _orient_outward(v, f, np.zeros(3))


def _unit_torus(nu: int, nv: int, tube_ratio: float) -> tuple[np.ndarray, np.ndarray]:
    """Torus in the xz-plane with ring radius 1 and tube radius ``tube_ratio``."""
    R, r = 1.0, tube_ratio
    verts = []
    for i in range(nu):
        u = 2 * math.pi * i / nu
        for j in range(nv):
            w = 2 * math.pi * j / nv
            verts.append([(R + r * math.cos(w)) * math.cos(u), r * math.sin(w), (R + r * math.cos(w)) * math.sin(u)])
    v = np.array(verts, dtype=np.float64)
    f = []
    for i in range(nu):
        for j in range(nv):
            a = i * nv + j
            b = ((i + 1) % nu) * nv + j
            c = ((i + 1) % nu) * nv + (j + 1) % nv
            d = i * nv + (j + 1) % nv
            f += [[a, b, c], [a, c, d]]
    f = np.array(f, dtype=np.int64)
    # orient each face away from the tube's centre circle
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    cen = (a + b + c) / 3.0
    ring = cen.copy()
    ring[:, 1] = 0.0
    ring /= np.linalg.norm(ring, axis=1, keepdims=True)
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, cen - ring) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a uniform unit quaternion (Shoemake 1992)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1 - u1), math.sqrt(u1)
    x, y, z, w = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2), b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ]
    )


def axis_rotation(axis: np.ndarray, angle: float) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def _merge(parts: list[tuple[np.ndarray, np.ndarray]]) -> tuple[np.ndarray, np.ndarray]:
    vs, fs, off = [], [], 0
    for v, f in parts:
        vs.append(v)
        fs.append(f + off)
        off += v.shape[0]
    return np.concatenate(vs, 0), np.concatenate(fs, 0)


def _as_mesh(v: np.ndarray, f: np.ndarray) -> Mesh:
    return Mesh(np.ascontiguousarray(v, dtype=np.float32), np.ascontiguousarray(f, dtype=np.int32))


def icosphere(level: int, radius: float, center) -> Mesh:
    v, f = _unit_icosphere(level)
    return _as_mesh(v * radius + np.asarray(center, dtype=np.float64), f)


def ground_quad(y0: float, lo: float = 0.0, hi: float = 1.0) -> Mesh:
    """Axis-aligned one-sided quad at height ``y0`` spanning x, z in [lo, hi]; normal +y."""
    v = np.array([[lo, y0, lo], [hi, y0, lo], [hi, y0, hi], [lo, y0, hi]], dtype=np.float64)
    f = np.array([[0, 2, 1], [0, 3, 2]], dtype=np.int64)
    return _as_mesh(v, f)


def room_box() -> tuple[np.ndarray, np.ndarray]:
    """The unit cube's six walls, two triangles each, normals pointing into the room."""
    v, f = _unit_box()
    v = (v + 1.0) * 0.5
    return v, f[:, [0, 2, 1]]


PRIM_KINDS = ("box", "sphere", "torus")


def _primitive(kind: str, detail: str) -> tuple[np.ndarray, np.ndarray]:
    """Unit primitive (bounding radius 1) for the given kind and detail level."""
    if kind == "box":
        v, f = _unit_box()
        return v / math.sqrt(3.0), f
    if kind == "sphere":
        return _unit_icosphere({"low": 2, "mid": 3, "high": 4}[detail])
    if kind == "torus":
        nu, nv = {"low": (32, 12), "mid": (32, 12), "high": (64, 24)}[detail]
        v, f = _unit_torus(nu, nv, 0.3)
        return v / 1.3, f
    raise ValueError(kind)


@dataclass
class Placement:
    kind: str
    center: np.ndarray
    scale: float
    rotation: np.ndarray


def random_placements(rng: np.random.Generator, n: int, smin: float = 0.02, smax: float = 0.2,
                      margin: float = 0.0) -> list[Placement]:
    out = []
    for _ in range(n):
        kind = PRIM_KINDS[int(rng.integers(0, 3))]
        s = math.exp(rng.uniform(math.log(smin), math.log(smax)))
        c = rng.uniform(s + margin, 1.0 - s - margin, size=3)
        out.append(Placement(kind, c, s, random_rotation(rng)))
    return out


def place(kind: str, detail: str, p: Placement, rot: np.ndarray | None = None, shift=None) -> tuple[np.ndarray, np.ndarray]:
    v, f = _primitive(kind, detail)
    R = p.rotation if rot is None else rot @ p.rotation
    c = p.center if shift is None else p.center + shift
    return (v * p.scale) @ R.T + c, f


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------


@dataclass
class Workload:
    """One configuration of the method: scene + grid sizes + parameters.

    ``beta_vox`` and ``d_vox`` are in coarse voxels; :meth:`beta` and :meth:`d`
    give them in world units.
    """

    name: str
    mesh: Mesh
    nc: int
    nf: int
    beta_vox: float
    d_vox: float
    rays: int
    frames: int
    alpha: float = 1.0
    seed: int = 0  # Philox key
    scene_seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def hc(self) -> float:
        return 1.0 / self.nc

    @property
    def hf(self) -> float:
        return 1.0 / self.nf

    @property
    def beta(self) -> float:
        return float(np.float32(self.beta_vox * self.hc))

    @property
    def d(self) -> float:
        return float(np.float32(self.d_vox * self.hc))


def tiny_scene() -> Mesh:
    """Icosphere level 2 (320 triangles, r = 0.3, centre 0.5) over a ground quad at y = 0.15."""
    s = icosphere(2, 0.3, (0.5, 0.5, 0.5))
    q = ground_quad(0.15)
    v, f = _merge([(s.vertices.astype(np.float64), s.faces.astype(np.int64)),
                   (q.vertices.astype(np.float64), q.faces.astype(np.int64))])
    return _as_mesh(v, f)


def room_scene(seed: int = 1, n_prims: int = 300, detail: str = "mid") -> Mesh:
    """Axis-aligned room (walls on the domain faces) with ``n_prims`` random primitives."""
    rng = np.random.default_rng(seed)
    parts = [room_box()]
    for p in random_placements(rng, n_prims):
        parts.append(place(p.kind, detail, p))
    return _as_mesh(*_merge(parts))


class DynamicScene:
    """Room with many primitives; a fixed seeded 20% subset moves rigidly every frame."""

    def __init__(self, seed: int = 2, n_prims: int = 366, detail: str = "high", moving_frac: float = 0.2):
        rng = np.random.default_rng(seed)
        self.placements = random_placements(rng, n_prims, margin=0.05)
        self.detail = detail
        nmov = int(round(moving_frac * n_prims))
        self.moving = set(int(i) for i in rng.choice(n_prims, size=nmov, replace=False))
        self.axes = {i: rng.normal(size=3) for i in self.moving}
        self.rates = {i: float(rng.uniform(0.02, 0.1)) for i in self.moving}
        self.radii = {i: float(rng.uniform(0.0, 0.05)) for i in self.moving}
        self.phases = {i: float(rng.uniform(0, 2 * math.pi)) for i in self.moving}
        self._static = [place(p.kind, detail, p) for p in self.placements]

    def mesh(self, frame: int = 0) -> Mesh:
        parts = [room_box()]
        for i, p in enumerate(self.placements):
            if i in self.moving:
                rot = axis_rotation(self.axes[i], self.rates[i] * frame)
                ph = self.phases[i] + 0.05 * frame
                shift = self.radii[i] * np.array([math.cos(ph), 0.0, math.sin(ph)])
                parts.append(place(p.kind, self.detail, p, rot=rot, shift=shift))
            else:
                parts.append(self._static[i])
        return _as_mesh(*_merge(parts))


    def moving_transform(self, i: int, frame: int) -> np.ndarray:
        """Rigid object-to-world rows (3 x 4) taking moving primitive i from its frame-0 placement to frame
        ``frame``: x_f = rot_f (x_0 - c - s_0) + c + s_f."""
        p = self.placements[i]
        rot = axis_rotation(self.axes[i], self.rates[i] * frame)
        s0 = self.radii[i] * np.array([math.cos(self.phases[i]), 0.0, math.sin(self.phases[i])])
        ph = self.phases[i] + 0.05 * frame
        sf = self.radii[i] * np.array([math.cos(ph), 0.0, math.sin(ph)])
        t = p.center + sf - rot @ (p.center + s0)
        return np.concatenate([rot, t[:, None]], axis=1)

    def parts(self):
        """The same scene as rigid parts: part 0 is everything static (identity transform), parts 1.. are the
        moving primitives at their frame-0 placement.  Returns (vertices, faces, part face offsets, moving ids)."""
        static = [room_box()] + [self._static[i] for i in range(len(self.placements)) if i not in self.moving]
        moving = sorted(self.moving)
        chunks = [_merge(static)] + [place(self.placements[i].kind, self.detail, self.placements[i],
                                           rot=np.eye(3), shift=self.radii[i] * np.array(
                                               [math.cos(self.phases[i]), 0.0, math.sin(self.phases[i])]))
                                     for i in moving]
        offs = [0]
        for _, f in chunks:
            offs.append(offs[-1] + len(f))
        v, f = _merge(chunks)
        return v.astype(np.float32), f.astype(np.int32), offs, moving

    def part_transforms(self, frame: int) -> np.ndarray:
        """float32 [1 + moving, 12]: identity for the static part, then each moving primitive's transform."""
        rows = [np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)]
        rows += [self.moving_transform(i, frame) for i in sorted(self.moving)]
        return np.stack([r.reshape(12) for r in rows]).astype(np.float32)


def rigid_parts(seed: int = 6):
    """A small scene of three rigid parts for tests: a ground quad (part 0), an icosphere and a torus, with
    seeded rigid transforms.  Returns (object vertices, faces, part face offsets, transforms [3, 12])."""
    rng = np.random.default_rng(seed)
    quad = ground_quad(0.15)
    sph = _unit_icosphere(2)
    tor = _unit_torus(24, 8, 0.3)
    parts = [(quad.vertices.astype(np.float64), quad.faces), (sph[0] * 0.18, sph[1]), (tor[0] * 0.12, tor[1])]
    offs = [0]
    for _, f in parts:
        offs.append(offs[-1] + len(f))
    v, f = _merge(parts)
    T = [np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)]
    for c in ((0.35, 0.45, 0.5), (0.7, 0.4, 0.55)):
        T.append(np.concatenate([random_rotation(rng), np.asarray(c)[:, None]], axis=1))
    return v.astype(np.float32), f.astype(np.int32), offs, np.stack([t.reshape(12) for t in T]).astype(np.float32)


def batched_scenes(n_scenes: int = 64, seed0: int = 3) -> list[Workload]:
    """``n_scenes`` independent scenes of uneven size (1k-100k triangles, log-uniform)."""
    out = []
    for s in range(n_scenes):
        rng = np.random.default_rng(seed0 * 1000 + s)
        target = int(round(math.exp(rng.uniform(math.log(1e3), math.log(1e5)))))
        nc = int(rng.choice([32, 64, 128]))
        parts, tris = [], 0
        while tris < target:
            p = random_placements(rng, 1)[0]
            detail = "low" if rng.random() < 0.5 else "mid"
            v, f = place(p.kind, detail, p)
            parts.append((v, f))
            tris += f.shape[0]
        mesh = _as_mesh(*_merge(parts))
        out.append(Workload(f"batched[{s}]", mesh, nc, 2 * nc, 0.5, 2.0, 8, 16, 1.0, 0, s))
    return out


def perturbed_sphere(freq: int = 22, radius: float = 0.3, amp: float = 0.05, seed: int = 4) -> Mesh:
    """Geodesic sphere (20 * freq**2 triangles) with a seeded smooth radial perturbation."""
    rng = np.random.default_rng(seed)
    v, f = _unit_geodesic(freq)
    dirs = rng.normal(size=(6, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    freqs = rng.uniform(1.0, 3.0, size=6)
    phases = rng.uniform(0, 2 * math.pi, size=6)
    noise = np.zeros(v.shape[0])
    for d_, fr, ph in zip(dirs, freqs, phases):
        noise += np.sin(fr * (v @ d_) * math.pi + ph)
    noise /= np.max(np.abs(noise))
    r = radius * (1.0 + amp * noise)
    return _as_mesh(v * r[:, None] + 0.5, f)


def workload(name: str) -> Workload:
    """The named workload.

    tiny     icosphere + ground quad, coarse 32^3 / fine 64^3, beta 0.5, d 2, 4 rays x 8 frames
    room     room + 300 primitives (~200k triangles), 128^3 / 256^3, d 3, 16 rays x 64 frames
    dynamic  room + 366 primitives (~1M triangles, 20% animated), 256^3 / 512^3, 8 rays x 120 frames
    diff     perturbed geodesic sphere (9,680 triangles), 64^3 / 128^3, 32 rays x 16 frames
    """
    if name == "tiny":
        return Workload("tiny", tiny_scene(), 32, 64, 0.5, 2.0, 4, 8, 1.0, 0, 0)
    if name == "room":
        return Workload("room", room_scene(1), 128, 256, 0.5, 3.0, 16, 64, 1.0, 0, 1)
    if name == "dynamic":
        dyn = DynamicScene(2)
        return Workload("dynamic", dyn.mesh(0), 256, 512, 0.5, 3.0, 8, 120, 0.9, 0, 2, {"scene": dyn})
    if name == "diff":
        return Workload("diff", perturbed_sphere(), 64, 128, 0.5, 2.0, 32, 16, 1.0, 0, 4)
    raise ValueError(f"unknown workload {name!r}")


def random_soup(seed: int, nt: int, lo: float = -0.2, hi: float = 1.2, size: float = 0.1) -> Mesh:
    """Random triangle soup for edge-case tests (vertices may leave the unit cube)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(lo + size, hi - size, size=(nt, 1, 3))
    v = c + rng.uniform(-size, size, size=(nt, 3, 3))
    f = np.arange(3 * nt, dtype=np.int64).reshape(nt, 3)
    return _as_mesh(v.reshape(-1, 3), f)
