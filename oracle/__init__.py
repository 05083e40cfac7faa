"""CPU oracle of the RTSDF SDF-generation path (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never loads it, and it shares no
code with the GPU path.  The arithmetic lives in ``rtsdf_oracle.c`` (plain C,
double precision, OpenMP over independent voxels/texels); this module only
builds that file with gcc and marshals numpy arrays through ctypes.

Functions mirror the steps of the method (paper Sec. 2.1-2.2):
``voxelize``, ``jfa`` / ``jfa_pass``, ``coarse``, ``select_threshold``,
``select``, ``coarse_trilinear``, ``select_field``, ``philox4x64_10``,
``direction``, ``Scene.closest_hits``,
``Scene.trace_frame`` and ``Scene.fine_grad``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rtsdf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain IEEE double/float, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i32, u32, u64, f32, f64 = C.c_int, C.c_uint32, C.c_uint64, C.c_float, C.c_double
        L.oracle_num_threads.restype = i32
        L.oracle_voxelize.argtypes = [P, i32, P, i32, P, f32, i32, P]
        L.oracle_jfa_pass.argtypes = [i32, i32, P, P]
        L.oracle_jfa.argtypes = [i32, P, P]
        L.oracle_jfa_steps.argtypes = [i32, P, P, i32, P]
        L.oracle_coarse.argtypes = [i32, P, f32, f32, P, P]
        L.oracle_select_threshold.argtypes = [f32, f32, f32]
        L.oracle_select.argtypes = [i32, P, i32, i32, P, P, i32, P]
        L.oracle_coarse_trilinear.argtypes = [i32, P, i32, P]
        L.oracle_select_field.argtypes = [i32, P, f32, P, P, i32, P]
        L.oracle_philox4x64_10.argtypes = [P, P, P]
        L.oracle_direction.argtypes = [u64, u64, u32, u32, u32, P]
        L.oracle_texel_origin.argtypes = [i32, P, f32, i32, P]
        L.oracle_scene_create.argtypes = [P, i32, P, i32, i32]
        L.oracle_scene_create.restype = P
        L.oracle_scene_create_f64.argtypes = [P, i32, P, i32, i32]
        L.oracle_scene_create_f64.restype = P
        L.oracle_scene_destroy.argtypes = [P]
        L.oracle_eq1.argtypes = [f64, f64, f32, f64, P]
        L.oracle_eq1.restype = f64
        L.oracle_fine_value.argtypes = [f64, f32, i32, i32, i32, f64]
        L.oracle_fine_value.restype = f64
        L.oracle_closest_hits.argtypes = [P, i32, P, P, P, P, P, P]
        L.oracle_trace_frame.argtypes = [P, i32, P, i32, P, f32, P, P, i32, i32, u32, u64, u32, f64,
                                         P, P, P, P, P, P, P, P, P, P, i32, f64]
        L.oracle_fine_grad.argtypes = [P, i32, P, f32, u64, u32, P, P, P, P, P, P, i32]
        L.oracle_directions.argtypes = [i32, P, P, P, u64, u32, P]
        L.oracle_point_distance.argtypes = [P, i32, P, P, P]
        L.oracle_instance_world.argtypes = [i32, P, P, P, P]
        L.oracle_shadow.argtypes = [i32, P, f32, P, i32, P, P, f32, f32, i32, f32, f32, i32, P, f32, P]
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def voxelize(vertices, faces, lo, h: float, n: int) -> np.ndarray:
    """Occupied-voxel seeds: own linear index where occupied, else -1 (shape n^3, x fastest)."""
    v, f = _c(vertices, np.float32), _c(faces, np.int32)
    lo = _c(lo, np.float32)
    seeds = np.empty(n ** 3, np.int32)
    rc = lib().oracle_voxelize(_p(v), v.shape[0], _p(f), f.shape[0], _p(lo), float(h), int(n), _p(seeds))
    if rc != 0:
        raise ValueError("oracle_voxelize: invalid arguments (vertex outside the grown domain or bad index)")
    return seeds


def jfa_pass(n: int, k: int, seeds: np.ndarray) -> np.ndarray:
    s = _c(seeds, np.int32)
    out = np.empty_like(s)
    lib().oracle_jfa_pass(int(n), int(k), _p(s), _p(out))
    return out


def jfa(n: int, seeds: np.ndarray) -> np.ndarray:
    s = _c(seeds, np.int32)
    out = np.empty_like(s)
    if lib().oracle_jfa(int(n), _p(s), _p(out)) != 0:
        raise ValueError("oracle_jfa: n must be a power of two")
    return out


def jfa_steps(n: int, seeds: np.ndarray, steps) -> np.ndarray:
    """Jump flooding with an explicit pass schedule (one oracle_jfa_pass per step, in order)."""
    s = _c(seeds, np.int32)
    st = np.ascontiguousarray(steps, np.int32)
    out = np.empty_like(s)
    if lib().oracle_jfa_steps(int(n), _p(s), _p(st), int(st.size), _p(out)) != 0:
        raise ValueError("oracle_jfa_steps: bad schedule")
    return out


def coarse(n: int, seeds: np.ndarray, h: float, beta: float):
    s = _c(seeds, np.int32)
    d2 = np.empty(n ** 3, np.int32)
    c = np.empty(n ** 3, np.float32)
    lib().oracle_coarse(int(n), _p(s), float(h), float(beta), _p(d2), _p(c))
    return d2, c


def select_threshold(hc: float, beta: float, d: float) -> int:
    return int(lib().oracle_select_threshold(float(hc), float(beta), float(d)))


def select(nc: int, dist2: np.ndarray, nf: int, K: int):
    d2 = _c(dist2, np.int32)
    mask = np.empty(nf ** 3, np.uint8)
    queue = np.empty(nf ** 3, np.int32)
    cnt = C.c_int(0)
    rc = lib().oracle_select(int(nc), _p(d2), int(nf), int(K), _p(mask), _p(queue), nf ** 3, C.byref(cnt))
    if rc != 0:
        raise ValueError("oracle_select failed")
    return mask, queue[: cnt.value].copy()


def coarse_trilinear(nc: int, c: np.ndarray, nf: int) -> np.ndarray:
    """Coarse SDF sampled trilinearly at the fine texel centres (float32)."""
    cc = _c(c, np.float32)
    out = np.empty(nf ** 3, np.float32)
    if lib().oracle_coarse_trilinear(int(nc), _p(cc), int(nf), _p(out)) != 0:
        raise ValueError("oracle_coarse_trilinear: invalid arguments")
    return out


def select_field(n: int, field: np.ndarray, d: float):
    """Texels with field <= d: mask and Morton-ordered queue."""
    fl = _c(field, np.float32)
    mask = np.empty(n ** 3, np.uint8)
    queue = np.empty(n ** 3, np.int32)
    cnt = C.c_int(0)
    if lib().oracle_select_field(int(n), _p(fl), float(d), _p(mask), _p(queue), n ** 3, C.byref(cnt)) != 0:
        raise ValueError("oracle_select_field failed")
    return mask, queue[: cnt.value].copy()


def instance_world(obj_vertices, part, transforms) -> np.ndarray:
    """World positions (float32 [nv, 3]) of vertices given in their part's object space."""
    o = _c(np.asarray(obj_vertices, np.float32).reshape(-1, 3), np.float32)
    pa = _c(part, np.int32)
    T = _c(np.asarray(transforms, np.float32).reshape(-1, 12), np.float32)
    out = np.empty_like(o)
    lib().oracle_instance_world(o.shape[0], _p(o), _p(pa), _p(T), _p(out))
    return out


def philox4x64_10(counter, key) -> np.ndarray:
    ctr = _c(counter, np.uint64)
    k = _c(key, np.uint64)
    out = np.empty(4, np.uint64)
    lib().oracle_philox4x64_10(_p(ctr), _p(k), _p(out))
    return out


def direction(seed: int, texel: int, frame: int, ray: int, scene: int = 0):
    out = np.empty(3, np.float32)
    attempt = lib().oracle_direction(seed, texel, frame, ray, scene, _p(out))
    return out, int(attempt)


def directions(texel, frame, ray, seed: int = 0, scene: int = 0) -> np.ndarray:
    """Directions for many (texel, frame, ray) keys, float32 [n, 3]."""
    t = _c(texel, np.int32)
    fr = _c(np.broadcast_to(frame, t.shape), np.uint32)
    r = _c(np.broadcast_to(ray, t.shape), np.int32)
    out = np.empty((t.shape[0], 3), np.float32)
    lib().oracle_directions(t.shape[0], _p(t), _p(fr), _p(r), int(seed), int(scene), _p(out))
    return out


def shadow(n: int, lo, h: float, sdf, points, light, k: float, eps: float, max_steps: int, max_step: float,
           max_dist: float, penumbra: int = 0, jitter=None, jitter_scale: float = 0.0) -> np.ndarray:
    """Soft-shadow visibility of each point (Sec. 2.3), float32 [np].  penumbra 0: cone term k s / t;
    1: triangulated between consecutive samples.  jitter [np] in [0, 1) moves each march's start by
    jitter * jitter_scale towards the light."""
    lo = _c(lo, np.float32)
    s = _c(sdf, np.float32)
    pts = _c(points, np.float32).reshape(-1, 3)
    l = _c(light, np.float32)
    jt = None if jitter is None else _c(jitter, np.float32)
    out = np.empty(pts.shape[0], np.float32)
    lib().oracle_shadow(int(n), _p(lo), float(h), _p(s), pts.shape[0], _p(pts), _p(l), float(k), float(eps),
                        int(max_steps), float(max_step), float(max_dist), int(penumbra), _p(jt),
                        float(jitter_scale), _p(out))
    return out


def texel_origin(nf: int, lo, h: float, j: int) -> np.ndarray:
    lo = _c(lo, np.float32)
    out = np.empty(3, np.float32)
    lib().oracle_texel_origin(int(nf), _p(lo), float(h), int(j), _p(out))
    return out


def eq1(alpha: float, u_prev: float, c: float, r_t: float):
    """Eq. (1) on the unsigned state; returns (u_t, source) with source 1 = rays, 0 = kept, 2 = decayed."""
    src = C.c_int(-1)
    u = lib().oracle_eq1(float(alpha), float(u_prev), float(c), float(r_t), C.byref(src))
    return float(u), int(src.value)


SIGN_POLICIES = {"vote": 0, "shell": 1}


def fine_value(u: float, c: float, nfront: int, nback: int, sign_policy: str = "vote", shell: float = 0.0) -> float:
    return float(lib().oracle_fine_value(float(u), float(c), int(nfront), int(nback), SIGN_POLICIES[sign_policy],
                                         float(shell)))


class TraceState:
    """Per-texel accumulation state of the oracle (double precision)."""

    def __init__(self, nf: int):
        n = nf ** 3
        self.u = np.full(n, np.inf)
        self.nfront = np.zeros(n, np.int32)
        self.nback = np.zeros(n, np.int32)
        self.arg_frame = np.full(n, -1, np.int32)
        self.arg_ray = np.full(n, -1, np.int32)
        self.arg_tri = np.full(n, -1, np.int32)
        self.arg_amb = np.zeros(n, np.uint8)
        self.texel_amb = np.zeros(n, np.uint8)
        self.fine = np.zeros(n)
        self.rmin = np.full(n, np.inf)

    def copy(self) -> "TraceState":
        o = TraceState.__new__(TraceState)
        for k, v in self.__dict__.items():
            setattr(o, k, v.copy())
        return o


class Scene:
    """Triangle scene for closest-hit queries (optionally with a median-split hierarchy)."""

    def __init__(self, vertices, faces, use_bvh: bool = True):
        """``vertices`` float32 (as the GPU sees them) or float64 (finite-difference checks)."""
        self.f = _c(faces, np.int32)
        if np.asarray(vertices).dtype == np.float64:
            self.v = _c(vertices, np.float64)
            self.h = lib().oracle_scene_create_f64(_p(self.v), self.v.shape[0], _p(self.f), self.f.shape[0],
                                                   int(use_bvh))
        else:
            self.v = _c(vertices, np.float32)
            self.h = lib().oracle_scene_create(_p(self.v), self.v.shape[0], _p(self.f), self.f.shape[0],
                                               int(use_bvh))

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_scene_destroy(self.h)
            self.h = None

    def closest_hits(self, origins, dirs):
        o = _c(origins, np.float64).reshape(-1, 3)
        d = _c(dirs, np.float64).reshape(-1, 3)
        n = o.shape[0]
        t = np.empty(n)
        tri = np.empty(n, np.int32)
        front = np.empty(n, np.int32)
        amb = np.empty(n, np.int32)
        lib().oracle_closest_hits(self.h, n, _p(o), _p(d), _p(t), _p(tri), _p(front), _p(amb))
        return t, tri, front, amb

    def trace_frame(self, nc: int, coarse_sdf, nf: int, lo, hf: float, mask, rays: int, frame: int,
                    seed: int, scene: int, alpha: float, state: TraceState, texels=None, sign_policy: str = "vote",
                    shell: float = 0.0) -> TraceState:
        cs = _c(coarse_sdf, np.float32)
        m = _c(mask, np.uint8)
        lo = _c(lo, np.float32)
        tx = None if texels is None else _c(texels, np.int32)
        ntex = -1 if tx is None else tx.shape[0]
        rc = lib().oracle_trace_frame(
            self.h, int(nc), _p(cs), int(nf), _p(lo), float(hf), _p(m), _p(tx), ntex, int(rays),
            int(frame), int(seed), int(scene), float(alpha),
            _p(state.u), _p(state.nfront), _p(state.nback), _p(state.arg_frame), _p(state.arg_ray),
            _p(state.arg_tri), _p(state.arg_amb), _p(state.texel_amb), _p(state.fine), _p(state.rmin),
            SIGN_POLICIES[sign_policy],
            float(shell))
        if rc != 0:
            raise ValueError("oracle_trace_frame: invalid arguments")
        return state

    def point_distance(self, points):
        """Exact unsigned distance from each point to the mesh (float64) and the nearest triangle."""
        pts = _c(np.asarray(points, np.float64).reshape(-1, 3), np.float64)
        dist = np.empty(pts.shape[0])
        tri = np.empty(pts.shape[0], np.int32)
        lib().oracle_point_distance(self.h, pts.shape[0], _p(pts), _p(dist), _p(tri))
        return dist, tri

    def fine_grad(self, nf: int, lo, hf: float, seed: int, scene: int, state: TraceState, grad_f,
                  sign_policy: str = "vote") -> np.ndarray:
        lo = _c(lo, np.float32)
        g = _c(grad_f, np.float64)
        out = np.zeros(self.v.shape[0] * 3)
        lib().oracle_fine_grad(self.h, int(nf), _p(lo), float(hf), int(seed), int(scene), _p(state.fine),
                               _p(state.arg_frame), _p(state.arg_ray), _p(state.arg_tri), _p(g), _p(out),
                               SIGN_POLICIES[sign_policy])
        return out.reshape(-1, 3)


def run_frames(mesh_v, mesh_f, nc: int, nf: int, beta: float, d: float, rays: int, frames, seed: int = 0,
               scene: int = 0, alpha: float = 1.0, lo=(0.0, 0.0, 0.0), texels=None, use_bvh: bool = True,
               state: TraceState | None = None, side: float = 1.0, sampling: str = "point",
               sign_policy: str = "vote", shell: float = 0.0):
    """Whole oracle pipeline for a static mesh over the given frame indices, on
    the cube [lo, lo + side]^3.  ``sampling="trilinear"`` selects and fills
    with the trilinearly sampled coarse SDF instead of the containing voxel's;
    ``sign_policy``/``shell`` choose how traced distances are signed.

    Returns a dict with the coarse stage outputs and the final trace state.
    """
    lo = np.asarray(lo, np.float32)
    hc = np.float32(side) / np.float32(nc)
    hf = np.float32(side) / np.float32(nf)
    seeds0 = voxelize(mesh_v, mesh_f, lo, hc, nc)
    seeds = jfa(nc, seeds0)
    d2, c = coarse(nc, seeds, hc, beta)
    K = select_threshold(hc, beta, d)
    if sampling == "point":
        mask, queue = select(nc, d2, nf, K)
        ng, cg = nc, c
    elif sampling == "trilinear":
        cg = coarse_trilinear(nc, c, nf)
        mask, queue = select_field(nf, cg, d)
        ng = nf
    else:
        raise ValueError(f"unknown sampling {sampling!r}")
    sc = Scene(mesh_v, mesh_f, use_bvh)
    st = TraceState(nf) if state is None else state
    for fr in frames:
        sc.trace_frame(ng, cg, nf, lo, hf, mask, rays, fr, seed, scene, alpha, st, texels, sign_policy, shell)
    out = dict(seeds0=seeds0, seeds=seeds, dist2=d2, coarse=c, K=K, mask=mask, queue=queue, state=st, scene=sc)
    if sampling == "trilinear":
        out["coarse_fine"] = cg
    return out
