"""ctypes binding of ``librtsdf.so`` (the C ABI declared in include/rtsdf.h).

Functions keep the C names and only marshal arguments: torch tensors are
passed as device pointers, the stream defaults to torch's current stream, and
a non-zero status raises :class:`RtsdfError`.  All computation happens in the
library's HIP kernels; there is no fallback path -- importing this module on a
machine without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

from .build import LIB

_P = C.c_void_p
_i32, _u32, _u64, _f32, _sz = C.c_int32, C.c_uint32, C.c_uint64, C.c_float, C.c_size_t

OK, EINVAL, ENOMEM, EHIP, EDEVICE = 0, -1, -2, -3, -4
ERR_FACE_INDEX, ERR_VERTEX_RANGE, ERR_QUEUE_FULL, ERR_BATCH, ERR_TRANSFORM, ERR_FRAME = 1, 2, 4, 8, 16, 32


class Grid(C.Structure):
    """Cubic grid: ``n`` cells per axis of size ``h`` from corner ``lo``."""

    _fields_ = [("lo", C.c_float * 3), ("h", C.c_float), ("n", C.c_int32)]

    @classmethod
    def make(cls, n: int, h: float | None = None, lo=(0.0, 0.0, 0.0)) -> "Grid":
        g = cls()
        g.lo[0], g.lo[1], g.lo[2] = (float(x) for x in lo)
        g.h = float(1.0 / n) if h is None else float(h)
        g.n = int(n)
        return g


class Accum(C.Structure):
    _fields_ = [("u", _P), ("hits", _P), ("arg_tri", _P), ("arg_ray", _P)]


class ShadowParams(C.Structure):
    _fields_ = [("light_dir", _f32 * 3), ("k", _f32), ("eps", _f32), ("max_steps", _i32), ("max_step", _f32),
                ("max_dist", _f32), ("penumbra", _i32), ("jitter_scale", _f32)]


class FrameDesc(C.Structure):
    _fields_ = [("vertices", _P), ("nv", _i32), ("faces", _P), ("nt", _i32), ("scene", _P), ("refit", _i32),
                ("coarse", Grid), ("fine", Grid), ("beta", _f32), ("d", _f32), ("rays_per_texel", _i32),
                ("seed", _u64), ("scene_id", _u32), ("alpha", _f32), ("seeds", _P), ("scratch", _P),
                ("dist2", _P), ("coarse_sdf", _P), ("mask", _P), ("queue", _P), ("queue_cap", _i32),
                ("count", _P), ("select_workspace", _P), ("state", Accum), ("fine_sdf", _P),
                ("trace_workspace", _P), ("frame_counter", _P), ("fine_c", _P),
                ("jfa_steps", _P), ("jfa_nsteps", _i32), ("transforms", _P), ("world_vertices", _P)]


class BatchScene(C.Structure):
    _fields_ = [("vertices", _P), ("nv", _i32), ("faces", _P), ("nt", _i32), ("lo", C.c_float * 3), ("side", _f32),
                ("coarse_n", _i32), ("fine_n", _i32), ("beta", _f32), ("d", _f32), ("rays_per_texel", _i32),
                ("alpha", _f32), ("scene_id", _u32), ("sign_policy", _i32), ("shell", _f32)]


class BatchView(C.Structure):
    _fields_ = [("coarse", Grid), ("fine", Grid), ("seeds", _P), ("dist2", _P), ("coarse_sdf", _P), ("mask", _P),
                ("queue", _P), ("count", _P), ("state", Accum), ("fine_sdf", _P), ("scene", _P)]


class TraceTuning(C.Structure):
    _fields_ = [("refill", _i32), ("blocks_per_cu", _i32), ("stats", _i32), ("loop", _i32),
                ("bin_directions", _i32), ("stack_lds", _i32), ("tile_texels", _i32), ("bvh_width", _i32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class JfaTuning(C.Structure):
    _fields_ = [("near_stage", _i32), ("far_order", _i32)]


class SceneInfo(C.Structure):
    _fields_ = [("nv", _i32), ("nt", _i32), ("nodes", _i32), ("max_depth", _i32), ("leaf_size", _i32),
                ("device_bytes", C.c_int64), ("references", _i32), ("instances", _i32)]


class RtsdfError(RuntimeError):
    def __init__(self, fn: str, status: int, bits: int = 0):
        self.status, self.bits = status, bits
        msg = f"{fn} failed: {_lib.rtsdf_status_string(status).decode()} ({status})"
        if bits:
            msg += f", device error bits 0x{bits:x}"
        super().__init__(msg)


def _load():
    path = LIB  # always the in-tree build of the checked-out sources
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2210_04449_amd.build` (hipcc, gfx950)")
    L = C.CDLL(path)
    sig = {
        "rtsdf_status_string": ([_i32], C.c_char_p),
        "rtsdf_version": ([], _i32),
        "rtsdf_sync_status": ([_P, C.POINTER(_u32)], _i32),
        "rtsdf_copy": ([_P, _P, _sz, _P], _i32),
        "rtsdf_voxelize": ([_P, _i32, _P, _i32, Grid, _P, _P], _i32),
        "rtsdf_jfa": ([Grid, _P, _P, _f32, _P, _P, _P], _i32),
        "rtsdf_jfa_steps": ([Grid, _P, _P, C.POINTER(_i32), _i32, _f32, _P, _P, _P], _i32),
        "rtsdf_select_workspace_size": ([_i32], _sz),
        "rtsdf_select": ([Grid, _P, Grid, _f32, _f32, _P, _P, _i32, _P, _P, _P], _i32),
        "rtsdf_select_noalloc": ([Grid, _P, Grid, _f32, _f32, _P, _P, _i32, _P, _P], _i32),
        "rtsdf_select_noalloc_max_bytes": ([], _sz),
        "rtsdf_coarse_trilinear": ([Grid, _P, Grid, _P, _P], _i32),
        "rtsdf_select_field": ([Grid, _P, _f32, _P, _P, _i32, _P, _P, _P], _i32),
        "rtsdf_scene_create": ([_P, _i32, _P, _i32, _i32, C.POINTER(_P), _P], _i32),
        "rtsdf_scene_refit": ([_P, _P, _P], _i32),
        "rtsdf_scene_info_get": ([_P, C.POINTER(SceneInfo)], _i32),
        "rtsdf_scene_hierarchy": ([_P, _i32, _P, _P, _P, _P], _i32),
        "rtsdf_scene_destroy": ([_P], None),
        "rtsdf_accum_reset": ([Grid, Accum, _P], _i32),
        "rtsdf_trace_workspace_size": ([], _sz),
        "rtsdf_trace_accumulate": ([_P, Grid, _P, Grid, _P, _P, _P, _i32, _i32, _u32, _P, _u64, _u32, _f32,
                                    Accum, _P, _P, _P], _i32),
        "rtsdf_trace_config": ([C.POINTER(TraceTuning)], _i32),
        "rtsdf_trace_config_get": ([C.POINTER(TraceTuning)], _i32),
        "rtsdf_jfa_config": ([_i32, C.POINTER(JfaTuning)], _i32),
        "rtsdf_jfa_config_get": ([_i32, C.POINTER(JfaTuning)], _i32),
        "rtsdf_scene_set_tuning": ([_P, C.POINTER(TraceTuning)], _i32),
        "rtsdf_scene_get_tuning": ([_P, C.POINTER(TraceTuning)], _i32),
        "rtsdf_batch_set_tuning": ([_P, C.POINTER(TraceTuning)], _i32),
        "rtsdf_sqrt": ([_P, C.c_int64, _P, _P], _i32),
        "rtsdf_sort_pairs_workspace_size": ([_i32], _sz),
        "rtsdf_sort_pairs": ([_P, _P, _i32, _i32, _P, _P], _i32),
        "rtsdf_directions": ([_P, _P, _P, _i32, _u64, _u32, _P, _P], _i32),
        "rtsdf_closest_hits": ([_P, _P, _P, _i32, _P, _P, _P, _P], _i32),
        "rtsdf_trace_backward": ([_P, Grid, Accum, _P, _P, _u64, _u32, _P, _P], _i32),
        "rtsdf_shadow": ([Grid, _P, _P, _i32, _P, _f32, _f32, _i32, _f32, _f32, _P, _P], _i32),
        "rtsdf_scene_set_sign": ([_P, _i32, _f32], _i32),
        "rtsdf_scene_enable_rebuild": ([_P, _P], _i32),
        "rtsdf_scene_rebuild": ([_P, _P, _P], _i32),
        "rtsdf_scene_create_instanced": ([_P, _i32, _P, _i32, C.POINTER(_i32), _i32, _P, _i32, C.POINTER(_P), _P],
                                         _i32),
        "rtsdf_scene_set_transforms": ([_P, _P, _P, _P], _i32),
        "rtsdf_scene_world_vertices": ([_P, _P, _P], _i32),
        "rtsdf_point_distance": ([_P, _P, _i32, _P, _P, _P], _i32),
        "rtsdf_texel_distance": ([_P, Grid, _P, _i32, _P, _P, _P], _i32),
        "rtsdf_shadow_ex": ([Grid, _P, _P, _i32, C.POINTER(ShadowParams), _P, _P, _P], _i32),
        "rtsdf_frame_graph_create": ([C.POINTER(FrameDesc), C.POINTER(_P), _P], _i32),
        "rtsdf_frame_graph_launch": ([_P, _P], _i32),
        "rtsdf_frame_graph_destroy": ([_P], None),
        "rtsdf_batch_create": ([C.POINTER(BatchScene), _i32, _u64, _i32, C.POINTER(_P), _P], _i32),
        "rtsdf_batch_reset": ([_P, _P], _i32),
        "rtsdf_batch_step": ([_P, _u32, _P, _P], _i32),
        "rtsdf_batch_outputs": ([_P, _i32, C.POINTER(BatchView)], _i32),
        "rtsdf_batch_graph_create": ([_P, _P, C.POINTER(_P), _P], _i32),
        "rtsdf_batch_destroy": ([_P], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


_lib = _load()


def lib():
    return _lib


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("rtsdf: tensors must be on the GPU")
        if not t.is_contiguous():
            raise ValueError("rtsdf: tensors must be contiguous")
        return t.data_ptr()
    return int(t)


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _check(fn: str, status: int):
    if status != OK:
        raise RtsdfError(fn, status)


def _dtype(t: torch.Tensor, dt: torch.dtype, name: str):
    if t.dtype != dt:
        raise TypeError(f"rtsdf: {name} must be {dt}, got {t.dtype}")


def rtsdf_version() -> int:
    return int(_lib.rtsdf_version())


def rtsdf_sync_status(stream=None) -> int:
    """Synchronise and return the device error bits (raises nothing)."""
    bits = _u32(0)
    st = _lib.rtsdf_sync_status(_stream(stream), C.byref(bits))
    if st not in (OK, EDEVICE):
        raise RtsdfError("rtsdf_sync_status", st)
    return int(bits.value)


def rtsdf_voxelize(vertices, faces, coarse: Grid, seeds, stream=None):
    _dtype(vertices, torch.float32, "vertices")
    _dtype(faces, torch.int32, "faces")
    _dtype(seeds, torch.int32, "seeds")
    _check("rtsdf_voxelize", _lib.rtsdf_voxelize(_ptr(vertices), vertices.shape[0], _ptr(faces), faces.shape[0],
                                                 coarse, _ptr(seeds), _stream(stream)))


def rtsdf_jfa(coarse: Grid, seeds, scratch, beta: float, dist2, coarse_sdf, stream=None):
    _check("rtsdf_jfa", _lib.rtsdf_jfa(coarse, _ptr(seeds), _ptr(scratch), float(beta), _ptr(dist2),
                                       _ptr(coarse_sdf), _stream(stream)))


def jfa_schedule(n: int, variant: str = "jfa") -> list[int]:
    """Pass steps of a jump-flooding variant: "jfa" (n/2 .. 1), "jfa+1", "jfa+2", "1+jfa"."""
    base = []
    k = n // 2
    while k >= 1:
        base.append(k)
        k //= 2
    if variant == "jfa":
        return base
    if variant == "jfa+1":
        return base + [1]
    if variant == "jfa+2":
        return base + [2, 1]
    if variant == "1+jfa":
        return [1] + base
    raise ValueError(f"unknown jump-flooding variant {variant!r}")


def rtsdf_jfa_steps(coarse: Grid, seeds, scratch, steps, beta: float, dist2, coarse_sdf, stream=None):
    arr = (_i32 * len(steps))(*[int(k) for k in steps])
    _check("rtsdf_jfa_steps", _lib.rtsdf_jfa_steps(coarse, _ptr(seeds), _ptr(scratch), arr, len(steps), float(beta),
                                                   _ptr(dist2), _ptr(coarse_sdf), _stream(stream)))


def rtsdf_select_workspace_size(coarse_n: int) -> int:
    return int(_lib.rtsdf_select_workspace_size(int(coarse_n)))


def rtsdf_select(coarse: Grid, dist2, fine: Grid, beta: float, d: float, mask, queue, count, workspace,
                 stream=None):
    cap = 0 if queue is None else queue.numel()
    _check("rtsdf_select", _lib.rtsdf_select(coarse, _ptr(dist2), fine, float(beta), float(d), _ptr(mask),
                                             _ptr(queue), cap, _ptr(count), _ptr(workspace), _stream(stream)))


def rtsdf_select_noalloc(coarse: Grid, dist2, fine: Grid, beta: float, d: float, mask, queue, count, stream=None):
    """rtsdf_select without a workspace: its scratch is the library's static per-device array (calls that
    overlap on one GPU race on it)."""
    cap = 0 if queue is None else queue.numel()
    _check("rtsdf_select_noalloc", _lib.rtsdf_select_noalloc(coarse, _ptr(dist2), fine, float(beta), float(d),
                                                             _ptr(mask), _ptr(queue), cap, _ptr(count),
                                                             _stream(stream)))


def rtsdf_coarse_trilinear(coarse: Grid, coarse_sdf, fine: Grid, fine_c, stream=None):
    _check("rtsdf_coarse_trilinear", _lib.rtsdf_coarse_trilinear(coarse, _ptr(coarse_sdf), fine, _ptr(fine_c),
                                                                 _stream(stream)))


def rtsdf_select_field(grid: Grid, field, d: float, mask, queue, count, workspace, stream=None):
    cap = 0 if queue is None else queue.numel()
    _check("rtsdf_select_field", _lib.rtsdf_select_field(grid, _ptr(field), float(d), _ptr(mask), _ptr(queue), cap,
                                                         _ptr(count), _ptr(workspace), _stream(stream)))


SIGN_POLICIES = {"vote": 0, "shell": 1}  # RTSDF_SIGN_VOTE, RTSDF_SIGN_SHELL


class Scene:
    """Owning handle of an ``rtsdf_scene`` (device triangles + hierarchy)."""

    def __init__(self, vertices, faces, leaf_size: int = 4, stream=None):
        _dtype(vertices, torch.float32, "vertices")
        _dtype(faces, torch.int32, "faces")
        h = _P()
        _check("rtsdf_scene_create", _lib.rtsdf_scene_create(_ptr(vertices), vertices.shape[0], _ptr(faces),
                                                             faces.shape[0], int(leaf_size), C.byref(h),
                                                             _stream(stream)))
        self.handle = h

    def refit(self, vertices, stream=None):
        _check("rtsdf_scene_refit", _lib.rtsdf_scene_refit(self.handle, _ptr(vertices), _stream(stream)))

    @classmethod
    def instanced(cls, vertices, faces, instance_faces, transforms, leaf_size: int = 4, stream=None) -> "Scene":
        """Two-level scene of rigid parts: part i owns faces instance_faces[i]:instance_faces[i+1] (host ints),
        vertices are in object space, transforms float32 [ninst, 12] (device) are object-to-world rows."""
        _dtype(vertices, torch.float32, "vertices")
        _dtype(faces, torch.int32, "faces")
        _dtype(transforms, torch.float32, "transforms")
        offs = [int(x) for x in instance_faces]
        arr = (_i32 * len(offs))(*offs)
        h = _P()
        _check("rtsdf_scene_create_instanced", _lib.rtsdf_scene_create_instanced(
            _ptr(vertices), vertices.shape[0], _ptr(faces), faces.shape[0], arr, len(offs) - 1, _ptr(transforms),
            int(leaf_size), C.byref(h), _stream(stream)))
        self = cls.__new__(cls)
        self.handle = h
        return self

    def set_transforms(self, transforms, world_vertices=None, stream=None):
        _check("rtsdf_scene_set_transforms", _lib.rtsdf_scene_set_transforms(self.handle, _ptr(transforms),
                                                                             _ptr(world_vertices), _stream(stream)))

    def world_vertices(self, out, stream=None):
        _check("rtsdf_scene_world_vertices", _lib.rtsdf_scene_world_vertices(self.handle, _ptr(out), _stream(stream)))

    def set_sign(self, policy: str = "vote", shell: float = 0.0):
        """How traced distances are signed: "vote" (front/back hit counts) or "shell" (distance - shell)."""
        _check("rtsdf_scene_set_sign", _lib.rtsdf_scene_set_sign(self.handle, SIGN_POLICIES[policy], float(shell)))

    def enable_rebuild(self, stream=None):
        """Replace the hierarchy by one rebuilt on the device (linear BVH); later rebuild() calls redo it."""
        _check("rtsdf_scene_enable_rebuild", _lib.rtsdf_scene_enable_rebuild(self.handle, _stream(stream)))

    def rebuild(self, vertices, stream=None):
        _check("rtsdf_scene_rebuild", _lib.rtsdf_scene_rebuild(self.handle, _ptr(vertices), _stream(stream)))

    def set_tuning(self, **kw):
        """Give this scene its own tracer tuning (fields of rtsdf_trace_tuning over the tuning it uses now);
        clear_tuning() goes back to the process default."""
        t = TraceTuning(**{**self.tuning().as_dict(), **kw})
        _check("rtsdf_scene_set_tuning", _lib.rtsdf_scene_set_tuning(self.handle, C.byref(t)))

    def clear_tuning(self):
        _check("rtsdf_scene_set_tuning", _lib.rtsdf_scene_set_tuning(self.handle, None))

    def tuning(self) -> TraceTuning:
        t = TraceTuning()
        _check("rtsdf_scene_get_tuning", _lib.rtsdf_scene_get_tuning(self.handle, C.byref(t)))
        return t

    def info(self) -> SceneInfo:
        inf = SceneInfo()
        _check("rtsdf_scene_info_get", _lib.rtsdf_scene_info_get(self.handle, C.byref(inf)))
        return inf

    def hierarchy(self, stream=None):
        """Host copy of the hierarchy: boxes float32 [nodes, 2, 6] (lo xyz, hi xyz per child slot), links int32
        [nodes, 2, 2] ((j, 0) internal child j, (-1 - first, count) leaf), parents int32 [nodes]."""
        import numpy as np
        n = self.info().nodes
        boxes = np.zeros((max(n, 1), 2, 6), np.float32)
        links = np.zeros((max(n, 1), 2, 2), np.int32)
        parents = np.zeros(max(n, 1), np.int32)
        _check("rtsdf_scene_hierarchy", _lib.rtsdf_scene_hierarchy(
            self.handle, n, boxes.ctypes.data_as(_P), links.ctypes.data_as(_P), parents.ctypes.data_as(_P),
            _stream(stream)))
        return boxes[:n], links[:n], parents[:n]

    def close(self):
        if getattr(self, "handle", None):
            _lib.rtsdf_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AccumState:
    """Per-texel accumulation state (u, hits, arg_tri, arg_ray) as torch tensors."""

    def __init__(self, fine: Grid, device="cuda"):
        n = fine.n ** 3
        self.u = torch.empty(n, dtype=torch.float32, device=device)
        self.hits = torch.empty(n, dtype=torch.int32, device=device)
        self.arg_tri = torch.empty(n, dtype=torch.int32, device=device)
        self.arg_ray = torch.empty(n, dtype=torch.int32, device=device)
        rtsdf_accum_reset(fine, self)

    @classmethod
    def wrap(cls, u, hits, arg_tri, arg_ray) -> "AccumState":
        """A state over existing tensors (no reset)."""
        s = cls.__new__(cls)
        s.u, s.hits, s.arg_tri, s.arg_ray = u, hits, arg_tri, arg_ray
        return s

    def struct(self) -> Accum:
        return Accum(_ptr(self.u), _ptr(self.hits), _ptr(self.arg_tri), _ptr(self.arg_ray))

    def tensors(self) -> dict:
        return {"u": self.u, "hits": self.hits, "arg_tri": self.arg_tri, "arg_ray": self.arg_ray}


def rtsdf_accum_reset(fine: Grid, state: AccumState, stream=None):
    _check("rtsdf_accum_reset", _lib.rtsdf_accum_reset(fine, state.struct(), _stream(stream)))


def rtsdf_trace_workspace_size() -> int:
    return int(_lib.rtsdf_trace_workspace_size())


def rtsdf_trace_config_get() -> TraceTuning:
    t = TraceTuning()
    _check("rtsdf_trace_config_get", _lib.rtsdf_trace_config_get(C.byref(t)))
    return t


def rtsdf_trace_config(**kw) -> TraceTuning:
    """Update the tracer tuning (fields of rtsdf_trace_tuning); returns the previous one."""
    old = rtsdf_trace_config_get()
    t = TraceTuning(**{**old.as_dict(), **kw})
    _check("rtsdf_trace_config", _lib.rtsdf_trace_config(C.byref(t)))
    return old


def rtsdf_jfa_config_get(n: int, field: str = "near_stage") -> int:
    """One field of the jump-flooding tuning for grids of side n: "near_stage" (0 automatic, 1 seeds, 2 seed
    pairs) or "far_order" (0 automatic, 1 slab order, 2 coset order, 3 coset order in brick pairs, 4 in 2 x 2 brick
    quads)."""
    t = JfaTuning()
    _check("rtsdf_jfa_config_get", _lib.rtsdf_jfa_config_get(int(n), C.byref(t)))
    return int(getattr(t, field))


def rtsdf_jfa_config(n: int, near_stage: int | None = None, far_order: int | None = None):
    """Set the near-pass staging and/or the far-pass brick order for grids of side n (a field left None keeps
    its setting); returns the previous value of the field set (a (near_stage, far_order) pair when both are)."""
    t = JfaTuning()
    _check("rtsdf_jfa_config_get", _lib.rtsdf_jfa_config_get(int(n), C.byref(t)))
    old = (int(t.near_stage), int(t.far_order))
    if near_stage is not None:
        t.near_stage = int(near_stage)
    if far_order is not None:
        t.far_order = int(far_order)
    _check("rtsdf_jfa_config", _lib.rtsdf_jfa_config(int(n), C.byref(t)))
    if near_stage is not None and far_order is not None:
        return old
    return old[1] if far_order is not None else old[0]


def rtsdf_trace_accumulate(scene: Scene, coarse: Grid, coarse_sdf, fine: Grid, mask, queue, count,
                           rays_per_texel: int, frame: int, seed: int, scene_id: int, alpha: float,
                           state: AccumState, fine_sdf, workspace, frame_ptr=None, stream=None):
    _check("rtsdf_trace_accumulate", _lib.rtsdf_trace_accumulate(
        scene.handle, coarse, _ptr(coarse_sdf), fine, _ptr(mask), _ptr(queue), _ptr(count), queue.numel(),
        int(rays_per_texel), int(frame), _ptr(frame_ptr), int(seed), int(scene_id), float(alpha), state.struct(),
        _ptr(fine_sdf), _ptr(workspace), _stream(stream)))


def rtsdf_sort_pairs(keys, values, bits: int = 32, stream=None):
    """Stable radix sort of (uint32 keys as int32 tensor, int32 values) in place by the low `bits` key bits."""
    _dtype(keys, torch.int32, "keys")
    _dtype(values, torch.int32, "values")
    n = keys.numel()
    if values.numel() != n:
        raise ValueError("rtsdf_sort_pairs: keys and values differ in length")
    ws = torch.empty(max(int(_lib.rtsdf_sort_pairs_workspace_size(n)), 1), dtype=torch.uint8, device=keys.device)
    _check("rtsdf_sort_pairs", _lib.rtsdf_sort_pairs(_ptr(keys), _ptr(values), n, int(bits), _ptr(ws),
                                                     _stream(stream)))


def rtsdf_sqrt(x, out, stream=None):
    """The library's float32 square root (the one every stage uses), element-wise."""
    _dtype(x, torch.float32, "x")
    _dtype(out, torch.float32, "out")
    if out.numel() < x.numel():
        raise ValueError("rtsdf_sqrt: out is shorter than x")
    _check("rtsdf_sqrt", _lib.rtsdf_sqrt(_ptr(x), x.numel(), _ptr(out), _stream(stream)))


def rtsdf_directions(texel, frame, ray, seed: int, scene_id: int, out, stream=None):
    n = texel.numel()
    _check("rtsdf_directions", _lib.rtsdf_directions(_ptr(texel), _ptr(frame), _ptr(ray), n, int(seed),
                                                     int(scene_id), _ptr(out), _stream(stream)))


def rtsdf_closest_hits(scene: Scene, origins, dirs, t_out, tri_out, front_out, stream=None):
    n = origins.shape[0]
    _check("rtsdf_closest_hits", _lib.rtsdf_closest_hits(scene.handle, _ptr(origins), _ptr(dirs), n, _ptr(t_out),
                                                         _ptr(tri_out), _ptr(front_out), _stream(stream)))


def rtsdf_trace_backward(scene: Scene, fine: Grid, state: AccumState, fine_sdf, grad_fine, seed: int,
                         scene_id: int, grad_v, stream=None):
    _check("rtsdf_trace_backward", _lib.rtsdf_trace_backward(scene.handle, fine, state.struct(), _ptr(fine_sdf),
                                                             _ptr(grad_fine), int(seed), int(scene_id),
                                                             _ptr(grad_v), _stream(stream)))


def rtsdf_shadow(fine: Grid, fine_sdf, points, light_dir, k: float, eps: float, max_steps: int, max_step: float,
                 max_dist: float, visibility, stream=None):
    ld = (C.c_float * 3)(*[float(x) for x in light_dir])
    _check("rtsdf_shadow", _lib.rtsdf_shadow(fine, _ptr(fine_sdf), _ptr(points), points.shape[0], ld, float(k),
                                             float(eps), int(max_steps), float(max_step), float(max_dist),
                                             _ptr(visibility), _stream(stream)))


def rtsdf_point_distance(scene: "Scene", points, dist, tri=None, stream=None):
    _check("rtsdf_point_distance", _lib.rtsdf_point_distance(scene.handle, _ptr(points), points.shape[0], _ptr(dist),
                                                             _ptr(tri), _stream(stream)))


def rtsdf_texel_distance(scene: "Scene", grid: Grid, texels, dist, tri=None, stream=None):
    """Distance at texel centres; texels=None means every texel of the grid (n = grid.n^3)."""
    count = grid.n ** 3 if texels is None else texels.numel()
    _check("rtsdf_texel_distance", _lib.rtsdf_texel_distance(scene.handle, grid, _ptr(texels), count, _ptr(dist),
                                                             _ptr(tri), _stream(stream)))


def rtsdf_shadow_ex(fine: Grid, fine_sdf, points, light_dir, k: float, eps: float, max_steps: int, max_step: float,
                    max_dist: float, visibility, penumbra: int = 0, jitter=None, jitter_scale: float = 0.0,
                    stream=None):
    P = ShadowParams((_f32 * 3)(*[float(x) for x in light_dir]), float(k), float(eps), int(max_steps),
                     float(max_step), float(max_dist), int(penumbra), float(jitter_scale))
    _check("rtsdf_shadow_ex", _lib.rtsdf_shadow_ex(fine, _ptr(fine_sdf), _ptr(points), points.shape[0], C.byref(P),
                                                   _ptr(jitter), _ptr(visibility), _stream(stream)))


class FrameGraph:
    """Owning handle of an ``rtsdf_frame_graph`` (one captured SDF update)."""

    def __init__(self, desc: FrameDesc | None, keepalive=(), stream=None, handle=None):
        self._desc = desc
        self._keep = keepalive
        if handle is not None:
            self.handle = handle
            return
        h = _P()
        _check("rtsdf_frame_graph_create", _lib.rtsdf_frame_graph_create(C.byref(desc), C.byref(h), _stream(stream)))
        self.handle = h

    def launch(self, stream=None):
        _check("rtsdf_frame_graph_launch", _lib.rtsdf_frame_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            _lib.rtsdf_frame_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev_view(ptr: int, n: int, dtype: torch.dtype, device) -> torch.Tensor:
    """A copy (on the current stream) of n elements of library-owned device memory."""
    out = torch.empty(n, dtype=dtype, device=device)
    _check("rtsdf_copy", _lib.rtsdf_copy(_ptr(out), int(ptr), out.numel() * out.element_size(), _stream(None)))
    return out


class Batch:
    """Owning handle of an ``rtsdf_batch``: many scenes, one launch per stage."""

    def __init__(self, scenes: list[dict], seed: int = 0, leaf_size: int = 4, stream=None):
        arr = (BatchScene * len(scenes))()
        self._keep = []
        for i, d in enumerate(scenes):
            v = d["vertices"].contiguous()
            f = d["faces"].contiguous()
            _dtype(v, torch.float32, "vertices")
            _dtype(f, torch.int32, "faces")
            self._keep += [v, f]
            b = arr[i]
            b.vertices, b.nv, b.faces, b.nt = _ptr(v), v.shape[0], _ptr(f), f.shape[0]
            lo = d.get("lo", (0.0, 0.0, 0.0))
            b.lo[0], b.lo[1], b.lo[2] = (float(x) for x in lo)
            b.side = float(d.get("side", 1.0))
            b.coarse_n, b.fine_n = int(d["coarse_n"]), int(d["fine_n"])
            b.beta, b.d = float(d["beta"]), float(d["d"])
            b.rays_per_texel, b.alpha, b.scene_id = int(d["rays"]), float(d.get("alpha", 1.0)), int(d.get("scene_id", i))
            b.sign_policy = SIGN_POLICIES[d.get("sign_policy", "vote")]
            b.shell = float(d.get("shell", 0.0))
        h = _P()
        _check("rtsdf_batch_create", _lib.rtsdf_batch_create(arr, len(scenes), int(seed), int(leaf_size), C.byref(h),
                                                             _stream(stream)))
        self.handle = h
        self.n = len(scenes)
        self.descriptors = [dict(fine_n=int(d["fine_n"]), coarse_n=int(d["coarse_n"]), nt=int(d["faces"].shape[0]),
                                 rays=int(d["rays"])) for d in scenes]
        self._keep = []  # the batch copied the meshes

    def step(self, frame: int, frame_ptr=None, stream=None):
        _check("rtsdf_batch_step", _lib.rtsdf_batch_step(self.handle, int(frame), _ptr(frame_ptr), _stream(stream)))

    def set_tuning(self, **kw):
        """Give this batch its own tracer tuning (fields of rtsdf_trace_tuning over the process default)."""
        t = TraceTuning(**{**rtsdf_trace_config_get().as_dict(), **getattr(self, "_tuning", {}), **kw})
        _check("rtsdf_batch_set_tuning", _lib.rtsdf_batch_set_tuning(self.handle, C.byref(t)))
        self._tuning = t.as_dict()

    def clear_tuning(self):
        _check("rtsdf_batch_set_tuning", _lib.rtsdf_batch_set_tuning(self.handle, None))
        self._tuning = {}

    def reset(self, stream=None):
        _check("rtsdf_batch_reset", _lib.rtsdf_batch_reset(self.handle, _stream(stream)))

    def view(self, i: int) -> BatchView:
        v = BatchView()
        _check("rtsdf_batch_outputs", _lib.rtsdf_batch_outputs(self.handle, int(i), C.byref(v)))
        return v

    def tensors(self, i: int, device="cuda") -> dict:
        """Copies of scene i's outputs as device tensors."""
        v = self.view(i)
        nc3, nf3 = v.coarse.n ** 3, v.fine.n ** 3
        return {
            "seeds": _dev_view(v.seeds, nc3, torch.int32, device),
            "dist2": _dev_view(v.dist2, nc3, torch.int32, device),
            "coarse_sdf": _dev_view(v.coarse_sdf, nc3, torch.float32, device),
            "mask": _dev_view(v.mask, nf3, torch.uint8, device),
            "count": _dev_view(v.count, 1, torch.int32, device),
            "queue": _dev_view(v.queue, nf3, torch.int32, device),
            "u": _dev_view(v.state.u, nf3, torch.float32, device),
            "hits": _dev_view(v.state.hits, nf3, torch.int32, device),
            "arg_tri": _dev_view(v.state.arg_tri, nf3, torch.int32, device),
            "arg_ray": _dev_view(v.state.arg_ray, nf3, torch.int32, device),
            "fine_sdf": _dev_view(v.fine_sdf, nf3, torch.float32, device),
        }

    def make_graph(self, first_frame: int = 0, stream=None) -> FrameGraph:
        self.frame_counter = torch.full((1,), int(first_frame), dtype=torch.int32, device="cuda")
        h = _P()
        _check("rtsdf_batch_graph_create", _lib.rtsdf_batch_graph_create(self.handle, _ptr(self.frame_counter),
                                                                         C.byref(h), _stream(stream)))
        return FrameGraph(None, keepalive=(self,), handle=h)

    def close(self):
        if getattr(self, "handle", None):
            _lib.rtsdf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
