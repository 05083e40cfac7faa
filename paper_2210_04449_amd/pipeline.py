"""Per-frame SDF update on one GPU: voxelize -> jump flood -> select -> trace.

`Pipeline` owns every device buffer of the path (torch tensors used only as
device memory) and calls the C ABI in the order of the paper's design
(Sec. 2): coarse SDF by voxelization + jump flooding (Sec. 2.1), selection of
the fine texels near surfaces and ray-traced temporal accumulation
(Sec. 2.2).

``sampling`` chooses how a fine texel reads the coarse SDF for the selection
test c <= d and for c_t of Eq. (1): ``"point"`` (the coarse voxel containing
the texel centre) or ``"trilinear"`` (the coarse field interpolated at the
texel centre; the tracer then works on the fine grid alone).  ``sign_policy``
"vote" signs traced distances by the front/back vote of Sec. 2.2; "shell"
outputs the unsigned distance minus ``shell`` (open or thin surfaces).
``parts=(part_faces, transforms)`` builds a two-level scene of rigid parts
(vertices in object space; ``set_transforms`` moves them).  ``rebuild``
chooses how ``set_vertices`` updates a single-level hierarchy for moved
geometry: ``None`` (default) keeps the host-built SAH hierarchy while the
scene is static and switches to rebuilding it on the device at the first
``set_vertices`` (a refitted hierarchy loosens frame after frame under
continuous motion); ``True`` rebuilds on the device from the start;
``False`` always refits.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import rtsdf as R


class Pipeline:
    def __init__(self, vertices: torch.Tensor, faces: torch.Tensor, nc: int, nf: int, beta: float, d: float,
                 rays: int, seed: int = 0, scene_id: int = 0, alpha: float = 1.0, lo=(0.0, 0.0, 0.0),
                 side: float = 1.0, leaf_size: int = 4, queue_cap: int | None = None, device="cuda",
                 jfa_variant: str = "jfa", sampling: str = "point", sign_policy: str = "vote",
                 shell: float = 0.0, parts=None, rebuild: bool | None = None):
        if sampling not in ("point", "trilinear"):
            raise ValueError(f"sampling must be 'point' or 'trilinear', not {sampling!r}")
        self.sampling = sampling
        self.leaf_size = int(leaf_size)
        self.device = torch.device(device)
        self.vertices = vertices.to(self.device, torch.float32).contiguous()
        self.faces = faces.to(self.device, torch.int32).contiguous()
        self.coarse = R.Grid.make(nc, side / nc, lo)
        self.fine = R.Grid.make(nf, side / nf, lo)
        self.nc, self.nf = nc, nf
        self.jfa_steps = None if jfa_variant == "jfa" else R.jfa_schedule(nc, jfa_variant)
        self.beta, self.d = float(beta), float(d)
        self.rays, self.seed, self.scene_id, self.alpha = int(rays), int(seed), int(scene_id), float(alpha)
        dev = self.device
        i32, f32 = torch.int32, torch.float32
        self.seeds = torch.empty(nc ** 3, dtype=i32, device=dev)
        self.scratch = torch.empty(nc ** 3, dtype=i32, device=dev)
        self.dist2 = torch.empty(nc ** 3, dtype=i32, device=dev)
        self.coarse_sdf = torch.empty(nc ** 3, dtype=f32, device=dev)
        self.mask = torch.empty(nf ** 3, dtype=torch.uint8, device=dev)
        self.queue = torch.empty(nf ** 3 if queue_cap is None else int(queue_cap), dtype=i32, device=dev)
        self.count = torch.zeros(1, dtype=i32, device=dev)
        tri = sampling == "trilinear"
        self.fine_c = torch.empty(nf ** 3, dtype=f32, device=dev) if tri else None
        self.sel_ws = torch.empty(R.rtsdf_select_workspace_size(nf if tri else nc), dtype=torch.uint8, device=dev)
        self.trace_ws = torch.empty(R.rtsdf_trace_workspace_size(), dtype=torch.uint8, device=dev)
        self.fine_sdf = torch.empty(nf ** 3, dtype=f32, device=dev)
        self.state = R.AccumState(self.fine, dev)
        if parts is None:
            self.scene = R.Scene(self.vertices, self.faces, leaf_size)
        else:
            # rigid parts: `vertices` are in object space; voxelization reads the world positions the scene
            # computes from the transforms
            part_faces, transforms = parts
            self.obj_vertices = self.vertices
            self.vertices = torch.empty_like(self.obj_vertices)
            self.transforms = transforms.to(self.device, torch.float32).contiguous().clone()  # read by graphs
            self.scene = R.Scene.instanced(self.obj_vertices, self.faces, part_faces, self.transforms, leaf_size)
            self.scene.world_vertices(self.vertices)
        self.parts = parts is not None
        self.rebuild_policy = None if rebuild is None else bool(rebuild)
        self.rebuild = False  # whether set_vertices rebuilds the hierarchy on the device (else it refits)
        if rebuild:
            self._enable_rebuild()
        self.scene.set_sign(sign_policy, shell)

    # -- stages ----------------------------------------------------------
    def voxelize(self, stream=None):
        R.rtsdf_voxelize(self.vertices, self.faces, self.coarse, self.seeds, stream)

    def jfa(self, stream=None):
        if self.jfa_steps is None:
            R.rtsdf_jfa(self.coarse, self.seeds, self.scratch, self.beta, self.dist2, self.coarse_sdf, stream)
        else:
            R.rtsdf_jfa_steps(self.coarse, self.seeds, self.scratch, self.jfa_steps, self.beta, self.dist2,
                              self.coarse_sdf, stream)

    def select(self, stream=None):
        if self.fine_c is None:
            R.rtsdf_select(self.coarse, self.dist2, self.fine, self.beta, self.d, self.mask, self.queue, self.count,
                           self.sel_ws, stream)
        else:
            R.rtsdf_coarse_trilinear(self.coarse, self.coarse_sdf, self.fine, self.fine_c, stream)
            R.rtsdf_select_field(self.fine, self.fine_c, self.d, self.mask, self.queue, self.count, self.sel_ws,
                                 stream)

    def trace_field(self):
        """(grid, field) the tracer reads c_t from: the coarse SDF, or its trilinear samples on the fine grid."""
        return (self.coarse, self.coarse_sdf) if self.fine_c is None else (self.fine, self.fine_c)

    def trace(self, frame: int, stream=None, frame_ptr=None):
        cgrid, cfield = self.trace_field()
        R.rtsdf_trace_accumulate(self.scene, cgrid, cfield, self.fine, self.mask, self.queue,
                                 self.count, self.rays, frame, self.seed, self.scene_id, self.alpha, self.state,
                                 self.fine_sdf, self.trace_ws, frame_ptr=frame_ptr, stream=stream)

    def step(self, frame: int, stream=None):
        """One SDF update (all stages) for frame index `frame`."""
        self.voxelize(stream)
        self.jfa(stream)
        self.select(stream)
        self.trace(frame, stream)

    def _enable_rebuild(self):
        if not self.rebuild and not self.parts and self.faces.shape[0] > 1:
            self.scene.enable_rebuild()
            self.rebuild = True

    def make_graph(self, first_frame: int = 0, refit: bool = False) -> "R.FrameGraph":
        """Capture one whole update as a HIP graph; each launch advances the frame index.  With refit, each
        launch updates the hierarchy from `self.vertices` as they are then (a device rebuild, or a refit
        with rebuild=False), or for rigid parts applies `self.transforms`."""
        if refit and self.rebuild_policy is None:
            self._enable_rebuild()
        self.frame_counter = torch.full((1,), int(first_frame), dtype=torch.int32, device=self.device)
        D = R.FrameDesc()
        D.vertices, D.nv = self.vertices.data_ptr(), self.vertices.shape[0]
        D.faces, D.nt = self.faces.data_ptr(), self.faces.shape[0]
        D.scene, D.refit = self.scene.handle, (2 if self.rebuild else 1) if refit else 0
        D.coarse, D.fine = self.coarse, self.fine
        D.beta, D.d, D.rays_per_texel = self.beta, self.d, self.rays
        D.seed, D.scene_id, D.alpha = self.seed, self.scene_id, self.alpha
        D.seeds, D.scratch, D.dist2 = self.seeds.data_ptr(), self.scratch.data_ptr(), self.dist2.data_ptr()
        D.coarse_sdf, D.mask = self.coarse_sdf.data_ptr(), self.mask.data_ptr()
        D.queue, D.queue_cap, D.count = self.queue.data_ptr(), self.queue.numel(), self.count.data_ptr()
        D.select_workspace = self.sel_ws.data_ptr()
        D.state = self.state.struct()
        D.fine_sdf, D.trace_workspace = self.fine_sdf.data_ptr(), self.trace_ws.data_ptr()
        D.frame_counter = self.frame_counter.data_ptr()
        D.fine_c = None if self.fine_c is None else self.fine_c.data_ptr()
        if self.parts:  # each launch applies self.transforms (update it in place between launches)
            D.transforms, D.world_vertices = self.transforms.data_ptr(), self.vertices.data_ptr()
        steps = None
        if self.jfa_steps is not None:
            steps = (C.c_int32 * len(self.jfa_steps))(*self.jfa_steps)  # read during create only
            D.jfa_steps, D.jfa_nsteps = C.cast(steps, C.c_void_p), len(self.jfa_steps)
        return R.FrameGraph(D, keepalive=(self, steps))

    def set_vertices(self, vertices: torch.Tensor, stream=None):
        """New positions for the same topology (animated scenes): refit the hierarchy."""
        if self.parts:
            raise RuntimeError("a scene of rigid parts moves by set_transforms")
        self.vertices.copy_(vertices)
        if self.rebuild_policy is None:
            self._enable_rebuild()
        if self.rebuild:
            self.scene.rebuild(self.vertices, stream)
        else:
            self.scene.refit(self.vertices, stream)

    def set_transforms(self, transforms: torch.Tensor, stream=None):
        """New object-to-world transforms of the rigid parts: top-level refit and world positions."""
        if not self.parts:
            raise RuntimeError("set_transforms needs a scene of rigid parts")
        if transforms.data_ptr() != self.transforms.data_ptr():
            self.transforms.copy_(transforms)
        self.scene.set_transforms(self.transforms, self.vertices, stream)

    def reset(self):
        R.rtsdf_accum_reset(self.fine, self.state)

    def selected(self) -> int:
        return int(self.count.item())

    def close(self):
        self.scene.close()
