"""The 4-wide copy of the hierarchy (tuning bvh_width 4) on the GPU:

* the tiny workload over all texels and the room workload on a sample, each
  against the oracle with the exact checks of compare_trace;
* a refitted moving scene (20 % of primitives moving, alpha 0.9) traced with
  the wide copy, against the oracle frame by frame;
* traces with width 4 equal those with width 2 (the closest hit is the
  minimum over all references whatever the traversal order; only rays whose
  two best candidates tie within rounding may differ, at most one texel in
  10^5);
* the refusals: a two-level scene, and a scene rebuilding on the device
  (which drops the copy).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth.scenes import DynamicScene, workload

pytestmark = pytest.mark.gpu


def say(*a):
    print("[wide]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    return R


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pipe(w, width, **kw):
    from paper_2210_04449_amd.pipeline import Pipeline
    p = Pipeline(cu(w.mesh.vertices), cu(w.mesh.faces), w.nc, w.nf, w.beta, w.d, w.rays, seed=0,
                 scene_id=w.scene_seed, alpha=w.alpha, **kw)
    p.scene.set_tuning(bvh_width=width)
    return p


def same(a, b, tol=1e-5):
    diff = ((a.fine_sdf != b.fine_sdf) | (a.state.u != b.state.u) | (a.state.hits != b.state.hits)
            | (a.state.arg_tri != b.state.arg_tri) | (a.state.arg_ray != b.state.arg_ray))
    n = int(diff.sum())
    if n:
        d = float((a.fine_sdf[diff].abs() - b.fine_sdf[diff].abs()).abs().max())
        print("texels differing:", n, "max |f| difference", d)
        if d > tol:
            return False
    return n <= max(1, diff.numel() // 100000)


@pytest.mark.parametrize("case", ["tiny", "room"])
def test_wide_against_oracle_and_two_wide(R, case):
    from test_gpu_parity import compare_trace
    w = workload(case)
    frames = range(w.frames) if case == "tiny" else range(2)
    say(case, "frames", len(frames))
    p4, p2 = pipe(w, 4), pipe(w, 2)
    assert p4.scene.tuning().bvh_width == 4
    for f in frames:
        p4.step(f)
        p2.step(f)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    assert same(p4, p2)
    sample = None
    if case == "room":
        sel = np.nonzero(p4.mask.cpu().numpy())[0]
        sample = np.sort(np.random.default_rng(5).choice(sel, 4000, replace=False)).astype(np.int32)
    ref = oracle.run_frames(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, frames, seed=0,
                            scene=w.scene_seed, texels=sample)
    print(compare_trace(p4, ref, sample=sample))
    p4.close()
    p2.close()


def test_wide_refit_moving_scene(R):
    from test_gpu_parity import compare_trace
    from paper_2210_04449_amd.pipeline import Pipeline
    say("refit moving")
    dyn = DynamicScene(7, n_prims=30, detail="low")
    nc, nf, rays, alpha = 32, 64, 4, 0.9
    beta, d = np.float32(0.5 / nc), np.float32(2.0 / nc)
    m0 = dyn.mesh(0)
    ps = {}
    for width in (4, 2):
        p = Pipeline(cu(m0.vertices), cu(m0.faces), nc, nf, float(beta), float(d), rays, scene_id=9, alpha=alpha,
                     rebuild=False)
        p.scene.set_tuning(bvh_width=width)
        ps[width] = p
    st = oracle.TraceState(nf)
    for f in range(5):
        m = dyn.mesh(f)
        for p in ps.values():
            p.set_vertices(cu(m.vertices))
            p.step(f)
        ref = oracle.run_frames(m.vertices, m.faces, nc, nf, beta, d, rays, [f], seed=0, scene=9, alpha=alpha,
                                state=st)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    assert same(ps[4], ps[2])
    print(compare_trace(ps[4], ref))


def test_wide_refusals(R):
    say("refusals")
    from paper_2210_04449_amd.pipeline import Pipeline
    w = workload("tiny")
    p = Pipeline(cu(w.mesh.vertices), cu(w.mesh.faces), w.nc, w.nf, w.beta, w.d, w.rays, rebuild=True)
    with pytest.raises(R.RtsdfError):
        p.scene.set_tuning(bvh_width=4)  # a rebuilding scene has no 4-wide copy
    dyn = DynamicScene(7, n_prims=6, detail="low")
    pv, pf, offs, _ = dyn.parts()
    q = Pipeline(cu(pv), cu(pf), 16, 32, 0.5 / 16, 2.0 / 16, 2, parts=(offs, cu(dyn.part_transforms(0))))
    with pytest.raises(R.RtsdfError):
        q.scene.set_tuning(bvh_width=4)
    # enabling the rebuild after the copy exists drops it: traces fall back to two-wide (and stay correct)
    r = Pipeline(cu(w.mesh.vertices), cu(w.mesh.faces), w.nc, w.nf, w.beta, w.d, w.rays, rebuild=False)
    r.scene.set_tuning(bvh_width=4)
    r.step(0)
    r.scene.enable_rebuild()
    r.step(1)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
