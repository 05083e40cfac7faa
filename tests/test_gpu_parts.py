"""Two-level scenes of rigid parts on the GPU, against the oracle on the world mesh.

* World positions from the parts' transforms are bit-exact with the oracle's
  (so voxelization, flooding and selection are too).
* Traced values match the oracle tracing the world mesh within 1e-5 x extent
  (the tracer works in each part's object space: the transform adds float32
  rounding of about 1e-7), sign / hit counts / argmin faces agree outside
  ambiguous rays, over several frames of motion with alpha 0.9.
* The same geometry as a single-level scene gives the same values to the same
  tolerance, and a static two-level scene is deterministic.
* Bad input: a vertex shared by two parts, a non-rigid transform (EINVAL at
  create, an error bit at set_transforms), calls that take single-level scenes.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth.scenes import DynamicScene, rigid_parts

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    return R


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def part_of_vertex(nv, f, offs):
    part = np.full(nv, -1, np.int32)
    for i in range(len(offs) - 1):
        part[np.unique(f[offs[i]:offs[i + 1]])] = i
    return part


def compare(p, ref):
    from test_gpu_parity import compare_trace
    return compare_trace(p, ref)


def test_parts_static_against_oracle(R):
    say("parts static")
    from paper_2210_04449_amd.pipeline import Pipeline
    v, f, offs, T = rigid_parts()
    nc, nf, rays, frames = 32, 64, 4, 4
    beta, d = np.float32(0.5 / nc), np.float32(2.0 / nc)
    p = Pipeline(cu(v), cu(f), nc, nf, float(beta), float(d), rays, scene_id=3, parts=(offs, cu(T)))
    info = p.scene.info()
    assert info.instances == 3 and info.nt == len(f)
    w = oracle.instance_world(v, part_of_vertex(len(v), f, offs), T)
    torch.cuda.synchronize()
    assert np.array_equal(p.vertices.cpu().numpy().view(np.int32), w.view(np.int32))
    for fr in range(frames):
        p.step(fr)
    torch.cuda.synchronize()
    ref = oracle.run_frames(w, f, nc, nf, beta, d, rays, range(frames), scene=3)
    assert np.array_equal(p.seeds.cpu().numpy(), ref["seeds"])
    stats = compare(p, ref)
    print(stats)
    assert stats["texels"] > 20000
    # the same world geometry as one hierarchy: same values within the tolerance
    flat = Pipeline(cu(w), cu(f), nc, nf, float(beta), float(d), rays, scene_id=3)
    for fr in range(frames):
        flat.step(fr)
    q = Pipeline(cu(v), cu(f), nc, nf, float(beta), float(d), rays, scene_id=3, parts=(offs, cu(T)))
    for fr in range(frames):
        q.step(fr)
    torch.cuda.synchronize()
    assert torch.equal(q.fine_sdf, p.fine_sdf) and torch.equal(q.state.hits, p.state.hits)  # deterministic
    sel = p.mask.bool()
    diff = (p.fine_sdf[sel].abs() - flat.fine_sdf[sel].abs()).abs()
    agree = (p.state.arg_tri[sel] == flat.state.arg_tri[sel]).float().mean().item()
    print("two-level vs one hierarchy: max |diff|", diff.max().item(), "argmin agreement", agree)
    assert agree > 0.999
    assert diff.quantile(0.999).item() <= TOL


def test_parts_moving_against_oracle(R):
    say("parts moving")
    from paper_2210_04449_amd.pipeline import Pipeline
    dyn = DynamicScene(7, n_prims=30, detail="low")
    v, f, offs, _ = dyn.parts()
    part = part_of_vertex(len(v), f, offs)
    nc, nf, rays, alpha = 32, 64, 4, 0.9
    beta, d = np.float32(0.5 / nc), np.float32(2.0 / nc)
    p = Pipeline(cu(v), cu(f), nc, nf, float(beta), float(d), rays, scene_id=9, alpha=alpha,
                 parts=(offs, cu(dyn.part_transforms(0))))
    st = oracle.TraceState(nf)
    for fr in range(5):
        T = dyn.part_transforms(fr)
        p.set_transforms(cu(T))
        p.step(fr)
        w = oracle.instance_world(v, part, T)
        ref = oracle.run_frames(w, f, nc, nf, beta, d, rays, [fr], seed=0, scene=9, alpha=alpha, state=st)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    assert np.array_equal(p.vertices.cpu().numpy().view(np.int32), w.view(np.int32))
    stats = compare(p, ref)
    print(stats)
    assert stats["texels"] > 10000


def test_parts_bad_input(R):
    say("parts bad input")
    v, f, offs, T = rigid_parts()
    # a vertex used by two parts
    f2 = f.copy()
    f2[offs[1], 0] = f[0, 0]
    with pytest.raises(R.RtsdfError):
        R.Scene.instanced(cu(v), cu(f2), offs, cu(T))
    # a scaled (non-rigid) transform
    T2 = T.copy()
    T2[1, :3] *= 1.5
    with pytest.raises(R.RtsdfError):
        R.Scene.instanced(cu(v), cu(f), offs, cu(T2))
    # offsets that do not cover the faces, or an empty part
    with pytest.raises(R.RtsdfError):
        R.Scene.instanced(cu(v), cu(f), [0, 2, 2, len(f)], cu(T))
    sc = R.Scene.instanced(cu(v), cu(f), offs, cu(T))
    sc.set_transforms(cu(T2))  # detected on the device: the error bit, the call itself goes on
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() & R.ERR_TRANSFORM
    sc.set_transforms(cu(T))
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    o = torch.zeros((4, 3), device="cuda")
    t = torch.empty(4, device="cuda")
    i = torch.empty(4, dtype=torch.int32, device="cuda")
    with pytest.raises(R.RtsdfError):
        R.rtsdf_closest_hits(sc, o, o, t, i, i)
    with pytest.raises(R.RtsdfError):
        R.rtsdf_point_distance(sc, o, t)
    with pytest.raises(R.RtsdfError):
        sc.refit(cu(v))
    with pytest.raises(R.RtsdfError):
        sc.hierarchy()  # the export takes single-level scenes
    sc.close()


def test_parts_without_static_world_and_without_movers(R):
    """Part 0 may be empty (every part moves), and a scene may have no moving part (static world only): both
    trace as the oracle on the world mesh."""
    say("parts edge layouts")
    from paper_2210_04449_amd.pipeline import Pipeline
    v, f, offs, T = rigid_parts()
    nc, nf, rays, frames = 32, 64, 4, 2
    beta, d = np.float32(0.5 / nc), np.float32(2.0 / nc)
    # drop the ground quad: parts = [empty static world, sphere, torus]
    keep = f[offs[1]:]
    used = np.unique(keep)
    remap = np.full(len(v), -1, np.int64)
    remap[used] = np.arange(len(used))
    v2, f2 = v[used], remap[keep].astype(np.int32)
    offs2 = [0, 0, offs[2] - offs[1], len(f2)]
    for verts, faces, o, tr in ((v2, f2, offs2, T), (v[:4], f[:2], [0, 2], T[:1])):
        p = Pipeline(cu(verts), cu(faces), nc, nf, float(beta), float(d), rays, scene_id=5, parts=(o, cu(tr)))
        for fr in range(frames):
            p.step(fr)
        torch.cuda.synchronize()
        w = oracle.instance_world(verts, part_of_vertex(len(verts), faces, o), tr)
        ref = oracle.run_frames(w, faces, nc, nf, beta, d, rays, range(frames), scene=5)
        print(len(o) - 1, "parts:", compare(p, ref))
        p.close()


def test_parts_graph_replays_eager(R):
    """A captured update of a two-level scene applies the transform buffer at each launch: replays equal the
    eager updates bit for bit while the parts move."""
    say("parts graph")
    from paper_2210_04449_amd.pipeline import Pipeline
    dyn = DynamicScene(7, n_prims=30, detail="low")
    v, f, offs, _ = dyn.parts()
    nc, nf, rays = 32, 64, 4
    beta, d = 0.5 / nc, 2.0 / nc
    mk = lambda: Pipeline(cu(v), cu(f), nc, nf, beta, d, rays, scene_id=9, alpha=0.9,  # noqa: E731
                          parts=(offs, cu(dyn.part_transforms(0))))
    eager, cap = mk(), mk()
    g = cap.make_graph(first_frame=0, refit=True)
    for fr in range(4):
        T = cu(dyn.part_transforms(fr + 1))
        eager.set_transforms(T)
        eager.step(fr)
        cap.transforms.copy_(T)
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(eager.vertices, cap.vertices) and torch.equal(eager.fine_sdf, cap.fine_sdf), fr
        assert torch.equal(eager.state.hits, cap.state.hits) and torch.equal(eager.mask, cap.mask), fr
    g.close()
