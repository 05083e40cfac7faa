"""Captured per-frame graphs and many-scene batches, on the GPU.

* A graph replay performs exactly the eager update (bitwise), replay after
  replay, with other GPU work and synchronisations in between, and advances
  its device-side frame counter; with refit it follows moving vertices.
* Every scene of a batch equals its own single-scene run bitwise (forward),
  for scenes of different triangle counts and grid sizes in one launch, and a
  captured batch step equals the eager batch step.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth.scenes import Workload, batched_scenes, icosphere, tiny_scene, workload

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    return R


def pipe(w, **kw):
    from paper_2210_04449_amd.pipeline import Pipeline
    return Pipeline(torch.from_numpy(w.mesh.vertices).cuda(), torch.from_numpy(w.mesh.faces).cuda(), w.nc, w.nf,
                    w.beta, w.d, w.rays, seed=kw.get("seed", 0), scene_id=w.scene_seed, alpha=kw.get("alpha", w.alpha))


def same_state(a, b):
    return (torch.equal(a.fine_sdf, b.fine_sdf) and torch.equal(a.state.u, b.state.u)
            and torch.equal(a.state.hits, b.state.hits) and torch.equal(a.state.arg_tri, b.state.arg_tri)
            and torch.equal(a.state.arg_ray, b.state.arg_ray))


def test_graph_replays_match_eager(R):
    say("graph replay")
    w = workload("tiny")
    eager, cap = pipe(w), pipe(w)
    g = cap.make_graph(first_frame=0)
    scratch = torch.zeros(1 << 20, device="cuda")
    for f in range(6):
        eager.step(f)
        g.launch()
        scratch.add_(1.0)  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert int(cap.frame_counter.item()) == f + 1
        assert same_state(eager, cap), f
        assert torch.equal(eager.seeds, cap.seeds) and torch.equal(eager.mask, cap.mask)
    g.close()


def test_graph_with_refit_follows_moving_vertices(R):
    say("graph refit")
    s = icosphere(2, 0.25, (0.5, 0.5, 0.5))
    w = Workload("moving", s, 32, 64, 0.5, 2.0, 4, 4, alpha=0.75)
    eager, cap = pipe(w), pipe(w)
    g = cap.make_graph(first_frame=0, refit=True)
    base = torch.from_numpy(s.vertices).cuda()
    for f in range(4):
        moved = base + torch.tensor([0.01 * f, 0.005 * f, 0.0], device="cuda")
        eager.set_vertices(moved)
        eager.step(f)
        cap.vertices.copy_(moved)
        g.launch()
        torch.cuda.synchronize()
        assert same_state(eager, cap), f
    g.close()


def _batch_workloads(n=6):
    ws = batched_scenes(n, seed0=3)
    ws.append(workload("tiny"))
    return ws


def test_batch_matches_single_scene_runs(R):
    say("batch vs single")
    ws = _batch_workloads()
    B = R.Batch([dict(vertices=torch.from_numpy(w.mesh.vertices).cuda(), faces=torch.from_numpy(w.mesh.faces).cuda(),
                      coarse_n=w.nc, fine_n=w.nf, beta=w.beta, d=w.d, rays=w.rays, alpha=w.alpha,
                      scene_id=w.scene_seed) for w in ws], seed=0)
    frames = 3
    for f in range(frames):
        B.step(f)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    for i, w in enumerate(ws):
        say("batch scene", i, w.mesh.nt, w.nc, w.nf)
        p = pipe(w)
        for f in range(frames):
            p.step(f)
        torch.cuda.synchronize()
        t = B.tensors(i)
        torch.cuda.synchronize()
        assert torch.equal(t["seeds"], p.seeds)
        assert torch.equal(t["dist2"], p.dist2)
        assert torch.equal(t["mask"], p.mask)
        assert int(t["count"].item()) == p.selected()
        assert torch.equal(t["queue"][: p.selected()], p.queue[: p.selected()])
        assert torch.equal(t["fine_sdf"], p.fine_sdf)
        assert torch.equal(t["u"], p.state.u) and torch.equal(t["hits"], p.state.hits)
        assert torch.equal(t["arg_tri"], p.state.arg_tri)
    B.close()


def test_batch_graph_matches_eager_batch(R):
    say("batch graph")
    ws = _batch_workloads(3)
    scenes = [dict(vertices=torch.from_numpy(w.mesh.vertices).cuda(), faces=torch.from_numpy(w.mesh.faces).cuda(),
                   coarse_n=w.nc, fine_n=w.nf, beta=w.beta, d=w.d, rays=w.rays, alpha=w.alpha,
                   scene_id=w.scene_seed) for w in ws]
    A, B = R.Batch(scenes), R.Batch(scenes)
    g = B.make_graph(first_frame=0)
    for f in range(4):
        A.step(f)
        g.launch()
        torch.cuda.synchronize()
        for i in range(len(ws)):
            assert torch.equal(A.tensors(i)["fine_sdf"], B.tensors(i)["fine_sdf"]), (f, i)
    g.close()
    A.close()
    B.close()


def test_batch_scene_against_oracle(R):
    say("batch scene vs oracle")
    w = workload("tiny")
    other = batched_scenes(2, seed0=5)
    B = R.Batch([dict(vertices=torch.from_numpy(x.mesh.vertices).cuda(), faces=torch.from_numpy(x.mesh.faces).cuda(),
                      coarse_n=x.nc, fine_n=x.nf, beta=x.beta, d=x.d, rays=x.rays, scene_id=x.scene_seed)
                 for x in [other[0], w, other[1]]], seed=0)
    for f in range(2):
        B.step(f)
    torch.cuda.synchronize()
    t = B.tensors(1)
    ref = oracle.run_frames(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, range(2), seed=0,
                            scene=w.scene_seed)
    assert np.array_equal(t["mask"].cpu().numpy(), ref["mask"])
    st = ref["state"]
    fine = t["fine_sdf"].cpu().numpy().astype(np.float64)
    sel = np.nonzero(ref["mask"])[0]
    good = sel[st.arg_amb[sel] == 0]
    assert np.max(np.abs(np.abs(fine[good]) - np.abs(st.fine[good]))) <= 1e-5
    B.close()
