"""Workloads at their full benchmark sizes.

The moving-scene workload at its full size (935,508 triangles, coarse 256^3, fine 512^3, 8 rays per texel,
alpha 0.9), in the configurations the benchmark times: refit of the creation hierarchy and a device rebuild,
over two frames of motion, against the oracle.

The oracle recomputes voxelization, flooding and selection at full size every frame (the coarse grid and the
selection mask are compared whole) and traces a seeded sample of 4,000 texel indices drawn uniformly over the
fine grid, independently of either side (about half of them are selected); traced values agree within the
trace tolerance, signs, hit counts and argmin triangles outside ambiguous rays.

The batched workload with all 64 scenes: each scene of the batch equals its single-scene run bit for bit.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth.scenes import workload

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_moving_scene_full_size_sampled():
    say("moving scene full size: refit and rebuild")
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    from paper_2210_04449_amd.pipeline import Pipeline
    from test_gpu_parity import compare_trace
    w = workload("dynamic")
    dyn = w.extra["scene"]
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(w.nf ** 3, 4000, replace=False)).astype(np.int32)
    mk = lambda rb: Pipeline(cu(w.mesh.vertices), cu(w.mesh.faces), w.nc, w.nf, w.beta, w.d, w.rays,  # noqa: E731
                             seed=w.seed, scene_id=w.scene_seed, alpha=w.alpha, rebuild=rb)
    pipes = {"refit": mk(False), "rebuild": mk(True)}
    st = oracle.TraceState(w.nf)
    for fr in range(2):
        m = dyn.mesh(fr)
        for p in pipes.values():
            p.set_vertices(cu(m.vertices))
            p.step(fr)
        ref = oracle.run_frames(m.vertices, m.faces, w.nc, w.nf, w.beta, w.d, w.rays, [fr], seed=w.seed,
                                scene=w.scene_seed, alpha=w.alpha, state=st, texels=sample)
        say("frame", fr, "oracle done")
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    for name, p in pipes.items():
        assert np.array_equal(p.seeds.cpu().numpy(), ref["seeds"]), name
        stats = compare_trace(p, ref, sample=sample)
        print(name, stats)
        assert stats["texels"] > 1000
        p.close()


def test_batch_full_configuration_matches_single_scene_runs():
    """All 64 scenes of the batched workload (1.23 M triangles, coarse 32/64/128) in one batch: every scene's
    seeds, mask, queue, fine SDF and state equal a single-scene run of the same scene bit for bit (the
    single-scene path is the one compared with the oracle)."""
    say("batch, full configuration")
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    from paper_2210_04449_amd.pipeline import Pipeline
    from synth.scenes import batched_scenes
    ws = batched_scenes(64)
    B = R.Batch([dict(vertices=cu(w.mesh.vertices), faces=cu(w.mesh.faces), coarse_n=w.nc, fine_n=w.nf,
                      beta=w.beta, d=w.d, rays=w.rays, alpha=w.alpha, scene_id=w.scene_seed) for w in ws], seed=0)
    frames = 2
    for f in range(frames):
        B.step(f)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    for i, w in enumerate(ws):
        p = Pipeline(cu(w.mesh.vertices), cu(w.mesh.faces), w.nc, w.nf, w.beta, w.d, w.rays, seed=0,
                     scene_id=w.scene_seed, alpha=w.alpha)
        for f in range(frames):
            p.step(f)
        torch.cuda.synchronize()
        t = B.tensors(i)
        n = p.selected()
        ok = (torch.equal(t["seeds"], p.seeds) and torch.equal(t["mask"], p.mask) and int(t["count"].item()) == n
              and torch.equal(t["queue"][:n], p.queue[:n]) and torch.equal(t["fine_sdf"], p.fine_sdf)
              and torch.equal(t["u"], p.state.u) and torch.equal(t["hits"], p.state.hits)
              and torch.equal(t["arg_tri"], p.state.arg_tri))
        assert ok, (i, w.mesh.nt, w.nc)
        p.close()
    B.close()
