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


def test_differentiable_full_size_gradient_sampled():
    """The differentiable workload (9,680-triangle perturbed sphere, 64^3 / 128^3, 32 rays x 16 frames): on a
    seeded sample of 2,000 texels from the oracle's own selection, the traced state matches the oracle, and the
    vertex gradient of a loss on those texels (sum of (f - sphere SDF)^2 where both sides took the same argmin ray)
    matches the oracle's analytic gradient within 1e-4 relative L2."""
    say("differentiable workload full size")
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    from paper_2210_04449_amd.pipeline import Pipeline
    from test_gpu_parity import compare_trace
    w = workload("diff")
    m = w.mesh
    frames = range(w.frames)
    lo = np.zeros(3, np.float32)
    hc, hf = np.float32(1.0 / w.nc), np.float32(1.0 / w.nf)
    beta, d = np.float32(w.beta), np.float32(w.d)
    d2, _ = oracle.coarse(w.nc, oracle.jfa(w.nc, oracle.voxelize(m.vertices, m.faces, lo, hc, w.nc)), hc, beta)
    _, queue = oracle.select(w.nc, d2, w.nf, oracle.select_threshold(hc, beta, d))
    sample = np.sort(np.random.default_rng(7).choice(queue, 2000, replace=False)).astype(np.int32)
    ref = oracle.run_frames(m.vertices, m.faces, w.nc, w.nf, beta, d, w.rays, frames, seed=w.seed,
                            scene=w.scene_seed, alpha=w.alpha, texels=sample)
    st = ref["state"]
    p = Pipeline(cu(m.vertices), cu(m.faces), w.nc, w.nf, float(beta), float(d), w.rays, seed=w.seed,
                 scene_id=w.scene_seed, alpha=w.alpha)
    for f in frames:
        p.step(f)
    torch.cuda.synchronize()
    # 512 rays per texel: about one texel in six has some ray crossing near a triangle edge
    stats = compare_trace(p, ref, sample=sample, max_flagged=0.25)
    print(stats)
    assert stats["texels"] == len(sample) and stats["exact_hits"] > 1400 and stats["exact_arg"] > 1800
    fine = p.fine_sdf.cpu().numpy().astype(np.float64)
    at, ar = p.state.arg_tri.cpu().numpy(), p.state.arg_ray.cpu().numpy()
    j = sample.astype(np.int64)
    P = (np.stack([j % w.nf, (j // w.nf) % w.nf, j // w.nf ** 2], 1) + 0.5) / w.nf
    target = np.linalg.norm(P - 0.5, axis=1) - 0.3
    agree = ((at[j] == st.arg_tri[j]) & (ar[j] == ((st.arg_frame[j] << 8) | np.maximum(st.arg_ray[j], 0)))
             & (st.arg_amb[j] == 0) & (np.sign(fine[j]) == np.sign(st.fine[j])))
    assert agree.mean() > 0.99
    gf = np.zeros(w.nf ** 3)
    gf[j] = np.where(agree, 2 * (fine[j] - target), 0.0)
    gv = torch.zeros(m.nv * 3, dtype=torch.float32, device="cuda")
    R.rtsdf_trace_backward(p.scene, p.fine, p.state, p.fine_sdf, cu(gf.astype(np.float32)), w.seed, w.scene_seed, gv)
    got = gv.cpu().numpy().reshape(-1, 3).astype(np.float64)
    want = oracle.Scene(m.vertices, m.faces).fine_grad(w.nf, lo, hf, w.seed, w.scene_seed, st, gf)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("grad rel L2", rel, "nonzero vertices", int((np.abs(want).sum(1) > 0).sum()))
    assert np.linalg.norm(want) > 0 and rel <= 1e-4
    p.close()
