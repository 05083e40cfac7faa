"""The moving-scene workload at its full size (935,508 triangles, coarse 256^3, fine 512^3, 8 rays per texel,
alpha 0.9), in the configurations the benchmark times: refit of the creation hierarchy and a device rebuild,
over two frames of motion, against the oracle.

The oracle recomputes voxelization, flooding and selection at full size every frame (the coarse grid and the
selection mask are compared whole) and traces a seeded sample of 4,000 texel indices drawn uniformly over the
fine grid, independently of either side (about half of them are selected); traced values agree within the
trace tolerance, signs, hit counts and argmin triangles outside ambiguous rays.
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
