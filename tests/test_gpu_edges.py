"""Edge cases of the whole update on the GPU, against the oracle or against
properties that hold whatever the input:

* a scene without triangles (nothing selected; every fine value is +inf);
* a queue too small for the selection (flagged; the texels that fit get the
  values of an unbounded run, texel by texel);
* degenerate (zero-area) triangles mixed into a mesh;
* a grid that is not the unit cube (offset origin, side 2);
* one ray per texel, 64 rays per texel, and alpha = 0 (pure decay).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth.scenes import Mesh, icosphere, tiny_scene, workload

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


def pipe(v, f, nc, nf, beta, d, rays, **kw):
    from paper_2210_04449_amd.pipeline import Pipeline
    return Pipeline(torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda(),
                    torch.from_numpy(np.ascontiguousarray(f, np.int32)).cuda(), nc, nf, beta, d, rays, **kw)


def check_against(p, ref, side=1.0):
    from test_gpu_parity import compare_trace
    return compare_trace(p, ref, tol=TOL * side)["texels"]


def test_scene_without_triangles(R):
    say("no triangles")
    nc, nf = 16, 32
    v = np.zeros((3, 3), np.float32)
    f = np.zeros((0, 3), np.int32)
    p = pipe(v, f, nc, nf, 0.5 / nc, 2.0 / nc, 4)
    for fr in range(2):
        p.step(fr)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    assert p.selected() == 0
    assert bool(torch.isinf(p.fine_sdf).all()) and bool((p.fine_sdf > 0).all())
    assert bool(torch.isinf(p.state.u).all()) and bool((p.state.hits == 0).all())


def test_queue_overflow_keeps_texels_that_fit(R):
    say("queue overflow")
    w = workload("tiny")
    full = pipe(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, scene_id=w.scene_seed)
    full.step(0)
    torch.cuda.synchronize()
    n = full.selected()
    cap = n // 3
    small = pipe(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, scene_id=w.scene_seed,
                 queue_cap=cap)
    small.step(0)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() != 0  # the select stage reports the full queue
    assert small.selected() == n       # the count is the true selection size
    q = small.queue[:cap].long()
    assert torch.equal(q, full.queue[:cap].long())
    for a, b in ((small.fine_sdf, full.fine_sdf), (small.state.u, full.state.u), (small.state.hits, full.state.hits),
                 (small.state.arg_tri, full.state.arg_tri)):
        assert torch.equal(a[q], b[q])
    assert R.rtsdf_sync_status() == 0  # cleared by the previous read


def test_degenerate_triangles_mixed_in(R):
    say("degenerate triangles")
    m = tiny_scene()
    rng = np.random.default_rng(3)
    nv = m.vertices.shape[0]
    extra_v = rng.uniform(0.2, 0.8, (30, 3)).astype(np.float32)
    v = np.concatenate([m.vertices, extra_v])
    # zero-area triangles: repeated vertices, and three collinear points
    deg = [[nv + i, nv + i, nv + i + 1] for i in range(0, 20, 2)]
    a, b = extra_v[20], extra_v[21]
    v = np.concatenate([v, np.stack([a, (a + b) / 2, b]).astype(np.float32)])
    deg.append([len(v) - 3, len(v) - 2, len(v) - 1])
    f = np.concatenate([m.faces, np.array(deg, np.int32)])
    nc, nf, rays = 32, 64, 4
    beta, d = float(np.float32(0.5 / nc)), float(np.float32(2.0 / nc))
    p = pipe(v, f, nc, nf, beta, d, rays)
    for fr in range(3):
        p.step(fr)
    torch.cuda.synchronize()
    ref = oracle.run_frames(v, f, nc, nf, beta, d, rays, range(3))
    assert np.array_equal(p.seeds.cpu().numpy(), ref["seeds"])
    assert check_against(p, ref) > 10000


def test_offset_grid_side_two(R):
    say("offset grid")
    m = tiny_scene()
    lo, side = np.array([-1.5, 0.25, 2.0], np.float32), 2.0
    v = (m.vertices.astype(np.float64) * side + lo).astype(np.float32)
    nc, nf, rays = 32, 64, 4
    beta, d = float(np.float32(0.5 * side / nc)), float(np.float32(2.0 * side / nc))
    p = pipe(v, m.faces, nc, nf, beta, d, rays, lo=tuple(float(x) for x in lo), side=side)
    for fr in range(2):
        p.step(fr)
    torch.cuda.synchronize()
    ref = oracle.run_frames(v, m.faces, nc, nf, beta, d, rays, range(2), lo=lo, side=side)
    assert np.array_equal(p.seeds.cpu().numpy(), ref["seeds"])
    assert np.array_equal(p.coarse_sdf.cpu().numpy().view(np.int32), ref["coarse"].view(np.int32))
    assert check_against(p, ref, side) > 10000


@pytest.mark.parametrize("rays,alpha", [(1, 1.0), (64, 1.0), (4, 0.0)])
def test_ray_count_limits_and_pure_decay(R, rays, alpha):
    say("rays", rays, "alpha", alpha)
    s = icosphere(2, 0.3, (0.5, 0.5, 0.5))
    nc, nf = 16, 32
    beta, d = float(np.float32(0.5 / nc)), float(np.float32(2.0 / nc))
    p = pipe(s.vertices, s.faces, nc, nf, beta, d, rays, alpha=alpha)
    for fr in range(3):
        p.step(fr)
    torch.cuda.synchronize()
    ref = oracle.run_frames(s.vertices, s.faces, nc, nf, beta, d, rays, range(3), alpha=alpha)
    assert check_against(p, ref) > 1000


def test_shell_sign_policy_against_oracle(R):
    """Shell policy (open or thin surfaces): fine = u - shell for traced texels, the coarse value elsewhere; the
    one-sided ground quad of the tiny scene no longer leaves a negative region below it."""
    say("shell sign policy")
    w = workload("tiny")
    shell = 1.0 / 128
    p = pipe(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, scene_id=w.scene_seed,
             sign_policy="shell", shell=shell)
    for fr in range(w.frames):
        p.step(fr)
    torch.cuda.synchronize()
    ref = oracle.run_frames(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, range(w.frames),
                            scene=w.scene_seed, sign_policy="shell", shell=shell)
    st = ref["state"]
    mask = p.mask.cpu().numpy()
    assert np.array_equal(mask, ref["mask"])
    fine = p.fine_sdf.cpu().numpy().astype(np.float64)
    sel = np.nonzero(mask)[0]
    good = sel[st.arg_amb[sel] == 0]
    assert np.max(np.abs(fine[good] - st.fine[good])) <= TOL
    unsel = np.nonzero(mask == 0)[0]
    assert np.array_equal(fine[unsel], st.fine[unsel])
    assert fine[sel].min() >= -shell - TOL  # nothing is inside a shell deeper than its half-thickness
    # the vote run of the same frames: same state, signed output
    v = pipe(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, scene_id=w.scene_seed)
    for fr in range(w.frames):
        v.step(fr)
    torch.cuda.synchronize()
    assert torch.equal(v.state.u, p.state.u) and torch.equal(v.state.hits, p.state.hits)
    assert (v.fine_sdf < -shell).sum().item() > 1000


def test_shell_gradient_and_batch(R):
    say("shell gradient / batch")
    from synth.scenes import Workload
    nc, nf, rays, frames = 32, 64, 8, 3
    s = icosphere(2, 0.28, (0.5, 0.5, 0.5))
    w = Workload("g", s, nc, nf, 0.5, 2.0, rays, frames)
    shell = 0.01
    p = pipe(s.vertices, s.faces, nc, nf, w.beta, w.d, rays, sign_policy="shell", shell=shell)
    for fr in range(frames):
        p.step(fr)
    ref = oracle.run_frames(s.vertices, s.faces, nc, nf, w.beta, w.d, rays, range(frames), sign_policy="shell",
                            shell=shell)
    st = ref["state"]
    at, ar = p.state.arg_tri.cpu().numpy(), p.state.arg_ray.cpu().numpy()
    agree = (at == st.arg_tri) & (ar == ((st.arg_frame << 8) | np.maximum(st.arg_ray, 0))) & (st.arg_amb == 0)
    fine = p.fine_sdf.cpu().numpy().astype(np.float64)
    gf = np.where(agree & (p.mask.cpu().numpy() == 1), 2 * fine, 0.0)
    gv = torch.zeros(s.nv * 3, dtype=torch.float32, device="cuda")
    R.rtsdf_trace_backward(p.scene, p.fine, p.state, p.fine_sdf, torch.from_numpy(gf.astype(np.float32)).cuda(),
                           0, 0, gv)
    got = gv.cpu().numpy().reshape(-1, 3).astype(np.float64)
    want = oracle.Scene(s.vertices, s.faces).fine_grad(nf, np.zeros(3, np.float32), np.float32(1 / nf), 0, 0, st, gf,
                                                       sign_policy="shell")
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("shell grad rel L2", rel)
    assert rel <= 1e-4
    # a batched scene with the shell policy equals its single-scene run bit for bit
    B = R.Batch([dict(vertices=torch.from_numpy(s.vertices).cuda(), faces=torch.from_numpy(s.faces).cuda(),
                      coarse_n=nc, fine_n=nf, beta=w.beta, d=w.d, rays=rays, scene_id=0, sign_policy="shell",
                      shell=shell)], seed=0)
    for fr in range(frames):
        B.step(fr)
    t = B.tensors(0)
    torch.cuda.synchronize()
    assert torch.equal(t["fine_sdf"], p.fine_sdf) and torch.equal(t["u"], p.state.u)
    B.close()
