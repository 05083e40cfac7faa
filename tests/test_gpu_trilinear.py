"""GPU parity of trilinear coarse sampling (the smoother reading of c for the
selection test c <= d and for c_t of Eq. (1), Sec. 2.2), through the C ABI.

Bit-exact against the oracle: the interpolated field at the fine texel centres
(every float operation is rounded once in a fixed order on both sides), the
field selection's mask / queue / count, including a queue overflow.  The
pipeline in trilinear mode matches the oracle's trilinear pipeline as the
point-sampled one does (traced values within 1e-5 x extent, unselected texels
bit-exact).  A captured frame graph in trilinear mode, or with a jump-flooding
pass schedule other than n/2, ..., 1, replays the eager update bitwise.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth.scenes import room_scene, tiny_scene, workload

pytestmark = pytest.mark.gpu

LO = np.zeros(3, np.float32)


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


def oracle_coarse(mesh, nc):
    h = np.float32(1.0 / nc)
    d2, c = oracle.coarse(nc, oracle.jfa(nc, oracle.voxelize(mesh.vertices, mesh.faces, LO, h, nc)), h,
                          np.float32(0.5) * h)
    return d2, c


def gpu_trilinear(R, c, nc, nf):
    out = torch.full((nf ** 3,), -3.0, dtype=torch.float32, device="cuda")
    R.rtsdf_coarse_trilinear(R.Grid.make(nc), cu(c), R.Grid.make(nf), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_select_field(R, field, n, d, cap=None):
    mask = torch.empty(n ** 3, dtype=torch.uint8, device="cuda")
    queue = torch.full((n ** 3 if cap is None else cap,), -7, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = torch.empty(R.rtsdf_select_workspace_size(n), dtype=torch.uint8, device="cuda")
    R.rtsdf_select_field(R.Grid.make(n), cu(field), float(d), mask, queue, count, ws)
    torch.cuda.synchronize()
    return mask.cpu().numpy(), queue.cpu().numpy(), int(count.item())


@pytest.mark.parametrize("case,nc,nf", [("tiny", 16, 16), ("tiny", 32, 64), ("tiny", 8, 128), ("room", 128, 256),
                                        ("room", 64, 512)])
def test_coarse_trilinear_bit_exact(R, case, nc, nf):
    say("coarse trilinear", case, nc, nf)
    mesh = tiny_scene() if case == "tiny" else room_scene(1)
    _, c = oracle_coarse(mesh, nc)
    want = oracle.coarse_trilinear(nc, c, nf)
    got = gpu_trilinear(R, c, nc, nf)
    assert np.array_equal(got.view(np.int32), want.view(np.int32))


def test_coarse_trilinear_random_and_infinite(R):
    say("coarse trilinear random / inf")
    rng = np.random.default_rng(9)
    nc, nf = 16, 64
    c = rng.uniform(-0.2, 0.7, nc ** 3).astype(np.float32)
    c[rng.choice(nc ** 3, 5, replace=False)] = np.inf
    got = gpu_trilinear(R, c, nc, nf)
    assert np.array_equal(got.view(np.int32), oracle.coarse_trilinear(nc, c, nf).view(np.int32))
    empty = gpu_trilinear(R, np.full(8 ** 3, np.inf, np.float32), 8, 32)
    assert np.all(np.isposinf(empty))


@pytest.mark.parametrize("case,nc,nf,dv", [("tiny", 32, 64, 2.0), ("tiny", 32, 64, 0.0), ("tiny", 16, 128, 1.5),
                                           ("room", 128, 256, 3.0), ("room", 64, 512, 1.0)])
def test_select_field_bit_exact(R, case, nc, nf, dv):
    say("select field", case, nc, nf, dv)
    mesh = tiny_scene() if case == "tiny" else room_scene(1)
    _, c = oracle_coarse(mesh, nc)
    field = oracle.coarse_trilinear(nc, c, nf)
    d = np.float32(dv) * np.float32(1.0 / nc)
    want_mask, want_q = oracle.select_field(nf, field, d)
    mask, queue, count = gpu_select_field(R, field, nf, d)
    assert count == len(want_q) and count > 0
    assert np.array_equal(mask, want_mask)
    assert np.array_equal(queue[:count], want_q)
    assert np.all(queue[count:] == -7)


def test_select_field_edges(R):
    say("select field edges")
    n = 32
    rng = np.random.default_rng(2)
    f = rng.uniform(-1, 1, n ** 3).astype(np.float32)
    f[::7] = np.nan  # NaN never selects
    for d in (-np.inf, -0.5, 0.0, 0.999, np.inf):
        want_mask, want_q = oracle.select_field(n, f, np.float32(d))
        mask, queue, count = gpu_select_field(R, f, n, d)
        assert count == len(want_q) and np.array_equal(mask, want_mask) and np.array_equal(queue[:count], want_q)
    _, want_q = oracle.select_field(n, f, np.float32(0.0))
    cap = 1001
    _, queue, count = gpu_select_field(R, f, n, 0.0, cap=cap)
    assert R.rtsdf_sync_status() & R.ERR_QUEUE_FULL
    assert count == len(want_q) and np.array_equal(queue, want_q[:cap])
    # smallest grid: 4^3
    f4 = rng.uniform(-1, 1, 64).astype(np.float32)
    want_mask, want_q = oracle.select_field(4, f4, np.float32(0.1))
    mask, queue, count = gpu_select_field(R, f4, 4, 0.1)
    assert np.array_equal(mask, want_mask) and np.array_equal(queue[:count], want_q)


def pipe(w, **kw):
    from paper_2210_04449_amd.pipeline import Pipeline
    return Pipeline(cu(w.mesh.vertices), cu(w.mesh.faces), w.nc, w.nf, w.beta, w.d, w.rays, seed=0,
                    scene_id=w.scene_seed, alpha=kw.get("alpha", w.alpha), sampling=kw.get("sampling", "point"),
                    jfa_variant=kw.get("jfa_variant", "jfa"))


def test_trilinear_pipeline_tiny_all_texels(R):
    say("trilinear pipeline tiny")
    from test_gpu_parity import compare_trace
    w = workload("tiny")
    p = pipe(w, sampling="trilinear")
    for fr in range(w.frames):
        p.step(fr)
    torch.cuda.synchronize()
    ref = oracle.run_frames(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, range(w.frames),
                            seed=0, scene=w.scene_seed, sampling="trilinear")
    assert np.array_equal(p.fine_c.cpu().numpy().view(np.int32), ref["coarse_fine"].view(np.int32))
    assert np.array_equal(p.queue[: p.selected()].cpu().numpy(), ref["queue"])
    stats = compare_trace(p, ref)
    print(stats)
    # the interpolated field selects a different band than point sampling
    point = oracle.run_frames(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, range(0), seed=0,
                              scene=w.scene_seed)
    assert not np.array_equal(point["mask"], ref["mask"])


def test_trilinear_pipeline_room_sampled(R):
    say("trilinear pipeline room sampled")
    from test_gpu_parity import compare_trace
    w = workload("room")
    p = pipe(w, sampling="trilinear")
    for fr in range(2):
        p.step(fr)
    torch.cuda.synchronize()
    sel = np.nonzero(p.mask.cpu().numpy())[0]
    rng = np.random.default_rng(4)
    unsel = np.nonzero(p.mask.cpu().numpy() == 0)[0]
    sample = np.sort(np.concatenate([rng.choice(sel, 5000, replace=False),
                                     rng.choice(unsel, 1000, replace=False)])).astype(np.int32)
    ref = oracle.run_frames(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, range(2), seed=0,
                            scene=w.scene_seed, texels=sample, sampling="trilinear")
    print(compare_trace(p, ref, sample=sample))


def same_state(a, b):
    return (torch.equal(a.fine_sdf, b.fine_sdf) and torch.equal(a.state.u, b.state.u)
            and torch.equal(a.state.hits, b.state.hits) and torch.equal(a.state.arg_tri, b.state.arg_tri)
            and torch.equal(a.state.arg_ray, b.state.arg_ray) and torch.equal(a.mask, b.mask))


@pytest.mark.parametrize("opts", [dict(sampling="trilinear"), dict(jfa_variant="jfa+2"),
                                  dict(sampling="trilinear", jfa_variant="1+jfa")])
def test_graph_options_replay_eager(R, opts):
    say("graph options", opts)
    w = workload("tiny")
    eager, cap = pipe(w, **opts), pipe(w, **opts)
    g = cap.make_graph(first_frame=0)
    for f in range(4):
        eager.step(f)
        g.launch()
        torch.cuda.synchronize()
        assert same_state(eager, cap), (opts, f)
        assert torch.equal(eager.seeds, cap.seeds) and torch.equal(eager.dist2, cap.dist2)
    g.close()
    # the schedule really ran: it is the oracle's for that schedule
    if "jfa_variant" in opts:
        import paper_2210_04449_amd.rtsdf as RR
        s0 = oracle.voxelize(w.mesh.vertices, w.mesh.faces, LO, np.float32(1.0 / w.nc), w.nc)
        want = oracle.jfa_steps(w.nc, s0, RR.jfa_schedule(w.nc, opts["jfa_variant"]))
        assert np.array_equal(cap.seeds.cpu().numpy(), want)
