"""GPU parity of every stage against the CPU oracle, through the C ABI.

Bit-exact: voxel occupancy, jump-flooding seeds, D^2 and the coarse SDF, the
selection mask / queue / count, the ray directions, shadow visibility.
Within 1e-5 x scene extent (the unit cube): traced fine-SDF values against
the oracle's float64 distances, excluding texels whose argmin ray the oracle
flags as ambiguous for a float32 evaluation (those are counted).  Exact:
sign, front/back hit counts and the argmin record (frame, ray, triangle) of
every traced texel the oracle does not flag (a flagged texel had an
ambiguous ray or two candidate distances within float rounding).
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from synth.scenes import Mesh, ground_quad, icosphere, random_soup, room_scene, tiny_scene, workload

pytestmark = pytest.mark.gpu

LO = np.zeros(3, np.float32)
TOL = 1e-5  # x scene extent (1)


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    return R


def cu(a, dt=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dt is not None:
        t = t.to(dt)
    return t.cuda()


def gpu_coarse(R, mesh: Mesh, n: int, beta_vox: float = 0.5):
    g = R.Grid.make(n)
    v, f = cu(mesh.vertices), cu(mesh.faces)
    seeds0 = torch.empty(n ** 3, dtype=torch.int32, device="cuda")
    R.rtsdf_voxelize(v, f, g, seeds0)
    seeds = seeds0.clone()
    scratch = torch.empty_like(seeds)
    d2 = torch.empty_like(seeds)
    c = torch.empty(n ** 3, dtype=torch.float32, device="cuda")
    beta = np.float32(beta_vox) * np.float32(1.0 / n)
    R.rtsdf_jfa(g, seeds, scratch, float(beta), d2, c)
    torch.cuda.synchronize()
    return seeds0.cpu().numpy(), seeds.cpu().numpy(), d2.cpu().numpy(), c.cpu().numpy()


# ------------------------------------------------------------ voxelize ----

@pytest.mark.parametrize("case,n", [("tiny", 32), ("tiny", 64), ("room", 128), ("soup", 32), ("room", 256)])
def test_voxelize_bit_exact(R, case, n):
    say("voxelize", case, n)
    mesh = {"tiny": tiny_scene, "room": lambda: room_scene(1), "soup": lambda: random_soup(5, 3000)}[case]()
    want = oracle.voxelize(mesh.vertices, mesh.faces, LO, np.float32(1.0 / n), n)
    got, _, _, _ = gpu_coarse(R, mesh, n)
    assert np.array_equal(got, want), int((got != want).sum())
    assert R.rtsdf_sync_status() == 0


def test_voxelize_empty_and_errors(R):
    say("voxelize errors")
    n = 16
    g = R.Grid.make(n)
    seeds = torch.empty(n ** 3, dtype=torch.int32, device="cuda")
    v = cu(np.zeros((0, 3), np.float32))
    f = cu(np.zeros((0, 3), np.int32))
    R.rtsdf_voxelize(v, f, g, seeds)
    assert int((seeds >= 0).sum()) == 0
    # one face with an index out of range and one with a vertex far outside:
    # both are skipped and reported; the good triangle is still voxelized
    m = ground_quad(0.3)
    verts = np.concatenate([m.vertices, [[0.5, 5.0, 0.5]]]).astype(np.float32)
    faces = np.array([[0, 2, 1], [0, 1, 9], [0, 1, 4]], np.int32)
    R.rtsdf_voxelize(cu(verts), cu(faces), g, seeds)
    bits = R.rtsdf_sync_status()
    assert bits & R.ERR_FACE_INDEX and bits & R.ERR_VERTEX_RANGE
    want = oracle.voxelize(m.vertices, faces[:1], LO, np.float32(1 / n), n)
    assert np.array_equal(seeds.cpu().numpy(), want)
    assert R.rtsdf_sync_status() == 0  # cleared


# ----------------------------------------------------------------- jfa ----

@pytest.mark.parametrize("case,n", [("tiny", 8), ("tiny", 16), ("tiny", 32), ("soup", 64), ("room", 128),
                                    ("room", 256)])
def test_jfa_bit_exact(R, case, n):
    say("jfa", case, n)
    mesh = {"tiny": tiny_scene, "room": lambda: room_scene(1), "soup": lambda: random_soup(9, 400)}[case]()
    s0, s, d2, c = gpu_coarse(R, mesh, n)
    want_s = oracle.jfa(n, s0)
    beta = np.float32(0.5) * np.float32(1.0 / n)
    want_d2, want_c = oracle.coarse(n, want_s, np.float32(1.0 / n), beta)
    assert np.array_equal(s, want_s), int((s != want_s).sum())
    assert np.array_equal(d2, want_d2)
    assert np.array_equal(c.view(np.int32), want_c.view(np.int32))


@pytest.mark.parametrize("stage", [1, 2])
@pytest.mark.parametrize("case,n", [("tiny", 8), ("tiny", 32), ("room", 128), ("room", 256)])
def test_jfa_near_stagings_bit_exact(R, case, n, stage):
    """Both stagings of the step-2 and step-1 passes (seeds alone, or seed pairs) give the oracle's seeds, D^2
    and coarse SDF."""
    say("jfa near staging", stage, case, n)
    mesh = {"tiny": tiny_scene, "room": lambda: room_scene(1)}[case]()
    old = R.rtsdf_jfa_config(n, stage)
    try:
        s0, s, d2, c = gpu_coarse(R, mesh, n)
    finally:
        R.rtsdf_jfa_config(n, old)
    want_s = oracle.jfa(n, s0)
    beta = np.float32(0.5) * np.float32(1.0 / n)
    want_d2, want_c = oracle.coarse(n, want_s, np.float32(1.0 / n), beta)
    assert np.array_equal(s, want_s), int((s != want_s).sum())
    assert np.array_equal(d2, want_d2)
    assert np.array_equal(c.view(np.int32), want_c.view(np.int32))


@pytest.mark.parametrize("order", [1, 2, 3, 4])
@pytest.mark.parametrize("case,n,steps", [("tiny", 8, None), ("tiny", 16, None), ("tiny", 32, None),
                                          ("soup", 64, None), ("room", 128, None), ("room", 256, None),
                                          ("soup", 64, [8, 32, 16, 8, 4, 2, 1]),
                                          ("room", 128, [1, 16, 64, 32, 8, 4, 2, 1]),
                                          ("sparse", 16, None), ("sparse", 64, None), ("sparse", 128, None),
                                          ("sparse", 256, None), ("sparse", 128, [32, 64, 16, 4, 8, 2, 1])])
def test_jfa_far_orders_bit_exact(R, case, n, steps, order):
    """Every brick order of the far passes (slab order, coset order, coset order in brick pairs or 2 x 2 quads)
    gives the oracle's seeds, D^2 and coarse SDF, also for schedules whose first far pass reads the caller's
    linear seeds (step below n/2 first) or follows a near pass, and for a few isolated seeds (every voxel's seed
    arrives from far away, through every pass)."""
    say("jfa far order", order, case, n, steps)
    steps = steps or R.jfa_schedule(n, "jfa")
    g = R.Grid.make(n)
    if case == "sparse":
        s0 = np.full(n ** 3, -1, np.int32)
        own = np.random.default_rng(n).choice(n ** 3, size=7, replace=False)
        s0[own] = own
        seeds = cu(s0)
    else:
        mesh = {"tiny": tiny_scene, "room": lambda: room_scene(1), "soup": lambda: random_soup(9, 400)}[case]()
        seeds = torch.empty(n ** 3, dtype=torch.int32, device="cuda")
        R.rtsdf_voxelize(cu(mesh.vertices), cu(mesh.faces), g, seeds)
        s0 = seeds.cpu().numpy()
    scratch, d2 = torch.empty_like(seeds), torch.empty_like(seeds)
    c = torch.empty(n ** 3, dtype=torch.float32, device="cuda")
    old = R.rtsdf_jfa_config(n, far_order=order)
    try:
        R.rtsdf_jfa_steps(g, seeds, scratch, steps, float(np.float32(0.5) * np.float32(1.0 / n)), d2, c)
        torch.cuda.synchronize()
    finally:
        R.rtsdf_jfa_config(n, far_order=old)
    s, d2, c = seeds.cpu().numpy(), d2.cpu().numpy(), c.cpu().numpy()
    want_s = oracle.jfa_steps(n, s0, steps)
    beta = np.float32(0.5) * np.float32(1.0 / n)
    want_d2, want_c = oracle.coarse(n, want_s, np.float32(1.0 / n), beta)
    assert np.array_equal(s, want_s), int((s != want_s).sum())
    assert np.array_equal(d2, want_d2)
    assert np.array_equal(c.view(np.int32), want_c.view(np.int32))


@pytest.mark.parametrize("variant", ["jfa+1", "jfa+2", "1+jfa"])
@pytest.mark.parametrize("case,n", [("tiny", 8), ("tiny", 16), ("tiny", 32), ("soup", 64), ("room", 128),
                                    ("room", 256)])
def test_jfa_schedules_bit_exact(R, case, n, variant):
    """The error-reducing pass schedules (extra step-1/step-2 passes) against the oracle's passes."""
    say("jfa schedule", variant, case, n)
    mesh = {"tiny": tiny_scene, "room": lambda: room_scene(1), "soup": lambda: random_soup(9, 400)}[case]()
    g = R.Grid.make(n)
    seeds0 = torch.empty(n ** 3, dtype=torch.int32, device="cuda")
    R.rtsdf_voxelize(cu(mesh.vertices), cu(mesh.faces), g, seeds0)
    seeds = seeds0.clone()
    scratch, d2 = torch.empty_like(seeds), torch.empty_like(seeds)
    c = torch.empty(n ** 3, dtype=torch.float32, device="cuda")
    beta = np.float32(0.5) * np.float32(1.0 / n)
    steps = R.jfa_schedule(n, variant)
    R.rtsdf_jfa_steps(g, seeds, scratch, steps, float(beta), d2, c)
    torch.cuda.synchronize()
    want_s = oracle.jfa_steps(n, seeds0.cpu().numpy(), steps)
    want_d2, want_c = oracle.coarse(n, want_s, np.float32(1.0 / n), beta)
    got = seeds.cpu().numpy()
    assert np.array_equal(got, want_s), int((got != want_s).sum())
    assert np.array_equal(d2.cpu().numpy(), want_d2)
    assert np.array_equal(c.cpu().numpy().view(np.int32), want_c.view(np.int32))


def test_jfa_steps_rejects_bad_schedules(R):
    n = 16
    g = R.Grid.make(n)
    seeds = cu(np.full(n ** 3, -1, np.int32))
    scratch, d2 = torch.empty_like(seeds), torch.empty_like(seeds)
    c = torch.empty(n ** 3, dtype=torch.float32, device="cuda")
    for bad in ([], [8, 4, 2], [3, 1], [16, 1], [0, 1]):
        with pytest.raises(R.RtsdfError):
            R.rtsdf_jfa_steps(g, seeds, scratch, bad, 0.0, d2, c)


def test_jfa_single_seed_and_empty(R):
    for n, q in [(8, 0), (32, 32 ** 3 - 1), (64, 12345), (256, 256 ** 3 // 2 + 77)]:
        say("jfa single seed", n, q)
        g = R.Grid.make(n)
        s0 = np.full(n ** 3, -1, np.int32)
        s0[q] = q
        seeds = cu(s0)
        scratch, d2 = torch.empty_like(seeds), torch.empty_like(seeds)
        c = torch.empty(n ** 3, dtype=torch.float32, device="cuda")
        R.rtsdf_jfa(g, seeds, scratch, 0.0, d2, c)
        assert bool((seeds == q).all())
        want_d2, want_c = oracle.coarse(n, np.full(n ** 3, q, np.int32), np.float32(1 / n), 0.0)
        assert np.array_equal(d2.cpu().numpy(), want_d2)
        assert np.array_equal(c.cpu().numpy().view(np.int32), want_c.view(np.int32))
    say("jfa empty")
    n = 16
    seeds = cu(np.full(n ** 3, -1, np.int32))
    scratch, d2 = torch.empty_like(seeds), torch.empty_like(seeds)
    c = torch.empty(n ** 3, dtype=torch.float32, device="cuda")
    R.rtsdf_jfa(R.Grid.make(n), seeds, scratch, 0.01, d2, c)
    assert bool((seeds == -1).all()) and bool((d2 == 2 ** 31 - 1).all()) and bool(torch.isinf(c).all())


# -------------------------------------------------------------- select ----

def gpu_select(R, d2, nc, nf, beta, d, cap=None):
    cg, fg = R.Grid.make(nc), R.Grid.make(nf)
    mask = torch.empty(nf ** 3, dtype=torch.uint8, device="cuda")
    queue = torch.full((nf ** 3 if cap is None else cap,), -7, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = torch.empty(R.rtsdf_select_workspace_size(nc), dtype=torch.uint8, device="cuda")
    R.rtsdf_select(cg, cu(d2), fg, float(beta), float(d), mask, queue, count, ws)
    torch.cuda.synchronize()
    return mask.cpu().numpy(), queue.cpu().numpy(), int(count.item())


@pytest.mark.parametrize("case,nc,nf,dv", [("tiny", 32, 64, 2.0), ("tiny", 32, 128, 2.0), ("room", 128, 256, 3.0),
                                           ("tiny", 16, 16, 1.0), ("room", 64, 512, 0.0)])
def test_select_bit_exact(R, case, nc, nf, dv):
    say("select", case, nc, nf, dv)
    mesh = tiny_scene() if case == "tiny" else room_scene(1)
    h = np.float32(1.0 / nc)
    s0 = oracle.voxelize(mesh.vertices, mesh.faces, LO, h, nc)
    d2, _ = oracle.coarse(nc, oracle.jfa(nc, s0), h, np.float32(0.5) * h)
    beta, d = np.float32(0.5) * h, np.float32(dv) * h
    K = oracle.select_threshold(h, beta, d)
    want_mask, want_q = oracle.select(nc, d2, nf, K)
    mask, queue, count = gpu_select(R, d2, nc, nf, beta, d)
    assert count == len(want_q)
    assert np.array_equal(mask, want_mask)
    assert np.array_equal(queue[:count], want_q)


def test_select_overflow(R):
    say("select overflow")
    nc, nf = 32, 64
    mesh = tiny_scene()
    h = np.float32(1.0 / nc)
    d2, _ = oracle.coarse(nc, oracle.jfa(nc, oracle.voxelize(mesh.vertices, mesh.faces, LO, h, nc)), h,
                          np.float32(0.5) * h)
    beta, d = np.float32(0.5) * h, np.float32(2) * h
    _, want_q = oracle.select(nc, d2, nf, oracle.select_threshold(h, beta, d))
    cap = 1000
    _, queue, count = gpu_select(R, d2, nc, nf, beta, d, cap=cap)
    assert R.rtsdf_sync_status() & R.ERR_QUEUE_FULL
    assert count == len(want_q)
    assert np.array_equal(queue, want_q[:cap])


# ---------------------------------------------------------- directions ----

def test_directions_bit_exact(R):
    say("directions")
    rng = np.random.default_rng(0)
    n = 1 << 20
    texel = rng.integers(0, 2 ** 27, n).astype(np.int32)
    frame = rng.integers(0, 2 ** 23, n).astype(np.uint32)
    ray = rng.integers(0, 64, n).astype(np.int32)
    for seed, scene in [(0, 0), (12345678901, 7)]:
        out = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        R.rtsdf_directions(cu(texel), cu(frame.view(np.int32)), cu(ray), seed, scene, out)
        got = out.cpu().numpy()
        want = oracle.directions(texel, frame, ray, seed, scene)
        assert np.array_equal(got.view(np.int32), want.view(np.int32)), int((got != want).any(1).sum())


# --------------------------------------------------------- closest hit ----

@pytest.mark.parametrize("case", ["tiny", "room"])
def test_closest_hits(R, case):
    say("closest hits", case)
    mesh = tiny_scene() if case == "tiny" else room_scene(1)
    rng = np.random.default_rng(1)
    n = 200000
    o = rng.uniform(0.0, 1.0, (n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3)).astype(np.float32)
    sc = R.Scene(cu(mesh.vertices), cu(mesh.faces))
    t = torch.empty(n, dtype=torch.float32, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    fr = torch.empty(n, dtype=torch.int32, device="cuda")
    R.rtsdf_closest_hits(sc, cu(o), cu(d), t, tri, fr)
    t, tri, fr = t.cpu().numpy(), tri.cpu().numpy(), fr.cpu().numpy()
    ot, otri, ofr, amb = oracle.Scene(mesh.vertices, mesh.faces).closest_hits(o.astype(np.float64), d.astype(np.float64))
    ok = amb == 0
    assert ok.mean() > 0.99
    assert np.array_equal(tri[ok], otri[ok])
    hit = ok & (otri >= 0)
    assert np.all(np.abs(t[hit] - ot[hit]) * np.linalg.norm(d[hit], axis=1) <= TOL)
    assert np.array_equal(fr[hit], ofr[hit])
    info = sc.info()
    assert info.nt == mesh.nt and info.max_depth < 64
    sc.close()


# ----------------------------------------------------------- pipeline ----

def run_gpu(R, w, frames, seed=0, alpha=None):
    from paper_2210_04449_amd.pipeline import Pipeline
    p = Pipeline(cu(w.mesh.vertices), cu(w.mesh.faces), w.nc, w.nf, w.beta, w.d, w.rays, seed=seed,
                 scene_id=w.scene_seed, alpha=w.alpha if alpha is None else alpha)
    for fr in frames:
        p.step(fr)
    torch.cuda.synchronize()
    return p


def compare_trace(p, ref, sample=None, max_flagged=0.1, tol=TOL):
    """GPU trace state against the oracle's.

    The oracle's per-texel flags say what a float32 evaluation may legitimately get differently: bit 0 of
    ``texel_amb`` (some ray of the texel was ambiguous: its front/back counts and sign may differ), bit 1 (two
    candidate distances within float rounding: the argmin record may differ), and ``arg_amb`` (the argmin
    ray itself is ambiguous: its distance may differ beyond rounding).  Every selected texel must agree
    exactly in sign and hit counts unless bit 0 is set, in its argmin record (frame, ray, triangle) unless
    bit 1 or arg_amb is set, and in |f| within the tolerance unless arg_amb is set (and in f itself where
    the sign is exact).  At most `max_flagged` of the texels may be excluded from either exact check."""
    st = ref["state"]
    fine = p.fine_sdf.cpu().numpy()
    u = p.state.u.cpu().numpy()
    hits = p.state.hits.cpu().numpy().view(np.uint32)
    at = p.state.arg_tri.cpu().numpy()
    ar = p.state.arg_ray.cpu().numpy()
    mask = p.mask.cpu().numpy()
    assert np.array_equal(mask, ref["mask"])
    idx = np.nonzero(mask)[0] if sample is None else sample
    sel = idx[mask[idx] == 1]
    unsel = idx[mask[idx] == 0]
    assert np.array_equal(fine[unsel].astype(np.float64), st.fine[unsel])
    amb = st.arg_amb[sel] == 1
    good = sel[~amb]
    err = np.abs(np.abs(fine[good].astype(np.float64)) - np.abs(st.fine[good]))
    assert err.max(initial=0) <= tol, (err.max(), np.sum(err > tol))
    fin = np.isfinite(st.u[good])
    assert np.array_equal(np.isfinite(u[good]), fin)
    ray_flag = (st.texel_amb[sel] & 1) != 0
    arg_flag = ((st.texel_amb[sel] & 2) != 0) | amb
    assert ray_flag.mean() <= max_flagged and arg_flag.mean() <= max_flagged, (ray_flag.mean(), arg_flag.mean())
    ex_hits, ex_arg = sel[~ray_flag], sel[~arg_flag]
    ex_both = sel[~ray_flag & ~arg_flag]
    want_ar = np.where(st.arg_tri >= 0, (st.arg_frame << 8) | np.maximum(st.arg_ray, 0), -1)
    bad = {
        "sign": (ex_hits, np.sign(fine[ex_hits]) != np.sign(st.fine[ex_hits])),
        "front": (ex_hits, (hits[ex_hits] & 0xFFFF) != st.nfront[ex_hits]),
        "back": (ex_hits, (hits[ex_hits] >> 16) != st.nback[ex_hits]),
        "arg_tri": (ex_arg, at[ex_arg] != st.arg_tri[ex_arg]),
        "arg_ray": (ex_arg, ar[ex_arg] != want_ar[ex_arg]),
        "signed_value": (ex_both, np.abs(fine[ex_both].astype(np.float64) - st.fine[ex_both]) > tol),
    }
    for k, (ex, b) in bad.items():
        if b.any():
            i = ex[np.argmax(b)]
            raise AssertionError(f"{k}: {int(b.sum())} of {len(ex)} unflagged texels differ; first texel {i}: "
                                 f"gpu f {fine[i]} hits {hits[i] & 0xFFFF}/{hits[i] >> 16} arg {at[i]}/{ar[i]}; "
                                 f"oracle f {st.fine[i]} hits {st.nfront[i]}/{st.nback[i]} "
                                 f"arg {st.arg_tri[i]}/{st.arg_frame[i]}/{st.arg_ray[i]}")
    return dict(texels=len(sel), exact_hits=len(ex_hits), exact_arg=len(ex_arg), ray_flagged=int(ray_flag.sum()),
                tie_or_arg_flagged=int(arg_flag.sum()), ambiguous_argmin=int(amb.sum()),
                max_err=float(err.max(initial=0)))


def test_trace_tiny_all_texels(R):
    say("trace tiny all frames")
    w = workload("tiny")
    p = run_gpu(R, w, range(w.frames))
    ref = oracle.run_frames(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, range(w.frames),
                            seed=0, scene=w.scene_seed)
    stats = compare_trace(p, ref)
    print(stats)
    assert stats["texels"] > 50000


def test_trace_determinism_and_resume(R):
    say("trace determinism")
    w = workload("tiny")
    a = run_gpu(R, w, range(6))
    b = run_gpu(R, w, range(6))
    assert torch.equal(a.fine_sdf, b.fine_sdf) and torch.equal(a.state.hits, b.state.hits)
    # frames keyed by index: 0..2 then 3..5 on a copied state equals 0..5
    c = run_gpu(R, w, range(3))
    for fr in range(3, 6):
        c.step(fr)
    torch.cuda.synchronize()
    assert torch.equal(a.fine_sdf, c.fine_sdf) and torch.equal(a.state.u, c.state.u)


@pytest.mark.parametrize("case", ["tiny", "room"])
def test_trace_tunings_agree_bitwise(R, case):
    """The tracer's tuning (loop shape, refill threshold, LDS stack depth,
    direction sorting, workgroups per CU, tile size) changes speed only: every setting
    gives the default setting's state and output bit for bit."""
    w = workload(case)
    frames = range(3) if case == "tiny" else range(1)
    default = R.rtsdf_trace_config_get().as_dict()
    settings = [dict(loop=0), dict(loop=1), dict(loop=2), dict(loop=3, refill=16), dict(loop=1, stack_lds=24),
                dict(loop=2, stack_lds=16, bin_directions=0), dict(loop=2, blocks_per_cu=2),
                dict(tile_texels=16, blocks_per_cu=3), dict(tile_texels=32, blocks_per_cu=5, stack_lds=16),
                dict(blocks_per_cu=4, refill=16, tile_texels=16), dict(loop=4), dict(loop=4, refill=16, stack_lds=16),
                dict(loop=4, tile_texels=16, blocks_per_cu=3, bin_directions=0)]
    try:
        say("tunings", case, "default", default)
        ref = run_gpu(R, w, frames)
        for t in settings:
            say("tunings", case, t)
            R.rtsdf_trace_config(**{**default, **t})
            p = run_gpu(R, w, frames)
            assert R.rtsdf_sync_status() == 0
            for a, b in ((p.fine_sdf, ref.fine_sdf), (p.state.u, ref.state.u), (p.state.hits, ref.state.hits),
                         (p.state.arg_tri, ref.state.arg_tri), (p.state.arg_ray, ref.state.arg_ray)):
                assert torch.equal(a, b), t
            p.close()
            del p
            R.rtsdf_trace_config(**default)
    finally:
        R.rtsdf_trace_config(**default)


def test_two_tile_contexts_in_use(R):
    """Instrumented room traces: a wavefront starts its next tile while rays of the last one are still in
    flight (the two tile contexts), and with small tiles some rounds wait for every lane first (the next tile
    must wait for a context still holding rays of the tile before); the state equals the plain run's."""
    say("two tile contexts")
    w = workload("room")
    default = R.rtsdf_trace_config_get().as_dict()
    try:
        ref = run_gpu(R, w, range(1))
        for t in (dict(), dict(tile_texels=16)):
            R.rtsdf_trace_config(**{**default, **t, "stats": 1})
            p = run_gpu(R, w, range(1))
            ctr = p.trace_ws[8:88].view(torch.int64).cpu().tolist()
            tiles, early, drains = ctr[6] // 64, ctr[8] // 64, ctr[9] // 64
            print(t, "tiles", tiles, "started early", early, "drain rounds", drains)
            assert ctr[2] == int(p.count.item()) * w.rays  # every ray traced once
            assert 0.5 * tiles < early < tiles
            if t:
                assert drains > 0
            assert torch.equal(p.fine_sdf, ref.fine_sdf) and torch.equal(p.state.u, ref.state.u)
            assert torch.equal(p.state.hits, ref.state.hits) and torch.equal(p.state.arg_ray, ref.state.arg_ray)
            p.close()
            R.rtsdf_trace_config(**default)
        ref.close()
    finally:
        R.rtsdf_trace_config(**default)


def test_trace_room_sampled(R):
    say("trace room sampled, 8 frames")
    w = workload("room")
    frames = range(8)
    p = run_gpu(R, w, frames)
    mask = p.mask.cpu().numpy()
    rng = np.random.default_rng(3)
    sel = np.nonzero(mask)[0]
    sample = np.sort(rng.choice(sel, 6000, replace=False)).astype(np.int32)
    ref = oracle.run_frames(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, frames,
                            seed=0, scene=w.scene_seed, texels=sample)
    stats = compare_trace(p, ref, sample=sample)
    print(stats)


def test_trace_decay_alpha(R):
    say("trace alpha 0.75")
    w = workload("tiny")
    p = run_gpu(R, w, range(4), alpha=0.75)
    ref = oracle.run_frames(w.mesh.vertices, w.mesh.faces, w.nc, w.nf, w.beta, w.d, w.rays, range(4), seed=0,
                            scene=w.scene_seed, alpha=0.75)
    compare_trace(p, ref)


def test_trace_moving_scene_alpha(R):
    """Dynamic workload in small: a room whose seeded 20% subset of primitives
    moves every frame, refit per frame, alpha 0.9; the oracle rebuilds its
    hierarchy for each frame's mesh and carries the accumulation state."""
    say("trace moving scene alpha 0.9")
    from synth.scenes import DynamicScene
    from paper_2210_04449_amd.pipeline import Pipeline
    dyn = DynamicScene(7, n_prims=30, detail="low")
    nc, nf, rays, alpha = 32, 64, 4, 0.9
    m0 = dyn.mesh(0)
    beta, d = np.float32(0.5 / nc), np.float32(2.0 / nc)
    p = Pipeline(cu(m0.vertices), cu(m0.faces), nc, nf, float(beta), float(d), rays, scene_id=9, alpha=alpha)
    st = oracle.TraceState(nf)
    for f in range(5):
        m = dyn.mesh(f)
        p.set_vertices(cu(m.vertices))
        p.step(f)
        ref = oracle.run_frames(m.vertices, m.faces, nc, nf, beta, d, rays, [f], seed=0, scene=9, alpha=alpha,
                                state=st)
    torch.cuda.synchronize()
    stats = compare_trace(p, ref)
    print(stats)
    assert stats["texels"] > 10000


# ------------------------------------------------------------- refit ----

def test_refit_matches_moved_mesh(R):
    say("refit")
    mesh = room_scene(1, n_prims=40)
    sc = R.Scene(cu(mesh.vertices), cu(mesh.faces))
    rng = np.random.default_rng(4)
    moved = mesh.vertices + rng.normal(0, 0.01, mesh.vertices.shape).astype(np.float32)
    moved = np.clip(moved, 0, 1).astype(np.float32)
    sc.refit(cu(moved))
    n = 100000
    o = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3)).astype(np.float32)
    t = torch.empty(n, dtype=torch.float32, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    fr = torch.empty(n, dtype=torch.int32, device="cuda")
    R.rtsdf_closest_hits(sc, cu(o), cu(d), t, tri, fr)
    ot, otri, _, amb = oracle.Scene(moved, mesh.faces).closest_hits(o.astype(np.float64), d.astype(np.float64))
    ok = amb == 0
    assert np.array_equal(tri.cpu().numpy()[ok], otri[ok])


# ---------------------------------------------------------- gradient ----

def test_backward_matches_oracle_gradient(R):
    say("backward")
    nc, nf, rays, frames = 32, 64, 8, 3
    s = icosphere(2, 0.28, (0.5, 0.5, 0.5))
    from synth.scenes import Workload
    w = Workload("g", s, nc, nf, 0.5, 2.0, rays, frames)
    p = run_gpu(R, w, range(frames))
    ref = oracle.run_frames(s.vertices, s.faces, nc, nf, w.beta, w.d, rays, range(frames))
    st = ref["state"]
    fine = p.fine_sdf.cpu().numpy().astype(np.float64)
    j = np.arange(nf ** 3)
    P = (np.stack([j % nf, (j // nf) % nf, j // nf ** 2], 1) + 0.5) / nf
    target = np.linalg.norm(P - 0.5, axis=1) - 0.28
    at = p.state.arg_tri.cpu().numpy()
    ar = p.state.arg_ray.cpu().numpy()
    agree = (at == st.arg_tri) & (ar == ((st.arg_frame << 8) | np.maximum(st.arg_ray, 0))) & (st.arg_amb == 0)
    agree &= np.sign(fine) == np.sign(st.fine)
    gf = np.where(agree & (p.mask.cpu().numpy() == 1), 2 * (fine - target), 0.0)
    gv = torch.zeros(s.nv * 3, dtype=torch.float32, device="cuda")
    R.rtsdf_trace_backward(p.scene, p.fine, p.state, p.fine_sdf, cu(gf.astype(np.float32)), 0, 0, gv)
    got = gv.cpu().numpy().reshape(-1, 3).astype(np.float64)
    want = oracle.Scene(s.vertices, s.faces).fine_grad(nf, LO, np.float32(1 / nf), 0, 0, st, gf)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("grad rel L2", rel)
    assert rel <= 1e-4


# ------------------------------------------------------------ shadow ----

def test_shadow_bit_exact(R):
    say("shadow")
    w = workload("tiny")
    p = run_gpu(R, w, range(4))
    sdf = p.fine_sdf.cpu().numpy()
    rng = np.random.default_rng(6)
    pts = np.column_stack([rng.uniform(0, 1, 20000), np.full(20000, 0.16), rng.uniform(0, 1, 20000)]).astype(np.float32)
    light = np.array([0.3, 0.9, 0.2], np.float32)
    light /= np.linalg.norm(light)
    vis = torch.empty(len(pts), dtype=torch.float32, device="cuda")
    h = 1.0 / w.nf
    R.rtsdf_shadow(p.fine, p.fine_sdf, cu(pts), light, 8.0, h, 96, 2 * h, 2.0, vis)
    got = vis.cpu().numpy()
    want = oracle.shadow(w.nf, LO, np.float32(h), sdf, pts, light, 8.0, h, 96, 2 * h, 2.0)
    assert np.array_equal(got.view(np.int32), want.view(np.int32)), int((got != want).sum())
    assert (got == 0).mean() > 0.05 and (got == 1).mean() > 0.05  # umbra and lit points both present


@pytest.mark.parametrize("penumbra,jittered", [(0, True), (1, False), (1, True)])
def test_shadow_triangulated_and_jittered_bit_exact(R, penumbra, jittered):
    say("shadow ex", penumbra, jittered)
    w = workload("tiny")
    p = run_gpu(R, w, range(4))
    sdf = p.fine_sdf.cpu().numpy()
    rng = np.random.default_rng(7)
    n = 30001  # ragged against the 256-lane workgroups
    pts = np.column_stack([rng.uniform(0, 1, n), np.full(n, 0.16), rng.uniform(0, 1, n)]).astype(np.float32)
    pts[:5] = [[-0.5, 0.2, 0.5], [0.5, 1.5, 0.5], [0.5, 0.16, 0.5], [0.0, 0.16, 0.0], [0.999, 0.16, 0.999]]
    light = np.array([0.3, 0.9, 0.2], np.float32)
    light /= np.linalg.norm(light)
    jit = rng.uniform(0, 1, n).astype(np.float32) if jittered else None
    h = 1.0 / w.nf
    vis = torch.empty(n, dtype=torch.float32, device="cuda")
    R.rtsdf_shadow_ex(p.fine, p.fine_sdf, cu(pts), light, 8.0, h, 96, 2 * h, 2.0, vis, penumbra=penumbra,
                      jitter=None if jit is None else cu(jit), jitter_scale=2 * h)
    got = vis.cpu().numpy()
    want = oracle.shadow(w.nf, LO, np.float32(h), sdf, pts, light, 8.0, h, 96, 2 * h, 2.0, penumbra=penumbra,
                         jitter=jit, jitter_scale=2 * h)
    assert np.array_equal(got.view(np.int32), want.view(np.int32)), int((got != want).sum())
    assert (got == 0).mean() > 0.05 and (got == 1).mean() > 0.01
    if penumbra == 0 and not jittered:
        return
    # the options change the penumbra, not the umbra test
    base = oracle.shadow(w.nf, LO, np.float32(h), sdf, pts, light, 8.0, h, 96, 2 * h, 2.0)
    assert not np.array_equal(base, got)
