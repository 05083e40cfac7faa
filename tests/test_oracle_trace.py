"""Pins of the oracle's ray tracing and temporal accumulation (paper Sec. 2.2,
Eq. (1)) and of its vertex gradient.

* closest hits: analytic ray/plane distances, the circumsphere/insphere
  bracket of a tessellated sphere, and the hierarchy against a plain loop over
  all triangles;
* traced distances: never below the exact point-to-mesh distance (computed
  here with a separate closest-point-on-triangle routine), converging to it as
  the ray count grows, and distributed as the closed form for a half-space;
* Eq. (1) and the sign rule: hand-computed cases in tests/golden/eq1_cases.json
  and the inside/outside behaviour the paper describes;
* gradient: float64 central finite differences.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from synth.scenes import ground_quad, icosphere, tiny_scene

LO = np.zeros(3, np.float32)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eq1_cases.json")


def _num(x):
    return math.inf if x == "inf" else float(x)


def point_mesh_distance(P, V, F, chunk=1024):
    """Exact distance from points to a triangle mesh (closest point on each
    triangle by projection onto the plane, else onto the nearest edge)."""
    T = V.astype(np.float64)[F]
    A, B, C = T[:, 0], T[:, 1], T[:, 2]
    n = np.cross(B - A, C - A)
    nn = np.einsum("ij,ij->i", n, n)
    out = np.empty(len(P))

    def seg(p, a, b):
        ab = b - a
        t = np.clip(np.einsum("ptk,tk->pt", p[:, None, :] - a[None], ab) / np.einsum("tk,tk->t", ab, ab), 0, 1)
        q = a[None] + t[..., None] * ab[None]
        return np.linalg.norm(p[:, None, :] - q, axis=-1)

    for s in range(0, len(P), chunk):
        p = P[s:s + chunk].astype(np.float64)
        d = np.minimum(np.minimum(seg(p, A, B), seg(p, B, C)), seg(p, C, A))
        # projection inside the triangle?
        w = p[:, None, :] - A[None]
        dist_plane = np.einsum("ptk,tk->pt", w, n) / np.sqrt(nn)
        proj = p[:, None, :] - dist_plane[..., None] * (n / np.sqrt(nn)[:, None])[None]
        inside = np.ones(d.shape, bool)
        for a, b in ((A, B), (B, C), (C, A)):
            inside &= np.einsum("ptk,tk->pt", np.cross(b - a, proj - a[None]), n) >= 0
        d = np.where(inside, np.abs(dist_plane), d)
        out[s:s + chunk] = d.min(1)
    return out


def test_ray_plane_analytic():
    q = ground_quad(0.15)
    sc = oracle.Scene(q.vertices, q.faces, use_bvh=False)
    rng = np.random.default_rng(1)
    o = np.column_stack([rng.uniform(0.2, 0.8, 4000), rng.uniform(0.16, 0.9, 4000), rng.uniform(0.2, 0.8, 4000)])
    d = rng.normal(size=(4000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t, tri, front, amb = sc.closest_hits(o, d)
    y0 = float(np.float32(0.15))
    tp = (y0 - o[:, 1]) / d[:, 1]
    hitp = o + tp[:, None] * d
    inside = (d[:, 1] < 0) & (hitp[:, 0] > 0) & (hitp[:, 0] < 1) & (hitp[:, 2] > 0) & (hitp[:, 2] < 1)
    assert np.all(tri[~inside] == -1)
    assert np.allclose(t[inside], tp[inside], rtol=1e-12, atol=1e-14)
    assert np.all(front[inside] == 1)  # the quad faces +y, rays come from above
    # from below, the same quad is hit on its back face
    t2, tri2, front2, _ = sc.closest_hits(o * [1, 0, 1] + [0, 0.1, 0], d * [1, -1, 1])
    assert np.all(front2[tri2 >= 0] == 0)


def test_sphere_bracket():
    R = 0.3
    s = icosphere(2, R, (0.5, 0.5, 0.5))
    v = s.vertices.astype(np.float64) - 0.5
    tri = v[s.faces]
    nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    r_in = np.min(np.abs(np.einsum("ij,ij->i", tri.mean(1), nrm)))
    r_out = np.max(np.linalg.norm(v, axis=1))
    sc = oracle.Scene(s.vertices, s.faces)
    rng = np.random.default_rng(2)
    o = rng.normal(size=(5000, 3))
    o = 0.5 + o / np.linalg.norm(o, axis=1, keepdims=True) * 0.45
    target = 0.5 + rng.uniform(-0.35, 0.35, size=(5000, 3))
    d = target - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t, trid, front, _ = sc.closest_hits(o, d)

    def entry(rad):
        oc = o - 0.5
        b = np.einsum("ij,ij->i", oc, d)
        c = np.einsum("ij,ij->i", oc, oc) - rad * rad
        disc = b * b - c
        return np.where(disc >= 0, -b - np.sqrt(np.maximum(disc, 0)), np.nan)

    t_out, t_in = entry(r_out), entry(r_in)
    hits_in = ~np.isnan(t_in)
    assert np.all(trid[hits_in] >= 0)
    assert np.all(t[hits_in] >= t_out[hits_in] - 1e-12)
    assert np.all(t[hits_in] <= t_in[hits_in] + 1e-12)
    assert np.all(trid[np.isnan(t_out)] == -1)
    assert np.all(front[trid >= 0] == 1)


def test_hierarchy_equals_plain_loop(tiny):
    m = tiny.mesh
    a = oracle.Scene(m.vertices, m.faces, use_bvh=True)
    b = oracle.Scene(m.vertices, m.faces, use_bvh=False)
    rng = np.random.default_rng(3)
    o = rng.uniform(0, 1, size=(20000, 3))
    d = rng.normal(size=(20000, 3))
    ra, rb = a.closest_hits(o, d), b.closest_hits(o, d)
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)


@pytest.fixture(scope="module")
def tiny_run():
    w = tiny_scene()
    return oracle.run_frames(w.vertices, w.faces, 32, 64, np.float32(0.5 / 32), np.float32(2 / 32), 4, range(8)), w


def test_traced_never_below_exact_distance(tiny_run):
    r, m = tiny_run
    st = r["state"]
    sel = np.nonzero(r["mask"])[0]
    nf = 64
    P = (np.stack([sel % nf, (sel // nf) % nf, sel // nf ** 2], 1) + 0.5) / nf
    exact = point_mesh_distance(P, m.vertices, m.faces)
    u = st.u[sel]
    fin = np.isfinite(u)
    assert fin.mean() > 0.99
    assert np.all(u[fin] >= exact[fin] * (1 - 1e-9) - 1e-12)
    # |f| equals the state where finite; otherwise the coarse value
    assert np.allclose(np.abs(st.fine[sel][fin]), u[fin])


def test_converges_with_more_rays():
    m = tiny_scene()
    nf = 32
    sub = np.arange(0, nf ** 3, 7)
    excess = []
    for frames in (1, 4, 16):
        r = oracle.run_frames(m.vertices, m.faces, 16, nf, np.float32(0.5 / 16), np.float32(2 / 16), 4,
                              range(frames), texels=sub)
        sel = sub[r["mask"][sub] == 1]
        P = (np.stack([sel % nf, (sel // nf) % nf, sel // nf ** 2], 1) + 0.5) / nf
        exact = point_mesh_distance(P, m.vertices, m.faces)
        u = r["state"].u[sel]
        excess.append(np.mean(np.where(np.isfinite(u), u / exact - 1, 1.0)))
    assert excess[0] > excess[1] > excess[2]
    assert excess[2] < 0.1


def test_half_space_distribution(tiny_run):
    # Texels above the ground quad, far from the sphere: the minimum over n
    # rays of the distance to a plane at distance D satisfies
    #   P(r <= D (1 + delta)) = 1 - (1 - delta / (2 (1 + delta)))^n
    # (the y component of a uniform direction is uniform on [-1, 1]).
    r, m = tiny_run
    st = r["state"]
    nf, n_rays = 64, 32
    y0 = float(np.float32(0.15))
    dmax = 1.0
    sel = np.nonzero(r["mask"])[0]
    P = (np.stack([sel % nf, (sel // nf) % nf, sel // nf ** 2], 1) + 0.5) / nf
    D = P[:, 1] - y0
    rad = D * math.sqrt((1 + dmax) ** 2 - 1)
    ok = (D > 0) & (P[:, 0] - rad > 0) & (P[:, 0] + rad < 1) & (P[:, 2] - rad > 0) & (P[:, 2] + rad < 1)
    sph = icosphere(2, 0.3, (0.5, 0.5, 0.5))
    ds = point_mesh_distance(P[ok], sph.vertices, sph.faces)
    idx = np.nonzero(ok)[0][ds > D[ok] * (1 + dmax)]
    ratio = st.u[sel[idx]] / D[idx]
    N = len(ratio)
    assert N > 2000
    assert np.all(ratio >= 1 - 1e-9)
    for delta in (0.005, 0.02, 0.05, 0.1, 0.3, 1.0):
        F = 1 - (1 - delta / (2 * (1 + delta))) ** n_rays
        k = np.sum(ratio <= 1 + delta)
        assert abs(k - N * F) <= 5 * math.sqrt(N * F * (1 - F)) + 1, (delta, k, N * F)


def test_sign_inside_outside(tiny_run):
    r, m = tiny_run
    st = r["state"]
    nf = 64
    sel = np.nonzero(r["mask"])[0]
    P = (np.stack([sel % nf, (sel // nf) % nf, sel // nf ** 2], 1) + 0.5) / nf
    rr = np.linalg.norm(P - 0.5, axis=1)
    inside = rr < 0.27  # strictly inside the icosphere (inradius > 0.28)
    assert inside.sum() > 100
    assert np.all(st.nback[sel[inside]] > st.nfront[sel[inside]])
    assert np.all(st.fine[sel[inside]] < 0)
    # above the ground and outside the sphere: front faces dominate or tie
    above = (P[:, 1] > 0.16) & (rr > 0.31)
    assert np.all(st.nfront[sel[above]] >= st.nback[sel[above]])
    assert np.all(st.fine[sel[above]] > 0)
    # below the one-sided ground quad only its back face is visible: negative
    below = P[:, 1] < 0.149
    assert below.sum() > 100
    assert np.all(st.fine[sel[below]] < 0)


def test_unselected_take_coarse_value(tiny_run):
    r, _ = tiny_run
    st = r["state"]
    nf, nc = 64, 32
    j = np.nonzero(r["mask"] == 0)[0]
    x, y, z = j % nf, (j // nf) % nf, j // nf ** 2
    c = r["coarse"][x // 2 + nc * (y // 2 + nc * (z // 2))]
    assert np.array_equal(st.fine[j], c.astype(np.float64))
    assert np.all(np.isinf(st.u[j])) and np.all(st.arg_tri[j] == -1)


def test_eq1_golden():
    g = json.load(open(GOLDEN))
    for case in g["eq1"]:
        u, src = oracle.eq1(_num(case["alpha"]), _num(case["u_prev"]), _num(case["c"]), _num(case["r_t"]))
        assert u == _num(case["u_t"]), case
        assert src == case["source"], case
    for case in g["sign"]:
        assert oracle.fine_value(_num(case["u"]), _num(case["c"]), case["nfront"], case["nback"]) == _num(case["f"])


def test_argmin_record_reproduces_value(tiny_run):
    # The stored (frame, ray, triangle) regenerates the ray whose distance is u.
    r, m = tiny_run
    st = r["state"]
    nf = 64
    sc = oracle.Scene(m.vertices, m.faces)
    sel = np.nonzero((r["mask"] == 1) & (st.arg_tri >= 0))[0][::97]
    o = np.array([oracle.texel_origin(nf, LO, np.float32(1 / nf), j) for j in sel], np.float64)
    d = np.array([oracle.direction(0, j, st.arg_frame[j], st.arg_ray[j])[0] for j in sel], np.float64)
    t, tri, _, _ = sc.closest_hits(o, d)
    assert np.array_equal(tri, st.arg_tri[sel])
    assert np.allclose(t * np.linalg.norm(d, axis=1), st.u[sel], rtol=0, atol=0)


def test_gradient_matches_central_differences():
    # Loss L = sum over traced texels of (f - s)^2 with s the analytic sphere
    # SDF; float64 central differences (h = 1e-4) over texels whose discrete
    # state (argmin frame/ray/triangle and sign) is the same at +h and -h.
    nc, nf, rays, frames = 16, 32, 8, 2
    s = icosphere(1, 0.25, (0.5, 0.5, 0.5))
    v64 = s.vertices.astype(np.float64)
    f = s.faces
    base = oracle.run_frames(s.vertices, f, nc, nf, np.float32(0.5 / nc), np.float32(2 / nc), rays, range(frames))
    c, mask = base["coarse"], base["mask"]
    hf = np.float32(1 / nf)
    sel = np.nonzero(mask)[0]
    P = (np.stack([sel % nf, (sel // nf) % nf, sel // nf ** 2], 1) + 0.5) / nf
    target = np.zeros(nf ** 3)
    target[sel] = np.linalg.norm(P - 0.5, axis=1) - 0.25

    def run(v):
        sc = oracle.Scene(v, f)
        st = oracle.TraceState(nf)
        for fr in range(frames):
            sc.trace_frame(nc, c, nf, LO, hf, mask, rays, fr, 0, 0, 1.0, st)
        return sc, st

    sc0, st0 = run(v64)
    rng = np.random.default_rng(5)
    h = 1e-4
    checked = 0
    for _ in range(12):
        vi, ax = int(rng.integers(0, len(v64))), int(rng.integers(0, 3))
        vp, vm = v64.copy(), v64.copy()
        vp[vi, ax] += h
        vm[vi, ax] -= h
        _, sp = run(vp)
        _, sm = run(vm)
        stable = (st0.arg_tri >= 0) & (mask == 1)
        for other in (sp, sm):
            stable &= (other.arg_tri == st0.arg_tri) & (other.arg_frame == st0.arg_frame)
            stable &= (other.arg_ray == st0.arg_ray) & (np.sign(other.fine) == np.sign(st0.fine))
        Lp = np.sum((sp.fine[stable] - target[stable]) ** 2)
        Lm = np.sum((sm.fine[stable] - target[stable]) ** 2)
        fd = (Lp - Lm) / (2 * h)
        gf = np.where(stable, 2 * (st0.fine - target), 0.0)
        an = sc0.fine_grad(nf, LO, hf, 0, 0, st0, gf)[vi, ax]
        if abs(fd) < 1e-9 and abs(an) < 1e-9:
            continue
        assert abs(fd - an) <= 1e-5 * max(abs(fd), abs(an)) + 1e-9, (vi, ax, fd, an)
        checked += 1
    assert checked >= 6


def test_shell_sign_policy(tiny_run):
    """Shell policy: the output is the unsigned traced distance minus the shell half-thickness, so the one-sided
    ground quad no longer makes the region below it negative; the state and the hits are the vote run's."""
    r, m = tiny_run
    shell = 1.0 / 128
    rs = oracle.run_frames(m.vertices, m.faces, 32, 64, np.float32(0.5 / 32), np.float32(2 / 32), 4, range(8),
                           sign_policy="shell", shell=shell)
    a, b = r["state"], rs["state"]
    assert np.array_equal(a.u, b.u) and np.array_equal(a.nfront, b.nfront) and np.array_equal(a.arg_tri, b.arg_tri)
    traced = np.isfinite(a.u)
    assert np.array_equal(b.fine[traced], np.abs(a.fine[traced]) - shell)
    assert np.array_equal(b.fine[~traced], a.fine[~traced])
    nf = 64
    sel = np.nonzero(r["mask"].astype(bool) & traced)[0]
    P = (np.stack([sel % nf, (sel // nf) % nf, sel // nf ** 2], 1) + 0.5) / nf
    below = P[:, 1] < 0.149
    assert np.all(a.fine[sel[below]] < 0) and np.all(b.fine[sel[below]] > -shell)
    assert oracle.fine_value(0.25, 0.5, 1, 3, "shell", 0.0625) == 0.1875
    assert oracle.fine_value(np.inf, 0.5, 1, 3, "shell", 0.0625) == 0.5


def test_ambiguity_second_surface_at_the_same_distance():
    """A ray whose closest hit has another triangle at the same distance (a duplicated quad) is ambiguous,
    wherever it crosses; with the duplicate removed the same rays are not (away from the diagonal edge)."""
    q = ground_quad(0.15)
    dup = np.concatenate([q.faces, q.faces[:, ::-1]]).astype(np.int32)  # same plane, both windings
    rng = np.random.default_rng(11)
    o = np.column_stack([rng.uniform(0.3, 0.7, 3000), np.full(3000, 0.5), rng.uniform(0.3, 0.7, 3000)])
    d = np.column_stack([rng.uniform(-0.2, 0.2, 3000), -np.ones(3000), rng.uniform(-0.2, 0.2, 3000)])
    hit = np.abs(np.abs(o[:, 0] + (0.35 / 1) * d[:, 0] - (o[:, 2] + 0.35 * d[:, 2])))  # distance to the diagonal
    _, tri1, _, amb1 = oracle.Scene(q.vertices, q.faces, use_bvh=False).closest_hits(o, d)
    _, tri2, _, amb2 = oracle.Scene(q.vertices, dup, use_bvh=False).closest_hits(o, d)
    assert np.all(tri1 >= 0) and np.all(tri2 >= 0)
    assert np.all(amb2 == 1)
    assert np.all(amb1[hit > 1e-3] == 0)


def test_ambiguity_interpenetrating_surfaces():
    """Two planes crossing along a line: rays hitting near the crossing line (within the tie margin of the
    other plane) are ambiguous, rays far from it are not."""
    y0 = 0.4
    a = np.array([[0, y0, 0], [1, y0, 0], [1, y0, 1], [0, y0, 1]], np.float32)  # horizontal
    b = np.array([[0.5, 0, 0], [0.5, 0, 1], [0.5, 1, 1], [0.5, 1, 0]], np.float32)  # vertical x = 0.5
    v = np.concatenate([a, b])
    f = np.array([[0, 2, 1], [0, 3, 2], [4, 6, 5], [4, 7, 6]], np.int32)
    sc = oracle.Scene(v, f, use_bvh=False)
    xs = np.array([0.5 + 1e-9, 0.5 + 1e-8, 0.45, 0.3])
    o = np.column_stack([xs - 0.3, np.full(4, y0 + 0.3), np.full(4, 0.37)])
    d = np.tile([0.3, -0.3, 0.0], (4, 1))  # crosses y0 at x = xs, lands just past the vertical plane or away
    t, tri, _, amb = sc.closest_hits(o, d)
    assert list(amb) == [1, 1, 0, 0], amb


def test_texel_flags_near_tied_rays_and_history():
    """The per-texel flag: set when two rays of a frame land within the tie margin, kept while the texel
    stays selected, reset when it is unselected; and on the tiny scene only a small fraction is flagged."""
    w = tiny_scene()
    nc, nf, rays = 32, 64, 4
    r = oracle.run_frames(w.vertices, w.faces, nc, nf, np.float32(0.5 / nc), np.float32(2 / nc), rays, range(4))
    st, mask = r["state"], r["mask"]
    sel = np.nonzero(mask)[0]
    assert np.all(st.texel_amb[mask == 0] == 0)
    assert np.all((st.texel_amb[sel] & 1) >= st.arg_amb[sel])  # an ambiguous argmin ray flags its texel
    frac = (st.texel_amb[sel] != 0).mean()
    assert 0 < frac < 0.02, frac
    # the flag is sticky over frames: a fresh state over frames 0..1 flags a subset of frames 0..3's
    r2 = oracle.run_frames(w.vertices, w.faces, nc, nf, np.float32(0.5 / nc), np.float32(2 / nc), rays, range(2))
    assert np.all((r2["state"].texel_amb[sel] & ~st.texel_amb[sel]) == 0)
    # a texel traced with two identical frames: every ray ties with the history -> flagged
    st3 = oracle.TraceState(nf)
    sc = r["scene"]
    t = sel[:200].astype(np.int32)
    lo, hf = np.zeros(3, np.float32), np.float32(1 / nf)
    sc.trace_frame(nc, r["coarse"], nf, lo, hf, mask, rays, 5, 0, 0, 1.0, st3, t)
    finite = np.isfinite(st3.u[t])
    sc.trace_frame(nc, r["coarse"], nf, lo, hf, mask, rays, 5, 0, 0, 1.0, st3, t)
    assert np.all((st3.texel_amb[t][finite] & 2) == 2)
