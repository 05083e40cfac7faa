"""Pins of the oracle's soft-shadow march (Sec. 2.3) by closed forms.

The march visits t_0, t_0 + step, ... with step = max(min(s, max_step), eps);
on fields where that sequence is known in closed form, the visibility is too:

* a constant field S: every sample is S, the samples are evenly spaced, the cone
  term k S / t is smallest at the last sample, and the triangulated term (two
  equal spheres a step D apart meet at y = D / 2 behind the current point, at
  radius sqrt(S^2 - D^2 / 4)) is k sqrt(S^2 - D^2/4) / (t - D/2);
* a linear field s = y (distance to the plane y = 0) with the light rising at
  angle theta and a step capped below every sample: t_i = t_0 + i m,
  s_i = p_y + t_i sin(theta), and the spheres meet at
  y = m cos^2(theta) / 2 + s sin(theta) (terms whose circle lies behind the
  march's start, t - y <= 0, bound nothing);
* a wall in the light's way gives 0; no samples (max_steps 0, max_dist below
  the start, a point outside the grid) give 1;
* jitter moves the first sample to eps + jitter * scale.
The linear field is reproduced exactly by trilinear sampling between texel
centres, so these are exact statements about the march up to float32
rounding of t (a few ulps per step).
"""
import math

import numpy as np

import oracle

N = 64
H = np.float32(1.0 / N)
LO = np.zeros(3, np.float32)


def const_field(S):
    return np.full(N ** 3, S, np.float32)


def run(sdf, pts, light, k, eps, max_steps, max_step, max_dist, **kw):
    return oracle.shadow(N, LO, H, sdf, np.asarray(pts, np.float32), np.asarray(light, np.float32), k, eps,
                         max_steps, max_step, max_dist, **kw)


def samples(t0, step, max_dist, max_steps):
    t = [t0]
    while len(t) < max_steps and t[-1] + step <= max_dist:
        t.append(t[-1] + step)
    return np.array(t)


def test_constant_field_cone_and_triangulated():
    S, eps, k, max_dist = 0.125, 1 / 64, 2.0, 0.8
    pts = [[0.5, 0.05, 0.5]]
    t = samples(eps, S, max_dist, 1000)
    assert len(t) == 7
    cone = run(const_field(S), pts, [0, 1, 0], k, eps, 1000, 1.0, max_dist)[0]
    assert math.isclose(cone, min(1.0, k * S / t[-1]), rel_tol=1e-6)
    tri = run(const_field(S), pts, [0, 1, 0], k, eps, 1000, 1.0, max_dist, penumbra=1)[0]
    want = min(1.0, k * S / t[0], k * math.sqrt(S * S - S * S / 4) / (t[-1] - S / 2))
    assert math.isclose(tri, want, rel_tol=1e-6)
    assert tri != cone


def test_max_step_clamp_triangulated():
    S, m, eps, k, max_dist = 0.3, 0.05, 1 / 64, 1.5, 0.6
    pts = [[0.5, 0.1, 0.5]]
    t = samples(eps, m, max_dist, 1000)
    got = run(const_field(S), pts, [0, 1, 0], k, eps, 1000, m, max_dist, penumbra=1)[0]
    want = min(1.0, k * S / t[0], k * math.sqrt(S * S - m * m / 4) / (t[-1] - m / 2))
    assert math.isclose(got, want, rel_tol=1e-5)
    # the step count limit cuts the march at the same samples
    got5 = run(const_field(S), pts, [0, 1, 0], k, eps, 5, m, max_dist, penumbra=1)[0]
    t5 = samples(eps, m, max_dist, 5)
    assert math.isclose(got5, min(1.0, k * S / t5[0], k * math.sqrt(S * S - m * m / 4) / (t5[-1] - m / 2)),
                        rel_tol=1e-5)


def test_linear_field_rising_light():
    # s(q) = q_y: exact distance to the plane y = 0 at every texel centre
    j = np.arange(N ** 3)
    yc = ((j // N) % N + 0.5) / N
    sdf = yc.astype(np.float32)
    theta = math.radians(20)
    light = np.array([math.cos(theta), math.sin(theta), 0.0], np.float32)
    p = np.array([0.1, 0.12, 0.5], np.float32)
    m, eps, k = 1 / 128, 1 / 64, 3.0
    max_dist = 0.7  # stays between the outermost texel centres
    sin_t = float(light[1])
    cos2 = float(light[0]) ** 2 + float(light[2]) ** 2
    t = samples(eps, m, max_dist, 10000)
    s = float(p[1]) + t * sin_t
    assert np.all(s > m)  # the cap is the step everywhere
    cone = run(sdf, [p], light, k, eps, 10000, m, max_dist)[0]
    assert math.isclose(cone, min(1.0, float(np.min(k * s / t))), rel_tol=2e-5)
    y = m * cos2 / 2 + s[1:] * sin_t
    d = np.sqrt(s[1:] ** 2 - y ** 2)
    ahead = t[1:] - y > 0  # a circle behind the start of the march bounds nothing
    assert ahead.sum() > 10 and not ahead.all()
    tri_terms = np.concatenate([[k * s[0] / t[0]], (k * d / (t[1:] - y))[ahead]])
    tri = run(sdf, [p], light, k, eps, 10000, m, max_dist, penumbra=1)[0]
    assert math.isclose(tri, min(1.0, float(tri_terms.min())), rel_tol=2e-5)


def test_wall_blocks_and_empty_marches_are_lit():
    j = np.arange(N ** 3)
    yc = ((j // N) % N + 0.5) / N
    wall = (0.7 - yc).astype(np.float32)  # distance to the plane y = 0.7 from below
    for pen in (0, 1):
        assert run(wall, [[0.5, 0.2, 0.5]], [0, 1, 0], 4.0, 1 / 64, 64, 1.0, 2.0, penumbra=pen)[0] == 0.0
        assert run(wall, [[0.5, 0.2, 0.5]], [0, 1, 0], 4.0, 1 / 64, 0, 1.0, 2.0, penumbra=pen)[0] == 1.0
        assert run(wall, [[0.5, 0.2, 0.5]], [0, 1, 0], 4.0, 1 / 64, 64, 1.0, 1 / 128, penumbra=pen)[0] == 1.0
        assert run(wall, [[1.5, 0.2, 0.5]], [0, 1, 0], 4.0, 1 / 64, 64, 1.0, 2.0, penumbra=pen)[0] == 1.0


def test_jitter_moves_the_first_sample():
    S, eps, k, max_dist = 0.125, 1 / 64, 0.25, 0.8
    pts = np.array([[0.5, 0.05, 0.5]] * 3, np.float32)
    jit = np.array([0.0, 0.5, 0.9375], np.float32)
    scale = 1 / 32
    got = run(const_field(S), pts, [0, 1, 0], k, eps, 1000, 1.0, max_dist, jitter=jit, jitter_scale=scale)
    for g, jv in zip(got, jit):
        t = samples(eps + float(jv) * scale, S, max_dist, 1000)
        assert math.isclose(g, min(1.0, k * S / t[-1]), rel_tol=1e-6)
    # zero jitter equals no jitter
    nojit = run(const_field(S), pts[:1], [0, 1, 0], k, eps, 1000, 1.0, max_dist)
    assert got[0] == nojit[0]
