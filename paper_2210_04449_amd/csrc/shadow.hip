// Soft shadows from the fine SDF (paper Sec. 2.3): sphere tracing from each
// shaded point towards a directional light, stopping after a maximum number
// of steps or when the field drops below eps (at least one voxel, so a
// surface does not shadow itself); the field is sampled trilinearly, not at
// the nearest texel, and the step is capped (the paper notes the cap removes
// banding at the price of more samples).  The penumbra term is the running
// minimum of k * s / t (the cone estimate of the SDF shadow technique the
// paper cites), or, with triangulation between consecutive samples (the
// banding fix the paper takes from Aaltonen 2018), k * d / (t - y) with the
// clearance d and position y estimated where the two samples' empty spheres
// intersect.  The start of the march can be jittered towards the light by a
// caller-supplied amount per point (the paper jitters the origin and filters
// the noise over time).
//
// Every float operation below is an explicitly rounded intrinsic in a fixed
// order, so the march (including its data-dependent stopping decisions) is
// reproducible exactly on another IEEE machine.
#include "common.hpp"

namespace rtsdf {

__device__ __forceinline__ float lerp_rn(float a, float b, float f) { return rn_add(a, rn_mul(f, rn_sub(b, a))); }

// coordinate of q along one axis in texel-centre units, clamped to [0, n-1];
// false if q is outside the grid box
__device__ __forceinline__ bool grid_coord(float q, float lo, float h, int n, int &i, float &f)
{
    const float g = rn_sub(rn_div(rn_sub(q, lo), h), 0.5f);
    if (g < -0.5f || g > (float)n - 0.5f) return false;
    const float gc = fminf(fmaxf(g, 0.0f), (float)(n - 1));
    i = min((int)floorf(gc), n - 2);
    f = rn_sub(gc, (float)i);
    return true;
}

struct ShadowArgs {
    rtsdf_grid g;
    const float *sdf, *pts, *jitter;
    int np;
    float lx, ly, lz, k, eps, max_step, max_dist, jitter_scale;
    int max_steps, penumbra;
};

__global__ void __launch_bounds__(256) shadow_kernel(ShadowArgs A, float *__restrict__ vis_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.np) return;
    const rtsdf_grid &g = A.g;
    const float *__restrict__ sdf = A.sdf;
    const int n = g.n;
    const float px = A.pts[3 * p], py = A.pts[3 * p + 1], pz = A.pts[3 * p + 2];
    const float eps = A.eps, k = A.k;
    float vis = 1.0f, t = eps;
    if (A.jitter) t = rn_add(eps, rn_mul(A.jitter[p], A.jitter_scale));
    bool have_prev = false;
    float t_prev = 0.0f, s_prev = 0.0f;
    for (int step = 0; step < A.max_steps; ++step) {
        if (t > A.max_dist) break;
        const float qx = rn_add(px, rn_mul(t, A.lx));
        const float qy = rn_add(py, rn_mul(t, A.ly));
        const float qz = rn_add(pz, rn_mul(t, A.lz));
        int ix, iy, iz;
        float fx, fy, fz;
        if (!grid_coord(qx, g.lo[0], g.h, n, ix, fx) || !grid_coord(qy, g.lo[1], g.h, n, iy, fy) ||
            !grid_coord(qz, g.lo[2], g.h, n, iz, fz))
            break;
        const int64_t b = ix + (int64_t)n * (iy + (int64_t)n * iz);
        const int64_t sy = n, sz = (int64_t)n * n;
        const float c00 = lerp_rn(sdf[b], sdf[b + 1], fx);
        const float c10 = lerp_rn(sdf[b + sy], sdf[b + sy + 1], fx);
        const float c01 = lerp_rn(sdf[b + sz], sdf[b + sz + 1], fx);
        const float c11 = lerp_rn(sdf[b + sy + sz], sdf[b + sy + sz + 1], fx);
        const float s = lerp_rn(lerp_rn(c00, c10, fy), lerp_rn(c01, c11, fy), fz);
        if (s < eps) {
            vis = 0.0f;
            break;
        }
        if (A.penumbra == 1 && have_prev) {
            // the empty spheres of radius s_prev (at t_prev) and s (at t)
            // intersect on a circle y behind the current sample; its radius d
            // is the estimated clearance of the ray
            const float D = rn_sub(t, t_prev);
            const float ss = rn_mul(s, s);
            const float num = rn_sub(rn_add(rn_mul(D, D), ss), rn_mul(s_prev, s_prev));
            const float y = fminf(fmaxf(rn_div(num, rn_add(D, D)), 0.0f), s);
            const float d = rn_sqrt(fmaxf(rn_sub(ss, rn_mul(y, y)), 0.0f));
            const float w = rn_sub(t, y);
            if (w > 0.0f) vis = fminf(vis, rn_div(rn_mul(k, d), w));
        } else {
            vis = fminf(vis, rn_div(rn_mul(k, s), t));
        }
        have_prev = true;
        t_prev = t;
        s_prev = s;
        t = rn_add(t, fmaxf(fminf(s, A.max_step), eps));
    }
    vis_out[p] = fmaxf(vis, 0.0f);
}

}  // namespace rtsdf

static int shadow_launch(rtsdf_grid fine, const float *fine_sdf, const float *points, int32_t np,
                         const rtsdf_shadow_params &P, const float *jitter, float *visibility, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!grid_ok(fine) || fine.n < 2 || !fine_sdf || np < 0 || (np > 0 && (!points || !visibility)))
        return RTSDF_EINVAL;
    if (!(P.eps > 0.0f) || P.max_steps < 0 || !(P.max_step > 0.0f) || !(P.k > 0.0f) || !(P.max_dist >= 0.0f))
        return RTSDF_EINVAL;
    if (P.penumbra != 0 && P.penumbra != 1) return RTSDF_EINVAL;
    if (jitter && !(P.jitter_scale >= 0.0f)) return RTSDF_EINVAL;
    if (np == 0) return RTSDF_OK;
    const ShadowArgs A{fine,         fine_sdf, points, jitter,     np,         P.light_dir[0],
                       P.light_dir[1], P.light_dir[2], P.k, P.eps, P.max_step, P.max_dist,
                       P.jitter_scale, P.max_steps, P.penumbra};
    shadow_kernel<<<dim3((np + 255) / 256), dim3(256), 0, as_stream(stream)>>>(A, visibility);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

extern "C" int rtsdf_shadow(rtsdf_grid fine, const float *fine_sdf, const float *points, int32_t np,
                            const float light_dir[3], float k, float eps, int32_t max_steps, float max_step,
                            float max_dist, float *visibility, rtsdf_stream stream)
{
    if (!light_dir) return RTSDF_EINVAL;
    rtsdf_shadow_params P{};
    P.light_dir[0] = light_dir[0];
    P.light_dir[1] = light_dir[1];
    P.light_dir[2] = light_dir[2];
    P.k = k;
    P.eps = eps;
    P.max_steps = max_steps;
    P.max_step = max_step;
    P.max_dist = max_dist;
    P.penumbra = 0;
    P.jitter_scale = 0.0f;
    return shadow_launch(fine, fine_sdf, points, np, P, nullptr, visibility, stream);
}

extern "C" int rtsdf_shadow_ex(rtsdf_grid fine, const float *fine_sdf, const float *points, int32_t np,
                               const rtsdf_shadow_params *params, const float *jitter, float *visibility,
                               rtsdf_stream stream)
{
    if (!params) return RTSDF_EINVAL;
    return shadow_launch(fine, fine_sdf, points, np, *params, jitter, visibility, stream);
}
