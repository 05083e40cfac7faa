// Soft shadows from the fine SDF (paper Sec. 2.3): sphere tracing from each
// shaded point towards a directional light, stopping after a maximum number
// of steps or when the field drops below eps (at least one voxel, so a
// surface does not shadow itself); the field is sampled trilinearly, not at
// the nearest texel, and the step is capped (the paper notes the cap removes
// banding at the price of more samples).  The penumbra term is the running
// minimum of k * s / t (the cone estimate of the SDF shadow technique the
// paper cites).
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

__global__ void __launch_bounds__(256) shadow_kernel(rtsdf_grid g, const float *__restrict__ sdf,
                                                     const float *__restrict__ pts, int np, float lx, float ly,
                                                     float lz, float k, float eps, int max_steps, float max_step,
                                                     float max_dist, float *__restrict__ vis_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int n = g.n;
    const float px = pts[3 * p], py = pts[3 * p + 1], pz = pts[3 * p + 2];
    float vis = 1.0f, t = eps;
    for (int step = 0; step < max_steps; ++step) {
        if (t > max_dist) break;
        const float qx = rn_add(px, rn_mul(t, lx));
        const float qy = rn_add(py, rn_mul(t, ly));
        const float qz = rn_add(pz, rn_mul(t, lz));
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
        vis = fminf(vis, rn_div(rn_mul(k, s), t));
        t = rn_add(t, fmaxf(fminf(s, max_step), eps));
    }
    vis_out[p] = fmaxf(vis, 0.0f);
}

}  // namespace rtsdf

extern "C" int rtsdf_shadow(rtsdf_grid fine, const float *fine_sdf, const float *points, int32_t np,
                            const float light_dir[3], float k, float eps, int32_t max_steps, float max_step,
                            float max_dist, float *visibility, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!grid_ok(fine) || fine.n < 2 || !fine_sdf || np < 0 || (np > 0 && (!points || !visibility)) || !light_dir)
        return RTSDF_EINVAL;
    if (!(eps > 0.0f) || max_steps < 0 || !(max_step > 0.0f) || !(k > 0.0f) || !(max_dist >= 0.0f)) return RTSDF_EINVAL;
    if (np == 0) return RTSDF_OK;
    shadow_kernel<<<dim3((np + 255) / 256), dim3(256), 0, as_stream(stream)>>>(
        fine, fine_sdf, points, np, light_dir[0], light_dir[1], light_dir[2], k, eps, max_steps, max_step, max_dist,
        visibility);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}
