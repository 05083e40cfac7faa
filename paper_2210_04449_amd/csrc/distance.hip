// Exact unsigned distance from points to the mesh: the quantity the traced
// fine SDF approximates from above (Sec. 2.2 keeps the smallest hit distance
// of random rays, and every hit lies on the mesh, so for the current geometry
// the traced value can never be below it).  Used to measure the method's
// accuracy and, for moving scenes, the stale history that the decay alpha of
// Eq. (1) is there to forget (a traced value below the current exact distance
// can only come from geometry that has moved away).
//
// One lane per point, best-first descent of the same two-wide hierarchy the
// tracer uses: at a node the nearer child box (squared point-box distance) is
// visited first and the farther one is pushed with its distance, a popped
// entry is dropped when its box is no nearer than the best triangle so far.
// Leaves test whole triangles (a split reference's box bounds its piece; the
// pieces cover the triangle, so the piece holding the closest point is never
// pruned and testing the whole triangle there is exact).  Closest point on a
// triangle by its Voronoi regions (vertex, edge and face regions, as in
// Ericson, Real-Time Collision Detection, 2005, Sec. 5.1.5), in float32.
#include "common.hpp"

namespace rtsdf {

__device__ __forceinline__ float dot3f(float ax, float ay, float az, float bx, float by, float bz)
{
    return ax * bx + ay * by + az * bz;
}

// squared distance from p to the closest point of segment [a, a + e]
__device__ __forceinline__ float seg_dist2(float px, float py, float pz, float ax, float ay, float az, float ex,
                                           float ey, float ez)
{
    const float ee = dot3f(ex, ey, ez, ex, ey, ez);
    float t = ee > 0.0f ? dot3f(px - ax, py - ay, pz - az, ex, ey, ez) / ee : 0.0f;
    t = fminf(fmaxf(t, 0.0f), 1.0f);
    const float qx = ax + t * ex - px, qy = ay + t * ey - py, qz = az + t * ez - pz;
    return dot3f(qx, qy, qz, qx, qy, qz);
}

__device__ __forceinline__ float point_tri_dist2(float px, float py, float pz, float4 A, float4 B, float4 Cv)
{
    const float abx = B.x - A.x, aby = B.y - A.y, abz = B.z - A.z;
    const float acx = Cv.x - A.x, acy = Cv.y - A.y, acz = Cv.z - A.z;
    const float apx = px - A.x, apy = py - A.y, apz = pz - A.z;
    float qx, qy, qz;
    const float d1 = dot3f(abx, aby, abz, apx, apy, apz), d2 = dot3f(acx, acy, acz, apx, apy, apz);
    const float bpx = px - B.x, bpy = py - B.y, bpz = pz - B.z;
    const float d3 = dot3f(abx, aby, abz, bpx, bpy, bpz), d4 = dot3f(acx, acy, acz, bpx, bpy, bpz);
    const float cpx = px - Cv.x, cpy = py - Cv.y, cpz = pz - Cv.z;
    const float d5 = dot3f(abx, aby, abz, cpx, cpy, cpz), d6 = dot3f(acx, acy, acz, cpx, cpy, cpz);
    const float vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
    if (d1 <= 0.0f && d2 <= 0.0f) {  // vertex A
        qx = A.x, qy = A.y, qz = A.z;
    } else if (d3 >= 0.0f && d4 <= d3) {  // vertex B
        qx = B.x, qy = B.y, qz = B.z;
    } else if (d6 >= 0.0f && d5 <= d6) {  // vertex C
        qx = Cv.x, qy = Cv.y, qz = Cv.z;
    } else if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) {  // edge AB
        const float t = d1 / (d1 - d3);
        qx = A.x + t * abx, qy = A.y + t * aby, qz = A.z + t * abz;
    } else if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {  // edge AC
        const float t = d2 / (d2 - d6);
        qx = A.x + t * acx, qy = A.y + t * acy, qz = A.z + t * acz;
    } else if (va <= 0.0f && d4 - d3 >= 0.0f && d5 - d6 >= 0.0f) {  // edge BC
        const float t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        qx = B.x + t * (Cv.x - B.x), qy = B.y + t * (Cv.y - B.y), qz = B.z + t * (Cv.z - B.z);
    } else {
        const float sum = va + vb + vc;
        if (!(sum > 0.0f) || isinf(sum)) {  // degenerate (zero area): nearest of the three edges
            return fminf(fminf(seg_dist2(px, py, pz, A.x, A.y, A.z, abx, aby, abz),
                               seg_dist2(px, py, pz, A.x, A.y, A.z, acx, acy, acz)),
                         seg_dist2(px, py, pz, B.x, B.y, B.z, Cv.x - B.x, Cv.y - B.y, Cv.z - B.z));
        }
        const float v = vb / sum, w = vc / sum;  // face region
        qx = A.x + abx * v + acx * w, qy = A.y + aby * v + acy * w, qz = A.z + abz * v + acz * w;
    }
    const float dx = qx - px, dy = qy - py, dz = qz - pz;
    return dot3f(dx, dy, dz, dx, dy, dz);
}

// squared distance from p to the box [lo, hi]; +inf for an empty box
__device__ __forceinline__ float box_dist2(float px, float py, float pz, float x0, float x1, float y0, float y1,
                                           float z0, float z1)
{
    if (!(x0 <= x1) || !(y0 <= y1) || !(z0 <= z1)) return __builtin_inff();
    const float dx = fmaxf(fmaxf(x0 - px, px - x1), 0.0f);
    const float dy = fmaxf(fmaxf(y0 - py, py - y1), 0.0f);
    const float dz = fmaxf(fmaxf(z0 - pz, pz - z1), 0.0f);
    return dx * dx + dy * dy + dz * dz;
}

constexpr int kDistBlock = 128;

template <int SD, bool TEXELS>
__global__ void __launch_bounds__(kDistBlock) point_distance_kernel(BvhView S, int nt, const float *__restrict__ pts,
                                                                    rtsdf_grid g, const int32_t *__restrict__ texels,
                                                                    int n, float *__restrict__ dist_out,
                                                                    int32_t *__restrict__ tri_out)
{
    __shared__ int stk_node[kDistBlock / kWave][SD][kWave];
    __shared__ float stk_d2[kDistBlock / kWave][SD][kWave];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float px, py, pz;
    if (TEXELS) {
        const int j = texels ? texels[i] : i;
        const int nn = g.n;
        px = texel_coord(g.lo[0], j % nn, g.h);
        py = texel_coord(g.lo[1], (j / nn) % nn, g.h);
        pz = texel_coord(g.lo[2], j / (nn * nn), g.h);
    } else {
        px = pts[3 * i], py = pts[3 * i + 1], pz = pts[3 * i + 2];
    }
    float best = __builtin_inff();
    int best_id = -1;
    int sp = 0;
    int node = nt > 0 ? 0 : kDone;
    while (node != kDone) {
        if (node >= 0) {
            const BvhNode *nd = node_ptr(S.nodes, node);
            const float4 a = nd->xy0, b = nd->xy1, z = nd->z01;
            const int4 m = nd->meta;
            const float e0 = box_dist2(px, py, pz, a.x, a.y, a.z, a.w, z.x, z.y);
            const float e1 = box_dist2(px, py, pz, b.x, b.y, b.z, b.w, z.z, z.w);
            const bool h0 = e0 <= best, h1 = e1 <= best;  // ties kept: a tie in distance may hold a lower id
            const bool first0 = h0 && (!h1 || e0 <= e1);
            if (h0 && h1) {
                stk_node[wave][sp][lane] = first0 ? m.y : m.x;
                stk_d2[wave][sp][lane] = first0 ? e1 : e0;
                ++sp;
            }
            if (h0 || h1) {
                node = first0 ? m.x : m.y;
                continue;
            }
        } else {
            const int first = leaf_first(node), cnt = leaf_count(node);
            for (int k = first; k < first + cnt; ++k) {
                const float4 *tp = reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(S.tris) +
                                                                    rec48(k));
                const float4 A = tp[0], B = tp[1], Cv = tp[2];
                const int id = __float_as_int(A.w);
                const float d2 = point_tri_dist2(px, py, pz, A, B, Cv);
                if (d2 < best || (d2 == best && id < best_id)) {
                    best = d2;
                    best_id = id;
                }
            }
        }
        // pop the next entry that can still hold a point no farther than the best
        node = kDone;
        while (sp > 0) {
            --sp;
            if (stk_d2[wave][sp][lane] <= best) {
                node = stk_node[wave][sp][lane];
                break;
            }
        }
    }
    dist_out[i] = best_id >= 0 ? __builtin_sqrtf(best) : __builtin_inff();
    if (tri_out) tri_out[i] = best_id;
}

static int point_distance_launch(const rtsdf_scene *scene, const float *points, rtsdf_grid g, bool texel_mode,
                                 const int32_t *texels, int32_t n, float *dist, int32_t *tri, rtsdf_stream stream)
{
    if (scene->ninst > 0) return RTSDF_EINVAL;  // single-level scenes only
    if (n == 0) return RTSDF_OK;
    const int sd = stack_depth_for(scene);
    if (sd > 64) return RTSDF_EINVAL;
    const BvhView S{scene->nodes, scene->tris, scene->tmap};
    const dim3 grid((unsigned)((n + kDistBlock - 1) / kDistBlock)), block(kDistBlock);
    hipStream_t s = as_stream(stream);
    if (texel_mode) {
        if (sd <= 32)
            point_distance_kernel<32, true><<<grid, block, 0, s>>>(S, scene->nt, nullptr, g, texels, n, dist, tri);
        else
            point_distance_kernel<64, true><<<grid, block, 0, s>>>(S, scene->nt, nullptr, g, texels, n, dist, tri);
    } else {
        if (sd <= 32)
            point_distance_kernel<32, false><<<grid, block, 0, s>>>(S, scene->nt, points, g, nullptr, n, dist, tri);
        else
            point_distance_kernel<64, false><<<grid, block, 0, s>>>(S, scene->nt, points, g, nullptr, n, dist, tri);
    }
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

}  // namespace rtsdf

extern "C" int rtsdf_point_distance(const rtsdf_scene *scene, const float *points, int32_t n, float *dist,
                                    int32_t *tri, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scene || n < 0 || (n > 0 && (!points || !dist))) return RTSDF_EINVAL;
    return point_distance_launch(scene, points, rtsdf_grid{}, false, nullptr, n, dist, tri, stream);
}

extern "C" int rtsdf_texel_distance(const rtsdf_scene *scene, rtsdf_grid grid, const int32_t *texels, int32_t n,
                                    float *dist, int32_t *tri, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scene || !grid_ok(grid) || grid.n > 1024 || n < 0 || (n > 0 && !dist)) return RTSDF_EINVAL;
    if (!texels && (int64_t)n != (int64_t)grid.n * grid.n * grid.n) return RTSDF_EINVAL;
    return point_distance_launch(scene, nullptr, grid, true, texels, n, dist, tri, stream);
}
