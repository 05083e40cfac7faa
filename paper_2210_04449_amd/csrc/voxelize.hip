// Voxelization of a triangle mesh into the coarse grid (paper Sec. 2.1).
//
// The paper renders the scene three times with an orthographic camera along
// +x, +y and +z, depth writes off, and marks the voxel under every fragment.
// gfx950 has no raster pipeline, so this is a compute kernel that applies an
// exact integer version of that rule: vertices snapped to 1/256 voxel, a
// column covered when its centre is inside or on the projected triangle, and
// the voxel holding the triangle's depth at that centre marked.
//
// Work mapping: one lane per (triangle, axis), dealt to wavefronts with a
// stride.  A lane rasterizes its own
// projection when the bounding box holds at most kSmallPixels column centres;
// larger projections (room walls cover whole faces of the grid) are flagged
// and then rasterized by the whole wavefront, one after another, with the 64
// lanes striding over the box, so a few huge triangles do not serialise one
// lane.
#include "common.hpp"

namespace rtsdf {

constexpr int kSmallPixels = 16;

struct VoxTri {
    int64_t px[3], py[3], z[3];  // projected snapped coordinates, depth
    int64_t area2;               // > 0 (counter-clockwise after the swap)
    int i0, i1, j0, j1;          // column range (inclusive)
    int axis;
};

__device__ __forceinline__ int64_t floor_div_pos(int64_t a, int64_t b)  // b > 0
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) --q;
    return q;
}

__device__ __forceinline__ bool snap(const float *__restrict__ v, int vi, const rtsdf_grid &g, int64_t X[3])
{
    const double side = (double)g.n * (double)g.h;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double rel = (double)v[3 * vi + a] - (double)g.lo[a];
        if (!(rel >= -side && rel <= 2.0 * side)) return false;
        X[a] = (int64_t)__builtin_rint(rel / (double)g.h * 256.0);
    }
    return true;
}

// Sets up the projection of triangle t along `axis`; false if it covers
// nothing (zero area or box outside the grid).
__device__ bool vox_setup(const int64_t X[3][3], int axis, int n, VoxTri &T)
{
    const int e1 = (axis + 1) % 3, e2 = (axis + 2) % 3;
    for (int k = 0; k < 3; ++k) {
        T.px[k] = X[k][e1];
        T.py[k] = X[k][e2];
        T.z[k] = X[k][axis];
    }
    int64_t area2 = (T.px[1] - T.px[0]) * (T.py[2] - T.py[0]) - (T.py[1] - T.py[0]) * (T.px[2] - T.px[0]);
    if (area2 == 0) return false;
    if (area2 < 0) {
        int64_t tx = T.px[1], ty = T.py[1], tz = T.z[1];
        T.px[1] = T.px[2]; T.py[1] = T.py[2]; T.z[1] = T.z[2];
        T.px[2] = tx; T.py[2] = ty; T.z[2] = tz;
        area2 = -area2;
    }
    T.area2 = area2;
    T.axis = axis;
    const int64_t minx = min(T.px[0], min(T.px[1], T.px[2])), maxx = max(T.px[0], max(T.px[1], T.px[2]));
    const int64_t miny = min(T.py[0], min(T.py[1], T.py[2])), maxy = max(T.py[0], max(T.py[1], T.py[2]));
    // column centre 256 i + 128 within [min, max]
    int64_t i0 = floor_div_pos(minx - 128 + 255, 256), i1 = floor_div_pos(maxx - 128, 256);
    int64_t j0 = floor_div_pos(miny - 128 + 255, 256), j1 = floor_div_pos(maxy - 128, 256);
    i0 = max(i0, (int64_t)0);
    j0 = max(j0, (int64_t)0);
    i1 = min(i1, (int64_t)n - 1);
    j1 = min(j1, (int64_t)n - 1);
    if (i0 > i1 || j0 > j1) return false;
    T.i0 = (int)i0; T.i1 = (int)i1; T.j0 = (int)j0; T.j1 = (int)j1;
    return true;
}

// Tests column (i, j); marks the voxel if covered.
__device__ __forceinline__ void vox_column(const VoxTri &T, int i, int j, int n, int32_t *__restrict__ seeds)
{
    const int64_t cx = 256 * (int64_t)i + 128, cy = 256 * (int64_t)j + 128;
    const int64_t w0 = (T.px[2] - T.px[1]) * (cy - T.py[1]) - (T.py[2] - T.py[1]) * (cx - T.px[1]);
    const int64_t w1 = (T.px[0] - T.px[2]) * (cy - T.py[2]) - (T.py[0] - T.py[2]) * (cx - T.px[2]);
    const int64_t w2 = (T.px[1] - T.px[0]) * (cy - T.py[0]) - (T.py[1] - T.py[0]) * (cx - T.px[0]);
    if ((w0 | w1 | w2) < 0) return;
    const int64_t num = w0 * T.z[0] + w1 * T.z[1] + w2 * T.z[2];
    const int64_t den = T.area2 * 256;
    int64_t L;
    if (num == (int64_t)n * den) {
        L = n - 1;
    } else {
        // floor(num / den) from a double estimate, corrected exactly (the
        // estimate is off by at most one; num < 2^56, den < 2^45).
        L = (int64_t)floor((double)num / (double)den);
        if (L * den > num) --L;
        if ((L + 1) * den <= num) ++L;
        if (L < 0 || L >= n) return;
    }
    int q[3];
    const int a = T.axis;
    q[a] = (int)L;
    q[(a + 1) % 3] = i;
    q[(a + 2) % 3] = j;
    const int idx = q[0] + n * (q[1] + n * q[2]);
    seeds[idx] = idx;
}

// Lane part of one (triangle, axis) item: snap, set up, rasterize a small
// projection directly; returns true when the projection is large and left to
// the whole wavefront.
__device__ __forceinline__ bool vox_item(const float *__restrict__ v, int nv, const int32_t *__restrict__ f, int t,
                                         int axis, const rtsdf_grid &g, int32_t *__restrict__ seeds, VoxTri &T)
{
    int vid[3] = {f[3 * t], f[3 * t + 1], f[3 * t + 2]};
    for (int k = 0; k < 3; ++k)
        if (vid[k] < 0 || vid[k] >= nv) {
            if (axis == 0) raise_error(RTSDF_ERR_FACE_INDEX);
            return false;
        }
    int64_t X[3][3];
    for (int k = 0; k < 3; ++k)
        if (!snap(v, vid[k], g, X[k])) {
            if (axis == 0) raise_error(RTSDF_ERR_VERTEX_RANGE);
            return false;
        }
    if (!vox_setup(X, axis, g.n, T)) return false;
    const int npix = (T.i1 - T.i0 + 1) * (T.j1 - T.j0 + 1);
    if (npix <= kSmallPixels) {
        for (int j = T.j0; j <= T.j1; ++j)
            for (int i = T.i0; i <= T.i1; ++i) vox_column(T, i, j, g.n, seeds);
        return false;
    }
    return true;
}

// Large projections of the wavefront's lanes, rasterized by all 64 lanes in
// turn; `seeds` / `n` may differ per lane (many scenes per launch).
__device__ __forceinline__ void vox_wave_big(bool big, const VoxTri &T, int32_t *seeds, int n)
{
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t pending = __ballot(big);
    while (pending) {
        const int src = __ffsll((unsigned long long)pending) - 1;
        pending &= pending - 1;
        VoxTri B;
        for (int k = 0; k < 3; ++k) {
            B.px[k] = __shfl(T.px[k], src);
            B.py[k] = __shfl(T.py[k], src);
            B.z[k] = __shfl(T.z[k], src);
        }
        B.area2 = __shfl(T.area2, src);
        B.i0 = __shfl(T.i0, src);
        B.i1 = __shfl(T.i1, src);
        B.j0 = __shfl(T.j0, src);
        B.j1 = __shfl(T.j1, src);
        B.axis = __shfl(T.axis, src);
        int32_t *bs = reinterpret_cast<int32_t *>(__shfl((long long)reinterpret_cast<intptr_t>(seeds), src));
        const int bn = __shfl(n, src);
        const int w = B.i1 - B.i0 + 1;
        const int npix = w * (B.j1 - B.j0 + 1);
        for (int p = lane; p < npix; p += kWave) vox_column(B, B.i0 + p % w, B.j0 + p / w, bn, bs);
    }
}

__global__ void __launch_bounds__(256) voxelize_kernel(const float *__restrict__ v, int nv,
                                                       const int32_t *__restrict__ f, int nt, rtsdf_grid g,
                                                       int32_t *__restrict__ seeds)
{
    // items are dealt to wavefronts with a stride (lane l of wavefront w takes item l * waves + w), so the
    // large projections of consecutive triangles (the walls of a room come one after another) land in
    // different wavefronts instead of queueing in one
    const int64_t total = 3 * (int64_t)nt;
    const int64_t waves = (total + kWave - 1) / kWave;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t item = (gid & (kWave - 1)) * waves + (gid >> 6);
    VoxTri T;
    bool big = false;
    if ((gid >> 6) < waves && item < total) big = vox_item(v, nv, f, (int)(item / 3), (int)(item % 3), g, seeds, T);
    vox_wave_big(big, T, seeds, g.n);
}

}  // namespace rtsdf

extern "C" int rtsdf_voxelize(const float *vertices, int32_t nv, const int32_t *faces, int32_t nt,
                              rtsdf_grid coarse, int32_t *seeds, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!grid_ok(coarse) || !is_pow2(coarse.n) || coarse.n < 8 || coarse.n > 256) return RTSDF_EINVAL;
    if (!seeds || nv < 0 || nt < 0 || (nt > 0 && (!vertices || !faces))) return RTSDF_EINVAL;
    if ((int64_t)nt * 3 > (int64_t)INT32_MAX) return RTSDF_EINVAL;
    hipStream_t s = as_stream(stream);
    const int64_t nvox = (int64_t)coarse.n * coarse.n * coarse.n;
    int rc = launch_fill<int32_t>(seeds, -1, nvox, s);
    if (rc != RTSDF_OK) return rc;
    if (nt == 0) return RTSDF_OK;
    const int64_t items = 3 * (int64_t)nt;
    voxelize_kernel<<<dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s>>>(vertices, nv, faces, nt, coarse, seeds);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}
