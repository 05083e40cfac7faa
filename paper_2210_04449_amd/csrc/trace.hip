// Fine-SDF ray tracing and temporal accumulation (paper Sec. 2.2, Eq. (1)),
// the vertex gradient of the traced distances, and two helper entry points
// (directions, closest hits) that expose the same arithmetic.
//
// Per selected texel and frame, rays_per_texel rays leave the texel centre
// towards uniformly random points of the unit sphere; each ray's closest hit
// distance is found in the bounding volume hierarchy; the smallest of the
// frame is r_t, which enters Eq. (1); front/back counts of the closest hits
// vote the sign.
//
// Random directions: Philox4x64 with 10 rounds (Salmon et al., SC'11) keyed
// by (seed, 0) with counter (texel, frame << 32 | ray, scene, attempt); 32-bit
// halves become odd multiples of 2^-23 in (-1, 1); Marsaglia's 1972 mapping of
// the first pair inside the unit disc gives the direction.  Every float
// operation there is an explicitly rounded intrinsic, so the directions are
// reproducible bit for bit on any IEEE machine.
//
// Closest hit: software traversal of the two-wide hierarchy with a per-lane
// stack in LDS (its depth is the hierarchy's depth, so it never overflows)
// and the watertight ray/triangle test of Woop, Benthin and Wald (JCGT 2013):
// vertices are mapped into a ray space where the ray is the +z axis (a
// per-ray affine map: axis permutation plus shear), 2D edge functions decide
// coverage (re-evaluated in double when one is exactly zero), so a ray that
// crosses a shared edge hits at least one of its triangles.  Ties in t go to
// the lower triangle index; t must be > 0.
//
// Work distribution: persistent wavefronts; one lane owns one selected texel
// and traces its rays one after another.  Lanes whose texel is finished are
// refilled from the compacted queue by one atomic add per wavefront (ballot +
// mbcnt to hand out the slots), so the queue is consumed in Morton order and
// no lane waits for a whole wavefront of texels to finish.
#include <algorithm>

#include "common.hpp"

namespace rtsdf {

// ------------------------------------------------------------------ RNG ----

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t y0 = hi1 ^ c[1] ^ k0, y2 = hi0 ^ c[3] ^ k1;
        c[0] = y0;
        c[1] = lo1;
        c[2] = y2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ float uniform_pm1(uint32_t h)
{
    return (float)((int32_t)((h >> 9) << 1) + 1 - 8388608) * 0x1p-23f;
}

__device__ __forceinline__ float3 sphere_dir(uint64_t seed, uint32_t texel, uint32_t frame, uint32_t ray, uint32_t scene)
{
    for (uint32_t attempt = 0; attempt < 8; ++attempt) {
        uint64_t c[4] = {(uint64_t)texel, ((uint64_t)frame << 32) | ray, (uint64_t)scene, (uint64_t)attempt};
        philox4x64_10(c, seed, 0);
        for (int p = 0; p < 4; ++p) {
            const float x1 = uniform_pm1((uint32_t)c[p]);
            const float x2 = uniform_pm1((uint32_t)(c[p] >> 32));
            const float s = rn_add(rn_mul(x1, x1), rn_mul(x2, x2));
            if (s < 1.0f) {
                const float q = rn_sqrt(rn_sub(1.0f, s));
                return make_float3(rn_mul(rn_mul(2.0f, x1), q), rn_mul(rn_mul(2.0f, x2), q),
                                   rn_sub(1.0f, rn_mul(2.0f, s)));
            }
        }
    }
    return make_float3(0.0f, 0.0f, 1.0f);
}

// texel centre: lo + (i + 1/2) h per axis, float ops rounded once each
__device__ __forceinline__ float texel_coord(float lo, int i, float h)
{
    return rn_add(lo, rn_mul(rn_add((float)i, 0.5f), h));
}

// ------------------------------------------------------------- geometry ----

struct RaySetup {
    float ix, iy, iz;    // 1 / direction (zero components replaced by +-1e-12)
    float oix, oiy, oiz; // origin * inverse
    float ox, oy, oz;    // origin
    float dx, dy, dz;    // direction
};

// |direction|, which turns a hit's ray parameter into a distance (computed where it is needed, from the
// stored direction, so the traversal loop does not keep it; the fused multiply-adds are spelled out so every
// kernel rounds it alike)
__device__ __forceinline__ float ray_len(const RaySetup &R)
{
    return __builtin_amdgcn_sqrtf(fmaf(R.dz, R.dz, fmaf(R.dy, R.dy, R.dx * R.dx)));
}

__device__ __forceinline__ float safe_inv(float d)
{
    const float a = fabsf(d) < 1e-12f ? copysignf(1e-12f, d) : d;
    return __builtin_amdgcn_rcpf(a);
}

__device__ __forceinline__ void ray_setup(float ox, float oy, float oz, float dx, float dy, float dz, RaySetup &R)
{
    R.ix = safe_inv(dx);
    R.iy = safe_inv(dy);
    R.iz = safe_inv(dz);
    R.oix = ox * R.ix;
    R.oiy = oy * R.iy;
    R.oiz = oz * R.iz;
    R.ox = ox;
    R.oy = oy;
    R.oz = oz;
    R.dx = dx;
    R.dy = dy;
    R.dz = dz;
}

// Watertight ray/triangle test (Woop, Benthin and Wald 2013): the vertices are
// taken into a ray space where the ray is the +z axis (permute so the largest
// direction component is z, then shear), and the three 2-D edge functions
// decide; edges shared by two triangles get the same values in both, so no
// ray passes between them.  Zero edge functions are recomputed in double
// precision.  Returns t of a front-face hit, -t of a back-face hit, 0 for a
// miss (hits have t > 0).
__device__ __noinline__ float tri_watertight(float ox, float oy, float oz, float dx, float dy, float dz,
                                             const float4 *tp)
{
    const float4 a = tp[0], b = tp[1], c = tp[2];
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    int kz = ay > ax ? 1 : 0;
    if (az > fmaxf(ax, ay)) kz = 2;
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    const float d[3] = {dx, dy, dz};
    if (d[kz] < 0.0f) {
        const int t = kx;
        kx = ky;
        ky = t;
    }
    // the shear only has to be the same for every triangle a ray meets, not correctly rounded
    const float Sz = __builtin_amdgcn_rcpf(d[kz]), Sx = d[kx] * Sz, Sy = d[ky] * Sz;
    const float o[3] = {ox, oy, oz};
    const float va[3] = {a.x - o[0], a.y - o[1], a.z - o[2]};
    const float vb[3] = {b.x - o[0], b.y - o[1], b.z - o[2]};
    const float vc[3] = {c.x - o[0], c.y - o[1], c.z - o[2]};
    const float Ax = va[kx] - Sx * va[kz], Ay = va[ky] - Sy * va[kz];
    const float Bx = vb[kx] - Sx * vb[kz], By = vb[ky] - Sy * vb[kz];
    const float Cx = vc[kx] - Sx * vc[kz], Cy = vc[ky] - Sy * vc[kz];
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0.0f;
    const float det = U + V + W;
    if (det == 0.0f) return 0.0f;
    const float T = U * (Sz * va[kz]) + V * (Sz * vb[kz]) + W * (Sz * vc[kz]);
    const float t = T / det;
    if (!(t > 0.0f)) return 0.0f;
    return det > 0.0f ? t : -t;
}

// Fast test through the triangle's precomputed map (see the scene layout):
// t from the plane coordinate, then the barycentrics at the crossing.  Where
// the smallest barycentric is within a rounding margin of zero -- the ray
// passes near an edge or a vertex -- the decision is left to the watertight
// test, so rays cannot slip between neighbouring triangles.  Updates the
// closest hit (t, leaf-order index) with ties going to the lower original
// triangle id.
constexpr float kEdgeMargin = 0x1p-12f;  // relative to the magnitude of the terms of the barycentrics

// Whether the ray (origin o, direction d) meets the triangle at leaf-order index i (rows r0, r1, r2 of its
// map) at some 0 < t <= tlim; the distance t and the facing (front: the ray meets the front face).  The
// decision and t do not depend on tlim, which only filters the result: whichever bound a traversal holds when
// it tests the triangle, the closest hit over all tested triangles is the same.
__device__ __forceinline__ bool tri_hit_rows(float ox, float oy, float oz, float dx, float dy, float dz, float4 r0,
                                             float4 r1, float4 r2, const float4 *tris, int i, float tlim, float &t,
                                             bool &fr)
{
    const float pz = fmaf(r2.x, ox, fmaf(r2.y, oy, fmaf(r2.z, oz, r2.w)));
    const float qz = fmaf(r2.x, dx, fmaf(r2.y, dy, r2.z * dz));
    const float p0 = fmaf(r0.x, ox, fmaf(r0.y, oy, fmaf(r0.z, oz, r0.w)));
    const float q0 = fmaf(r0.x, dx, fmaf(r0.y, dy, r0.z * dz));
    const float p1 = fmaf(r1.x, ox, fmaf(r1.y, oy, fmaf(r1.z, oz, r1.w)));
    const float q1 = fmaf(r1.x, dx, fmaf(r1.y, dy, r1.z * dz));
    t = -pz * __builtin_amdgcn_rcpf(qz);
    const float b1 = fmaf(t, q0, p0), b2 = fmaf(t, q1, p1);
    const float bmin = fminf(1.0f - b1 - b2, fminf(b1, b2));
    const float margin = kEdgeMargin * (fmaf(t, fabsf(q0) + fabsf(q1), fabsf(p0) + fabsf(p1)) + 1.0f);
    const bool in_range = t > 0.0f && t <= 3.0e38f;
    bool hit = in_range && bmin > margin;
    fr = qz < 0.0f;
    if (in_range && !(bmin > margin) && !(bmin < -margin)) {
        // near an edge or a vertex (or not a number): the watertight test decides
        const float4 *tp = reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(tris) + rec48(i));
        const float h = tri_watertight(ox, oy, oz, dx, dy, dz, tp);
        t = fabsf(h);
        fr = h > 0.0f;
        hit = h != 0.0f;
    }
    return hit && t <= tlim;
}

__device__ __forceinline__ void tri_test_rows(const RaySetup &R, float4 r0, float4 r1, float4 r2, const float4 *tris,
                                              int i, float &tbest, int &ibest, bool &front)
{
    float t;
    bool fr;
    if (!tri_hit_rows(R.ox, R.oy, R.oz, R.dx, R.dy, R.dz, r0, r1, r2, tris, i, tbest, t, fr)) return;
    if (t == tbest) {  // equal distances: the lower original triangle id wins
        const float4 *tp = reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(tris) + rec48(i));
        const float4 *tb = reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(tris) + rec48(ibest));
        if (!(__float_as_int(tp[0].w) < __float_as_int(tb[0].w))) return;
    }
    tbest = t;
    ibest = i;
    front = fr;
}

__device__ __forceinline__ void tri_test(const RaySetup &R, const float4 *tmap, const float4 *tris, int i,
                                         float &tbest, int &ibest, bool &front)
{
    // the whole record in one round trip, and no branch before the decision
    const float4 *mp = reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(tmap) + rec48(i));
    tri_test_rows(R, mp[0], mp[1], mp[2], tris, i, tbest, ibest, front);
}

// original id of the triangle at leaf-order index i
__device__ __forceinline__ int tri_id(const float4 *tris, int i)
{
    return __float_as_int(reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(tris) + rec48(i))->w);
}

// slab test against a padded box: whether the ray meets it before tbest (a NaN slab misses), the entry
// distance and the exit distance (capped at tbest)
__device__ __forceinline__ bool box_hit2(const RaySetup &R, float lx, float hx, float ly, float hy, float lz, float hz,
                                         float tbest, float &t_entry, float &t_exit)
{
    const float x0 = fmaf(lx, R.ix, -R.oix), x1 = fmaf(hx, R.ix, -R.oix);
    const float y0 = fmaf(ly, R.iy, -R.oiy), y1 = fmaf(hy, R.iy, -R.oiy);
    const float z0 = fmaf(lz, R.iz, -R.oiz), z1 = fmaf(hz, R.iz, -R.oiz);
    const float tmin = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), 0.0f));
    const float tmax = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tbest));
    t_entry = tmin;
    t_exit = tmax;
    return tmin <= tmax;
}

__device__ __forceinline__ bool box_hit(const RaySetup &R, float lx, float hx, float ly, float hy, float lz, float hz,
                                        float tbest, float &t_entry)
{
    float t_exit;
    return box_hit2(R, lx, hx, ly, hy, lz, hz, tbest, t_entry, t_exit);
}

constexpr int kDone = INT32_MIN;

struct BvhView {
    const BvhNode *nodes;
    const float4 *tris;  // vertices (v0 carrying the original id), leaf order
    const float4 *tmap;  // triangle-space maps, leaf order
};

// One traversal step of one lane: an internal node tests both child boxes
// and descends into the nearer hit child (pushing the farther); a leaf tests
// its triangles; then the lane pops.  `stk` points at the lane's stack slot 0
// in LDS, entries `stride` words apart.
template <bool STATS = false>
__device__ __forceinline__ void trav_step(const BvhView &S, const RaySetup &R, int &node, int &sp, int *stk,
                                          int stride, float &tbest, int &ibest, bool &front, uint32_t *nodes_visited = nullptr,
                                          uint32_t *tris_tested = nullptr)
{
    if (node >= 0) {
        if (STATS) ++*nodes_visited;
        const BvhNode *nd = S.nodes + node;
        const float4 a = nd->xy0, b = nd->xy1, z = nd->z01;
        const int4 m = nd->meta;
        float t0, t1;
        const bool h0 = box_hit(R, a.x, a.y, a.z, a.w, z.x, z.y, tbest, t0);
        const bool h1 = box_hit(R, b.x, b.y, b.z, b.w, z.z, z.w, tbest, t1);
        if (h0 && h1) {
            const bool first0 = t0 <= t1;
            stk[sp * stride] = first0 ? m.y : m.x;
            ++sp;
            node = first0 ? m.x : m.y;
            return;
        }
        if (h0 || h1) {
            node = h0 ? m.x : m.y;
            return;
        }
    } else {
        const int first = leaf_first(node), cnt = leaf_count(node);
        if (STATS) *tris_tested += (uint32_t)cnt;
        for (int i = first; i < first + cnt; ++i) tri_test(R, S.tmap, S.tris, i, tbest, ibest, front);
    }
    node = sp > 0 ? stk[--sp * stride] : kDone;
}

// ------------------------------------------------------ persistent tracer ----

// Everything the tracer needs to know about one scene.
struct TraceScene {
    BvhView bvh;
    const BvhNode *nodes4;  // 4-wide copy (WIDE launches)
    int nt;
    const int32_t *queue;
    const int32_t *count;
    int32_t queue_cap;
    const float *coarse_sdf;
    int nc, logr, nf, lognf;
    float lox, loy, loz, hf;
    int rays;
    uint32_t scene_id;
    float alpha;
    int sign_policy;  // RTSDF_SIGN_VOTE or RTSDF_SIGN_SHELL
    float shell;
    float *u;
    uint32_t *hits;
    int32_t *arg_tri;
    int32_t *arg_ray;
    float *fine;
};

struct TraceArgs {
    TraceScene one;              // the scene of a single-scene launch
    const TraceScene *scenes;    // batched launch: per-scene records ...
    const int32_t *tile_offset;  // ... and the first global tile of each scene ([nscenes + 1])
    int nscenes;
    int32_t *cursor;             // global tile counter
    uint32_t frame;
    const uint32_t *frame_ptr;
    uint64_t seed;
    int32_t *spill;              // deep stack entries: [(depth - SL) * spill_stride + lane]
    int spill_stride;            // lanes in the launch
    int bin_directions;          // sort each tile's rays by direction bin
    int tile_cap;                // texels per wavefront tile at most (16, 32 or 64)
    float4 *dirs;                // per wavefront: kTileRays directions of its current tile
};

constexpr int kTraceWaves = 4;
constexpr int kTileRays = 768;  // rays per wavefront tile
constexpr int kTileTexels = 64;

// frame indices share the argmin record with the ray index (frame << 8 | ray)
constexpr uint32_t kMaxFrame = 1u << 23;

__host__ __device__ __forceinline__ int tile_texels_for(int rays, int cap)
{
    return rays >= kTileRays ? 1 : min(cap, kTileRays / rays);
}

typedef __attribute__((address_space(3))) int lds_int;

__device__ __forceinline__ const BvhNode *node_ptr(const BvhNode *base, int node)
{
    return reinterpret_cast<const BvhNode *>(reinterpret_cast<const char *>(base) + (uint32_t)node * 64u);
}

__device__ __forceinline__ const float4 *tri_ptr(const float4 *base, int tri)
{
    return reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + rec48(tri));
}

template <int SL>
__device__ __forceinline__ void stack_push(int stride, int &sp, lds_int *stk, int32_t *spill, int v)
{
    if (sp < SL) stk[sp * kWave] = v;
    else spill[__umul24((uint32_t)(sp - SL), (uint32_t)stride)] = v;  // stride < 2^24 lanes
    ++sp;
}

template <int SL>
__device__ __forceinline__ int stack_pop(int stride, int &sp, const lds_int *stk, const int32_t *spill)
{
    if (sp == 0) return kDone;
    --sp;
    int v;
    if (sp < SL) v = stk[sp * kWave];
    else v = spill[__umul24((uint32_t)(sp - SL), (uint32_t)stride)];
    return v;
}

// One internal node: test both children's boxes, descend into the nearer hit
// child and push the farther one; pop when neither is hit.
template <int SL, bool STATS>
__device__ __forceinline__ void inner_step(const BvhView &S, int stride, const RaySetup &R, int &node, int &sp,
                                           lds_int *stk, int32_t *spill, float tbest, uint32_t &st_nodes)
{
    if (STATS) ++st_nodes;
    const BvhNode *nd = node_ptr(S.nodes, node);
    const float4 a = nd->xy0, b = nd->xy1, z = nd->z01;
    const int4 m = nd->meta;
    float t0, t1;
    const bool h0 = box_hit(R, a.x, a.y, a.z, a.w, z.x, z.y, tbest, t0);
    const bool h1 = box_hit(R, b.x, b.y, b.z, b.w, z.z, z.w, tbest, t1);
    if (h0 && h1) {
        const bool first0 = t0 <= t1;
        stack_push<SL>(stride, sp, stk, spill, first0 ? m.y : m.x);
        node = first0 ? m.x : m.y;
    } else if (h0 || h1) {
        node = h0 ? m.x : m.y;
    } else {
        node = stack_pop<SL>(stride, sp, stk, spill);
    }
}

// Same, but a leaf child is opened at once (its triangle range becomes the
// lane's current work) instead of costing an iteration of its own.
template <int SL, bool STATS>
__device__ __forceinline__ void node_step(const BvhView &S, int stride, const RaySetup &R, int &node, int &sp,
                                          lds_int *stk, int32_t *spill, float tbest, int &tri_cur, int &tri_end,
                                          uint32_t &st_nodes)
{
    if (STATS) ++st_nodes;
    const BvhNode *nd = node_ptr(S.nodes, node);
    const float4 a = nd->xy0, b = nd->xy1, z = nd->z01;
    const int4 m = nd->meta;
    float t0, t1;
    const bool h0 = box_hit(R, a.x, a.y, a.z, a.w, z.x, z.y, tbest, t0);
    const bool h1 = box_hit(R, b.x, b.y, b.z, b.w, z.z, z.w, tbest, t1);
    if (h0 && h1) {
        const bool first0 = t0 <= t1;
        const int near = first0 ? m.x : m.y, far = first0 ? m.y : m.x;
        if (near < 0) {
            tri_cur = leaf_first(near);
            tri_end = tri_cur + leaf_count(near);
            node = far;
        } else {
            stack_push<SL>(stride, sp, stk, spill, far);
            node = near;
        }
    } else if (h0 || h1) {
        const int c = h0 ? m.x : m.y;
        if (c < 0) {
            tri_cur = leaf_first(c);
            tri_end = tri_cur + leaf_count(c);
            node = stack_pop<SL>(stride, sp, stk, spill);
        } else {
            node = c;
        }
    } else {
        node = stack_pop<SL>(stride, sp, stk, spill);
    }
}

// One 4-wide node (two records: children 0, 1 in a, b, z, m and 2, 3 in a2,
// b2, z2, m2): test the four boxes, order the hit children by entry
// distance (a five-comparator sorting network), go to the nearest (a leaf
// becomes the triangle range at once, the next nearest child is then next)
// and request pushes of the other hit children, farthest first.
__device__ __forceinline__ void swap_if_greater(float &ta, int &ca, float &tb, int &cb)
{
    const bool sw = ta > tb;
    const float t = sw ? tb : ta;
    tb = sw ? ta : tb;
    ta = t;
    const int c = sw ? cb : ca;
    cb = sw ? ca : cb;
    ca = c;
}

__device__ __forceinline__ void node4_step_regs(const RaySetup &R, float4 a, float4 b, float4 z, int2 m, float4 a2,
                                                float4 b2, float4 z2, int2 m2, int &node, float tbest, int &tri_cur,
                                                int &tri_end, bool &p1, bool &p2, bool &p3, int &v1, int &v2, int &v3,
                                                bool &pop)
{
    const float inf = __builtin_inff();
    float t0, t1, t2, t3;
    const bool h0 = box_hit(R, a.x, a.y, a.z, a.w, z.x, z.y, tbest, t0);
    const bool h1 = box_hit(R, b.x, b.y, b.z, b.w, z.z, z.w, tbest, t1);
    const bool h2 = box_hit(R, a2.x, a2.y, a2.z, a2.w, z2.x, z2.y, tbest, t2);
    const bool h3 = box_hit(R, b2.x, b2.y, b2.z, b2.w, z2.z, z2.w, tbest, t3);
    float e0 = h0 ? t0 : inf, e1 = h1 ? t1 : inf, e2 = h2 ? t2 : inf, e3 = h3 ? t3 : inf;
    int c0 = m.x, c1 = m.y, c2 = m2.x, c3 = m2.y;
    swap_if_greater(e0, c0, e1, c1);
    swap_if_greater(e2, c2, e3, c3);
    swap_if_greater(e0, c0, e2, c2);
    swap_if_greater(e1, c1, e3, c3);
    swap_if_greater(e1, c1, e2, c2);
    const bool any = e0 < inf;
    const bool leaf0 = any && c0 < 0;
    if (leaf0) {
        tri_cur = leaf_first(c0);
        tri_end = tri_cur + leaf_count(c0);
    }
    node = leaf0 ? c1 : c0;
    pop = !any || (leaf0 && !(e1 < inf));
    p3 = e3 < inf;
    p2 = e2 < inf;
    p1 = e1 < inf && !leaf0;
    v1 = c1;
    v2 = c2;
    v3 = c3;
}

// Lanes whose ray is finished (or that have none): a ballot of each compare, combined on the scalar unit (a
// ballot of the combined condition would first be materialised lane by lane).
__device__ __forceinline__ uint64_t wave_done(bool busy, int node, int tri_cur, int tri_end)
{
    return ~__builtin_amdgcn_ballot_w64(busy) |
           (__builtin_amdgcn_ballot_w64(node == kDone) & __builtin_amdgcn_ballot_w64(tri_cur >= tri_end));
}

// Same decisions as node_step, written as selects: the caller performs the
// (at most one) push and the (at most one) pop after the lane's work of the
// iteration, so every lane shares one copy of the stack code.
__device__ __forceinline__ void node_decide(bool h0, bool h1, bool first0, int4 m, int &node, int &tri_cur,
                                            int &tri_end, bool &push, int &push_val, bool &pop)
{
    const bool any = h0 || h1, both = h0 && h1;
    const int near = first0 ? m.x : m.y, far = first0 ? m.y : m.x;
    const bool near_leaf = any && near < 0;
    // a leaf child's triangles become the lane's range; otherwise the range is left empty (the lane is idle,
    // so its range is empty already)
    tri_cur = leaf_first(near);
    tri_end = tri_cur + (near_leaf ? leaf_count(near) : 0);
    // next: the nearer internal child; after a leaf child, the other hit child; else pop
    push = both && !near_leaf;
    push_val = far;
    pop = !any || (near_leaf && !both);
    node = near_leaf ? far : near;
}

__device__ __forceinline__ void node_step_regs(const RaySetup &R, float4 a, float4 b, float4 z, int4 m, int &node,
                                               float tbest, int &tri_cur, int &tri_end, bool &push, int &push_val,
                                               bool &pop)
{
    float t0, t1, e0, e1;
    const bool h0 = box_hit2(R, a.x, a.y, a.z, a.w, z.x, z.y, tbest, t0, e0);
    const bool h1 = box_hit2(R, b.x, b.y, b.z, b.w, z.z, z.w, tbest, t1, e1);
    // the nearer entry first; equal entries (the origin inside both boxes): the child the ray leaves first
    // (bitwise, so the compiler keeps it branch-free)
    const bool second = h1 & ((t1 < t0) | ((t1 == t0) & (e1 < e0)));
    node_decide(h0, h1, h0 & !second, m, node, tri_cur, tri_end, push, push_val, pop);
}

__device__ __forceinline__ void node_step_flat(const BvhView &S, const RaySetup &R, int &node, float tbest,
                                               int &tri_cur, int &tri_end, bool &push, int &push_val, bool &pop)
{
    const BvhNode *nd = node_ptr(S.nodes, node);
    node_step_regs(R, nd->xy0, nd->xy1, nd->z01, nd->meta, node, tbest, tri_cur, tri_end, push, push_val, pop);
}

// Octahedral direction bin (8 x 8 cells of the octahedral map, numbered in
// Morton order so consecutive bins are neighbours on the sphere).
constexpr int kBins = 64;
__device__ __forceinline__ int direction_bin(float3 d)
{
    const float s = fabsf(d.x) + fabsf(d.y) + fabsf(d.z);
    float u = d.x / s, v = d.y / s;
    if (d.z < 0.0f) {
        const float uu = (1.0f - fabsf(v)) * (u >= 0.0f ? 1.0f : -1.0f);
        const float vv = (1.0f - fabsf(u)) * (v >= 0.0f ? 1.0f : -1.0f);
        u = uu;
        v = vv;
    }
    const int bu = min(7, max(0, (int)((u + 1.0f) * 4.0f)));
    const int bv = min(7, max(0, (int)((v + 1.0f) * 4.0f)));
    return (bu & 1) | ((bv & 1) << 1) | ((bu & 2) << 1) | ((bv & 2) << 2) | ((bu & 4) << 2) | ((bv & 4) << 3);
}

// queued loop: triangle tests queued per wavefront (a power of two, at least two wavefronts' worth)
constexpr int kQueueCap = 128;
constexpr unsigned long long kBestInit = 0x7F800000FFFFFFFFull;  // t = +inf, no triangle
constexpr int kMaxQueuedRefs = 1 << 26;  // queue entries: leaf-order index << 6 | lane
static_assert(2 * kWave <= kQueueCap && (kQueueCap & (kQueueCap - 1)) == 0, "queue size");
static_assert(kBins <= kQueueCap, "the bin counters share the queue's words");

// A wavefront's LDS: the texel results of two tile contexts (the tile whose rays are handed out and the one
// before it, whose last rays may still be in flight; context c holds entries c * kTileTexels + slot), each
// lane's best hit key (queued loop) and the triangle-test queue, whose words hold the direction-bin counters
// while a tile's rays are sorted (the queue is empty then).
struct WaveTile {
    int32_t tex[2 * kTileTexels];
    unsigned long long key[2 * kTileTexels];  // min over rays of (distance bits << 32 | ray << 26 | triangle)
    uint32_t cnt[2 * kTileTexels];            // front | back << 16 for this frame
    unsigned long long best[kWave];  // each lane's ray: min of (t bits << 32 | triangle id << 1 | front)
    union {
        uint32_t q[kQueueCap];       // queued triangle tests: leaf-order index << 6 | lane of the ray
        uint32_t bin[kBins];         // bin counts, then bin cursors
    };
};

// Tiles of a scene: ceil(min(count, cap) / tile texels).
__device__ __forceinline__ int scene_tiles(const TraceScene &P, int cap)
{
    const int total = min(*P.count, P.queue_cap);
    const int tt = tile_texels_for(P.rays, cap);
    return total > 0 ? (total + tt - 1) / tt : 0;
}

// Global tile prefix of a batch: tile_offset[s] = sum of tiles of scenes < s.
__global__ void trace_tile_prefix(const TraceScene *scenes, int n, int cap, int32_t *tile_offset)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int acc = 0;
    for (int s = 0; s < n; ++s) {
        tile_offset[s] = acc;
        acc += scene_tiles(scenes[s], cap);
    }
    tile_offset[n] = acc;
}

// Persistent tracer.  Each wavefront repeatedly takes a tile of up to 64
// consecutive queue texels of one scene (Morton order: a compact block of the
// fine grid), draws all their rays' directions, sorts the rays by direction
// bin, and traces them in that order, so the lanes of a wavefront follow rays
// that start close together and point the same way.  Results are folded per
// texel with LDS atomics (a 64-bit min keeps the smallest distance, ties to
// the lowest ray index, together with its triangle; an add counts front and
// back hits), which makes them independent of the order rays complete in.  A
// wavefront holds two tile contexts: once its tile has handed out its last
// ray, it sorts the next tile's rays into the other context and refills its
// lanes from there while the first tile's last rays are still traced (a
// tile's Eq. (1) epilogue runs once its last ray is done), so lanes do not
// wait for the slowest ray of each tile.  Two-level scenes, and a next tile
// of another scene in a batch, start only once every lane is done (a part's
// exit re-reads its ray's direction by ray id; the traversal takes the
// scene's hierarchy as a wave-uniform value).
// Loop shapes (LOOP): 0 = phases per iteration
// (after Aila and Laine's "while-while" loop with postponed leaves: every lane
// walks internal nodes until it holds a leaf, then all held leaves are
// tested); 1 = one unit of work per lane per iteration (a triangle of the
// current leaf, else a node, else opening a popped leaf), which keeps more
// lanes busy on wave64; 2 = as 1, but each lane only requests its stack
// push/pop and one shared copy of the stack code runs after the work; 3 =
// as 2, but every lane fetches its node or its triangle's map into the same
// registers with one shared load sequence, so an iteration waits for memory
// once instead of once per kind of work; 4 = queued triangle tests (below).
// BATCHED launches serve many scenes: a global tile
// index is mapped to its scene through the tile prefix.  Instrumented runs
// (STATS) also count into 64-bit counters at workspace offsets 8, 16, ...:
// node visits, triangle tests, rays, traversal-loop iterations x 64, refill
// rounds x 64, lane-iterations with work (LOOP 1 and 2), tiles x 64, node
// visits that entered neither child box (LOOP 3), tiles started while lanes
// were still busy x 64, traversal rounds that waited for every lane before a
// next tile x 64.
template <int SL, int REFILL, int LOOP, bool STATS, bool BATCHED, bool INST = false, bool WIDE = false>
__global__ void __launch_bounds__(kTraceWaves * kWave) __attribute__((amdgpu_waves_per_eu(6, 8)))
trace_persistent(TraceArgs A)
{
    uint32_t st_nodes = 0, st_tris = 0, st_rays = 0, st_iters = 0, st_refills = 0, st_busy = 0, st_tiles = 0;
    uint32_t st_empty = 0, st_early = 0, st_drains = 0;
    __shared__ int stack_mem[kTraceWaves * SL * kWave];
    __shared__ WaveTile tiles[kTraceWaves];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    lds_int *stk = (lds_int *)(stack_mem + wave * SL * kWave + lane);
    WaveTile &T = tiles[wave];
    int32_t *spill = A.spill + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the wavefront's two direction buffers: by ray id (slot * R + ray), and the same rays in bin order as
    // (direction, ray id) records
    float4 *dirs = A.dirs + ((int64_t)blockIdx.x * kTraceWaves + wave) * (2 * kTileRays);
    float4 *recs = dirs + kTileRays;
    const int stride = A.spill_stride;
    const uint32_t frame = A.frame_ptr ? *A.frame_ptr : A.frame;
    if (frame >= kMaxFrame) {
        // a device frame counter past the argmin record's range: trace nothing (the state keeps the
        // previous frame's values) and report it
        if (blockIdx.x == 0 && threadIdx.x == 0) raise_error(RTSDF_ERR_FRAME);
        return;
    }
    const int single_tiles = BATCHED ? 0 : scene_tiles(A.one, A.tile_cap);
    const int all_tiles = BATCHED ? A.tile_offset[A.nscenes] : single_tiles;
    const auto scene_of = [&](int g) {  // last scene whose first tile is <= g
        int lo = 0, hi = A.nscenes - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.tile_offset[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        return __builtin_amdgcn_readfirstlane(lo);
    };

    // wave-uniform context state: -1 free, else rays not yet finished | texels << 16; and the scene (batches)
    int cstate[2] = {-1, -1}, cscene[2] = {0, 0};
    int cur = 0, pool = 0, nrays = 0;  // the context rays are handed out from
    uint32_t rdiv = 0;                 // its q / R multiplier (below)
    int gnext = -2;                    // the next tile: -2 not taken yet, -1 none left
    // lane state
    bool busy = false;
    int rid = 0;  // the lane's ray: (context * kTileTexels + texel slot) << 6 | ray index
    RaySetup Rs;
    float tbest = __builtin_inff();
    int ibest = -1, node = kDone, leaf = kDone, sp = 0;
    int tri_cur = 0, tri_end = 0;
    bool front = false;

    while (true) {
        // ---- start the next tile once the current one has handed out its last ray
        const bool any_busy = __builtin_amdgcn_ballot_w64(busy) != 0;
        if (pool >= nrays && cstate[cur ^ 1] < 0 && gnext != -1) {
            if (gnext == -2) {
                int g = 0;
                if (lane == 0) g = atomicAdd(A.cursor, 1);
                g = __builtin_amdgcn_readlane(g, 0);  // a wave-uniform (scalar) value
                gnext = g < all_tiles ? g : -1;
            }
            const int sn = gnext >= 0 && BATCHED ? scene_of(gnext) : 0;
            if (gnext >= 0 && (!any_busy || (!INST && (!BATCHED || sn == cscene[cur])))) {
                const int c = cur ^ 1, g = gnext;
                gnext = -2;
                const TraceScene &P = BATCHED ? A.scenes[sn] : A.one;
                if (STATS) {
                    ++st_tiles;
                    st_early += any_busy;
                }
                const int R = P.rays;
                // q / R as a multiply-high: exact for q < kTileRays and R <= 64 (the error of the rounded-up
                // reciprocal, q / 2^32, stays below the distance 1/R of q / R from the next integer)
                rdiv = R > 1 ? (uint32_t)(((1ull << 32) + (uint64_t)R - 1) / (uint64_t)R) : 0u;
                const int tile_texels = tile_texels_for(R, A.tile_cap);
                const int total = min(*P.count, P.queue_cap);
                const int base = (g - (BATCHED ? A.tile_offset[sn] : 0)) * tile_texels;
                const int nt = min(tile_texels, total - base);
                const uint64_t ntex_grid = (uint64_t)1 << (3 * P.lognf);
                const int c0 = c * kTileTexels;
                if (lane < nt) {
                    int j = P.queue[base + lane];
                    if (j < 0 || (uint64_t)j >= ntex_grid) j = -1;
                    T.tex[c0 + lane] = j;
                    T.key[c0 + lane] = ~0ull;
                    T.cnt[c0 + lane] = 0u;
                }
                T.bin[lane] = 0u;  // the queue is empty between traversal rounds
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                // ---- bin the tile's rays by direction (the bin rides in the direction record's w)
                nrays = nt * R;
#pragma unroll 1
                for (int q = lane; q < nrays; q += kWave) {
                    const int qs = R > 1 ? (int)__umulhi((uint32_t)q, rdiv) : q, qr = q - qs * R;
                    const int j = T.tex[c0 + qs];
                    int b = 0;
                    if (j >= 0) {
                        // drawn once at full width; the lane that later takes the ray reads it back
                        const float3 d = sphere_dir(A.seed, (uint32_t)j, frame, (uint32_t)qr, P.scene_id);
                        if (A.bin_directions) b = direction_bin(d);
                        dirs[q] = make_float4(d.x, d.y, d.z, __int_as_float(b));
                    }
                    atomicAdd(&T.bin[b], 1u);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
                {  // exclusive scan of the 64 bin counts, one per lane
                    const uint32_t cb = T.bin[lane];
                    uint32_t x = cb;
#pragma unroll
                    for (int off = 1; off < kWave; off <<= 1) {
                        const uint32_t y = __shfl_up(x, off);
                        if (lane >= off) x += y;
                    }
                    T.bin[lane] = x - cb;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
                // ---- the records in bin order (each lane re-reads the directions it stored)
#pragma unroll 1
                for (int q = lane; q < nrays; q += kWave) {
                    const int qs = R > 1 ? (int)__umulhi((uint32_t)q, rdiv) : q;
                    float4 d = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (T.tex[c0 + qs] >= 0) d = dirs[q];
                    const uint32_t pos = atomicAdd(&T.bin[__float_as_int(d.w)], 1u);
                    recs[pos] = make_float4(d.x, d.y, d.z, __int_as_float(q));
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");  // also orders the stored records
                __builtin_amdgcn_wave_barrier();
                cstate[c] = nrays | nt << 16;
                cscene[c] = sn;
                cur = c;
                pool = 0;
            }
        }

        // ---- refill idle lanes from the current tile, in bin order
        const TraceScene &P = BATCHED ? A.scenes[cscene[cur]] : A.one;
        const int R = P.rays;
        const int nfm = P.nf - 1;
        const BvhView S = P.bvh;
        const int scene_nt = P.nt;
        {
            const uint64_t need = __builtin_amdgcn_ballot_w64(!busy);
            if (need != 0 && pool < nrays) {
                if (STATS) ++st_refills;
                const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
                const int take = min(__popcll(need), nrays - pool);
                if (!busy && rank < take) {
                    const float4 d = recs[pool + rank];
                    const int q = __float_as_int(d.w);
                    const int qs = R > 1 ? (int)__umulhi((uint32_t)q, rdiv) : q;
                    rid = (cur * kTileTexels + qs) << 6 | (q - qs * R);
                    const int j = T.tex[cur * kTileTexels + qs];
                    if (j >= 0) {
                        const float ox = texel_coord(P.lox, j & nfm, P.hf);
                        const float oy = texel_coord(P.loy, (j >> P.lognf) & nfm, P.hf);
                        const float oz = texel_coord(P.loz, j >> (2 * P.lognf), P.hf);
                        ray_setup(ox, oy, oz, d.x, d.y, d.z, Rs);
                        node = scene_nt > 0 ? 0 : kDone;
                    } else {
                        node = kDone;
                    }
                    tbest = __builtin_inff();
                    ibest = -1;
                    front = false;
                    if (LOOP == 4) T.best[lane] = kBestInit;
                    leaf = kDone;
                    tri_cur = tri_end = 0;
                    sp = 0;
                    busy = true;
                }
                pool += take;
            }
        }
        if (__builtin_amdgcn_ballot_w64(busy) == 0) {
            // every context is finished (a context's epilogue runs when its last ray is done)
            if (pool >= nrays && gnext == -1) break;
            continue;
        }
        {
            // refill rounds go on while this tile has rays or the next one can start before every lane is
            // done; otherwise every lane finishes first
            const bool early = !INST && cstate[cur ^ 1] < 0 &&
                               (gnext == -2 || (gnext >= 0 && (!BATCHED || scene_of(gnext) == cscene[cur])));
            const int refill_at = __builtin_amdgcn_readfirstlane(pool < nrays || early ? REFILL : kWave);
            if (STATS) st_drains += refill_at == kWave && gnext != -1;  // every lane finishes before the next tile
            if (LOOP == 0) {
                while (true) {
                    if (busy && leaf == kDone && node < 0 && node != kDone) {
                        leaf = node;
                        node = stack_pop<SL>(stride, sp, stk, spill);
                    }
                    // phase 1: internal nodes until every busy lane holds a leaf or is done
                    while (__ballot(busy && node >= 0 && leaf == kDone)) {
                        if (busy && node >= 0) {
                            inner_step<SL, STATS>(S, stride, Rs, node, sp, stk, spill, tbest, st_nodes);
                            if (node < 0 && node != kDone && leaf == kDone) {
                                leaf = node;
                                node = stack_pop<SL>(stride, sp, stk, spill);
                            }
                        }
                    }
                    // phase 2: triangles of the held leaves
                    if (busy && leaf != kDone) {
                        const int first = leaf_first(leaf), cnt = leaf_count(leaf);
                        if (STATS) st_tris += (uint32_t)cnt;
                        for (int i = first; i < first + cnt; ++i) {
                            tri_test(Rs, S.tmap, S.tris, i, tbest, ibest, front);
                        }
                        leaf = kDone;
                    }
                    const uint64_t done = __ballot(!busy || (node == kDone && leaf == kDone));
                    if (__popcll(done) >= refill_at) break;
                }
            } else if (LOOP == 3) {
                while (true) {
                    if (STATS) {
                        ++st_iters;
                        st_busy += busy && (node != kDone || tri_cur < tri_end);
                    }
                    // one fetch per lane and iteration: the triangle's map or the node, into the same
                    // registers, so the wavefront waits for memory once whichever work its lanes do
                    const bool do_tri = busy && tri_cur < tri_end;
                    const bool do_node = busy && !do_tri && node >= 0;
                    // (lanes with neither load the root node, which every scene allocates, and ignore it)
                    const char *base =
                        do_tri ? reinterpret_cast<const char *>(S.tmap) + rec48(tri_cur)
                               : WIDE ? reinterpret_cast<const char *>(P.nodes4) + (uint32_t)(do_node ? node : 0) * 128u
                                      : reinterpret_cast<const char *>(S.nodes) + (uint32_t)(do_node ? node : 0) * 64u;
                    const float4 *q = reinterpret_cast<const float4 *>(base);
                    const float4 w0 = q[0], w1 = q[1], w2 = q[2];
                    const int2 w3 = *reinterpret_cast<const int2 *>(q + 3);  // the map array has 16 B of padding
                    // a wide node's second record (other lanes re-read their first 64 bytes)
                    float4 w4, w5, w6;
                    int2 w7;
                    if (WIDE) {
                        const float4 *q2 = do_node ? q + 4 : q;
                        w4 = q2[0];
                        w5 = q2[1];
                        w6 = q2[2];
                        w7 = *reinterpret_cast<const int2 *>(q2 + 3);
                    }
                    bool push = false, pop = false;
                    int push_val = 0;
                    bool p1 = false, p2 = false, p3 = false;
                    int v1 = 0, v2 = 0, v3 = 0;
                    if (do_tri) {
                        if (STATS) ++st_tris;
                        tri_test_rows(Rs, w0, w1, w2, S.tris, tri_cur, tbest, ibest, front);
                        ++tri_cur;
                    } else if (do_node) {
                        if (STATS) ++st_nodes;
                        if (INST && w3.y == kInstTag) {
                            // instance node of a two-level scene: its rows take the (world) ray into the
                            // part's object space; the return marker restores it
                            const float ox = w0.x * Rs.ox + w0.y * Rs.oy + w0.z * Rs.oz + w0.w;
                            const float oy = w1.x * Rs.ox + w1.y * Rs.oy + w1.z * Rs.oz + w1.w;
                            const float oz = w2.x * Rs.ox + w2.y * Rs.oy + w2.z * Rs.oz + w2.w;
                            const float dx = w0.x * Rs.dx + w0.y * Rs.dy + w0.z * Rs.dz;
                            const float dy = w1.x * Rs.dx + w1.y * Rs.dy + w1.z * Rs.dz;
                            const float dz = w2.x * Rs.dx + w2.y * Rs.dy + w2.z * Rs.dz;
                            ray_setup(ox, oy, oz, dx, dy, dz, Rs);
                            push = true;
                            push_val = kReturn;
                            node = w3.x;
                        } else if (WIDE) {
                            node4_step_regs(Rs, w0, w1, w2, w3, w4, w5, w6, w7, node, tbest, tri_cur, tri_end, p1, p2,
                                            p3, v1, v2, v3, pop);
                            if (STATS) st_empty += pop && tri_cur >= tri_end;  // no child box was entered
                        } else {
                            const int4 m = make_int4(w3.x, w3.y, 0, 0);
                            node_step_regs(Rs, w0, w1, w2, m, node, tbest, tri_cur, tri_end, push, push_val, pop);
                            if (STATS) st_empty += pop && tri_cur >= tri_end;  // neither child box was entered
                        }
                    } else if (INST && busy && node == kReturn) {
                        // the part is done (its last leaf's triangles too): the world ray again, as drawn
                        const int j = T.tex[rid >> 6];
                        const float4 d = dirs[((rid >> 6) & (kTileTexels - 1)) * R + (rid & 63)];
                        ray_setup(texel_coord(P.lox, j & nfm, P.hf), texel_coord(P.loy, (j >> P.lognf) & nfm, P.hf),
                                  texel_coord(P.loz, j >> (2 * P.lognf), P.hf), d.x, d.y, d.z, Rs);
                        pop = true;
                    } else if (busy && node != kDone) {
                        tri_cur = leaf_first(node);
                        tri_end = tri_cur + leaf_count(node);
                        pop = true;
                    }
                    if (WIDE) {  // farthest first, so the nearest is popped first
                        if (p3) stack_push<SL>(stride, sp, stk, spill, v3);
                        if (p2) stack_push<SL>(stride, sp, stk, spill, v2);
                        if (p1) stack_push<SL>(stride, sp, stk, spill, v1);
                    }
                    if (push) stack_push<SL>(stride, sp, stk, spill, push_val);
                    if (pop) node = stack_pop<SL>(stride, sp, stk, spill);
                    const uint64_t done = wave_done(busy, node, tri_cur, tri_end);
                    if (__popcll(done) >= refill_at) break;
                }
            } else if (LOOP == 4) {
                // Queued loop: a lane that reaches a leaf appends its triangles to the wavefront's queue
                // in LDS (two per iteration at most) and goes on with its traversal; once a wavefront's
                // worth of tests is queued, every lane takes one, whichever ray it belongs to, so the
                // triangle code runs at full width instead of in nearly every iteration for a few lanes.
                // Between flushes a lane culls boxes against its ray's best distance as of the last flush
                // (a larger bound only enters more boxes); the closest hit is the minimum of the
                // (t, triangle id, facing) keys of all tests, as in the other loops.
                int qh = 0, qt = 0;  // wave-uniform head and tail (entries at index & (kQueueCap - 1))
                const auto flush = [&](int nf) {
                    const bool act = lane < nf;
                    const uint32_t e = act ? T.q[(qh + lane) & (kQueueCap - 1)] : (uint32_t)lane;
                    const int owner = (int)(e & 63u), addr = owner << 2;
                    // the owner's ray, from its registers (every lane takes part in the permutes)
                    const float ox = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(Rs.ox)));
                    const float oy = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(Rs.oy)));
                    const float oz = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(Rs.oz)));
                    const float dx = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(Rs.dx)));
                    const float dy = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(Rs.dy)));
                    const float dz = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(Rs.dz)));
                    const float tb = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(tbest)));
                    if (act) {
                        if (STATS) ++st_tris;
                        const int i = (int)(e >> 6);
                        const float4 *mp = tri_ptr(S.tmap, i);
                        float t;
                        bool fr;
                        if (tri_hit_rows(ox, oy, oz, dx, dy, dz, mp[0], mp[1], mp[2], S.tris, i, tb, t, fr)) {
                            const unsigned long long key = ((unsigned long long)__float_as_uint(t) << 32) |
                                                           ((uint32_t)tri_id(S.tris, i) << 1) | (fr ? 1u : 0u);
                            atomicMin(&T.best[owner], key);
                        }
                    }
                    qh += nf;
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    tbest = __uint_as_float((uint32_t)(T.best[lane] >> 32));
                };
                while (true) {
                    if (STATS) {
                        ++st_iters;
                        st_busy += busy && (node != kDone || tri_cur < tri_end);
                    }
                    // ---- append up to two of the lane's pending triangles, as far as the queue has room
                    // (lanes without a ray hold an empty range)
                    const int c = min(tri_end - tri_cur, 2);
                    const uint64_t b1 = __builtin_amdgcn_ballot_w64(c >= 1), b2 = __builtin_amdgcn_ballot_w64(c >= 2);
                    // the lane's position: the requests of the lanes below it
                    const int pos = (int)__builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(b2 >> 32),
                        __builtin_amdgcn_mbcnt_lo(
                            (uint32_t)b2, __builtin_amdgcn_mbcnt_hi((uint32_t)(b1 >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)b1, 0u))));
                    int total = (int)(__popcll(b1) + __popcll(b2)), g = c;
                    if (qt - qh + total > kQueueCap) {  // rare: grant a prefix of the lanes
                        g = pos + c <= kQueueCap - (qt - qh) ? c : 0;
                        total = (int)(__popcll(__builtin_amdgcn_ballot_w64(g >= 1)) + __popcll(__builtin_amdgcn_ballot_w64(g >= 2)));
                    }
                    if (g > 0) {
                        const uint32_t e = ((uint32_t)tri_cur << 6) | (uint32_t)lane;
                        T.q[(qt + pos) & (kQueueCap - 1)] = e;
                        if (g > 1) T.q[(qt + pos + 1) & (kQueueCap - 1)] = e + 64u;
                        tri_cur += g;
                    }
                    qt += total;
                    // ---- the lane's traversal step: a node, or opening a popped leaf
                    const bool idle = busy && tri_cur >= tri_end;
                    const bool do_node = idle && node >= 0;
                    const float4 *q = reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(S.nodes) +
                                                                       (uint32_t)(do_node ? node : 0) * 64u);
                    const float4 w0 = q[0], w1 = q[1], w2 = q[2];
                    const int2 w3 = *reinterpret_cast<const int2 *>(q + 3);
                    bool push = false, pop = false;
                    int push_val = 0;
                    if (do_node) {
                        if (STATS) ++st_nodes;
                        const int4 m = make_int4(w3.x, w3.y, 0, 0);
                        node_step_regs(Rs, w0, w1, w2, m, node, tbest, tri_cur, tri_end, push, push_val, pop);
                        if (STATS) st_empty += pop && tri_cur >= tri_end;
                    } else if (idle && node != kDone) {
                        tri_cur = leaf_first(node);
                        tri_end = tri_cur + leaf_count(node);
                        pop = true;
                    }
                    if (push) stack_push<SL>(stride, sp, stk, spill, push_val);
                    if (pop) node = stack_pop<SL>(stride, sp, stk, spill);
                    // ---- a wavefront's worth of tests
                    if (qt - qh >= kWave) flush(kWave);
                    const uint64_t done = wave_done(busy, node, tri_cur, tri_end);
                    if (__popcll(done) >= refill_at) break;
                }
                // the rest of the queue (the finished rays' tests among them)
                while (qt - qh > 0) flush(min(qt - qh, kWave));
            } else if (LOOP == 2) {
                while (true) {
                    if (STATS) {
                        ++st_iters;
                        st_busy += busy && (node != kDone || tri_cur < tri_end);
                    }
                    bool push = false, pop = false;
                    int push_val = 0;
                    if (busy) {
                        if (tri_cur < tri_end) {
                            if (STATS) ++st_tris;
                            tri_test(Rs, S.tmap, S.tris, tri_cur, tbest, ibest, front);
                            ++tri_cur;
                        } else if (node >= 0) {
                            if (STATS) ++st_nodes;
                            node_step_flat(S, Rs, node, tbest, tri_cur, tri_end, push, push_val, pop);
                        } else if (node != kDone) {
                            tri_cur = leaf_first(node);
                            tri_end = tri_cur + leaf_count(node);
                            pop = true;
                        }
                    }
                    if (push) stack_push<SL>(stride, sp, stk, spill, push_val);
                    if (pop) node = stack_pop<SL>(stride, sp, stk, spill);
                    const uint64_t done = wave_done(busy, node, tri_cur, tri_end);
                    if (__popcll(done) >= refill_at) break;
                }
            } else {
                while (true) {
                    if (STATS) {
                        ++st_iters;
                        st_busy += busy && (node != kDone || tri_cur < tri_end);
                    }
                    if (busy) {
                        if (tri_cur < tri_end) {
                            if (STATS) ++st_tris;
                            tri_test(Rs, S.tmap, S.tris, tri_cur, tbest, ibest, front);
                            ++tri_cur;
                        } else if (node >= 0) {
                            node_step<SL, STATS>(S, stride, Rs, node, sp, stk, spill, tbest, tri_cur, tri_end,
                                                 st_nodes);
                        } else if (node != kDone) {
                            tri_cur = leaf_first(node);
                            tri_end = tri_cur + leaf_count(node);
                            node = stack_pop<SL>(stride, sp, stk, spill);
                        }
                    }
                    const uint64_t done = wave_done(busy, node, tri_cur, tri_end);
                    if (__popcll(done) >= refill_at) break;
                }
            }
            const bool fin = busy && node == kDone && leaf == kDone && tri_cur >= tri_end;
            if (fin) {
                if (STATS) ++st_rays;
                int id = -1;
                if (LOOP == 4) {
                    const unsigned long long kb = T.best[lane];
                    if (kb != kBestInit) {
                        tbest = __uint_as_float((uint32_t)(kb >> 32));
                        id = (int)((uint32_t)kb >> 1);
                        front = (kb & 1u) != 0u;
                    }
                } else if (ibest >= 0) {
                    id = tri_id(S.tris, ibest);
                }
                if (id >= 0) {
                    const float dist = tbest * ray_len(Rs);
                    const unsigned long long key = ((unsigned long long)__float_as_uint(dist) << 32) |
                                                   ((unsigned long long)(rid & 63) << 26) | (unsigned long long)id;
                    atomicMin(&T.key[rid >> 6], key);
                    atomicAdd(&T.cnt[rid >> 6], front ? 1u : 0x10000u);
                }
                busy = false;
            }
            const uint64_t fin1 = __builtin_amdgcn_ballot_w64(fin && rid >= (kTileTexels << 6));
            cstate[0] -= (int)__popcll(__builtin_amdgcn_ballot_w64(fin) & ~fin1);
            cstate[1] -= (int)__popcll(fin1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();

        // ---- Eq. (1) on the unsigned state, then the sign vote, for each tile whose last ray is done
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (cstate[c] < 0 || (cstate[c] & 0xFFFF) > 0) continue;
            const int nt = cstate[c] >> 16, e = c * kTileTexels + lane;
            cstate[c] = -1;
            const TraceScene &Q = BATCHED ? A.scenes[cscene[c]] : A.one;
            if (lane < nt && T.tex[e] >= 0) {
                const int j = T.tex[e];
                const unsigned long long key = T.key[e];
                const uint32_t fc = T.cnt[e];
                const float rmin = key == ~0ull ? __builtin_inff() : __uint_as_float((uint32_t)(key >> 32));
                const int argray = (int)((key >> 26) & 63u), argtri = (int)(key & ((1u << 26) - 1u));
                const int qm = Q.nf - 1;
                const int x = j & qm, y = (j >> Q.lognf) & qm, z = j >> (2 * Q.lognf);
                const float cs = Q.coarse_sdf[(x >> Q.logr) + Q.nc * ((y >> Q.logr) + Q.nc * (z >> Q.logr))];
                const float uprev = Q.u[j];
                const uint32_t h = Q.hits[j];
                const uint32_t F = min((h & 0xFFFFu) + (fc & 0xFFFFu), 0xFFFFu);
                const uint32_t B = min((h >> 16) + (fc >> 16), 0xFFFFu);
                float uu;
                if (Q.alpha == 1.0f) {
                    uu = uprev;
                } else {
                    // alpha = 0: no memory, the alpha u term is 0 even before the first hit (u = +inf)
                    uu = Q.alpha == 0.0f ? fmaxf(cs, 0.0f) : Q.alpha * uprev + (1.0f - Q.alpha) * fmaxf(cs, 0.0f);
                }
                if (rmin < uu) {
                    uu = rmin;
                    Q.arg_tri[j] = argtri;
                    Q.arg_ray[j] = (int32_t)((frame << 8) | (uint32_t)argray);
                } else if (Q.alpha != 1.0f) {
                    Q.arg_tri[j] = -1;
                    Q.arg_ray[j] = -1;
                }
                Q.u[j] = uu;
                Q.hits[j] = F | (B << 16);
                if (isinf(uu)) Q.fine[j] = cs;
                else if (Q.sign_policy == RTSDF_SIGN_SHELL) Q.fine[j] = uu - Q.shell;
                else Q.fine[j] = B > F ? -uu : uu;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (STATS) {
        unsigned long long *ctr = reinterpret_cast<unsigned long long *>(A.cursor + 2);
        atomicAdd(&ctr[0], (unsigned long long)st_nodes);
        atomicAdd(&ctr[1], (unsigned long long)st_tris);
        atomicAdd(&ctr[2], (unsigned long long)st_rays);
        atomicAdd(&ctr[3], (unsigned long long)st_iters);
        atomicAdd(&ctr[4], (unsigned long long)st_refills);
        atomicAdd(&ctr[5], (unsigned long long)st_busy);
        atomicAdd(&ctr[6], (unsigned long long)st_tiles);
        atomicAdd(&ctr[7], (unsigned long long)st_empty);
        atomicAdd(&ctr[8], (unsigned long long)st_early);
        atomicAdd(&ctr[9], (unsigned long long)st_drains);
    }
}

// Unselected texels: fine = coarse value, state reset (Eq. (1), case c > d).
__device__ __forceinline__ void fill_unselected_body(const uint8_t *__restrict__ mask,
                                                     const float *__restrict__ coarse_sdf, int nc, int logr, int lognf,
                                                     int64_t ntex, float *__restrict__ u, uint32_t *__restrict__ hits,
                                                     int32_t *__restrict__ arg_tri, int32_t *__restrict__ arg_ray,
                                                     float *__restrict__ fine, int64_t j)
{
    if (j >= ntex || mask[j]) return;
    const int nfm = (1 << lognf) - 1;
    const int x = (int)(j & nfm), y = (int)((j >> lognf) & nfm), z = (int)(j >> (2 * lognf));
    fine[j] = coarse_sdf[(x >> logr) + nc * ((y >> logr) + nc * (z >> logr))];
    if (u[j] != __builtin_inff() || hits[j] != 0u || arg_tri[j] != -1) {
        u[j] = __builtin_inff();
        hits[j] = 0u;
        arg_tri[j] = -1;
        arg_ray[j] = -1;
    }
}

__global__ void __launch_bounds__(256) trace_fill_unselected(const uint8_t *__restrict__ mask,
                                                             const float *__restrict__ coarse_sdf, int nc, int logr,
                                                             int lognf, int64_t ntex, float *__restrict__ u,
                                                             uint32_t *__restrict__ hits, int32_t *__restrict__ arg_tri,
                                                             int32_t *__restrict__ arg_ray, float *__restrict__ fine)
{
    fill_unselected_body(mask, coarse_sdf, nc, logr, lognf, ntex, u, hits, arg_tri, arg_ray, fine,
                         (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) accum_reset_kernel(int64_t n, float *u, uint32_t *hits, int32_t *at, int32_t *ar)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        u[i] = __builtin_inff();
        hits[i] = 0u;
        at[i] = -1;
        ar[i] = -1;
    }
}

// ---------------------------------------------------------- helpers ----

__global__ void directions_kernel(const int32_t *texel, const uint32_t *frame, const int32_t *ray, int n, uint64_t seed,
                                  uint32_t scene, float *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float3 d = sphere_dir(seed, (uint32_t)texel[i], frame[i], (uint32_t)ray[i], scene);
    out[3 * i] = d.x;
    out[3 * i + 1] = d.y;
    out[3 * i + 2] = d.z;
}

template <int SD>
__global__ void __launch_bounds__(256) closest_hits_kernel(BvhView S, int nt, const float *__restrict__ o,
                                                           const float *__restrict__ d, int n, float *t_out,
                                                           int32_t *tri_out, int32_t *front_out)
{
    __shared__ int stack_mem[4 * SD * kWave];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int *stk = stack_mem + wave * SD * kWave + lane;
    if (i >= n) return;
    RaySetup R;
    ray_setup(o[3 * i], o[3 * i + 1], o[3 * i + 2], d[3 * i], d[3 * i + 1], d[3 * i + 2], R);
    float tbest = __builtin_inff();
    int ibest = -1, node = nt > 0 ? 0 : kDone, sp = 0;
    bool front = false;
    while (node != kDone) trav_step(S, R, node, sp, stk, kWave, tbest, ibest, front);
    t_out[i] = ibest >= 0 ? tbest : __builtin_inff();
    tri_out[i] = ibest >= 0 ? tri_id(S.tris, ibest) : -1;
    front_out[i] = ibest >= 0 && front;
}

// Gradient scatter: dL/dv_i += dL/df * sign * |w| * b_i * n / (n . w).
__global__ void __launch_bounds__(256) trace_backward_kernel(const float *__restrict__ v, const int32_t *__restrict__ f,
                                                             int nt, int lognf, float lox, float loy, float loz,
                                                             float hf, const int32_t *__restrict__ arg_tri,
                                                             const int32_t *__restrict__ arg_ray,
                                                             const float *__restrict__ fine,
                                                             const float *__restrict__ grad, uint64_t seed,
                                                             uint32_t scene, float *grad_v, int64_t ntex, bool vote)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntex) return;
    const int tri = arg_tri[j];
    const float g = grad[j];
    if (tri < 0 || tri >= nt || g == 0.0f) return;
    const uint32_t key = (uint32_t)arg_ray[j];
    const int nfm = (1 << lognf) - 1;
    const float ox = texel_coord(lox, (int)(j & nfm), hf), oy = texel_coord(loy, (int)((j >> lognf) & nfm), hf),
                oz = texel_coord(loz, (int)(j >> (2 * lognf)), hf);
    const float3 w = sphere_dir(seed, (uint32_t)j, key >> 8, key & 0xFFu, scene);
    const int i0 = f[3 * tri], i1 = f[3 * tri + 1], i2 = f[3 * tri + 2];
    const float3 p0 = make_float3(v[3 * i0], v[3 * i0 + 1], v[3 * i0 + 2]);
    const float3 p1 = make_float3(v[3 * i1], v[3 * i1 + 1], v[3 * i1 + 2]);
    const float3 p2 = make_float3(v[3 * i2], v[3 * i2 + 1], v[3 * i2 + 2]);
    const float3 e1 = make_float3(p1.x - p0.x, p1.y - p0.y, p1.z - p0.z);
    const float3 e2 = make_float3(p2.x - p0.x, p2.y - p0.y, p2.z - p0.z);
    // Moller-Trumbore barycentrics of the recorded hit
    const float3 pv = make_float3(w.y * e2.z - w.z * e2.y, w.z * e2.x - w.x * e2.z, w.x * e2.y - w.y * e2.x);
    const float det = e1.x * pv.x + e1.y * pv.y + e1.z * pv.z;
    if (det == 0.0f) return;
    const float inv = 1.0f / det;
    const float3 s = make_float3(ox - p0.x, oy - p0.y, oz - p0.z);
    const float bu = (s.x * pv.x + s.y * pv.y + s.z * pv.z) * inv;
    const float3 q = make_float3(s.y * e1.z - s.z * e1.y, s.z * e1.x - s.x * e1.z, s.x * e1.y - s.y * e1.x);
    const float bv = (w.x * q.x + w.y * q.y + w.z * q.z) * inv;
    const float3 nrm = make_float3(e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z, e1.x * e2.y - e1.y * e2.x);
    const float nw = nrm.x * w.x + nrm.y * w.y + nrm.z * w.z;
    if (nw == 0.0f) return;
    const float len = sqrtf(w.x * w.x + w.y * w.y + w.z * w.z);
    const float sgn = !vote || fine[j] >= 0.0f ? 1.0f : -1.0f;  // a shell value is the distance minus a constant
    const float scale = g * sgn * len / nw;
    const float b[3] = {1.0f - bu - bv, bu, bv};
    const int vid[3] = {i0, i1, i2};
    for (int k = 0; k < 3; ++k) {
        atomicAdd(&grad_v[3 * vid[k]], scale * b[k] * nrm.x);
        atomicAdd(&grad_v[3 * vid[k] + 1], scale * b[k] * nrm.y);
        atomicAdd(&grad_v[3 * vid[k] + 2], scale * b[k] * nrm.z);
    }
}

// ------------------------------------------------------------- launch ----

static rtsdf_trace_tuning g_tuning = {28, 0, 0, 4, 1, 12, 64, 2};
constexpr int kMaxBlocksPerCu = 8;  // persistent workgroups per CU (direction buffers and spill area sized for this)
constexpr int kMinShortStack = 12;  // smallest LDS stack part (spill area sized for this)
constexpr int kMaxStackDepth = 64;  // deepest hierarchy the tracer takes

static bool tuning_ok(const rtsdf_trace_tuning &t)
{
    if (t.refill != 16 && t.refill != 28) return false;
    if (t.blocks_per_cu < 0 || t.blocks_per_cu > kMaxBlocksPerCu) return false;
    if (t.stats < 0 || t.stats > 1 || t.loop < 0 || t.loop > 4) return false;
    if (t.bin_directions < 0 || t.bin_directions > 1) return false;
    if (t.stack_lds != 12 && t.stack_lds != 16 && t.stack_lds != 24) return false;
    if (t.tile_texels != 16 && t.tile_texels != 32 && t.tile_texels != 64) return false;
    if (t.bvh_width != 2 && t.bvh_width != 4) return false;
    return true;
}

template <int SL, int REFILL, int LOOP, bool STATS, bool BATCHED, bool INST = false, bool WIDE = false>
static int launch_trace5(TraceArgs A, const rtsdf_trace_tuning &T, hipStream_t s)
{
    int per_cu = T.blocks_per_cu;
    if (per_cu <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, trace_persistent<SL, REFILL, LOOP, STATS, BATCHED>,
                                                         kTraceWaves * kWave, 0) != hipSuccess ||
            per_cu <= 0)
            per_cu = 2;
    }
    per_cu = std::min(per_cu, kMaxBlocksPerCu);
    const int blocks = num_cus() * per_cu;
    A.spill_stride = blocks * kTraceWaves * kWave;
    A.bin_directions = T.bin_directions;
    A.tile_cap = T.tile_texels;
    trace_persistent<SL, REFILL, LOOP, STATS, BATCHED, INST, WIDE><<<dim3(blocks), dim3(kTraceWaves * kWave), 0, s>>>(A);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

template <int SL, int REFILL, int LOOP, bool BATCHED>
static int launch_trace4(const TraceArgs &A, const rtsdf_trace_tuning &T, hipStream_t s)
{
    return T.stats ? launch_trace5<SL, REFILL, LOOP, true, BATCHED>(A, T, s)
                   : launch_trace5<SL, REFILL, LOOP, false, BATCHED>(A, T, s);
}

template <int SL, int REFILL, bool BATCHED>
static int launch_trace3(const TraceArgs &A, const rtsdf_trace_tuning &T, hipStream_t s)
{
    switch (T.loop) {
    case 0: return launch_trace4<SL, REFILL, 0, BATCHED>(A, T, s);
    case 1: return launch_trace4<SL, REFILL, 1, BATCHED>(A, T, s);
    case 2: return launch_trace4<SL, REFILL, 2, BATCHED>(A, T, s);
    case 4: return launch_trace4<SL, REFILL, 4, BATCHED>(A, T, s);
    default: return launch_trace4<SL, REFILL, 3, BATCHED>(A, T, s);
    }
}

template <int SL, bool BATCHED>
static int launch_trace2(const TraceArgs &A, const rtsdf_trace_tuning &T, hipStream_t s)
{
    return T.refill == 16 ? launch_trace3<SL, 16, BATCHED>(A, T, s) : launch_trace3<SL, 28, BATCHED>(A, T, s);
}

// two-level scenes: the one-fetch loop only
template <int SL, int REFILL>
static int launch_trace_inst2(const TraceArgs &A, const rtsdf_trace_tuning &T, hipStream_t s)
{
    return T.stats ? launch_trace5<SL, REFILL, 3, true, false, true>(A, T, s)
                   : launch_trace5<SL, REFILL, 3, false, false, true>(A, T, s);
}

template <int SL>
static int launch_trace_inst1(const TraceArgs &A, const rtsdf_trace_tuning &T, hipStream_t s)
{
    return T.refill == 16 ? launch_trace_inst2<SL, 16>(A, T, s) : launch_trace_inst2<SL, 28>(A, T, s);
}

static int launch_trace_inst(const TraceArgs &A, const rtsdf_trace_tuning &T, hipStream_t s)
{
    switch (T.stack_lds) {
    case 12: return launch_trace_inst1<12>(A, T, s);
    case 24: return launch_trace_inst1<24>(A, T, s);
    default: return launch_trace_inst1<16>(A, T, s);
    }
}

// 4-wide single-scene launches: the one-fetch loop only
template <int SL, int REFILL>
static int launch_trace_wide2(const TraceArgs &A, const rtsdf_trace_tuning &T, hipStream_t s)
{
    return T.stats ? launch_trace5<SL, REFILL, 3, true, false, false, true>(A, T, s)
                   : launch_trace5<SL, REFILL, 3, false, false, false, true>(A, T, s);
}

static int launch_trace_wide(const TraceArgs &A, const rtsdf_trace_tuning &T, hipStream_t s)
{
    switch (T.stack_lds) {
    case 12: return T.refill == 16 ? launch_trace_wide2<12, 16>(A, T, s) : launch_trace_wide2<12, 28>(A, T, s);
    case 24: return T.refill == 16 ? launch_trace_wide2<24, 16>(A, T, s) : launch_trace_wide2<24, 28>(A, T, s);
    default: return T.refill == 16 ? launch_trace_wide2<16, 16>(A, T, s) : launch_trace_wide2<16, 28>(A, T, s);
    }
}

template <bool BATCHED>
static int launch_trace(const TraceArgs &A, const rtsdf_trace_tuning &T, hipStream_t s)
{
    switch (T.stack_lds) {
    case 12: return launch_trace2<12, BATCHED>(A, T, s);
    case 24: return launch_trace2<24, BATCHED>(A, T, s);
    default: return launch_trace2<16, BATCHED>(A, T, s);
    }
}

static int stack_depth_for(const rtsdf_scene *sc) { return sc->max_depth + 1; }

// stack entries a 4-wide traversal can hold at once: up to three pushed at each wide level on the path
// (levels 0 .. depth4), plus one
static int wide_stack_depth(const rtsdf_scene *sc) { return 3 * (sc->depth4 + 1) + 1; }

// whether a trace of this scene with tuning T runs the 4-wide loop
static bool trace_wide(const rtsdf_scene *sc, const rtsdf_trace_tuning &T)
{
    return T.bvh_width == 4 && sc->nodes4 && sc->ninst == 0 && wide_stack_depth(sc) <= kMaxStackDepth;
}

// the tuning a trace of this scene uses: its own if set, else the process default
static const rtsdf_trace_tuning &tuning_for(const rtsdf_scene *sc)
{
    return sc->has_tuning ? sc->tuning : g_tuning;
}

// Trace workspace: 256 B of counters, the wavefronts' direction buffers, then
// the spill area for stack entries deeper than the LDS part (per lane of the
// largest launch, for the deepest hierarchy the tracer takes).  Everything a
// launch writes besides its outputs lives here, so launches with separate
// workspaces can run concurrently, on one scene too.
static size_t trace_lanes_max() { return (size_t)num_cus() * kMaxBlocksPerCu * kTraceWaves * kWave; }
static size_t dirs_bytes() { return (size_t)num_cus() * kMaxBlocksPerCu * kTraceWaves * 2 * kTileRays * sizeof(float4); }
static size_t spill_bytes() { return trace_lanes_max() * (kMaxStackDepth - kMinShortStack) * sizeof(int32_t); }
static size_t trace_ws_bytes() { return 256 + dirs_bytes() + spill_bytes(); }
static float4 *ws_dirs(void *ws) { return reinterpret_cast<float4 *>(static_cast<char *>(ws) + 256); }
static int32_t *ws_spill(void *ws) { return reinterpret_cast<int32_t *>(static_cast<char *>(ws) + 256 + dirs_bytes()); }

}  // namespace rtsdf

extern "C" int rtsdf_trace_config(const rtsdf_trace_tuning *t)
{
    if (!t || !rtsdf::tuning_ok(*t)) return RTSDF_EINVAL;
    rtsdf::g_tuning = *t;
    return RTSDF_OK;
}

extern "C" int rtsdf_scene_set_tuning(rtsdf_scene *scene, const rtsdf_trace_tuning *t)
{
    if (!scene || (t && !rtsdf::tuning_ok(*t))) return RTSDF_EINVAL;
    if (t && t->bvh_width == 4 && !scene->nodes4) {  // the 4-wide copy is built on first use
        const int rc = rtsdf::wide_build(scene, nullptr);
        if (rc != RTSDF_OK) return rc;
        if (rtsdf::wide_stack_depth(scene) > rtsdf::kMaxStackDepth) return RTSDF_EINVAL;
    }
    scene->has_tuning = t != nullptr;
    if (t) scene->tuning = *t;
    return RTSDF_OK;
}

extern "C" int rtsdf_scene_get_tuning(const rtsdf_scene *scene, rtsdf_trace_tuning *t)
{
    if (!scene || !t) return RTSDF_EINVAL;
    *t = rtsdf::tuning_for(scene);
    return RTSDF_OK;
}

extern "C" int rtsdf_trace_config_get(rtsdf_trace_tuning *t)
{
    if (!t) return RTSDF_EINVAL;
    *t = rtsdf::g_tuning;
    return RTSDF_OK;
}

extern "C" int rtsdf_accum_reset(rtsdf_grid fine, rtsdf_accum st, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!grid_ok(fine) || !st.u || !st.hits || !st.arg_tri || !st.arg_ray) return RTSDF_EINVAL;
    const int64_t n = (int64_t)fine.n * fine.n * fine.n;
    int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    accum_reset_kernel<<<dim3((unsigned)blocks), dim3(256), 0, as_stream(stream)>>>(n, st.u, st.hits, st.arg_tri, st.arg_ray);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

extern "C" size_t rtsdf_trace_workspace_size(void) { return rtsdf::trace_ws_bytes(); }

extern "C" int rtsdf_trace_accumulate(const rtsdf_scene *scene, rtsdf_grid coarse, const float *coarse_sdf,
                                      rtsdf_grid fine, const uint8_t *mask, const int32_t *queue, const int32_t *count,
                                      int32_t queue_cap, int32_t rays_per_texel, uint32_t frame,
                                      const uint32_t *frame_ptr, uint64_t seed, uint32_t scene_id, float alpha,
                                      rtsdf_accum st, float *fine_sdf, void *workspace, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scene || !grid_ok(coarse) || !grid_ok(fine) || !coarse_sdf || !mask || !count || !fine_sdf || !workspace)
        return RTSDF_EINVAL;
    if (!st.u || !st.hits || !st.arg_tri || !st.arg_ray) return RTSDF_EINVAL;
    if (!is_pow2(coarse.n) || !is_pow2(fine.n) || fine.n < coarse.n || fine.n > 1024) return RTSDF_EINVAL;
    if (queue_cap < 0 || (queue_cap > 0 && !queue)) return RTSDF_EINVAL;
    if (rays_per_texel < 1 || rays_per_texel > 64) return RTSDF_EINVAL;
    if (!(alpha >= 0.0f && alpha <= 1.0f)) return RTSDF_EINVAL;
    if (frame >= kMaxFrame && !frame_ptr) return RTSDF_EINVAL;
    const int sd = stack_depth_for(scene);
    if (sd > kMaxStackDepth) return RTSDF_EINVAL;
    rtsdf_trace_tuning T = tuning_for(scene);
    if (scene->nt >= (1 << 26)) return RTSDF_EINVAL;  // triangle ids share a 64-bit key with the distance
    if (T.loop == 4 && scene->nref >= kMaxQueuedRefs) T.loop = 3;  // queue entries hold 26-bit indices
    hipStream_t s = as_stream(stream);
    const int lognf = ilog2(fine.n), logr = ilog2(fine.n / coarse.n);
    const int64_t ntex = (int64_t)fine.n * fine.n * fine.n;
    trace_fill_unselected<<<dim3((unsigned)((ntex + 255) / 256)), dim3(256), 0, s>>>(
        mask, coarse_sdf, coarse.n, logr, lognf, ntex, st.u, st.hits, st.arg_tri, st.arg_ray, fine_sdf);
    RTSDF_CHECK_LAUNCH();
    int32_t *cursor = static_cast<int32_t *>(workspace);
    int rc = launch_fill<int32_t>(cursor, 0, T.stats ? 32 : 1, s);
    if (rc != RTSDF_OK) return rc;
    TraceArgs A{};
    TraceScene &P = A.one;
    P.bvh.nodes = scene->nodes;
    P.bvh.tris = scene->tris;
    P.bvh.tmap = scene->tmap;
    P.nodes4 = scene->nodes4;
    P.nt = scene->nt;
    P.queue = queue;
    P.count = count;
    P.queue_cap = queue_cap;
    P.coarse_sdf = coarse_sdf;
    P.nc = coarse.n;
    P.logr = logr;
    P.nf = fine.n;
    P.lognf = lognf;
    P.lox = fine.lo[0];
    P.loy = fine.lo[1];
    P.loz = fine.lo[2];
    P.hf = fine.h;
    P.rays = rays_per_texel;
    P.scene_id = scene_id;
    P.alpha = alpha;
    P.sign_policy = scene->sign_policy;
    P.shell = scene->shell;
    P.u = st.u;
    P.hits = st.hits;
    P.arg_tri = st.arg_tri;
    P.arg_ray = st.arg_ray;
    P.fine = fine_sdf;
    A.scenes = nullptr;
    A.tile_offset = nullptr;
    A.nscenes = 1;
    A.cursor = cursor;
    A.frame = frame;
    A.frame_ptr = frame_ptr;
    A.seed = seed;
    A.spill = ws_spill(workspace);
    A.spill_stride = 0;
    A.dirs = ws_dirs(workspace);
    if (scene->ninst > 0) return launch_trace_inst(A, T, s);
    return trace_wide(scene, T) ? launch_trace_wide(A, T, s) : launch_trace<false>(A, T, s);
}

extern "C" int rtsdf_directions(const int32_t *texel, const uint32_t *frame, const int32_t *ray, int32_t n,
                                uint64_t seed, uint32_t scene_id, float *out, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (n < 0 || (n > 0 && (!texel || !frame || !ray || !out))) return RTSDF_EINVAL;
    if (n == 0) return RTSDF_OK;
    directions_kernel<<<dim3((n + 255) / 256), dim3(256), 0, as_stream(stream)>>>(texel, frame, ray, n, seed, scene_id, out);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

extern "C" int rtsdf_closest_hits(const rtsdf_scene *scene, const float *origins, const float *dirs, int32_t n,
                                  float *t_out, int32_t *tri_out, int32_t *front_out, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scene || n < 0 || (n > 0 && (!origins || !dirs || !t_out || !tri_out || !front_out))) return RTSDF_EINVAL;
    if (scene->ninst > 0) return RTSDF_EINVAL;  // single-level scenes only
    if (n == 0) return RTSDF_OK;
    const int sd = stack_depth_for(scene);
    if (sd > kMaxStackDepth) return RTSDF_EINVAL;
    BvhView S{scene->nodes, scene->tris, scene->tmap};
    hipStream_t s = as_stream(stream);
    const dim3 g((n + 255) / 256), b(256);
    if (sd <= 32)
        closest_hits_kernel<32><<<g, b, 0, s>>>(S, scene->nt, origins, dirs, n, t_out, tri_out, front_out);
    else
        closest_hits_kernel<64><<<g, b, 0, s>>>(S, scene->nt, origins, dirs, n, t_out, tri_out, front_out);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

extern "C" int rtsdf_trace_backward(const rtsdf_scene *scene, rtsdf_grid fine, rtsdf_accum st, const float *fine_sdf,
                                    const float *grad_fine, uint64_t seed, uint32_t scene_id, float *grad_v,
                                    rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scene || !grid_ok(fine) || !is_pow2(fine.n) || !st.arg_tri || !st.arg_ray || !fine_sdf || !grad_fine || !grad_v)
        return RTSDF_EINVAL;
    const int64_t ntex = (int64_t)fine.n * fine.n * fine.n;
    trace_backward_kernel<<<dim3((unsigned)((ntex + 255) / 256)), dim3(256), 0, as_stream(stream)>>>(
        scene->vertices, scene->faces, scene->nt, ilog2(fine.n), fine.lo[0], fine.lo[1], fine.lo[2], fine.h, st.arg_tri,
        st.arg_ray, fine_sdf, grad_fine, seed, scene_id, grad_v, ntex, scene->sign_policy == RTSDF_SIGN_VOTE);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}
