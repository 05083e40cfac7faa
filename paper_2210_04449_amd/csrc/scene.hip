// Scene: triangles and their bounding volume hierarchy on the device.
//
// The paper does not say how its rays find their closest hits (it traces on
// an RTX 2080 Ti).  gfx950 has no ray-tracing units, so the library keeps a
// two-wide hierarchy in HBM and traverses it in software:
//
//   node (64 B): both children's boxes, so one node fetch tests two boxes
//     xy0 = (c0.lo.x, c0.hi.x, c0.lo.y, c0.hi.y)
//     xy1 = (c1.lo.x, c1.hi.x, c1.lo.y, c1.hi.y)
//     z01 = (c0.lo.z, c0.hi.z, c1.lo.z, c1.hi.z)
//     meta = (child0, child1, parent, 0)
//   child >= 0 is an internal node, child < 0 a leaf: -1 - (first << 5 | count)
//   with `count` triangles starting at `first` in the reordered triangle array.
//   triangle (48 B): (v0, id) (v1, path) (v2, -) as float4s, one per
//     reference, in leaf order; path = levels << 24 | (2-bit piece per level,
//     level 0 lowest), 0 for an unsplit triangle.
//   triangle map (48 B, same order): rows r0, r1, r2 of the affine map that
//     takes v0, v1, v2 to (0,0,0), (1,0,0), (0,1,0) and v0 + n to (0,0,1),
//     n = (v1 - v0) x (v2 - v0); a point p maps to (r_k . (p, 1))_k, so for a
//     ray the first two coordinates at the plane crossing are barycentrics
//     b1, b2 and the third is the signed distance along n in units of |n|.
//     Computed in double precision from the float vertices on the device (at
//     creation and at every refit); degenerate triangles get a map no ray hits.
//
// Build (host, at creation): binned surface-area heuristic (256 bins per axis),
// leaves of at most `leaf_size` references, depth capped (median splits below
// kMaxBuildDepth) so the traversal stack of the tracer never overflows.
// Large triangles are split into several *references* before the build (the
// early-split idea of Ernst and Greiner 2007): a triangle whose longest edge
// exceeds 1/32 of the scene size is subdivided at edge midpoints, recursively,
// and each piece becomes a reference with the piece's tight box that points at
// the whole original triangle.  Long thin boxes of big triangles otherwise
// inflate every node above them.  Leaves store one triangle record per
// reference (the same triangle can sit in several leaves; the closest hit is
// the same whichever copy reports it), and the record keeps the piece's
// subdivision path so a refit can recompute the piece's box from moved
// vertices.
// Boxes are padded outwards by 2^-17 * (scene scale) so the float slab test,
// whose rounding error is far below that, never rejects a box the ray enters.
// Refit (device): triangle records rewritten from new positions, boxes
// recomputed bottom-up, the last child to finish continuing to the parent.
#include <algorithm>
#include <memory>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace rtsdf {

constexpr int kMaxBuildDepth = 48;  // median splits below; stack depth <= 63
constexpr int kMaxLeaf = 31;
// second child code of an instance node (no leaf code reaches it: references stay below 2^26 - 1)
constexpr int kInstTag = INT32_MIN;
// stack entry marking the return from an instance to world space
constexpr int kReturn = INT32_MIN + 1;

struct alignas(16) BvhNode {
    float4 xy0, xy1, z01;
    int4 meta;
};

__host__ __device__ __forceinline__ int leaf_code(int first, int count) { return -1 - ((first << 5) | count); }
__host__ __device__ __forceinline__ int leaf_first(int code) { return (-1 - code) >> 5; }
__host__ __device__ __forceinline__ int leaf_count(int code) { return (-1 - code) & 31; }

}  // namespace rtsdf

struct rtsdf_lbvh;  // device rebuild buffers (rtsdf_scene_enable_rebuild)

struct rtsdf_scene {
    int nv = 0, nt = 0;
    int nnodes = 0;
    int max_depth = 0;
    int max_leaf = 0;
    int leaf_size = 0;                 // the leaf size asked for at creation (device rebuilds use it too)
    float pad = 0.f;
    int device = 0;
    rtsdf::BvhNode *nodes = nullptr;   // [nnodes]
    int nref = 0;                      // triangle references (>= nt: large triangles are split)
    float4 *tris = nullptr;            // [3 nref]
    float4 *tmap = nullptr;            // [3 nref + 1] triangle-space maps, leaf order (+ 16 B padding)
    int4 *leaf_faces = nullptr;        // [nref] (i0, i1, i2, original id) in leaf order
    float *vertices = nullptr;         // [3 nv] current positions
    int32_t *faces = nullptr;          // [3 nt]
    int32_t *refit_counter = nullptr;  // [nnodes]
    int32_t *start_nodes = nullptr;    // internal nodes with two leaf children
    int nstart = 0;
    bool has_tuning = false;           // tracer tuning of this scene (rtsdf_scene_set_tuning); else the
    rtsdf_trace_tuning tuning{};       // process default of rtsdf_trace_config
    int64_t bytes = 0;
    int sign_policy = RTSDF_SIGN_VOTE;  // how the tracer signs a traced distance
    float shell = 0.f;                  // RTSDF_SIGN_SHELL: half-thickness subtracted from the distance
    // two-level scenes (rtsdf_scene_create_instanced): nodes = [top level over static triangles and moving
    // parts] [instance nodes (ninst - 1)] [each moving part's own hierarchy]; `vertices` holds world positions
    int ninst = 0;
    int inst_base = 0;                 // node index of the first instance node
    float *obj_vertices = nullptr;     // [3 nv] object-space positions
    int32_t *vert_inst = nullptr;      // [nv] instance of each vertex, -1 for vertices no face uses
    float *inst_obj_box = nullptr;     // [nentries][6] object-space box of each entry (a subtree of a moving part)
    float *inst_world_box = nullptr;   // [nentries][6]
    float *transforms = nullptr;       // [ninst][12] current object-to-world rows (row 0, the static world, unused)
    int32_t *top_dirty = nullptr;      // top-level nodes above moving parts, deepest level first
    int32_t *top_level_off = nullptr;  // [top_levels + 1] offsets of the levels in top_dirty
    int top_levels = 0;
    int nentries = 0;                  // subtrees of moving parts that the top level holds
    int32_t *entry_part = nullptr;     // [nentries] part of each (1..ninst-1)
    rtsdf_lbvh *lbvh = nullptr;        // set once the scene rebuilds its hierarchy on the device
    // 4-wide copy of the hierarchy for the tracer (rtsdf_scene_set_tuning with bvh_width 4): node j is the two
    // records 2 j (children 0, 1) and 2 j + 1 (children 2, 3) in the two-child format; map4[4 j + k] is the
    // two-child slot (node << 1 | slot) whose box child k mirrors, -1 for an empty child
    rtsdf::BvhNode *nodes4 = nullptr;
    int32_t *map4 = nullptr;
    int nnodes4 = 0;
    int depth4 = 0;                    // deepest wide level (root = 0)
};

static void lbvh_free(rtsdf_lbvh *L);

namespace rtsdf {

constexpr int kMaxSplitLevels = 12;

// piece k of the midpoint subdivision of (a, b, c): 0 (a, ab, ca), 1 (ab, b, bc), 2 (ca, bc, c), 3 (ab, bc, ca)
template <typename T>
__host__ __device__ __forceinline__ void split_piece(T a[3], T b[3], T c[3], int k)
{
    for (int i = 0; i < 3; ++i) {
        const T ab = (a[i] + b[i]) * (T)0.5, bc = (b[i] + c[i]) * (T)0.5, ca = (c[i] + a[i]) * (T)0.5;
        switch (k) {
        case 0: b[i] = ab; c[i] = ca; break;
        case 1: a[i] = ab; c[i] = bc; break;
        case 2: a[i] = ca; b[i] = bc; break;
        default: a[i] = ab; b[i] = bc; c[i] = ca; break;
        }
    }
}

// the piece of (a, b, c) a path code names
template <typename T>
__host__ __device__ __forceinline__ void follow_path(T a[3], T b[3], T c[3], int path)
{
    const int levels = (path >> 24) & 15;
    for (int l = 0; l < levels; ++l) split_piece(a, b, c, (path >> (2 * l)) & 3);
}

namespace {

struct Aabb {
    float lo[3], hi[3];
    void reset()
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = INFINITY;
            hi[a] = -INFINITY;
        }
    }
    void grow(const Aabb &b)
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b.lo[a]);
            hi[a] = std::max(hi[a], b.hi[a]);
        }
    }
    void grow_pt(const float *p)
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
        }
    }
    double area() const
    {
        const double dx = std::max(0.0, (double)hi[0] - lo[0]), dy = std::max(0.0, (double)hi[1] - lo[1]),
                     dz = std::max(0.0, (double)hi[2] - lo[2]);
        return dx * dy + dy * dz + dz * dx;
    }
};

struct HostBuilder {
    const float *v;
    const int32_t *f;
    int nt;
    int leaf_size;
    float pad;
    std::vector<Aabb> tb;
    std::vector<float> cen;
    std::vector<int> idx;
    std::vector<BvhNode> nodes;
    int max_depth = 0, max_leaf = 0;
    // two-level scenes: the top level mixes triangle references with moving parts; item_part[item] is the
    // moving part's index (-1 for a triangle reference) and such an item becomes the child code
    // kInstItem + index, remapped to its instance node once the node count is known
    const std::vector<int> *item_part = nullptr;
    static constexpr int kInstItem = 1 << 30;

    int movers_in(int b, int e, int &one) const
    {
        if (!item_part) return 0;
        int n = 0;
        for (int i = b; i < e; ++i)
            if ((*item_part)[idx[i]] >= 0) {
                ++n;
                one = (*item_part)[idx[i]];
            }
        return n;
    }

    Aabb range_box(int b, int e) const
    {
        Aabb r;
        r.reset();
        for (int i = b; i < e; ++i) r.grow(tb[idx[i]]);
        return r;
    }

    void padded(const Aabb &b, float lo[3], float hi[3]) const
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::nextafter(b.lo[a] - pad, -INFINITY);
            hi[a] = std::nextafter(b.hi[a] + pad, INFINITY);
        }
    }

    // returns the child code for range [b, e)
    int build(int b, int e, int depth)
    {
        const int count = e - b;
        int one = -1;
        const int movers = movers_in(b, e, one);
        if (movers > 0) {  // a moving part is a child of its own; leaves hold triangle references only
            if (count == 1) {
                max_depth = std::max(max_depth, depth);
                return kInstItem + one;
            }
        } else if (count <= leaf_size || depth >= kMaxBuildDepth + 14) {
            if (count > kMaxLeaf) {  // cannot happen unless the depth cap bites; split by index
                return build_split(b, e, b + count / 2, depth);
            }
            max_depth = std::max(max_depth, depth);
            max_leaf = std::max(max_leaf, count);
            return leaf_code(b, count);
        }
        Aabb cb;
        cb.reset();
        for (int i = b; i < e; ++i) cb.grow_pt(&cen[3 * idx[i]]);
        int axis = 0;
        for (int a = 1; a < 3; ++a)
            if (cb.hi[a] - cb.lo[a] > cb.hi[axis] - cb.lo[axis]) axis = a;
        if (!(cb.hi[axis] > cb.lo[axis])) return build_split(b, e, b + count / 2, depth);
        if (depth >= kMaxBuildDepth) {  // median split on the longest axis
            const int mid = b + count / 2;
            std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e, [&](int x, int y) {
                return cen[3 * x + axis] < cen[3 * y + axis] || (cen[3 * x + axis] == cen[3 * y + axis] && x < y);
            });
            return build_split(b, e, mid, depth);
        }
        constexpr int NB = 256;
        double best_cost = INFINITY;
        int best_axis = -1, best_bin = -1;
        for (int a = 0; a < 3; ++a) {
            const float ext = cb.hi[a] - cb.lo[a];
            if (!(ext > 0)) continue;
            Aabb bins[NB];
            int cnt[NB] = {0};
            for (int k = 0; k < NB; ++k) bins[k].reset();
            const float scale = NB / ext;
            for (int i = b; i < e; ++i) {
                int k = (int)((cen[3 * idx[i] + a] - cb.lo[a]) * scale);
                k = std::min(std::max(k, 0), NB - 1);
                bins[k].grow(tb[idx[i]]);
                cnt[k]++;
            }
            double rarea[NB];
            int rcnt[NB];
            Aabb acc;
            acc.reset();
            int c = 0;
            for (int k = NB - 1; k > 0; --k) {
                acc.grow(bins[k]);
                c += cnt[k];
                rarea[k] = acc.area();
                rcnt[k] = c;
            }
            acc.reset();
            c = 0;
            for (int k = 0; k < NB - 1; ++k) {
                acc.grow(bins[k]);
                c += cnt[k];
                if (c == 0 || rcnt[k + 1] == 0) continue;
                const double cost = acc.area() * c + rarea[k + 1] * rcnt[k + 1];
                if (cost < best_cost) {
                    best_cost = cost;
                    best_axis = a;
                    best_bin = k;
                }
            }
        }
        if (best_axis < 0) return build_split(b, e, b + count / 2, depth);
        const Aabb box = range_box(b, e);
        const double leaf_cost = box.area() * count;
        if (movers == 0 && count <= 2 * leaf_size && best_cost + box.area() >= leaf_cost) {
            max_depth = std::max(max_depth, depth);
            max_leaf = std::max(max_leaf, count);
            return leaf_code(b, count);
        }
        const float ext = cb.hi[best_axis] - cb.lo[best_axis];
        const float scale = NB / ext;
        auto it = std::partition(idx.begin() + b, idx.begin() + e, [&](int t) {
            int k = (int)((cen[3 * t + best_axis] - cb.lo[best_axis]) * scale);
            k = std::min(std::max(k, 0), NB - 1);
            return k <= best_bin;
        });
        int mid = (int)(it - idx.begin());
        if (mid == b || mid == e) mid = b + count / 2;
        return build_split(b, e, mid, depth);
    }

    int build_split(int b, int e, int mid, int depth)
    {
        const int id = (int)nodes.size();
        nodes.emplace_back();
        const int c0 = build(b, mid, depth + 1);
        const int c1 = build(mid, e, depth + 1);
        float lo0[3], hi0[3], lo1[3], hi1[3];
        padded(range_box(b, mid), lo0, hi0);
        padded(range_box(mid, e), lo1, hi1);
        BvhNode &nd = nodes[id];
        nd.xy0 = make_float4(lo0[0], hi0[0], lo0[1], hi0[1]);
        nd.xy1 = make_float4(lo1[0], hi1[0], lo1[1], hi1[1]);
        nd.z01 = make_float4(lo0[2], hi0[2], lo1[2], hi1[2]);
        nd.meta = make_int4(c0, c1, -1, 0);
        if (c0 >= 0 && c0 < kInstItem) nodes[c0].meta.z = id;
        if (c1 >= 0 && c1 < kInstItem) nodes[c1].meta.z = id;
        return id;
    }
};

// References of the triangles (see the header comment): pieces of midpoint
// subdivision until the longest edge is at most 1/32 of the scene's largest
// extent; the length doubles while the count would exceed 3 nt + 1024.
void make_references(const std::vector<float> &hv, const std::vector<int32_t> &hf, int nt, std::vector<Aabb> &boxes,
                     std::vector<int32_t> &ref_tri, std::vector<int32_t> &ref_path)
{
    boxes.clear();
    ref_tri.clear();
    ref_path.clear();
    if (nt <= 0) return;
    double slo[3] = {INFINITY, INFINITY, INFINITY}, shi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < 3 * nt; ++i)
        for (int a = 0; a < 3; ++a) {
            slo[a] = std::min(slo[a], (double)hv[3 * hf[i] + a]);
            shi[a] = std::max(shi[a], (double)hv[3 * hf[i] + a]);
        }
    const double extent = std::max(shi[0] - slo[0], std::max(shi[1] - slo[1], shi[2] - slo[2]));
    const size_t cap = (size_t)std::min<int64_t>(3LL * nt + 1024, (1LL << 26) - 1);
    struct Piece {
        double a[3], b[3], c[3];
        int level, path;
    };
    std::vector<Piece> stack;
    for (double len = extent / 32.0;; len *= 2.0) {
        boxes.clear();
        ref_tri.clear();
        ref_path.clear();
        bool over = false;
        for (int t = 0; t < nt && !over; ++t) {
            Piece p0;
            for (int a = 0; a < 3; ++a) {
                p0.a[a] = hv[3 * hf[3 * t] + a];
                p0.b[a] = hv[3 * hf[3 * t + 1] + a];
                p0.c[a] = hv[3 * hf[3 * t + 2] + a];
            }
            p0.level = 0;
            p0.path = 0;
            stack.assign(1, p0);
            while (!stack.empty()) {
                const Piece p = stack.back();
                stack.pop_back();
                double e = 0.0;
                for (int a = 0; a < 3; ++a) {
                    e = std::max(e, std::fabs(p.a[a] - p.b[a]));
                    e = std::max(e, std::fabs(p.b[a] - p.c[a]));
                    e = std::max(e, std::fabs(p.c[a] - p.a[a]));
                }
                if (p.level < kMaxSplitLevels && e > len) {
                    for (int k = 0; k < 4; ++k) {
                        Piece q = p;
                        split_piece(q.a, q.b, q.c, k);
                        q.level = p.level + 1;
                        q.path = p.path | (k << (2 * p.level));
                        stack.push_back(q);
                    }
                    continue;
                }
                Aabb box;
                for (int a = 0; a < 3; ++a) {  // float box rounded outwards
                    const double l = std::min(p.a[a], std::min(p.b[a], p.c[a]));
                    const double h = std::max(p.a[a], std::max(p.b[a], p.c[a]));
                    float lf = (float)l, hf2 = (float)h;
                    if ((double)lf > l) lf = std::nextafter(lf, -INFINITY);
                    if ((double)hf2 < h) hf2 = std::nextafter(hf2, INFINITY);
                    box.lo[a] = lf;
                    box.hi[a] = hf2;
                }
                boxes.push_back(box);
                ref_tri.push_back(t);
                ref_path.push_back(p.level ? (p.level << 24) | p.path : 0);
            }
            over = ref_tri.size() > cap;
        }
        if (!over || len > 4.0 * extent) break;  // past 2 x extent nothing splits, so the loop ends
    }
}

}  // namespace

// ---------------------------------------------------------------- refit ----

// records rewritten from the new positions (id and subdivision path kept)
__global__ void refit_tris(const float *__restrict__ v, const int4 *__restrict__ lf, float4 *__restrict__ tris, int nref)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nref) return;
    const int4 q = lf[i];
    const float path = tris[3 * i + 1].w;
    const int ids[3] = {q.x, q.y, q.z};
    for (int k = 0; k < 3; ++k) {
        const float *p = v + 3 * ids[k];
        tris[3 * i + k] = make_float4(p[0], p[1], p[2], k == 0 ? __int_as_float(q.w) : (k == 1 ? path : 0.f));
    }
}

// Rows of [e1 e2 n]^-1 are (e2 x n, n x e1, e1 x e2) / |n|^2; the translation
// column sends v0 to the origin.
__global__ void tri_maps(const float4 *__restrict__ tris, float4 *__restrict__ tmap, int nt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    const float4 a = tris[3 * i], b = tris[3 * i + 1], c = tris[3 * i + 2];
    const double v0[3] = {a.x, a.y, a.z};
    const double e1[3] = {(double)b.x - a.x, (double)b.y - a.y, (double)b.z - a.z};
    const double e2[3] = {(double)c.x - a.x, (double)c.y - a.y, (double)c.z - a.z};
    const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    if (!(nn > 0.0) || !isfinite(nn)) {  // no plane: every point maps to z = 1, rays parallel to "it"
        tmap[3 * i] = make_float4(0.f, 0.f, 0.f, -1.f);
        tmap[3 * i + 1] = make_float4(0.f, 0.f, 0.f, -1.f);
        tmap[3 * i + 2] = make_float4(0.f, 0.f, 0.f, 1.f);
        return;
    }
    const double r[3][3] = {
        {e2[1] * n[2] - e2[2] * n[1], e2[2] * n[0] - e2[0] * n[2], e2[0] * n[1] - e2[1] * n[0]},
        {n[1] * e1[2] - n[2] * e1[1], n[2] * e1[0] - n[0] * e1[2], n[0] * e1[1] - n[1] * e1[0]},
        {n[0], n[1], n[2]}};
    for (int k = 0; k < 3; ++k) {
        const double x = r[k][0] / nn, y = r[k][1] / nn, z = r[k][2] / nn;
        const double w = -(x * v0[0] + y * v0[1] + z * v0[2]);
        tmap[3 * i + k] = make_float4((float)x, (float)y, (float)z, (float)w);
    }
}

__device__ __forceinline__ void leaf_box(const float4 *__restrict__ tris, int code, float pad, float lo[3], float hi[3])
{
    for (int a = 0; a < 3; ++a) {
        lo[a] = INFINITY;
        hi[a] = -INFINITY;
    }
    const int first = leaf_first(code), cnt = leaf_count(code);
    for (int i = first; i < first + cnt; ++i) {
        const float4 pa = tris[3 * i], pb = tris[3 * i + 1], pc = tris[3 * i + 2];
        float a[3] = {pa.x, pa.y, pa.z}, b[3] = {pb.x, pb.y, pb.z}, c[3] = {pc.x, pc.y, pc.z};
        follow_path(a, b, c, __float_as_int(pb.w));  // the reference's piece (rounding << pad)
        for (int ax = 0; ax < 3; ++ax) {
            lo[ax] = fminf(lo[ax], fminf(a[ax], fminf(b[ax], c[ax])));
            hi[ax] = fmaxf(hi[ax], fmaxf(a[ax], fmaxf(b[ax], c[ax])));
        }
    }
    for (int a = 0; a < 3; ++a) {
        lo[a] = nextafterf(lo[a] - pad, -INFINITY);
        hi[a] = nextafterf(hi[a] + pad, INFINITY);
    }
}

__device__ __forceinline__ void set_slot(BvhNode *nd, int slot, const float lo[3], const float hi[3])
{
    float *xy = slot == 0 ? &nd->xy0.x : &nd->xy1.x;
    xy[0] = lo[0]; xy[1] = hi[0]; xy[2] = lo[1]; xy[3] = hi[1];
    float *z = &nd->z01.x;
    z[2 * slot] = lo[2];
    z[2 * slot + 1] = hi[2];
}

__device__ __forceinline__ void get_slot(const BvhNode *nd, int slot, float lo[3], float hi[3])
{
    const float *xy = slot == 0 ? &nd->xy0.x : &nd->xy1.x;
    lo[0] = xy[0]; hi[0] = xy[1]; lo[1] = xy[2]; hi[1] = xy[3];
    const float *z = &nd->z01.x;
    lo[2] = z[2 * slot];
    hi[2] = z[2 * slot + 1];
}

// 4-wide copy: child k of wide node i takes the box of the two-child slot map[4 i + k] (after a refit of
// the two-child hierarchy).  Children 2 r and 2 r + 1 share a record but write different words.
__global__ void __launch_bounds__(256) wide_gather(BvhNode *__restrict__ wide, const int32_t *__restrict__ map,
                                                   const BvhNode *__restrict__ nodes, int nslots)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nslots) return;
    const int m = map[i];
    if (m < 0) return;
    float lo[3], hi[3];
    get_slot(&nodes[m >> 1], m & 1, lo, hi);
    set_slot(&wide[i >> 1], i & 1, lo, hi);
}

// Every thread starts at an internal node whose children are both leaves and
// climbs; at a node with two internal children only the second arrival goes on.
__global__ void refit_nodes(BvhNode *nodes, const float4 *__restrict__ tris, const int32_t *__restrict__ starts,
                            int nstart, int32_t *counter, float pad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nstart) return;
    int node = starts[i];
    while (node >= 0) {
        BvhNode *nd = &nodes[node];
        const int c[2] = {nd->meta.x, nd->meta.y};
        float lo[2][3], hi[2][3];
        for (int s = 0; s < 2; ++s) {
            if (c[s] < 0) {
                leaf_box(tris, c[s], pad, lo[s], hi[s]);
                set_slot(nd, s, lo[s], hi[s]);
            } else {
                // the child's own slots are final (it finished before us)
                const BvhNode *ch = &nodes[c[s]];
                float l2[3], h2[3];
                get_slot(ch, 0, lo[s], hi[s]);
                get_slot(ch, 1, l2, h2);
                for (int a = 0; a < 3; ++a) {
                    lo[s][a] = fminf(lo[s][a], l2[a]);
                    hi[s][a] = fmaxf(hi[s][a], h2[a]);
                }
                set_slot(nd, s, lo[s], hi[s]);
            }
        }
        __threadfence();
        const int parent = nd->meta.z;
        if (parent < 0) break;
        const BvhNode *pn = &nodes[parent];
        const int internal_children = (pn->meta.x >= 0) + (pn->meta.y >= 0);
        if (internal_children == 2) {
            const int old = atomicAdd(&counter[parent], 1);
            if (old == 0) break;  // the sibling subtree is not done yet; it will continue
            __threadfence();
        }
        node = parent;
    }
}

}  // namespace rtsdf

extern "C" void rtsdf_scene_destroy(rtsdf_scene *scene);

static int rtsdf_scene_create_impl(const float *vertices, int32_t nv, const int32_t *faces, int32_t nt,
                                   int32_t leaf_size, rtsdf_scene **out, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!out || nv < 0 || nt < 0 || (nt > 0 && (!vertices || !faces))) return RTSDF_EINVAL;
    if (leaf_size <= 0) leaf_size = 4;
    if (leaf_size > kMaxLeaf) return RTSDF_EINVAL;
    if ((int64_t)nt >= (int64_t)1 << 26) return RTSDF_EINVAL;
    *out = nullptr;
    hipStream_t s = as_stream(stream);
    std::vector<float> hv((size_t)3 * nv);
    std::vector<int32_t> hf((size_t)3 * nt);
    if (nv > 0) RTSDF_TRY(hipMemcpyAsync(hv.data(), vertices, sizeof(float) * 3 * nv, hipMemcpyDeviceToHost, s));
    if (nt > 0) RTSDF_TRY(hipMemcpyAsync(hf.data(), faces, sizeof(int32_t) * 3 * nt, hipMemcpyDeviceToHost, s));
    RTSDF_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < 3 * nt; ++i)
        if (hf[i] < 0 || hf[i] >= nv) return RTSDF_EINVAL;
    float scale = 1.0f;
    for (float x : hv) {
        if (!std::isfinite(x)) return RTSDF_EINVAL;
        scale = std::max(scale, std::fabs(x));
    }
    HostBuilder B{hv.data(), hf.data(), nt, leaf_size, std::ldexp(scale, -17), {}, {}, {}, {}};
    std::vector<int32_t> ref_tri, ref_path;
    make_references(hv, hf, nt, B.tb, ref_tri, ref_path);
    const int nref = (int)ref_tri.size();
    if (nref >= kMaxRefs) return RTSDF_EINVAL;
    B.cen.resize((size_t)3 * nref);
    B.idx.resize(nref);
    for (int r = 0; r < nref; ++r) {
        for (int a = 0; a < 3; ++a) B.cen[3 * r + a] = 0.5f * (B.tb[r].lo[a] + B.tb[r].hi[a]);
        B.idx[r] = r;
    }
    if (nref > 0) {
        const int code = B.build(0, nref, 0);  // an internal root is node 0
        if (code < 0) {
            // the whole mesh is one leaf: a root holding it and an empty leaf
            B.nodes.emplace_back();
            float lo[3], hi[3];
            B.padded(B.range_box(0, nref), lo, hi);
            BvhNode &nd = B.nodes[0];
            nd.xy0 = nd.xy1 = make_float4(lo[0], hi[0], lo[1], hi[1]);
            nd.z01 = make_float4(lo[2], hi[2], lo[2], hi[2]);
            nd.meta = make_int4(code, leaf_code(0, 0), -1, 0);
            B.max_depth = 1;
        }
    }
    std::unique_ptr<rtsdf_scene> sc(new rtsdf_scene());
    sc->nv = nv;
    sc->nt = nt;
    sc->nref = nref;
    sc->nnodes = (int)B.nodes.size();
    sc->max_depth = B.max_depth;
    sc->max_leaf = B.max_leaf;
    sc->leaf_size = leaf_size;
    sc->pad = B.pad;
    RTSDF_TRY(hipGetDevice(&sc->device));
    std::vector<float4> htri((size_t)3 * std::max(nref, 1));
    std::vector<int4> hlf(std::max(nref, 1));
    for (int i = 0; i < nref; ++i) {
        const int r = B.idx[i], t = ref_tri[r];
        for (int k = 0; k < 3; ++k) {
            const float *p = &hv[3 * hf[3 * t + k]];
            float w = 0.f;
            if (k == 0) std::memcpy(&w, &t, sizeof(float));
            if (k == 1) std::memcpy(&w, &ref_path[r], sizeof(float));
            htri[3 * i + k] = make_float4(p[0], p[1], p[2], w);
        }
        hlf[i] = make_int4(hf[3 * t], hf[3 * t + 1], hf[3 * t + 2], t);
    }
    std::vector<int32_t> starts;
    for (int i = 0; i < sc->nnodes; ++i)
        if (B.nodes[i].meta.x < 0 && B.nodes[i].meta.y < 0) starts.push_back(i);
    sc->nstart = (int)starts.size();
    auto alloc = [&](void **p, size_t bytes) -> bool {
        if (bytes == 0) bytes = 16;
        if (hipMalloc(p, bytes) != hipSuccess) return false;
        sc->bytes += (int64_t)bytes;
        return true;
    };
    const size_t nn = std::max(sc->nnodes, 1);
    if (!alloc((void **)&sc->nodes, sizeof(BvhNode) * nn) || !alloc((void **)&sc->tris, sizeof(float4) * htri.size()) ||
        !alloc((void **)&sc->tmap, sizeof(float4) * (htri.size() + 1)) ||  // +1: the tracer's fetch reads 64 B
        !alloc((void **)&sc->leaf_faces, sizeof(int4) * hlf.size()) ||
        !alloc((void **)&sc->vertices, sizeof(float) * 3 * std::max(nv, 1)) ||
        !alloc((void **)&sc->faces, sizeof(int32_t) * 3 * std::max(nt, 1)) ||
        !alloc((void **)&sc->refit_counter, sizeof(int32_t) * nn) ||
        !alloc((void **)&sc->start_nodes, sizeof(int32_t) * std::max<size_t>(starts.size(), 1))) {
        rtsdf_scene_destroy(sc.release());
        return RTSDF_ENOMEM;
    }
    bool ok = true;
    if (sc->nnodes) ok &= hipMemcpyAsync(sc->nodes, B.nodes.data(), sizeof(BvhNode) * sc->nnodes, hipMemcpyHostToDevice, s) == hipSuccess;
    ok &= hipMemcpyAsync(sc->tris, htri.data(), sizeof(float4) * htri.size(), hipMemcpyHostToDevice, s) == hipSuccess;
    ok &= hipMemcpyAsync(sc->leaf_faces, hlf.data(), sizeof(int4) * hlf.size(), hipMemcpyHostToDevice, s) == hipSuccess;
    if (nv) ok &= hipMemcpyAsync(sc->vertices, hv.data(), sizeof(float) * 3 * nv, hipMemcpyHostToDevice, s) == hipSuccess;
    if (nt) ok &= hipMemcpyAsync(sc->faces, hf.data(), sizeof(int32_t) * 3 * nt, hipMemcpyHostToDevice, s) == hipSuccess;
    if (!starts.empty())
        ok &= hipMemcpyAsync(sc->start_nodes, starts.data(), sizeof(int32_t) * starts.size(), hipMemcpyHostToDevice, s) == hipSuccess;
    if (ok && nref > 0) {
        tri_maps<<<dim3((nref + 255) / 256), dim3(256), 0, s>>>(sc->tris, sc->tmap, nref);
        ok &= hipGetLastError() == hipSuccess;
    }
    ok &= hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        rtsdf_scene_destroy(sc.release());
        return RTSDF_EHIP;
    }
    *out = sc.release();
    return RTSDF_OK;
}

namespace rtsdf {
static int lbvh_run(rtsdf_scene *sc, bool rebuild, hipStream_t s);
}

extern "C" int rtsdf_scene_create(const float *vertices, int32_t nv, const int32_t *faces, int32_t nt,
                                  int32_t leaf_size, rtsdf_scene **out, rtsdf_stream stream)
{
    return rtsdf_scene_create_impl(vertices, nv, faces, nt, leaf_size, out, stream);
}

extern "C" int rtsdf_scene_refit(rtsdf_scene *scene, const float *vertices, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scene || (scene->nv > 0 && !vertices)) return RTSDF_EINVAL;
    if (scene->ninst > 0) return RTSDF_EINVAL;  // two-level scenes move by rtsdf_scene_set_transforms
    hipStream_t s = as_stream(stream);
    if (scene->nv > 0 && vertices != scene->vertices)
        RTSDF_TRY(hipMemcpyAsync(scene->vertices, vertices, sizeof(float) * 3 * scene->nv, hipMemcpyDeviceToDevice, s));
    if (scene->nref == 0) return RTSDF_OK;
    if (scene->lbvh) return lbvh_run(scene, false, s);  // a rebuilt tree refits through its own tables
    refit_tris<<<dim3((scene->nref + 255) / 256), dim3(256), 0, s>>>(scene->vertices, scene->leaf_faces, scene->tris,
                                                                      scene->nref);
    RTSDF_CHECK_LAUNCH();
    tri_maps<<<dim3((scene->nref + 255) / 256), dim3(256), 0, s>>>(scene->tris, scene->tmap, scene->nref);
    RTSDF_CHECK_LAUNCH();
    int rc = launch_fill<int32_t>(scene->refit_counter, 0, scene->nnodes, s);
    if (rc != RTSDF_OK) return rc;
    refit_nodes<<<dim3((scene->nstart + 255) / 256), dim3(256), 0, s>>>(scene->nodes, scene->tris, scene->start_nodes,
                                                                         scene->nstart, scene->refit_counter, scene->pad);
    RTSDF_CHECK_LAUNCH();
    if (scene->nodes4) {
        const int nslots = 4 * scene->nnodes4;
        wide_gather<<<dim3((nslots + 255) / 256), dim3(256), 0, s>>>(scene->nodes4, scene->map4, scene->nodes, nslots);
        RTSDF_CHECK_LAUNCH();
    }
    return RTSDF_OK;
}

namespace rtsdf {

// Collapse the two-child hierarchy into a 4-wide one (host): a wide node takes
// the two children of its two-child node and keeps replacing its internal
// child of largest box area by that child's two children while it has fewer
// than four (the usual greedy collapse); leaves stay where they are.  The
// boxes are copies of two-child slots, so a hit in the wide tree is a hit in
// the two-child tree and traversal finds the same closest hit.
static int wide_build(rtsdf_scene *sc, hipStream_t s)
{
    if (sc->nodes4) return RTSDF_OK;
    if (sc->ninst > 0 || sc->lbvh || sc->nnodes < 1 || sc->nref < 1) return RTSDF_EINVAL;
    std::vector<BvhNode> h(sc->nnodes);
    RTSDF_TRY(hipMemcpyAsync(h.data(), sc->nodes, sizeof(BvhNode) * h.size(), hipMemcpyDeviceToHost, s));
    RTSDF_TRY(hipStreamSynchronize(s));
    std::vector<BvhNode> w;
    std::vector<int32_t> map;
    int depth4 = 0;
    struct Slot {
        int node, slot;
    };
    auto code_of = [&](const Slot &q) { return q.slot ? h[q.node].meta.y : h[q.node].meta.x; };
    auto area_of = [&](const Slot &q) {
        const BvhNode &nd = h[q.node];
        const float4 xy = q.slot ? nd.xy1 : nd.xy0;
        const float lz = q.slot ? nd.z01.z : nd.z01.x, hz = q.slot ? nd.z01.w : nd.z01.y;
        const double dx = std::max(0.0, (double)xy.y - xy.x), dy = std::max(0.0, (double)xy.w - xy.z),
                     dz = std::max(0.0, (double)hz - lz);
        return dx * dy + dy * dz + dz * dx;
    };
    // iterative: (two-child node, wide index) pairs still to fill; wide nodes are allocated when first referenced
    struct Todo {
        int node2, wide, depth;
    };
    std::vector<Todo> todo{{0, 0, 0}};
    w.resize(2);
    map.resize(4, -1);
    while (!todo.empty()) {
        const Todo t = todo.back();
        todo.pop_back();
        depth4 = std::max(depth4, t.depth);
        std::vector<Slot> kids{{t.node2, 0}, {t.node2, 1}};
        while (kids.size() < 4) {
            int best = -1;
            double best_area = -1.0;
            for (int k = 0; k < (int)kids.size(); ++k)
                if (code_of(kids[k]) >= 0 && area_of(kids[k]) > best_area) {
                    best = k;
                    best_area = area_of(kids[k]);
                }
            if (best < 0) break;
            const int c = code_of(kids[best]);
            kids[best] = Slot{c, 0};
            kids.insert(kids.begin() + best + 1, Slot{c, 1});
        }
        for (int k = 0; k < 4; ++k) {
            BvhNode &rec = w[2 * t.wide + (k >> 1)];
            float *xy = (k & 1) ? &rec.xy1.x : &rec.xy0.x;
            float *z = &rec.z01.x;
            int *m = (k & 1) ? &rec.meta.y : &rec.meta.x;
            if (k < (int)kids.size()) {
                const Slot &q = kids[k];
                const BvhNode &nd = h[q.node];
                const float4 sxy = q.slot ? nd.xy1 : nd.xy0;
                xy[0] = sxy.x; xy[1] = sxy.y; xy[2] = sxy.z; xy[3] = sxy.w;
                z[2 * (k & 1)] = q.slot ? nd.z01.z : nd.z01.x;
                z[2 * (k & 1) + 1] = q.slot ? nd.z01.w : nd.z01.y;
                map[4 * t.wide + k] = q.node << 1 | q.slot;
                const int c = code_of(q);
                if (c >= 0) {  // an internal child: a new wide node, filled later
                    const int wi = (int)w.size() / 2;
                    *m = wi;
                    todo.push_back(Todo{c, wi, t.depth + 1});
                    w.resize(w.size() + 2);
                    map.resize(map.size() + 4, -1);
                } else {
                    *m = c;
                }
            } else {
                // empty child: a point box far outside the scene (finite, so every slab distance stays finite
                // for any ray set-up; entered only by a ray aimed exactly at it, and then an empty leaf)
                xy[0] = xy[1] = xy[2] = xy[3] = 1e18f;
                z[2 * (k & 1)] = z[2 * (k & 1) + 1] = 1e18f;
                *m = leaf_code(0, 0);
            }
        }
    }
    const int nw = (int)w.size() / 2;
    BvhNode *dn = nullptr;
    int32_t *dm = nullptr;
    if (hipMalloc((void **)&dn, sizeof(BvhNode) * w.size()) != hipSuccess) return RTSDF_ENOMEM;
    if (hipMalloc((void **)&dm, sizeof(int32_t) * map.size()) != hipSuccess) {
        (void)hipFree(dn);
        return RTSDF_ENOMEM;
    }
    if (hipMemcpyAsync(dn, w.data(), sizeof(BvhNode) * w.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(dm, map.data(), sizeof(int32_t) * map.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipFree(dn);
        (void)hipFree(dm);
        return RTSDF_EHIP;
    }
    sc->nodes4 = dn;
    sc->map4 = dm;
    sc->nnodes4 = nw;
    sc->depth4 = depth4;
    sc->bytes += (int64_t)(sizeof(BvhNode) * w.size() + sizeof(int32_t) * map.size());
    return RTSDF_OK;
}

static void wide_free(rtsdf_scene *sc)
{
    (void)hipFree(sc->nodes4);
    (void)hipFree(sc->map4);
    sc->nodes4 = nullptr;
    sc->map4 = nullptr;
    sc->nnodes4 = 0;
    sc->depth4 = 0;
}

}  // namespace rtsdf

extern "C" int rtsdf_scene_set_sign(rtsdf_scene *scene, int32_t policy, float shell)
{
    if (!scene || (policy != RTSDF_SIGN_VOTE && policy != RTSDF_SIGN_SHELL)) return RTSDF_EINVAL;
    if (policy == RTSDF_SIGN_SHELL && !(shell >= 0.0f && shell < __builtin_inff())) return RTSDF_EINVAL;
    scene->sign_policy = policy;
    scene->shell = policy == RTSDF_SIGN_SHELL ? shell : 0.0f;
    return RTSDF_OK;
}

extern "C" int rtsdf_scene_info_get(const rtsdf_scene *scene, rtsdf_scene_info *info)
{
    if (!scene || !info) return RTSDF_EINVAL;
    info->nv = scene->nv;
    info->nt = scene->nt;
    info->references = scene->nref;
    info->nodes = scene->nnodes;
    info->max_depth = scene->max_depth;
    info->leaf_size = scene->max_leaf;
    info->device_bytes = scene->bytes;
    info->instances = scene->ninst;
    return RTSDF_OK;
}

extern "C" int rtsdf_scene_hierarchy(const rtsdf_scene *scene, int32_t cap, float *boxes, int32_t *links,
                                     int32_t *parents, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scene || scene->ninst > 0 || cap < scene->nnodes || (scene->nnodes > 0 && (!boxes || !links)))
        return RTSDF_EINVAL;
    const int n = scene->nnodes;
    if (n == 0) return RTSDF_OK;
    std::vector<BvhNode> h(n);
    hipStream_t s = as_stream(stream);
    RTSDF_TRY(hipMemcpyAsync(h.data(), scene->nodes, sizeof(BvhNode) * n, hipMemcpyDeviceToHost, s));
    RTSDF_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) {
        const BvhNode &nd = h[i];
        const float xy[2][4] = {{nd.xy0.x, nd.xy0.y, nd.xy0.z, nd.xy0.w}, {nd.xy1.x, nd.xy1.y, nd.xy1.z, nd.xy1.w}};
        const float z[4] = {nd.z01.x, nd.z01.y, nd.z01.z, nd.z01.w};
        const int c[2] = {nd.meta.x, nd.meta.y};
        for (int sl = 0; sl < 2; ++sl) {
            float *b = boxes + 12 * (size_t)i + 6 * sl;
            b[0] = xy[sl][0], b[1] = xy[sl][2], b[2] = z[2 * sl];          // lo x, y, z
            b[3] = xy[sl][1], b[4] = xy[sl][3], b[5] = z[2 * sl + 1];      // hi x, y, z
            int32_t *l = links + 4 * (size_t)i + 2 * sl;
            if (c[sl] >= 0) l[0] = c[sl], l[1] = 0;
            else l[0] = -1 - leaf_first(c[sl]), l[1] = leaf_count(c[sl]);
        }
        if (parents) parents[i] = nd.meta.z;
    }
    return RTSDF_OK;
}

extern "C" void rtsdf_scene_destroy(rtsdf_scene *scene)
{
    if (!scene) return;
    lbvh_free(scene->lbvh);
    (void)hipFree(scene->obj_vertices);
    (void)hipFree(scene->vert_inst);
    (void)hipFree(scene->inst_obj_box);
    (void)hipFree(scene->inst_world_box);
    (void)hipFree(scene->transforms);
    (void)hipFree(scene->top_dirty);
    (void)hipFree(scene->top_level_off);
    (void)hipFree(scene->entry_part);
    (void)hipFree(scene->nodes);
    (void)hipFree(scene->tris);
    (void)hipFree(scene->tmap);
    (void)hipFree(scene->leaf_faces);
    (void)hipFree(scene->vertices);
    (void)hipFree(scene->faces);
    (void)hipFree(scene->refit_counter);
    (void)hipFree(scene->start_nodes);
    rtsdf::wide_free(scene);
    delete scene;
}
