// Two-level scenes: a static world plus parts that move rigidly.
//
// Refitting one hierarchy over moving geometry keeps its topology while the
// boxes of moving parts sweep through their neighbours', so tracing slows
// frame after frame (on the moving-scene workload an update takes 20x longer
// after 48 frames of continuous motion).  Here part 0 is the static world and
// parts 1.. move rigidly: each moving part's hierarchy is built once in its
// object space and stays tight, and the top level is one surface-area-
// heuristic tree over the static triangles (references, as in a single-level
// scene) and *entries*: a moving part enters as kCutEntries subtrees of its
// own hierarchy (its cut opened largest box first, the re-braiding idea of
// Benthin et al. 2017), each a child of its own.  Per frame only the entries'
// boxes change: the nodes above them are refit level by level, deepest first.
//
// Node array: [top level] [instance nodes (one per entry)] [hierarchy of
// moving part 1] [part 2] ...  An instance node carries the rows of its
// part's world-to-object transform in the three box slots and (root of the
// entry's subtree, kInstTag) as its children: the tracer that reaches it moves its
// ray into object space, pushes kReturn and descends; reaching kReturn, once
// the part's last leaf is tested, brings the ray back to world space.  The
// transforms are rigid (rotation and translation), so the ray parameter t,
// and with it the closest-hit order, is the same in both spaces.  Triangle
// records carry the global face index, so hits, the argmin record and the
// gradient name faces of the whole mesh.  World vertex positions (for
// voxelization and the gradient) are recomputed from the object positions at
// every transform update, each coordinate as ((r0 x + r1 y) + r2 z) + t with
// every float operation rounded once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "common.hpp"

namespace rtsdf {

constexpr float kRigidTol = 1e-4f;  // |R R^T - I| entries and |det R - 1| accepted as rigid
// subtrees per moving part in the top level.  One: with rotating parts, opened pieces sweep the part's whole
// sphere and loosen the top level over time (8 pieces: 6 % faster on the first frame of the moving-scene
// workload, 44 % slower after 48 frames of motion)
constexpr int kCutEntries = 1;

__host__ __device__ inline bool rigid_ok(const float *m)
{
    float err = 0.0f;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const float d = m[4 * a] * m[4 * b] + m[4 * a + 1] * m[4 * b + 1] + m[4 * a + 2] * m[4 * b + 2];
            err = fmaxf(err, fabsf(d - (a == b ? 1.0f : 0.0f)));
        }
    const float det = m[0] * (m[5] * m[10] - m[6] * m[9]) - m[1] * (m[4] * m[10] - m[6] * m[8]) +
                      m[2] * (m[4] * m[9] - m[5] * m[8]);
    return err <= kRigidTol && fabsf(det - 1.0f) <= kRigidTol;
}

// entry k (a subtree of moving part part[k]): world-to-object rows into its instance node, its world box
__global__ void inst_update(const float *__restrict__ T, const int32_t *__restrict__ part, int nent, BvhNode *nodes,
                            int inst_base, const float *__restrict__ obj_box, float *__restrict__ world_box,
                            float pad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nent) return;
    float m[12];
    for (int q = 0; q < 12; ++q) m[q] = T[12 * part[k] + q];
    if (!rigid_ok(m)) raise_error(RTSDF_ERR_TRANSFORM);
    float inv[12];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) inv[4 * r + c] = m[4 * c + r];
        inv[4 * r + 3] = -(m[r] * m[3] + m[4 + r] * m[7] + m[8 + r] * m[11]);
    }
    BvhNode *nd = &nodes[inst_base + k];
    nd->xy0 = make_float4(inv[0], inv[1], inv[2], inv[3]);
    nd->xy1 = make_float4(inv[4], inv[5], inv[6], inv[7]);
    nd->z01 = make_float4(inv[8], inv[9], inv[10], inv[11]);
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    const float *b = obj_box + 6 * k;
    for (int corner = 0; corner < 8; ++corner) {
        const float p[3] = {b[(corner & 1) ? 3 : 0], b[(corner & 2) ? 4 : 1], b[(corner & 4) ? 5 : 2]};
        for (int a = 0; a < 3; ++a) {
            const float w = m[4 * a] * p[0] + m[4 * a + 1] * p[1] + m[4 * a + 2] * p[2] + m[4 * a + 3];
            lo[a] = fminf(lo[a], w);
            hi[a] = fmaxf(hi[a], w);
        }
    }
    for (int a = 0; a < 3; ++a) {
        world_box[6 * k + a] = nextafterf(lo[a] - pad, -__builtin_inff());
        world_box[6 * k + 3 + a] = nextafterf(hi[a] + pad, __builtin_inff());
    }
}

// the top-level nodes above moving parts, one level at a time from the deepest (one workgroup); a slot whose
// child is a leaf of static triangles keeps its box
__global__ void __launch_bounds__(256) top_refit(BvhNode *nodes, const int32_t *__restrict__ dirty,
                                                 const int32_t *__restrict__ level_off, int nlevels, int inst_base,
                                                 int nent, const float *__restrict__ world_box)
{
    for (int L = 0; L < nlevels; ++L) {
        for (int k = level_off[L] + (int)threadIdx.x; k < level_off[L + 1]; k += blockDim.x) {
            BvhNode *p = &nodes[dirty[k]];
            const int c[2] = {p->meta.x, p->meta.y};
            for (int s = 0; s < 2; ++s) {
                if (c[s] < 0) continue;
                float lo[3], hi[3];
                if (c[s] >= inst_base && c[s] < inst_base + nent) {
                    const float *b = world_box + 6 * (c[s] - inst_base);
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = b[a];
                        hi[a] = b[3 + a];
                    }
                } else {
                    float l2[3], h2[3];
                    get_slot(&nodes[c[s]], 0, lo, hi);
                    get_slot(&nodes[c[s]], 1, l2, h2);
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = fminf(lo[a], l2[a]);
                        hi[a] = fmaxf(hi[a], h2[a]);
                    }
                }
                set_slot(p, s, lo, hi);
            }
        }
        __syncthreads();
    }
}

__global__ void inst_world_vertices(const float *__restrict__ obj, const int32_t *__restrict__ vinst,
                                    const float *__restrict__ T, int nv, float *__restrict__ world,
                                    float *__restrict__ out)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const float x = obj[3 * v], y = obj[3 * v + 1], z = obj[3 * v + 2];
    const int i = vinst[v];
    float w[3] = {x, y, z};
    if (i > 0) {  // part 0 is the static world
        const float *m = T + 12 * i;
        for (int a = 0; a < 3; ++a)
            w[a] = rn_add(rn_add(rn_add(rn_mul(m[4 * a], x), rn_mul(m[4 * a + 1], y)), rn_mul(m[4 * a + 2], z)),
                          m[4 * a + 3]);
    }
    for (int a = 0; a < 3; ++a) {
        world[3 * v + a] = w[a];
        if (out) out[3 * v + a] = w[a];
    }
}

static int launch_transforms(rtsdf_scene *sc, float *world_out, hipStream_t s)
{
    const int nent = sc->nentries;
    if (nent > 0) {
        inst_update<<<dim3((nent + 63) / 64), dim3(64), 0, s>>>(sc->transforms, sc->entry_part, nent, sc->nodes,
                                                                sc->inst_base, sc->inst_obj_box, sc->inst_world_box,
                                                                sc->pad);
        RTSDF_CHECK_LAUNCH();
        top_refit<<<dim3(1), dim3(256), 0, s>>>(sc->nodes, sc->top_dirty, sc->top_level_off, sc->top_levels,
                                                sc->inst_base, nent, sc->inst_world_box);
        RTSDF_CHECK_LAUNCH();
    }
    if (sc->nv > 0) {
        inst_world_vertices<<<dim3((sc->nv + 255) / 256), dim3(256), 0, s>>>(sc->obj_vertices, sc->vert_inst,
                                                                              sc->transforms, sc->nv, sc->vertices,
                                                                              world_out);
        RTSDF_CHECK_LAUNCH();
    }
    return RTSDF_OK;
}

}  // namespace rtsdf

static int rtsdf_scene_create_instanced_impl(const float *vertices, int32_t nv, const int32_t *faces, int32_t nt,
                                             const int32_t *instance_faces, int32_t ninst, const float *transforms,
                                             int32_t leaf_size, rtsdf_scene **out, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!out || !instance_faces || !transforms || ninst < 1 || nv < 1 || nt < 1 || !vertices || !faces)
        return RTSDF_EINVAL;
    if (leaf_size <= 0) leaf_size = 4;
    if (leaf_size > kMaxLeaf || (int64_t)nt >= (int64_t)1 << 26 || ninst > (1 << 20)) return RTSDF_EINVAL;
    if (instance_faces[0] != 0 || instance_faces[ninst] != nt || instance_faces[1] < 0) return RTSDF_EINVAL;
    for (int i = 1; i < ninst; ++i)
        if (instance_faces[i + 1] <= instance_faces[i]) return RTSDF_EINVAL;  // every moving part has a face
    *out = nullptr;
    hipStream_t s = as_stream(stream);
    const int nmov = ninst - 1;
    std::vector<float> hv((size_t)3 * nv), hT((size_t)12 * ninst);
    std::vector<int32_t> hf((size_t)3 * nt);
    RTSDF_TRY(hipMemcpyAsync(hv.data(), vertices, sizeof(float) * hv.size(), hipMemcpyDeviceToHost, s));
    RTSDF_TRY(hipMemcpyAsync(hf.data(), faces, sizeof(int32_t) * hf.size(), hipMemcpyDeviceToHost, s));
    RTSDF_TRY(hipMemcpyAsync(hT.data(), transforms, sizeof(float) * hT.size(), hipMemcpyDeviceToHost, s));
    RTSDF_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> vinst(nv, -1);
    for (int i = 0; i < ninst; ++i)
        for (int t = instance_faces[i]; t < instance_faces[i + 1]; ++t)
            for (int k = 0; k < 3; ++k) {
                const int v = hf[3 * t + k];
                if (v < 0 || v >= nv) return RTSDF_EINVAL;
                if (vinst[v] >= 0 && vinst[v] != i) return RTSDF_EINVAL;  // a vertex belongs to one part
                vinst[v] = i;
            }
    float obj_scale = 1.0f;
    for (float x : hv) {
        if (!std::isfinite(x)) return RTSDF_EINVAL;
        obj_scale = std::max(obj_scale, std::fabs(x));
    }
    float scale = obj_scale;  // bounds world coordinates: |R p + t| <= |p| + |t|
    for (int i = 1; i < ninst; ++i) {
        for (int k = 0; k < 12; ++k)
            if (!std::isfinite(hT[12 * i + k])) return RTSDF_EINVAL;
        if (!rigid_ok(&hT[12 * i])) return RTSDF_EINVAL;
        for (int a = 0; a < 3; ++a) scale = std::max(scale, obj_scale + std::fabs(hT[12 * i + 4 * a + 3]));
    }
    const float pad = std::ldexp(scale, -17);

    // each moving part's own hierarchy, in object space
    struct Part {
        std::vector<BvhNode> nodes;
        std::vector<int32_t> ref_face, ref_path;  // leaf order, global face index
        int depth = 0, max_leaf = 0;
        Aabb box;
    };
    auto one_leaf_root = [&](HostBuilder &B, int code, int nitems) {  // a root holding one child and an empty leaf
        B.nodes.emplace_back();
        float lo[3], hi[3];
        B.padded(B.range_box(0, nitems), lo, hi);
        BvhNode &nd = B.nodes[0];
        nd.xy0 = nd.xy1 = make_float4(lo[0], hi[0], lo[1], hi[1]);
        nd.z01 = make_float4(lo[2], hi[2], lo[2], hi[2]);
        nd.meta = make_int4(code, leaf_code(0, 0), -1, 0);
        B.max_depth = std::max(B.max_depth, 1);
    };
    std::vector<Part> parts(nmov);
    for (int k = 0; k < nmov; ++k) {
        const int f0 = instance_faces[k + 1], nti = instance_faces[k + 2] - f0;
        std::vector<int32_t> sub(hf.begin() + 3 * (size_t)f0, hf.begin() + 3 * (size_t)(f0 + nti));
        HostBuilder B{hv.data(), sub.data(), nti, leaf_size, pad, {}, {}, {}, {}};
        std::vector<int32_t> ref_tri, ref_path;
        make_references(hv, sub, nti, B.tb, ref_tri, ref_path);
        const int nref = (int)ref_tri.size();
        B.cen.resize((size_t)3 * nref);
        B.idx.resize(nref);
        for (int r = 0; r < nref; ++r) {
            for (int a = 0; a < 3; ++a) B.cen[3 * r + a] = 0.5f * (B.tb[r].lo[a] + B.tb[r].hi[a]);
            B.idx[r] = r;
        }
        const int code = B.build(0, nref, 0);
        if (code < 0) one_leaf_root(B, code, nref);
        Part &P = parts[k];
        P.nodes = std::move(B.nodes);
        P.depth = B.max_depth;
        P.max_leaf = B.max_leaf;
        for (int q = 0; q < nref; ++q) {
            P.ref_face.push_back(f0 + ref_tri[B.idx[q]]);
            P.ref_path.push_back(ref_path[B.idx[q]]);
        }
        const BvhNode &r0 = P.nodes[0];  // the part's box: both slots of its root
        const float lo0[3] = {r0.xy0.x, r0.xy0.z, r0.z01.x}, hi0[3] = {r0.xy0.y, r0.xy0.w, r0.z01.y};
        const float lo1[3] = {r0.xy1.x, r0.xy1.z, r0.z01.z}, hi1[3] = {r0.xy1.y, r0.xy1.w, r0.z01.w};
        P.box.reset();
        P.box.grow_pt(lo0);  // (a one-leaf part repeats its box in both slots)
        P.box.grow_pt(hi0);
        P.box.grow_pt(lo1);
        P.box.grow_pt(hi1);
    }

    // entries: each moving part enters the top level as a few subtrees of its own hierarchy, the cut opened
    // largest object-space box first (re-braiding, after Benthin et al. 2017), so the top level can separate
    // a large part's pieces instead of testing one loose box around all of it
    struct Entry {
        int part;  // moving part index k (part k + 1)
        int code;  // subtree root in the part's own numbering: node index or leaf code
        Aabb box;  // object space
    };
    std::vector<Entry> entries;
    auto slot_box = [](const BvhNode &nd, int s) {
        Aabb b;
        b.reset();
        const float lo[3] = {s ? nd.xy1.x : nd.xy0.x, s ? nd.xy1.z : nd.xy0.z, s ? nd.z01.z : nd.z01.x};
        const float hi[3] = {s ? nd.xy1.y : nd.xy0.y, s ? nd.xy1.w : nd.xy0.w, s ? nd.z01.w : nd.z01.y};
        b.grow_pt(lo);
        b.grow_pt(hi);
        return b;
    };
    for (int k = 0; k < nmov; ++k) {
        std::vector<Entry> cut;
        auto add_children = [&](int node) {
            const BvhNode &nd = parts[k].nodes[node];
            for (int s2 = 0; s2 < 2; ++s2) {
                const int c = s2 ? nd.meta.y : nd.meta.x;
                if (c < 0 && leaf_count(c) == 0) continue;  // the empty leaf of a one-leaf part
                cut.push_back(Entry{k, c, slot_box(nd, s2)});
            }
        };
        cut.push_back(Entry{k, 0, parts[k].box});  // the whole part, then opened while the budget allows
        while ((int)cut.size() < kCutEntries) {
            int best = -1;
            for (int q = 0; q < (int)cut.size(); ++q)
                if (cut[q].code >= 0 && (best < 0 || cut[q].box.area() > cut[best].box.area())) best = q;
            if (best < 0) break;
            const int node = cut[best].code;
            cut.erase(cut.begin() + best);
            add_children(node);
        }
        entries.insert(entries.end(), cut.begin(), cut.end());
    }
    const int nent = (int)entries.size();

    // the top level: static triangle references and the entries' world boxes, one tree
    const int f_static = instance_faces[1];
    std::vector<int32_t> sub0(hf.begin(), hf.begin() + 3 * (size_t)f_static);
    HostBuilder T{hv.data(), sub0.data(), f_static, leaf_size, pad, {}, {}, {}, {}};
    std::vector<int32_t> ref_tri, ref_path;
    make_references(hv, sub0, f_static, T.tb, ref_tri, ref_path);
    const int nsref = (int)ref_tri.size();
    std::vector<int> item_part(nsref, -1);
    for (int e = 0; e < nent; ++e) {
        const float *m = &hT[12 * (entries[e].part + 1)];
        const Aabb &ob = entries[e].box;
        Aabb wb;
        wb.reset();
        for (int corner = 0; corner < 8; ++corner) {
            const float p[3] = {(corner & 1) ? ob.hi[0] : ob.lo[0], (corner & 2) ? ob.hi[1] : ob.lo[1],
                                (corner & 4) ? ob.hi[2] : ob.lo[2]};
            float w[3];
            for (int a = 0; a < 3; ++a) w[a] = m[4 * a] * p[0] + m[4 * a + 1] * p[1] + m[4 * a + 2] * p[2] + m[4 * a + 3];
            wb.grow_pt(w);
        }
        T.tb.push_back(wb);
        item_part.push_back(e);
    }
    const int nitems = (int)T.tb.size();
    T.cen.resize((size_t)3 * nitems);
    T.idx.resize(nitems);
    for (int r = 0; r < nitems; ++r) {
        for (int a = 0; a < 3; ++a) T.cen[3 * r + a] = 0.5f * (T.tb[r].lo[a] + T.tb[r].hi[a]);
        T.idx[r] = r;
    }
    T.item_part = &item_part;
    const int tcode = T.build(0, nitems, 0);
    if (tcode < 0 || tcode >= HostBuilder::kInstItem) one_leaf_root(T, tcode, nitems);
    const int ntop = (int)T.nodes.size(), inst_base = ntop;
    std::vector<BvhNode> nodes(T.nodes);
    std::vector<int> inst_parent(nent, -1);
    for (int id = 0; id < ntop; ++id) {
        int *ch[2] = {&nodes[id].meta.x, &nodes[id].meta.y};
        for (int *c : ch)
            if (*c >= HostBuilder::kInstItem) {
                inst_parent[*c - HostBuilder::kInstItem] = id;
                *c = inst_base + (*c - HostBuilder::kInstItem);
            }
    }
    // top-level records in item order; the positions of moving parts hold no triangle (no leaf points there)
    std::vector<float4> htri;
    std::vector<int4> hlf;
    for (int q = 0; q < nitems; ++q) {
        const int item = T.idx[q];
        if (item >= nsref) {
            const int none = -1;
            float w = 0.f;
            std::memcpy(&w, &none, sizeof(float));
            htri.push_back(make_float4(0.f, 0.f, 0.f, w));
            htri.push_back(make_float4(0.f, 0.f, 0.f, 0.f));
            htri.push_back(make_float4(0.f, 0.f, 0.f, 0.f));
            hlf.push_back(make_int4(0, 0, 0, -1));
            continue;
        }
        const int t = ref_tri[item], path = ref_path[item];
        for (int c = 0; c < 3; ++c) {
            const float *p = &hv[3 * hf[3 * t + c]];
            float w = 0.f;
            if (c == 0) std::memcpy(&w, &t, sizeof(float));
            if (c == 1) std::memcpy(&w, &path, sizeof(float));
            htri.push_back(make_float4(p[0], p[1], p[2], w));
        }
        hlf.push_back(make_int4(hf[3 * t], hf[3 * t + 1], hf[3 * t + 2], t));
    }
    // nodes above moving parts, grouped by depth, deepest first
    std::vector<int> depth(ntop, 0);
    for (int id = 0; id < ntop; ++id)  // preorder: a parent comes before its children
        for (int c : {nodes[id].meta.x, nodes[id].meta.y})
            if (c >= 0 && c < ntop) depth[c] = depth[id] + 1;
    std::vector<char> is_dirty(ntop, 0);
    int max_top = 0;
    for (int e = 0; e < nent; ++e) {
        max_top = std::max(max_top, depth[inst_parent[e]] + 1);
        for (int id = inst_parent[e]; id >= 0 && !is_dirty[id]; id = nodes[id].meta.z) is_dirty[id] = 1;
    }
    std::vector<int32_t> dirty, level_off;
    int max_d = 0;
    for (int id = 0; id < ntop; ++id)
        if (is_dirty[id]) max_d = std::max(max_d, depth[id]);
    for (int d = max_d; d >= 0; --d) {
        level_off.push_back((int)dirty.size());
        for (int id = 0; id < ntop; ++id)
            if (is_dirty[id] && depth[id] == d) dirty.push_back(id);
    }
    level_off.push_back((int)dirty.size());
    if (dirty.empty()) level_off.assign(1, 0);
    // instance nodes (one per entry), then each moving part's hierarchy
    nodes.resize((size_t)inst_base + nent);
    int max_part = 0, max_leaf = T.max_leaf;
    std::vector<int> part_nbase(nmov), part_rbase(nmov);
    for (int k = 0; k < nmov; ++k) {
        const int nbase = (int)nodes.size(), rbase = (int)hlf.size();
        part_nbase[k] = nbase;
        part_rbase[k] = rbase;
        for (const BvhNode &b : parts[k].nodes) {
            BvhNode nd = b;
            int *ch[2] = {&nd.meta.x, &nd.meta.y};
            for (int *c : ch) *c = *c >= 0 ? *c + nbase : leaf_code(leaf_first(*c) + rbase, leaf_count(*c));
            if (nd.meta.z >= 0) nd.meta.z += nbase;
            nodes.push_back(nd);
        }
        for (size_t q = 0; q < parts[k].ref_face.size(); ++q) {
            const int t = parts[k].ref_face[q], path = parts[k].ref_path[q];
            for (int c = 0; c < 3; ++c) {
                const float *p = &hv[3 * hf[3 * t + c]];
                float w = 0.f;
                if (c == 0) std::memcpy(&w, &t, sizeof(float));
                if (c == 1) std::memcpy(&w, &path, sizeof(float));
                htri.push_back(make_float4(p[0], p[1], p[2], w));
            }
            hlf.push_back(make_int4(hf[3 * t], hf[3 * t + 1], hf[3 * t + 2], t));
        }
        max_part = std::max(max_part, parts[k].depth);
        max_leaf = std::max(max_leaf, parts[k].max_leaf);
    }
    for (int e = 0; e < nent; ++e) {
        const Entry &E = entries[e];
        const int k = E.part;
        const int root = E.code >= 0 ? E.code + part_nbase[k]
                                     : leaf_code(leaf_first(E.code) + part_rbase[k], leaf_count(E.code));
        BvhNode &inode = nodes[inst_base + e];
        inode.xy0 = inode.xy1 = inode.z01 = make_float4(0.f, 0.f, 0.f, 0.f);  // rows written on the device
        inode.meta = make_int4(root, kInstTag, inst_parent[e], k + 1);
    }
    const int nref = (int)hlf.size();
    if (nref >= kMaxRefs) return RTSDF_EINVAL;
    std::vector<float> obox((size_t)6 * std::max(nent, 1));
    std::vector<int32_t> epart(std::max(nent, 1), 0);
    for (int e = 0; e < nent; ++e) {
        epart[e] = entries[e].part + 1;
        for (int a = 0; a < 3; ++a) {
            obox[6 * e + a] = entries[e].box.lo[a];
            obox[6 * e + 3 + a] = entries[e].box.hi[a];
        }
    }

    std::unique_ptr<rtsdf_scene> sc(new rtsdf_scene());
    sc->nv = nv;
    sc->nt = nt;
    sc->nref = nref;
    sc->nnodes = (int)nodes.size();
    // stack: pending top-level entries, the return marker, then the part's own entries
    sc->max_depth = std::max(T.max_depth, max_top) + 2 + max_part;
    sc->max_leaf = max_leaf;
    sc->pad = pad;
    sc->ninst = ninst;
    sc->inst_base = inst_base;
    sc->top_levels = (int)level_off.size() - 1;
    sc->nentries = nent;
    RTSDF_TRY(hipGetDevice(&sc->device));
    auto alloc = [&](void **p, size_t bytes) -> bool {
        if (bytes == 0) bytes = 16;
        if (hipMalloc(p, bytes) != hipSuccess) return false;
        sc->bytes += (int64_t)bytes;
        return true;
    };
    if (!alloc((void **)&sc->nodes, sizeof(BvhNode) * nodes.size()) ||
        !alloc((void **)&sc->tris, sizeof(float4) * htri.size()) ||
        !alloc((void **)&sc->tmap, sizeof(float4) * (htri.size() + 1)) ||  // +1: the tracer's fetch reads 64 B
        !alloc((void **)&sc->leaf_faces, sizeof(int4) * hlf.size()) ||
        !alloc((void **)&sc->vertices, sizeof(float) * 3 * nv) || !alloc((void **)&sc->faces, sizeof(int32_t) * 3 * nt) ||
        !alloc((void **)&sc->refit_counter, sizeof(int32_t)) || !alloc((void **)&sc->start_nodes, sizeof(int32_t)) ||
        !alloc((void **)&sc->obj_vertices, sizeof(float) * 3 * nv) ||
        !alloc((void **)&sc->vert_inst, sizeof(int32_t) * nv) ||
        !alloc((void **)&sc->inst_obj_box, sizeof(float) * obox.size()) ||
        !alloc((void **)&sc->inst_world_box, sizeof(float) * obox.size()) ||
        !alloc((void **)&sc->transforms, sizeof(float) * hT.size()) ||
        !alloc((void **)&sc->top_dirty, sizeof(int32_t) * std::max<size_t>(dirty.size(), 1)) ||
        !alloc((void **)&sc->top_level_off, sizeof(int32_t) * level_off.size()) ||
        !alloc((void **)&sc->entry_part, sizeof(int32_t) * epart.size())) {
        rtsdf_scene_destroy(sc.release());
        return RTSDF_ENOMEM;
    }
    bool ok = true;
    auto up = [&](void *dst, const void *src, size_t bytes) {
        if (bytes) ok &= hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    up(sc->nodes, nodes.data(), sizeof(BvhNode) * nodes.size());
    up(sc->tris, htri.data(), sizeof(float4) * htri.size());
    up(sc->leaf_faces, hlf.data(), sizeof(int4) * hlf.size());
    up(sc->obj_vertices, hv.data(), sizeof(float) * hv.size());
    up(sc->faces, hf.data(), sizeof(int32_t) * hf.size());
    up(sc->vert_inst, vinst.data(), sizeof(int32_t) * nv);
    up(sc->inst_obj_box, obox.data(), sizeof(float) * obox.size());
    up(sc->transforms, hT.data(), sizeof(float) * hT.size());
    up(sc->top_dirty, dirty.data(), sizeof(int32_t) * dirty.size());
    up(sc->top_level_off, level_off.data(), sizeof(int32_t) * level_off.size());
    up(sc->entry_part, epart.data(), sizeof(int32_t) * epart.size());
    if (ok) {
        tri_maps<<<dim3((nref + 255) / 256), dim3(256), 0, s>>>(sc->tris, sc->tmap, nref);
        ok &= hipGetLastError() == hipSuccess;
    }
    if (ok) ok = launch_transforms(sc.get(), nullptr, s) == RTSDF_OK;
    ok &= hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        rtsdf_scene_destroy(sc.release());
        return RTSDF_EHIP;
    }
    *out = sc.release();
    return RTSDF_OK;
}

extern "C" int rtsdf_scene_create_instanced(const float *vertices, int32_t nv, const int32_t *faces, int32_t nt,
                                            const int32_t *instance_faces, int32_t ninst, const float *transforms,
                                            int32_t leaf_size, rtsdf_scene **out, rtsdf_stream stream)
{
    int rc = rtsdf_scene_create_instanced_impl(vertices, nv, faces, nt, instance_faces, ninst, transforms, leaf_size,
                                               out, stream);
    if (rc != RTSDF_OK) return rc;
    if ((*out)->max_depth + 1 > 64) rc = RTSDF_EINVAL;  // deeper than the tracer's stack
    if (rc != RTSDF_OK) {
        rtsdf_scene_destroy(*out);
        *out = nullptr;
    }
    return rc;
}

extern "C" int rtsdf_scene_set_transforms(rtsdf_scene *scene, const float *transforms, float *world_vertices,
                                          rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scene || scene->ninst == 0 || !transforms) return RTSDF_EINVAL;
    hipStream_t s = as_stream(stream);
    if (transforms != scene->transforms)
        RTSDF_TRY(hipMemcpyAsync(scene->transforms, transforms, sizeof(float) * 12 * scene->ninst,
                                 hipMemcpyDeviceToDevice, s));
    return launch_transforms(scene, world_vertices, s);
}

extern "C" int rtsdf_scene_world_vertices(const rtsdf_scene *scene, float *out, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scene || (scene->nv > 0 && !out)) return RTSDF_EINVAL;
    if (scene->nv == 0) return RTSDF_OK;
    RTSDF_TRY(hipMemcpyAsync(out, scene->vertices, sizeof(float) * 3 * scene->nv, hipMemcpyDeviceToDevice,
                             as_stream(stream)));
    return RTSDF_OK;
}
