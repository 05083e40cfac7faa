// Many independent scenes per launch.
//
// A batch owns every buffer of its scenes in pooled device allocations and
// runs each stage of the SDF update for all scenes at once:
//
//   voxelize  one launch over all (scene, triangle, axis) items; an item finds
//             its scene by binary search over the per-scene item prefix;
//   JFA       per pass index, one launch per pass kind with blockIdx.y = scene.
//             Passes are right-aligned (a scene with fewer passes starts
//             later) so every scene's final step-1 pass, which writes the
//             outputs, happens in the same launch.  The per-(pass, scene)
//             plan is built on the host at creation;
//   select    count / scan / scatter / mask with blockIdx.y = scene;
//   trace     one persistent launch over all scenes: a wavefront takes a global
//             tile index and finds its scene through a device-side tile prefix
//             built after selection (the texel counts never leave the GPU).
//
// Grids of a batch: coarse n a power of two in [8, 128], fine n a power-of-two
// multiple of it (at most 1024).  Every scene's outputs are bit-identical to
// running it alone through the single-scene entry points.
#include <algorithm>
#include <array>
#include <vector>

#include "common.hpp"
#include "jfa_device.hpp"

namespace rtsdf {

struct BatchVox {
    const float *v;
    int nv;
    const int32_t *f;
    int nt;
    rtsdf_grid g;
    int32_t *seeds;
    int64_t item_begin;
};

enum JfaKind { kJfaNone = 0, kJfaConvert, kJfaFarBricks, kJfaFarLinear, kJfaNear2, kJfaFinal, kJfaKinds };

struct JfaStep {
    int kind;
    int n, logn, kb;
    const int32_t *src;
    int32_t *dst;
    int32_t *dist2;
    float *sdf;
    float h, beta;
};

struct SelScene {
    const int32_t *d2;
    int logn, K;
    uint32_t total;
    uint32_t *sums;
    uint32_t nblocks;
    int logr, nf;
    int32_t *queue;
    int32_t cap;
    int32_t *count;
    uint32_t *mask4;
    int64_t nquads;
};

struct FillScene {
    const uint8_t *mask;
    const float *coarse_sdf;
    int nc, logr, lognf;
    int64_t ntex;
    float *u;
    uint32_t *hits;
    int32_t *arg_tri, *arg_ray;
    float *fine;
};

__global__ void __launch_bounds__(256) voxelize_batch(const BatchVox *__restrict__ sc, int ns, int64_t items)
{
    // the same strided dealing of items to wavefronts as the single-scene kernel
    const int64_t waves = (items + kWave - 1) / kWave;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t item = (gid & (kWave - 1)) * waves + (gid >> 6);
    VoxTri T;
    bool big = false;
    int32_t *seeds = nullptr;
    int n = 0;
    if ((gid >> 6) < waves && item < items) {
        int lo = 0, hi = ns - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sc[mid].item_begin <= item) lo = mid;
            else hi = mid - 1;
        }
        const BatchVox &B = sc[lo];
        const int64_t local = item - B.item_begin;
        seeds = B.seeds;
        n = B.g.n;
        if (local < 3 * (int64_t)B.nt)
            big = vox_item(B.v, B.nv, B.f, (int)(local / 3), (int)(local % 3), B.g, B.seeds, T);
    }
    vox_wave_big(big, T, seeds, n);
}

// Flat launches: the workgroups of every scene that has work in a stage are
// numbered consecutively; a workgroup finds its scene by a binary search over
// the scenes' first workgroup numbers (the search is uniform per workgroup).
// A grid sized by the largest scene times the scene count would leave most
// workgroups of small scenes without work.
struct FlatRange {
    int32_t scene;
    uint32_t first;  // first workgroup number of the scene in this launch
    uint32_t count;  // its workgroups
};

__device__ __forceinline__ const FlatRange &flat_find(const FlatRange *__restrict__ r, int nr, uint32_t g)
{
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (r[mid].first <= g) lo = mid;
        else hi = mid - 1;
    }
    return r[__builtin_amdgcn_readfirstlane(lo)];
}

template <int KIND>
__global__ void __launch_bounds__(KIND == kJfaNear2 || KIND == kJfaFinal ? 512 : 256)
    jfa_batch(const JfaStep *__restrict__ plan, const FlatRange *__restrict__ ranges, int nr, int neg2)
{
    const FlatRange &fr = flat_find(ranges, nr, blockIdx.x);
    const JfaStep &st = plan[fr.scene];
    const uint32_t blk = blockIdx.x - fr.first, nblk = fr.count;
    if (KIND == kJfaConvert) {
        const int64_t nvox = (int64_t)st.n * st.n * st.n;
        const int64_t e = (int64_t)blk * blockDim.x + threadIdx.x;
        if (e < nvox) jfa_to_bricks_body(st.src, st.dst, st.n, st.logn, e);
    } else if (KIND == kJfaFarBricks && st.n >= 16) {
        // 2 x 2 brick quads per wavefront (a workgroup per 1024 voxels), as the single-scene passes
        jfa_far_quad_body<false>(st.src, st.dst, st.n, st.logn, st.kb, blk, nblk, neg2);
    } else if (KIND == kJfaFarBricks || KIND == kJfaFarLinear) {
        jfa_far_body<false, KIND == kJfaFarLinear>(st.src, st.dst, st.n, st.logn, st.kb, blk, nblk, neg2, 0);
    } else if (KIND == kJfaNear2) {
        jfa_near_body<2, true, false>(st.src, st.dst, st.n, st.logn, nullptr, nullptr, 0.f, 0.f, blk, nblk, neg2);
    } else {
        jfa_near_body<1, true, true>(st.src, st.dst, st.n, st.logn, st.dist2, st.sdf, st.h, st.beta, blk, nblk,
                                     neg2);
    }
}

__global__ void __launch_bounds__(kSelBlock) select_count_batch(const SelScene *__restrict__ sc,
                                                                 const FlatRange *__restrict__ ranges, int nr)
{
    const FlatRange &fr = flat_find(ranges, nr, blockIdx.x);
    const SelScene &S = sc[fr.scene];
    select_count_body(SelPred{S.d2, S.K, nullptr, 0.0f}, S.logn, S.total, S.sums, blockIdx.x - fr.first);
}

__global__ void __launch_bounds__(1024) select_scan_batch(const SelScene *__restrict__ sc)
{
    const SelScene &S = sc[blockIdx.y];
    select_scan_body(S.sums, S.nblocks, 1u << (3 * S.logr), S.count, S.cap);
}

__global__ void __launch_bounds__(kSelBlock) select_scatter_batch(const SelScene *__restrict__ sc,
                                                                   const FlatRange *__restrict__ ranges, int nr)
{
    const FlatRange &fr = flat_find(ranges, nr, blockIdx.x);
    const SelScene &S = sc[fr.scene];
    select_scatter_body(SelPred{S.d2, S.K, nullptr, 0.0f}, S.logn, S.total, S.sums, S.logr, S.nf, S.queue, S.cap,
                        blockIdx.x - fr.first);
}

__global__ void __launch_bounds__(256) select_mask_batch(const SelScene *__restrict__ sc,
                                                         const FlatRange *__restrict__ ranges, int nr)
{
    const FlatRange &fr = flat_find(ranges, nr, blockIdx.x);
    const SelScene &S = sc[fr.scene];
    select_mask_body(SelPred{S.d2, S.K, nullptr, 0.0f}, S.logn, S.logr, S.nf, S.nquads, S.mask4,
                     (int64_t)(blockIdx.x - fr.first) * blockDim.x + threadIdx.x);
}

constexpr int kFillPerThread = 8;  // texels per thread of the batched fill

__global__ void __launch_bounds__(256) fill_unselected_batch(const FillScene *__restrict__ sc,
                                                             const FlatRange *__restrict__ ranges, int nr)
{
    const FlatRange &fr = flat_find(ranges, nr, blockIdx.x);
    const FillScene &F = sc[fr.scene];
    const int64_t stride = (int64_t)fr.count * blockDim.x;
    for (int64_t j = (int64_t)(blockIdx.x - fr.first) * blockDim.x + threadIdx.x; j < F.ntex; j += stride)
        fill_unselected_body(F.mask, F.coarse_sdf, F.nc, F.logr, F.lognf, F.ntex, F.u, F.hits, F.arg_tri, F.arg_ray,
                             F.fine, j);
}

// host side: one segment of the range table per launch
struct FlatLaunch {
    int offset = 0, count = 0;  // entries in the device range table
    uint32_t blocks = 0;        // workgroups of the launch
};

}  // namespace rtsdf

struct rtsdf_batch {
    int n = 0;
    uint64_t seed = 0;
    std::vector<rtsdf_batch_scene> desc;
    std::vector<rtsdf_scene *> scenes;
    std::vector<rtsdf_grid> coarse, fine;
    std::vector<int64_t> coff, foff;  // element offsets into the coarse / fine pools
    int64_t ctotal = 0, ftotal = 0, items = 0;
    int max_passes = 0;
    // pools
    int32_t *seeds = nullptr, *scratch = nullptr, *dist2 = nullptr;
    float *coarse_sdf = nullptr;
    uint8_t *mask = nullptr;
    int32_t *queue = nullptr;
    float *u = nullptr;
    uint32_t *hits = nullptr;
    int32_t *arg_tri = nullptr, *arg_ray = nullptr;
    float *fine_sdf = nullptr;
    uint32_t *sel_sums = nullptr;
    int32_t *counts = nullptr;
    int32_t *tile_offset = nullptr;
    int32_t *cursor = nullptr;  // 32 words: cursor + instrumentation counters (64-bit, from word 2)
    float4 *dirs = nullptr;     // the tracer's per-wavefront direction buffers
    int32_t *spill = nullptr;   // the tracer's spill area (stack entries deeper than its LDS part)
    bool has_tuning = false;    // tracer tuning of this batch (rtsdf_batch_set_tuning); else the process default
    rtsdf_trace_tuning tuning{};
    // tables
    rtsdf::BatchVox *vox = nullptr;
    rtsdf::JfaStep *plan = nullptr;  // [max_passes + 1][n]
    rtsdf::SelScene *sel = nullptr;
    rtsdf::FillScene *fill = nullptr;
    rtsdf::TraceScene *trace = nullptr;
    rtsdf::FlatRange *ranges = nullptr;  // all launches' range tables
    std::vector<std::array<rtsdf::FlatLaunch, rtsdf::kJfaKinds>> jfa_launch;  // [pass][kind]
    rtsdf::FlatLaunch sel_launch, mask_launch, fill_launch;
    std::vector<void *> allocations;
};

namespace rtsdf {

static void batch_free(rtsdf_batch *b)
{
    for (void *p : b->allocations) (void)hipFree(p);
    b->allocations.clear();
    for (rtsdf_scene *s : b->scenes) rtsdf_scene_destroy(s);
    b->scenes.clear();
}

template <typename T>
static bool batch_alloc(rtsdf_batch *b, T **p, int64_t count)
{
    void *q = nullptr;
    if (hipMalloc(&q, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) != hipSuccess) return false;
    b->allocations.push_back(q);
    *p = static_cast<T *>(q);
    return true;
}

}  // namespace rtsdf

extern "C" int rtsdf_batch_create(const rtsdf_batch_scene *scenes, int32_t n, uint64_t seed, int32_t leaf_size,
                                  rtsdf_batch **out, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scenes || n <= 0 || !out) return RTSDF_EINVAL;
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        const rtsdf_batch_scene &d = scenes[i];
        if (d.nt < 0 || d.nv < 0 || (d.nt > 0 && (!d.vertices || !d.faces))) return RTSDF_EINVAL;
        if (!is_pow2(d.coarse_n) || d.coarse_n < 8 || d.coarse_n > 128) return RTSDF_EINVAL;
        if (!is_pow2(d.fine_n) || d.fine_n < d.coarse_n || d.fine_n > 1024) return RTSDF_EINVAL;
        if (!(d.side > 0.0f) || d.rays_per_texel < 1 || d.rays_per_texel > 64) return RTSDF_EINVAL;
        if (!(d.alpha >= 0.0f && d.alpha <= 1.0f) || !(d.beta == d.beta) || !(d.d == d.d)) return RTSDF_EINVAL;
        if (d.sign_policy != RTSDF_SIGN_VOTE && d.sign_policy != RTSDF_SIGN_SHELL) return RTSDF_EINVAL;
        if (d.sign_policy == RTSDF_SIGN_SHELL && !(d.shell >= 0.0f && d.shell < __builtin_inff())) return RTSDF_EINVAL;
        if (d.nt >= (1 << 26)) return RTSDF_EINVAL;
    }
    hipStream_t s = as_stream(stream);
    auto *B = new rtsdf_batch();
    B->n = n;
    B->seed = seed;
    B->desc.assign(scenes, scenes + n);
    auto fail = [&](int rc) {
        batch_free(B);
        delete B;
        return rc;
    };
    for (int i = 0; i < n; ++i) {
        const rtsdf_batch_scene &d = scenes[i];
        rtsdf_scene *sc = nullptr;
        const int rc = rtsdf_scene_create(d.vertices, d.nv, d.faces, d.nt, leaf_size, &sc, stream);
        if (rc != RTSDF_OK) return fail(rc);
        B->scenes.push_back(sc);
        if (sc->max_depth + 1 > 64) return fail(RTSDF_EINVAL);
        rtsdf_grid c, f;
        for (int a = 0; a < 3; ++a) c.lo[a] = f.lo[a] = d.lo[a];
        c.n = d.coarse_n;
        c.h = d.side / (float)d.coarse_n;
        f.n = d.fine_n;
        f.h = d.side / (float)d.fine_n;
        B->coarse.push_back(c);
        B->fine.push_back(f);
        B->coff.push_back(B->ctotal);
        B->foff.push_back(B->ftotal);
        B->ctotal += (int64_t)c.n * c.n * c.n;
        B->ftotal += (int64_t)f.n * f.n * f.n;
        B->max_passes = std::max(B->max_passes, ilog2(c.n));
    }
    const int64_t C = B->ctotal, F = B->ftotal;
    std::vector<uint32_t> sel_off(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        const uint32_t total = (uint32_t)((int64_t)B->coarse[i].n * B->coarse[i].n * B->coarse[i].n);
        sel_off[i + 1] = sel_off[i] + (total + kSelPerBlock - 1) / kSelPerBlock;
    }
    if (!batch_alloc(B, &B->seeds, C) || !batch_alloc(B, &B->scratch, C) || !batch_alloc(B, &B->dist2, C) ||
        !batch_alloc(B, &B->coarse_sdf, C) || !batch_alloc(B, &B->mask, F) || !batch_alloc(B, &B->queue, F) ||
        !batch_alloc(B, &B->u, F) || !batch_alloc(B, &B->hits, F) || !batch_alloc(B, &B->arg_tri, F) ||
        !batch_alloc(B, &B->arg_ray, F) || !batch_alloc(B, &B->fine_sdf, F) ||
        !batch_alloc(B, &B->sel_sums, sel_off[n]) || !batch_alloc(B, &B->counts, n) ||
        !batch_alloc(B, &B->tile_offset, n + 1) || !batch_alloc(B, &B->cursor, 32) ||
        !batch_alloc(B, &B->dirs, (int64_t)(dirs_bytes() / sizeof(float4))) ||
        !batch_alloc(B, &B->spill, (int64_t)(spill_bytes() / sizeof(int32_t))) || !batch_alloc(B, &B->vox, n) ||
        !batch_alloc(B, &B->plan, (int64_t)(B->max_passes + 1) * n) || !batch_alloc(B, &B->sel, n) ||
        !batch_alloc(B, &B->fill, n) || !batch_alloc(B, &B->trace, n))
        return fail(RTSDF_ENOMEM);

    std::vector<BatchVox> vox(n);
    std::vector<JfaStep> plan((size_t)(B->max_passes + 1) * n);
    std::vector<SelScene> sel(n);
    std::vector<FillScene> fill(n);
    std::vector<TraceScene> trace(n);
    std::vector<std::array<uint32_t, kJfaKinds>> jfa_blocks((size_t)(B->max_passes + 1) * n);  // [pass * n + scene]
    for (auto &a : jfa_blocks) a.fill(0);
    int64_t items = 0;
    for (int i = 0; i < n; ++i) {
        const rtsdf_batch_scene &d = scenes[i];
        const rtsdf_grid &c = B->coarse[i], &f = B->fine[i];
        int32_t *seeds = B->seeds + B->coff[i], *scratch = B->scratch + B->coff[i];
        const rtsdf_scene *sc = B->scenes[i];
        vox[i] = BatchVox{sc->vertices, d.nv, sc->faces, d.nt, c, seeds, items};
        items += 3 * (int64_t)d.nt;
        // pass plan (the same ping-pong as the single-scene call), right-aligned
        const int L = ilog2(c.n), nbp = L - 1, first = B->max_passes - L + 1;
        const int64_t nvox = (int64_t)c.n * c.n * c.n;
        auto put = [&](int pass, JfaStep st, uint32_t grid) {
            plan[(size_t)pass * n + i] = st;
            jfa_blocks[(size_t)pass * n + i][st.kind] = grid;
        };
        int32_t *bufs[2] = {seeds, scratch};
        const int32_t *cur;
        int next;
        bool linear_first = false;
        if (nbp % 2 == 0) {
            put(first - 1, JfaStep{kJfaConvert, c.n, L, 0, seeds, scratch, nullptr, nullptr, 0.f, 0.f},
                (uint32_t)(nvox / 256));
            cur = scratch;
            next = 0;
        } else {
            cur = seeds;
            next = 1;
            linear_first = true;
        }
        for (int j = 1; j <= nbp; ++j) {
            const int k = c.n >> j;
            int32_t *dst = bufs[next];
            if (k >= 4)
                put(first + j - 1,
                    JfaStep{(linear_first && j == 1) ? kJfaFarLinear : kJfaFarBricks, c.n, L, k / 4, cur, dst, nullptr,
                            nullptr, 0.f, 0.f},
                    (uint32_t)(!(linear_first && j == 1) && c.n >= 16 ? nvox / 1024 : nvox / 256));
            else
                put(first + j - 1, JfaStep{kJfaNear2, c.n, L, 0, cur, dst, nullptr, nullptr, 0.f, 0.f},
                    (uint32_t)(nvox / 512));
            cur = dst;
            next ^= 1;
        }
        put(B->max_passes,
            JfaStep{kJfaFinal, c.n, L, 0, cur, seeds, B->dist2 + B->coff[i], B->coarse_sdf + B->coff[i], c.h, d.beta},
            (uint32_t)(nvox / 512));
        // selection
        const int logr = ilog2(f.n / c.n);
        sel[i] = SelScene{B->dist2 + B->coff[i], L, select_threshold(c.h, d.beta, d.d), (uint32_t)nvox,
                          B->sel_sums + sel_off[i], sel_off[i + 1] - sel_off[i], logr, f.n, B->queue + B->foff[i],
                          (int32_t)((int64_t)f.n * f.n * f.n), B->counts + i,
                          reinterpret_cast<uint32_t *>(B->mask + B->foff[i]), (int64_t)f.n * f.n * f.n / 4};
        const int64_t ntex = (int64_t)f.n * f.n * f.n;
        fill[i] = FillScene{B->mask + B->foff[i], B->coarse_sdf + B->coff[i], c.n, logr, ilog2(f.n), ntex,
                            B->u + B->foff[i], B->hits + B->foff[i], B->arg_tri + B->foff[i], B->arg_ray + B->foff[i],
                            B->fine_sdf + B->foff[i]};
        TraceScene &P = trace[i];
        P.bvh.nodes = sc->nodes;
        P.bvh.tris = sc->tris;
        P.bvh.tmap = sc->tmap;
        P.nodes4 = nullptr;  // batches trace the two-child hierarchy
        P.nt = sc->nt;
        P.queue = B->queue + B->foff[i];
        P.count = B->counts + i;
        P.queue_cap = sel[i].cap;
        P.coarse_sdf = B->coarse_sdf + B->coff[i];
        P.nc = c.n;
        P.logr = logr;
        P.nf = f.n;
        P.lognf = ilog2(f.n);
        P.lox = f.lo[0];
        P.loy = f.lo[1];
        P.loz = f.lo[2];
        P.hf = f.h;
        P.rays = d.rays_per_texel;
        P.scene_id = d.scene_id;
        P.alpha = d.alpha;
        P.sign_policy = d.sign_policy;
        P.shell = d.sign_policy == RTSDF_SIGN_SHELL ? d.shell : 0.0f;
        P.u = B->u + B->foff[i];
        P.hits = B->hits + B->foff[i];
        P.arg_tri = B->arg_tri + B->foff[i];
        P.arg_ray = B->arg_ray + B->foff[i];
        P.fine = B->fine_sdf + B->foff[i];
    }
    B->items = items;
    // range tables of the flat launches
    std::vector<FlatRange> ranges;
    auto segment = [&](auto blocks_of) {
        FlatLaunch L;
        L.offset = (int)ranges.size();
        for (int i = 0; i < n; ++i) {
            const uint32_t b = blocks_of(i);
            if (b == 0) continue;
            ranges.push_back(FlatRange{i, L.blocks, b});
            L.blocks += b;
        }
        L.count = (int)ranges.size() - L.offset;
        return L;
    };
    B->jfa_launch.assign(B->max_passes + 1, {});
    for (int p = 0; p <= B->max_passes; ++p)
        for (int k = 1; k < kJfaKinds; ++k)
            B->jfa_launch[p][k] = segment([&](int i) { return jfa_blocks[(size_t)p * n + i][k]; });
    B->sel_launch = segment([&](int i) { return sel[i].nblocks; });
    B->mask_launch = segment([&](int i) { return (uint32_t)((sel[i].nquads + 255) / 256); });
    B->fill_launch = segment([&](int i) { return (uint32_t)((fill[i].ntex + 256 * kFillPerThread - 1) / (256 * kFillPerThread)); });
    if (!batch_alloc(B, &B->ranges, (int64_t)std::max<size_t>(ranges.size(), 1))) return fail(RTSDF_ENOMEM);
    bool ok = hipMemcpyAsync(B->vox, vox.data(), sizeof(BatchVox) * n, hipMemcpyHostToDevice, s) == hipSuccess;
    if (!ranges.empty())
        ok &= hipMemcpyAsync(B->ranges, ranges.data(), sizeof(FlatRange) * ranges.size(), hipMemcpyHostToDevice, s) ==
              hipSuccess;
    ok &= hipMemcpyAsync(B->plan, plan.data(), sizeof(JfaStep) * plan.size(), hipMemcpyHostToDevice, s) == hipSuccess;
    ok &= hipMemcpyAsync(B->sel, sel.data(), sizeof(SelScene) * n, hipMemcpyHostToDevice, s) == hipSuccess;
    ok &= hipMemcpyAsync(B->fill, fill.data(), sizeof(FillScene) * n, hipMemcpyHostToDevice, s) == hipSuccess;
    ok &= hipMemcpyAsync(B->trace, trace.data(), sizeof(TraceScene) * n, hipMemcpyHostToDevice, s) == hipSuccess;
    ok &= hipStreamSynchronize(s) == hipSuccess;
    if (!ok) return fail(RTSDF_EHIP);
    if (rtsdf_batch_reset(B, stream) != RTSDF_OK) return fail(RTSDF_EHIP);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(RTSDF_EHIP);
    *out = B;
    return RTSDF_OK;
}

extern "C" int rtsdf_batch_reset(rtsdf_batch *B, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!B) return RTSDF_EINVAL;
    hipStream_t s = as_stream(stream);
    int64_t blocks = std::min<int64_t>((B->ftotal + 255) / 256, 8192);
    accum_reset_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(B->ftotal, B->u, B->hits, B->arg_tri, B->arg_ray);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

extern "C" int rtsdf_batch_step(rtsdf_batch *B, uint32_t frame, const uint32_t *frame_ptr, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!B) return RTSDF_EINVAL;
    if (frame >= kMaxFrame && !frame_ptr) return RTSDF_EINVAL;
    hipStream_t s = as_stream(stream);
    const int n = B->n;
    rtsdf_trace_tuning T = B->has_tuning ? B->tuning : g_tuning;
    if (T.loop == 4)
        for (int i = 0; i < n; ++i)
            if (B->scenes[i]->nref >= kMaxQueuedRefs) T.loop = 3;  // queue entries hold 26-bit indices
    // voxelize
    int rc = launch_fill<int32_t>(B->seeds, -1, B->ctotal, s);
    if (rc != RTSDF_OK) return rc;
    if (B->items > 0) {
        voxelize_batch<<<dim3((unsigned)((B->items + 255) / 256)), dim3(256), 0, s>>>(B->vox, n, B->items);
        RTSDF_CHECK_LAUNCH();
    }
    // jump flooding, pass by pass
    for (int p = 0; p <= B->max_passes; ++p) {
        const JfaStep *plan = B->plan + (size_t)p * n;
        const auto &L = B->jfa_launch[p];
        const FlatRange *r = B->ranges;
        if (L[kJfaConvert].blocks)
            jfa_batch<kJfaConvert><<<dim3(L[kJfaConvert].blocks), dim3(256), 0, s>>>(
                plan, r + L[kJfaConvert].offset, L[kJfaConvert].count, -2);
        if (L[kJfaFarLinear].blocks)
            jfa_batch<kJfaFarLinear><<<dim3(L[kJfaFarLinear].blocks), dim3(256), 0, s>>>(
                plan, r + L[kJfaFarLinear].offset, L[kJfaFarLinear].count, -2);
        if (L[kJfaFarBricks].blocks)
            jfa_batch<kJfaFarBricks><<<dim3(L[kJfaFarBricks].blocks), dim3(256), 0, s>>>(
                plan, r + L[kJfaFarBricks].offset, L[kJfaFarBricks].count, -2);
        if (L[kJfaNear2].blocks)
            jfa_batch<kJfaNear2><<<dim3(L[kJfaNear2].blocks), dim3(512), 0, s>>>(plan, r + L[kJfaNear2].offset,
                                                                                  L[kJfaNear2].count, -2);
        if (L[kJfaFinal].blocks)
            jfa_batch<kJfaFinal><<<dim3(L[kJfaFinal].blocks), dim3(512), 0, s>>>(plan, r + L[kJfaFinal].offset,
                                                                                  L[kJfaFinal].count, -2);
        RTSDF_CHECK_LAUNCH();
    }
    // selection
    const FlatLaunch &SL = B->sel_launch, &ML = B->mask_launch, &FL = B->fill_launch;
    if (SL.blocks) select_count_batch<<<dim3(SL.blocks), dim3(kSelBlock), 0, s>>>(B->sel, B->ranges + SL.offset, SL.count);
    select_scan_batch<<<dim3(1, n), dim3(1024), 0, s>>>(B->sel);
    if (SL.blocks)
        select_scatter_batch<<<dim3(SL.blocks), dim3(kSelBlock), 0, s>>>(B->sel, B->ranges + SL.offset, SL.count);
    if (ML.blocks) select_mask_batch<<<dim3(ML.blocks), dim3(256), 0, s>>>(B->sel, B->ranges + ML.offset, ML.count);
    RTSDF_CHECK_LAUNCH();
    // tracing
    if (FL.blocks) fill_unselected_batch<<<dim3(FL.blocks), dim3(256), 0, s>>>(B->fill, B->ranges + FL.offset, FL.count);
    RTSDF_CHECK_LAUNCH();
    trace_tile_prefix<<<dim3(1), dim3(64), 0, s>>>(B->trace, n, T.tile_texels, B->tile_offset);
    RTSDF_CHECK_LAUNCH();
    rc = launch_fill<int32_t>(B->cursor, 0, T.stats ? 32 : 1, s);
    if (rc != RTSDF_OK) return rc;
    TraceArgs A{};
    A.scenes = B->trace;
    A.tile_offset = B->tile_offset;
    A.nscenes = n;
    A.cursor = B->cursor;
    A.frame = frame;
    A.frame_ptr = frame_ptr;
    A.seed = B->seed;
    A.spill = B->spill;
    A.dirs = B->dirs;
    return launch_trace<true>(A, T, s);
}

extern "C" int rtsdf_batch_set_tuning(rtsdf_batch *B, const rtsdf_trace_tuning *t)
{
    if (!B || (t && !rtsdf::tuning_ok(*t))) return RTSDF_EINVAL;
    B->has_tuning = t != nullptr;
    if (t) B->tuning = *t;
    return RTSDF_OK;
}

extern "C" int rtsdf_batch_outputs(const rtsdf_batch *B, int32_t i, rtsdf_batch_view *out)
{
    if (!B || !out || i < 0 || i >= B->n) return RTSDF_EINVAL;
    out->coarse = B->coarse[i];
    out->fine = B->fine[i];
    out->seeds = B->seeds + B->coff[i];
    out->dist2 = B->dist2 + B->coff[i];
    out->coarse_sdf = B->coarse_sdf + B->coff[i];
    out->mask = B->mask + B->foff[i];
    out->queue = B->queue + B->foff[i];
    out->count = B->counts + i;
    out->state.u = B->u + B->foff[i];
    out->state.hits = B->hits + B->foff[i];
    out->state.arg_tri = B->arg_tri + B->foff[i];
    out->state.arg_ray = B->arg_ray + B->foff[i];
    out->fine_sdf = B->fine_sdf + B->foff[i];
    out->scene = B->scenes[i];
    return RTSDF_OK;
}

extern "C" void rtsdf_batch_destroy(rtsdf_batch *B)
{
    if (!B) return;
    rtsdf::batch_free(B);
    delete B;
}
