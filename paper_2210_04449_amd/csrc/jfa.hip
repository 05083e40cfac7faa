// The JFA's translation unit: its kernels, the pass schedule and the
// rtsdf_jfa* entry points (the passes themselves are in jfa_device.hpp).
//
// Built apart from the rest of the library, with its device code compiled on
// the assumption that no float is a NaN: the only floating-point values here
// are the candidate keys (non-negative denormals, or a large finite value for
// a missing seed) and the finite coarse SDF.  Under that assumption the
// minimum of two keys is one v_min_f64; otherwise every new key first passes
// through a v_max_f64 that would quiet a signalling NaN, one more VALU
// instruction per candidate.  Host code is compiled as usual.
#include <atomic>

// The library's error word is defined in its main translation unit; this unit raises no errors, and renaming its
// copy keeps the two units' device variables apart.
#define g_error_word g_error_word_jfa_unit
#include "jfa_device.hpp"
#undef g_error_word

namespace rtsdf {

__global__ void __launch_bounds__(256) jfa_to_bricks(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                                     int n, int logn)
{
    jfa_to_bricks_body(src, dst, n, logn, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

template <bool WIDE, bool LINEAR_IN>
__global__ void __launch_bounds__(256) jfa_far(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                               int logn, int kb, int neg2, int coset)
{
    jfa_far_body<WIDE, LINEAR_IN>(src, dst, n, logn, kb, blockIdx.x, gridDim.x, neg2, coset);
}

template <bool WIDE>
__global__ void __launch_bounds__(256) jfa_far_pairs(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                                     int logn, int kb, int neg2)
{
    jfa_far_pair_body<WIDE>(src, dst, n, logn, kb, blockIdx.x, gridDim.x, neg2);
}

template <bool WIDE>
__global__ void __launch_bounds__(256) jfa_far_quads(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                                     int logn, int kb, int neg2)
{
    jfa_far_quad_body<WIDE>(src, dst, n, logn, kb, blockIdx.x, gridDim.x, neg2);
}

template <bool WIDE>
__global__ void __launch_bounds__(512) jfa_first_orbit(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                                       int n, int logn, int neg2)
{
    jfa_first_orbit_body<WIDE>(src, dst, n, logn, neg2, blockIdx.x, gridDim.x);
}

template <bool WIDE>
__global__ void __launch_bounds__(512) jfa_first_orbit4(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                                        int n, int logn, int neg2)
{
    jfa_first_orbit4_body<WIDE>(src, dst, n, logn, neg2, blockIdx.x, gridDim.x);
}

template <int K, bool PAIRS, bool FINAL, bool SMALL>
__global__ void __launch_bounds__(512) jfa_near(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                                int logn, int32_t *__restrict__ dist2, float *__restrict__ sdf,
                                                float h, float beta, int neg2)
{
    jfa_near_body<K, PAIRS, FINAL, SMALL>(src, dst, n, logn, dist2, sdf, h, beta, blockIdx.x, gridDim.x, neg2);
}

template <bool WIDE, bool PAIRS>
static int jfa_run(const rtsdf_grid &g, int32_t *seeds, int32_t *scratch, float beta, int32_t *dist2, float *sdf,
                   const int32_t *steps, int m, int order, hipStream_t s)
{
    const int n = g.n, logn = ilog2(n);
    const int64_t nvox = (int64_t)n * n * n;
    // far-pass brick order: 1 slab order, 2 coset order, 3 coset order in brick pairs, 4 in 2 x 2 brick quads
    // (a grid of 8^3 voxels has only two quads, under one workgroup: it takes pairs)
    if (order == 4 && nvox < 1024) order = 3;
    const int coset = order >= 2 ? 1 : 0;
    constexpr bool SMALL = PAIRS && !WIDE;  // n <= 128 with staged pairs: the two-instruction near-pass key
    const unsigned far_blocks = (unsigned)(nvox / 256);
    const unsigned near_blocks = (unsigned)(nvox / 512);
    const unsigned orbit_blocks = (unsigned)(nvox / 512);  // one orbit of eight bricks per workgroup
    const unsigned pair_blocks = (unsigned)(nvox / 512);   // four wavefronts of two bricks each per workgroup
    // one wavefront of four bricks per workgroup (measured 1-2 % faster than four wavefronts per workgroup)
    const unsigned quad_waves = (unsigned)(nvox / 256);
    // Passes 0 .. m-2 go brick layout to brick layout; the final pass (step 1) must read `scratch` and write the
    // caller's linear layout to `seeds` (and `dist2`, `sdf`).  When the first step is a far one it reads the
    // linear input directly, and the brick passes alternate between `dist2` (written only by the final pass,
    // and distinct from `seeds` and `scratch` since that pass reads one and writes the other) and `scratch`,
    // chosen so that the last one lands in `scratch`.  Otherwise the input is converted into `scratch` first,
    // and copied once more when the number of brick passes would leave the last one in the wrong buffer.
    const int npass = m - 1;
    const int32_t *cur = seeds;
    if (npass >= 1 && steps[0] >= 4) {
        for (int i = 0; i < npass; ++i) {
            const int k = steps[i];
            int32_t *dst = (npass - 1 - i) % 2 == 0 ? scratch : dist2;
            if (k >= 4) {
                if (i == 0 && k == n / 2 && n >= 32)
                    jfa_first_orbit4<WIDE><<<dim3(orbit_blocks / 4), dim3(512), 0, s>>>(cur, dst, n, logn, -2);
                else if (i == 0 && k == n / 2)
                    jfa_first_orbit<WIDE><<<dim3(orbit_blocks), dim3(512), 0, s>>>(cur, dst, n, logn, -2);
                else if (i == 0)
                    jfa_far<WIDE, true><<<dim3(far_blocks), dim3(256), 0, s>>>(cur, dst, n, logn, k / 4, -2, coset);
                else if (order == 4)
                    jfa_far_quads<WIDE><<<dim3(quad_waves), dim3(64), 0, s>>>(cur, dst, n, logn, k / 4, -2);
                else if (order == 3)
                    jfa_far_pairs<WIDE><<<dim3(pair_blocks), dim3(256), 0, s>>>(cur, dst, n, logn, k / 4, -2);
                else
                    jfa_far<WIDE, false><<<dim3(far_blocks), dim3(256), 0, s>>>(cur, dst, n, logn, k / 4, -2, coset);
            } else if (k == 2) {
                jfa_near<2, PAIRS, false, SMALL>
                    <<<dim3(near_blocks), dim3(512), 0, s>>>(cur, dst, n, logn, nullptr, nullptr, 0.f, 0.f, -2);
            } else {
                jfa_near<1, PAIRS, false, SMALL>
                    <<<dim3(near_blocks), dim3(512), 0, s>>>(cur, dst, n, logn, nullptr, nullptr, 0.f, 0.f, -2);
            }
            RTSDF_CHECK_LAUNCH();
            cur = dst;
        }
    } else {
        int32_t *bufs[2] = {seeds, scratch};
        int next = 0;  // index into bufs of the next destination
        jfa_to_bricks<<<dim3(far_blocks), dim3(256), 0, s>>>(seeds, scratch, n, logn);
        RTSDF_CHECK_LAUNCH();
        cur = scratch;
        if (npass % 2 == 1) {
            RTSDF_TRY(hipMemcpyAsync(seeds, scratch, sizeof(int32_t) * nvox, hipMemcpyDeviceToDevice, s));
            cur = seeds;
            next = 1;
        }
        for (int i = 0; i < npass; ++i) {
            const int k = steps[i];
            int32_t *dst = bufs[next];
            if (k >= 4 && order == 4) {
                jfa_far_quads<WIDE><<<dim3(quad_waves), dim3(64), 0, s>>>(cur, dst, n, logn, k / 4, -2);
            } else if (k >= 4 && order == 3) {
                jfa_far_pairs<WIDE><<<dim3(pair_blocks), dim3(256), 0, s>>>(cur, dst, n, logn, k / 4, -2);
            } else if (k >= 4) {
                jfa_far<WIDE, false><<<dim3(far_blocks), dim3(256), 0, s>>>(cur, dst, n, logn, k / 4, -2, coset);
            } else if (k == 2) {
                jfa_near<2, PAIRS, false, SMALL>
                    <<<dim3(near_blocks), dim3(512), 0, s>>>(cur, dst, n, logn, nullptr, nullptr, 0.f, 0.f, -2);
            } else {
                jfa_near<1, PAIRS, false, SMALL>
                    <<<dim3(near_blocks), dim3(512), 0, s>>>(cur, dst, n, logn, nullptr, nullptr, 0.f, 0.f, -2);
            }
            RTSDF_CHECK_LAUNCH();
            cur = dst;
            next ^= 1;
        }
    }
    // cur == scratch here by construction
    jfa_near<1, PAIRS, true, SMALL>
        <<<dim3(near_blocks), dim3(512), 0, s>>>(cur, seeds, n, logn, dist2, sdf, g.h, beta, -2);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

}  // namespace rtsdf

// near-pass staging and far-pass brick order per grid size (index log2 n - 3: n = 8 .. 256)
static std::atomic<int> g_near_stage[6];
static std::atomic<int> g_far_order[6];

extern "C" int rtsdf_jfa_config(int32_t n, const rtsdf_jfa_tuning *t)
{
    if (!t || n < 8 || n > 256 || !rtsdf::is_pow2(n) || t->near_stage < 0 || t->near_stage > 2 || t->far_order < 0 ||
        t->far_order > 4)
        return RTSDF_EINVAL;
    g_near_stage[rtsdf::ilog2(n) - 3].store(t->near_stage);
    g_far_order[rtsdf::ilog2(n) - 3].store(t->far_order);
    return RTSDF_OK;
}

extern "C" int rtsdf_jfa_config_get(int32_t n, rtsdf_jfa_tuning *t)
{
    if (!t || n < 8 || n > 256 || !rtsdf::is_pow2(n)) return RTSDF_EINVAL;
    t->near_stage = g_near_stage[rtsdf::ilog2(n) - 3].load();
    t->far_order = g_far_order[rtsdf::ilog2(n) - 3].load();
    return RTSDF_OK;
}

extern "C" int rtsdf_jfa_steps(rtsdf_grid coarse, int32_t *seeds, int32_t *scratch, const int32_t *steps,
                               int32_t nsteps, float beta, int32_t *dist2, float *coarse_sdf, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!grid_ok(coarse) || !is_pow2(coarse.n) || coarse.n < 8 || coarse.n > 256) return RTSDF_EINVAL;
    if (!seeds || !scratch || !dist2 || !coarse_sdf || seeds == scratch || dist2 == seeds || dist2 == scratch)
        return RTSDF_EINVAL;
    if (!(beta == beta)) return RTSDF_EINVAL;
    if (!steps || nsteps < 1 || nsteps > 64 || steps[nsteps - 1] != 1) return RTSDF_EINVAL;
    for (int i = 0; i < nsteps; ++i)
        if (steps[i] < 1 || steps[i] > coarse.n / 2 || !is_pow2(steps[i])) return RTSDF_EINVAL;
    hipStream_t s = as_stream(stream);
    const int stage = g_near_stage[ilog2(coarse.n) - 3].load();
    const bool pairs = stage != 1;
    int order = g_far_order[ilog2(coarse.n) - 3].load();
    if (order == 0) order = 4;  // automatic: coset order in 2 x 2 brick quads
    if (coarse.n <= 128)
        return pairs ? jfa_run<false, true>(coarse, seeds, scratch, beta, dist2, coarse_sdf, steps, nsteps, order, s)
                     : jfa_run<false, false>(coarse, seeds, scratch, beta, dist2, coarse_sdf, steps, nsteps, order, s);
    return pairs ? jfa_run<true, true>(coarse, seeds, scratch, beta, dist2, coarse_sdf, steps, nsteps, order, s)
                 : jfa_run<true, false>(coarse, seeds, scratch, beta, dist2, coarse_sdf, steps, nsteps, order, s);
}

extern "C" int rtsdf_jfa(rtsdf_grid coarse, int32_t *seeds, int32_t *scratch, float beta, int32_t *dist2,
                         float *coarse_sdf, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!grid_ok(coarse) || !is_pow2(coarse.n) || coarse.n < 8 || coarse.n > 256) return RTSDF_EINVAL;
    int32_t steps[16];
    int m = 0;
    for (int k = coarse.n / 2; k >= 1; k /= 2) steps[m++] = k;  // n/2, ..., 2, 1
    return rtsdf_jfa_steps(coarse, seeds, scratch, steps, m, beta, dist2, coarse_sdf, stream);
}
