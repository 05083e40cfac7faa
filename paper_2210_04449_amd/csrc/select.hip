// Selection of the fine texels to ray trace (paper Sec. 2.2; the case
// c <= d of Eq. (1)), as a stream compaction.
//
// A fine texel is selected when the coarse voxel containing its centre has
// D^2 <= K, K = floor(((d + beta) / h_c)^2), which is c <= d in exact
// arithmetic.  Since the fine size is a power-of-two multiple r of the coarse
// size, the r^3 fine children of a coarse voxel are consecutive in fine Morton
// order (their codes are (coarse code) * r^3 + child), so the queue is built by
// compacting the coarse voxels in Morton order and expanding each selected one
// into its r^3 children.
//
//   select_count   one coarse voxel per lane in Morton order; wavefront ballot
//                  + popcount, per-block totals
//   select_scan    one workgroup: exclusive prefix of the block totals
//   select_scatter ballot + mbcnt rank inside the wavefront, wave offsets
//                  through LDS, block offset from the scan; writes r^3 queue
//                  entries per selected voxel
//   select_mask    the linear uint8 mask, four texels per lane
// No workgroup ever waits on another, and the queue order is deterministic.
#include <mutex>

#include "common.hpp"

namespace rtsdf {

constexpr int kSelBlock = 256;
constexpr int kSelItems = 4;  // coarse voxels per lane per block
constexpr int kSelPerBlock = kSelBlock * kSelItems;

// What is compared: D^2 against the integer threshold K (point sampling of
// the coarse voxel), or a float field at the selection grid's own resolution
// against d (trilinear sampling, see rtsdf_coarse_trilinear).
struct SelPred {
    const int32_t *d2;
    int K;
    const float *field;
    float d;
};

template <bool FIELD>
__device__ __forceinline__ bool pred_at(const SelPred &p, int64_t idx)
{
    if (FIELD) return p.field[idx] <= p.d;
    return p.d2[idx] <= p.K;
}

template <bool FIELD>
__device__ __forceinline__ bool coarse_selected(const SelPred &p, uint32_t m, int logn)
{
    const uint32_t x = compact1by2(m), y = compact1by2(m >> 1), z = compact1by2(m >> 2);
    const int64_t idx = x + ((int64_t)y << logn) + ((int64_t)z << (2 * logn));
    return pred_at<FIELD>(p, idx);
}

__device__ __forceinline__ uint32_t wave_prefix(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <bool FIELD = false>
__device__ __forceinline__ void select_count_body(const SelPred &pr, int logn, uint32_t total,
                                                  uint32_t *__restrict__ block_sums, uint32_t blk)
{
    __shared__ uint32_t wsum[kSelBlock / kWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t cnt = 0;
    for (int it = 0; it < kSelItems; ++it) {
        const uint32_t m = blk * kSelPerBlock + it * kSelBlock + threadIdx.x;
        const bool sel = m < total && coarse_selected<FIELD>(pr, m, logn);
        cnt += (uint32_t)__popcll(__ballot(sel));
    }
    if (lane == 0) wsum[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kSelBlock / kWave; ++w) s += wsum[w];
        block_sums[blk] = s;
    }
}

template <bool FIELD>
__global__ void __launch_bounds__(kSelBlock) select_count(SelPred pr, int logn, uint32_t total,
                                                          uint32_t *__restrict__ block_sums)
{
    select_count_body<FIELD>(pr, logn, total, block_sums, blockIdx.x);
}

// Exclusive scan of nblocks totals in one workgroup of 1024 lanes; also the
// grand total -> count (texels = coarse * r3) and the overflow check.
__device__ __forceinline__ void select_scan_body(uint32_t *__restrict__ sums, uint32_t nblocks, uint32_t r3,
                                                 int32_t *__restrict__ count, int32_t cap)
{
    __shared__ uint32_t part[1024];
    const uint32_t t = threadIdx.x;
    const uint32_t per = (nblocks + 1023) / 1024;
    const uint32_t b0 = t * per;
    uint32_t local = 0;
    for (uint32_t i = 0; i < per; ++i)
        if (b0 + i < nblocks) local += sums[b0 + i];
    part[t] = local;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scan
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - local;  // exclusive
    for (uint32_t i = 0; i < per; ++i) {
        if (b0 + i < nblocks) {
            const uint32_t v = sums[b0 + i];
            sums[b0 + i] = run;
            run += v;
        }
    }
    if (t == 1023) {
        const uint64_t texels = (uint64_t)part[1023] * r3;
        *count = texels > (uint64_t)INT32_MAX ? INT32_MAX : (int32_t)texels;
        if (texels > (uint64_t)cap) raise_error(RTSDF_ERR_QUEUE_FULL);
    }
}

__global__ void __launch_bounds__(1024) select_scan(uint32_t *__restrict__ sums, uint32_t nblocks, uint32_t r3,
                                                    int32_t *__restrict__ count, int32_t cap)
{
    select_scan_body(sums, nblocks, r3, count, cap);
}

template <bool FIELD = false>
__device__ __forceinline__ void select_scatter_body(const SelPred &pr, int logn, uint32_t total,
                                                    const uint32_t *__restrict__ offsets, int logr, int nf,
                                                    int32_t *__restrict__ queue, int32_t cap, uint32_t blk)
{
    __shared__ uint32_t wsum[kSelItems][kSelBlock / kWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool sel[kSelItems];
    uint32_t rank[kSelItems];
    for (int it = 0; it < kSelItems; ++it) {
        const uint32_t m = blk * kSelPerBlock + it * kSelBlock + threadIdx.x;
        sel[it] = m < total && coarse_selected<FIELD>(pr, m, logn);
        const uint64_t bal = __ballot(sel[it]);
        rank[it] = wave_prefix(bal);
        if (lane == 0) wsum[it][wave] = (uint32_t)__popcll(bal);
    }
    __syncthreads();
    const uint32_t r3 = 1u << (3 * logr);
    uint32_t base = offsets[blk];
    for (int it = 0; it < kSelItems; ++it) {
        uint32_t before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[it][w];
        if (sel[it]) {
            const uint32_t m = blk * kSelPerBlock + it * kSelBlock + threadIdx.x;
            const uint64_t pos = ((uint64_t)(base + before + rank[it])) * r3;
            const uint32_t cx = compact1by2(m), cy = compact1by2(m >> 1), cz = compact1by2(m >> 2);
            for (uint32_t c = 0; c < r3; ++c) {
                if (pos + c >= (uint64_t)cap) break;
                const uint32_t fx = (cx << logr) | compact1by2(c), fy = (cy << logr) | compact1by2(c >> 1),
                               fz = (cz << logr) | compact1by2(c >> 2);
                queue[pos + c] = (int32_t)(fx + (uint32_t)nf * (fy + (uint32_t)nf * fz));
            }
        }
        for (int w = 0; w < kSelBlock / kWave; ++w) base += wsum[it][w];
    }
}

template <bool FIELD>
__global__ void __launch_bounds__(kSelBlock) select_scatter(SelPred pr, int logn, uint32_t total,
                                                            const uint32_t *__restrict__ offsets, int logr, int nf,
                                                            int32_t *__restrict__ queue, int32_t cap)
{
    select_scatter_body<FIELD>(pr, logn, total, offsets, logr, nf, queue, cap, blockIdx.x);
}

template <bool FIELD = false>
__device__ __forceinline__ void select_mask_body(const SelPred &pr, int logn, int logr, int nf, int64_t nquads,
                                                 uint32_t *__restrict__ mask4, int64_t q)
{
    if (q >= nquads) return;
    const int64_t j = q * 4;
    const int x = (int)(j % nf), y = (int)((j / nf) % nf), z = (int)(j / ((int64_t)nf * nf));
    const int cy = y >> logr, cz = z >> logr;
    const int64_t row = ((int64_t)cy << logn) + ((int64_t)cz << (2 * logn));
    uint32_t w = 0;
    for (int i = 0; i < 4; ++i) w |= (uint32_t)pred_at<FIELD>(pr, row + ((x + i) >> logr)) << (8 * i);
    mask4[q] = w;
}

template <bool FIELD>
__global__ void __launch_bounds__(256) select_mask(SelPred pr, int logn, int logr, int nf, int64_t nquads,
                                                   uint32_t *__restrict__ mask4)
{
    select_mask_body<FIELD>(pr, logn, logr, nf, nquads, mask4, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Trilinear value of the coarse SDF at fine texel centres.  Coarse values sit
// at voxel centres; a fine centre at coarse coordinate u = (j + 1/2) / r - 1/2
// (r = fine / coarse size) is clamped to [0, n - 1], split into the cell
// i0 = floor(u), i1 = min(i0 + 1, n - 1) and the weight t = u - i0 (all exact
// for power-of-two r), and interpolated along x, then y, then z with
// lerp(a, b, t) = a + t (b - a), each float operation rounded once.  A cell
// with an infinite corner (no seed anywhere) gives +inf.
__device__ __forceinline__ void tri_axis(int j, float inv_r, int nc, int &i0, int &i1, float &t)
{
    float u = rn_sub(rn_mul(rn_add((float)j, 0.5f), inv_r), 0.5f);
    u = fminf(fmaxf(u, 0.0f), (float)(nc - 1));
    i0 = (int)u;  // u >= 0: truncation is the floor
    i1 = min(i0 + 1, nc - 1);
    t = rn_sub(u, (float)i0);
}

__device__ __forceinline__ float lerp_c(float a, float b, float t) { return rn_add(a, rn_mul(t, rn_sub(b, a))); }

__global__ void __launch_bounds__(256) coarse_trilinear_kernel(const float *__restrict__ c, int nc, int lognf, int logr,
                                                               float *__restrict__ out, int64_t ntex)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntex) return;
    const int nfm = (1 << lognf) - 1;
    const int jx = (int)(j & nfm), jy = (int)((j >> lognf) & nfm), jz = (int)(j >> (2 * lognf));
    const float inv_r = 1.0f / (float)(1 << logr);  // exact
    int x0, x1, y0, y1, z0, z1;
    float tx, ty, tz;
    tri_axis(jx, inv_r, nc, x0, x1, tx);
    tri_axis(jy, inv_r, nc, y0, y1, ty);
    tri_axis(jz, inv_r, nc, z0, z1, tz);
    auto at = [&](int x, int y, int z) { return c[x + (int64_t)nc * (y + (int64_t)nc * z)]; };
    const float c000 = at(x0, y0, z0), c100 = at(x1, y0, z0), c010 = at(x0, y1, z0), c110 = at(x1, y1, z0);
    const float c001 = at(x0, y0, z1), c101 = at(x1, y0, z1), c011 = at(x0, y1, z1), c111 = at(x1, y1, z1);
    const float m = fmaxf(fmaxf(fmaxf(c000, c100), fmaxf(c010, c110)), fmaxf(fmaxf(c001, c101), fmaxf(c011, c111)));
    if (isinf(m)) {
        out[j] = __builtin_inff();
        return;
    }
    const float c00 = lerp_c(c000, c100, tx), c10 = lerp_c(c010, c110, tx);
    const float c01 = lerp_c(c001, c101, tx), c11 = lerp_c(c011, c111, tx);
    const float c0 = lerp_c(c00, c10, ty), c1 = lerp_c(c01, c11, ty);
    out[j] = lerp_c(c0, c1, tz);
}

// K = floor(((d + beta) / h_c)^2), -1 if d + beta < 0
inline int select_threshold(float hc, float beta, float d)
{
    const double q = ((double)d + (double)beta) / (double)hc;
    if (q < 0) return -1;
    const double k = floor(q * q);
    return k > (double)INT32_MAX ? INT32_MAX : (int)k;
}


// Point-sampled selection with the block sums in `sums` (at least
// rtsdf_select_workspace_size(coarse.n) bytes).  Every sum the launches read
// is written earlier in the same sequence (count, then scan), so `sums` needs
// no clearing.
static int select_run(rtsdf_grid coarse, const int32_t *dist2, rtsdf_grid fine, float beta, float d, uint8_t *mask,
                      int32_t *queue, int32_t queue_cap, int32_t *count, uint32_t *sums, hipStream_t s)
{
    const int logn = ilog2(coarse.n), logr = ilog2(fine.n / coarse.n);
    const int K = select_threshold(coarse.h, beta, d);
    const uint32_t total = (uint32_t)((int64_t)coarse.n * coarse.n * coarse.n);
    const uint32_t nblocks = (total + kSelPerBlock - 1) / kSelPerBlock;
    const SelPred pr{dist2, K, nullptr, 0.0f};
    select_count<false><<<dim3(nblocks), dim3(kSelBlock), 0, s>>>(pr, logn, total, sums);
    RTSDF_CHECK_LAUNCH();
    select_scan<<<dim3(1), dim3(1024), 0, s>>>(sums, nblocks, 1u << (3 * logr), count, queue_cap);
    RTSDF_CHECK_LAUNCH();
    select_scatter<false><<<dim3(nblocks), dim3(kSelBlock), 0, s>>>(pr, logn, total, sums, logr, fine.n, queue,
                                                                     queue_cap);
    RTSDF_CHECK_LAUNCH();
    const int64_t nquads = (int64_t)fine.n * fine.n * fine.n / 4;
    select_mask<false><<<dim3((unsigned)((nquads + 255) / 256)), dim3(256), 0, s>>>(
        pr, logn, logr, fine.n, nquads, reinterpret_cast<uint32_t *>(mask));
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

static bool select_args_ok(rtsdf_grid coarse, const int32_t *dist2, rtsdf_grid fine, float beta, float d,
                           const uint8_t *mask, const int32_t *queue, int32_t queue_cap, const int32_t *count)
{
    if (!grid_ok(coarse) || !grid_ok(fine) || !is_pow2(coarse.n) || coarse.n > 512) return false;
    if (!is_pow2(fine.n) || fine.n < coarse.n || fine.n > 1024 || fine.n < 4) return false;
    if ((double)fine.h * fine.n != (double)coarse.h * coarse.n) return false;
    if (fine.lo[0] != coarse.lo[0] || fine.lo[1] != coarse.lo[1] || fine.lo[2] != coarse.lo[2]) return false;
    if (!dist2 || !mask || !count || queue_cap < 0 || (queue_cap > 0 && !queue)) return false;
    if (!(beta == beta) || !(d == d)) return false;
    return true;
}

// Scratch of the allocation-free selection: the block sums of the largest
// coarse grid rtsdf_select takes (512^3 voxels -> 131,072 blocks), 512 KiB per
// device, held until the process ends.  Host code never passes `scratch`
// itself to a kernel (on the host it is only a stand-in for the symbol); it
// uses the device address hipGetSymbolAddress returns for each device.
constexpr size_t kSelScratchWords = ((size_t)512 * 512 * 512 + kSelPerBlock - 1) / kSelPerBlock + 64;
__device__ __align__(256) uint32_t scratch[kSelScratchWords];

constexpr int kMaxDevices = 64;
static uint32_t *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// The current device's address of `scratch`, looked up once per device.
static uint32_t *scratch_for_current_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = static_cast<uint32_t *>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace rtsdf

extern "C" size_t rtsdf_select_workspace_size(int32_t coarse_n)
{
    using namespace rtsdf;
    if (coarse_n <= 0) return 0;
    const int64_t total = (int64_t)coarse_n * coarse_n * coarse_n;
    return (size_t)(((total + kSelPerBlock - 1) / kSelPerBlock) * sizeof(uint32_t) + 256);
}

extern "C" int rtsdf_select(rtsdf_grid coarse, const int32_t *dist2, rtsdf_grid fine, float beta, float d,
                            uint8_t *mask, int32_t *queue, int32_t queue_cap, int32_t *count, void *workspace,
                            rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!select_args_ok(coarse, dist2, fine, beta, d, mask, queue, queue_cap, count) || !workspace)
        return RTSDF_EINVAL;
    return select_run(coarse, dist2, fine, beta, d, mask, queue, queue_cap, count, static_cast<uint32_t *>(workspace),
                      as_stream(stream));
}

extern "C" size_t rtsdf_select_noalloc_max_bytes(void) { return rtsdf::kSelScratchWords * sizeof(uint32_t); }

extern "C" int rtsdf_select_noalloc(rtsdf_grid coarse, const int32_t *dist2, rtsdf_grid fine, float beta, float d,
                                    uint8_t *mask, int32_t *queue, int32_t queue_cap, int32_t *count,
                                    rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!select_args_ok(coarse, dist2, fine, beta, d, mask, queue, queue_cap, count)) return RTSDF_EINVAL;
    if (rtsdf_select_workspace_size(coarse.n) > kSelScratchWords * sizeof(uint32_t)) return RTSDF_EINVAL;
    uint32_t *sums = scratch_for_current_device();
    if (!sums) return RTSDF_EHIP;
    return select_run(coarse, dist2, fine, beta, d, mask, queue, queue_cap, count, sums, as_stream(stream));
}

extern "C" int rtsdf_coarse_trilinear(rtsdf_grid coarse, const float *coarse_sdf, rtsdf_grid fine, float *fine_c,
                                      rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!grid_ok(coarse) || !grid_ok(fine) || !is_pow2(coarse.n) || !is_pow2(fine.n)) return RTSDF_EINVAL;
    if (fine.n < coarse.n || fine.n > 1024 || coarse.n > 512) return RTSDF_EINVAL;
    if ((double)fine.h * fine.n != (double)coarse.h * coarse.n) return RTSDF_EINVAL;
    if (fine.lo[0] != coarse.lo[0] || fine.lo[1] != coarse.lo[1] || fine.lo[2] != coarse.lo[2]) return RTSDF_EINVAL;
    if (!coarse_sdf || !fine_c) return RTSDF_EINVAL;
    const int64_t ntex = (int64_t)fine.n * fine.n * fine.n;
    coarse_trilinear_kernel<<<dim3((unsigned)((ntex + 255) / 256)), dim3(256), 0, as_stream(stream)>>>(
        coarse_sdf, coarse.n, ilog2(fine.n), ilog2(fine.n / coarse.n), fine_c, ntex);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

extern "C" int rtsdf_select_field(rtsdf_grid grid, const float *field, float d, uint8_t *mask, int32_t *queue,
                                  int32_t queue_cap, int32_t *count, void *workspace, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!grid_ok(grid) || !is_pow2(grid.n) || grid.n < 4 || grid.n > 1024) return RTSDF_EINVAL;
    if (!field || !mask || !count || !workspace || queue_cap < 0 || (queue_cap > 0 && !queue)) return RTSDF_EINVAL;
    if (!(d == d)) return RTSDF_EINVAL;
    hipStream_t s = as_stream(stream);
    const int logn = ilog2(grid.n);
    const uint32_t total = (uint32_t)((int64_t)grid.n * grid.n * grid.n);
    const uint32_t nblocks = (total + kSelPerBlock - 1) / kSelPerBlock;
    uint32_t *sums = static_cast<uint32_t *>(workspace);
    const SelPred pr{nullptr, 0, field, d};
    select_count<true><<<dim3(nblocks), dim3(kSelBlock), 0, s>>>(pr, logn, total, sums);
    RTSDF_CHECK_LAUNCH();
    select_scan<<<dim3(1), dim3(1024), 0, s>>>(sums, nblocks, 1u, count, queue_cap);
    RTSDF_CHECK_LAUNCH();
    select_scatter<true><<<dim3(nblocks), dim3(kSelBlock), 0, s>>>(pr, logn, total, sums, 0, grid.n, queue, queue_cap);
    RTSDF_CHECK_LAUNCH();
    const int64_t nquads = (int64_t)grid.n * grid.n * grid.n / 4;
    select_mask<true><<<dim3((unsigned)((nquads + 255) / 256)), dim3(256), 0, s>>>(
        pr, logn, 0, grid.n, nquads, reinterpret_cast<uint32_t *>(mask));
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}
