// 3D jump flooding and the coarse SDF (paper Sec. 2.1; the jump flooding of
// Rong & Tan extended to three dimensions).
//
// Pass k (k = n/2, ..., 1) gives every voxel the best of its own seed and the
// seeds of the 26 voxels at offsets k (i, j, l), i, j, l in {-1, 0, 1}: the
// smallest squared distance, ties to the lowest linear seed index.  After the
// last pass the coarse SDF is c = h sqrt(D^2) - beta.
//
// Layout between passes (internal): the grid is cut into 4x4x4 bricks of 64
// voxels stored contiguously (lane = lx + 4 ly + 16 lz), brick
// b = bx + B (by + B bz) (B = n / 4), so reading a brick is one coalesced
// 256-byte block.  A seed is packed as x | y << 8 | z << 16 (0xFFFFFFFF =
// none); packed order equals linear-index order.
//
// Candidate key.  Every pass stages the seeds it reads in LDS as pairs
// (s, w); with s' = 255 - s per coordinate byte, w = |s'|^2 - 3 * 255^2 +
// 2^18 = |s|^2 - 510 (sx + sy + sz) + 2^18 for a seed and w = 0x7F000000 for
// none.  For the voxel p, with p' = 255 - p per coordinate byte packed the
// same way, the key is the 64-bit word (w + 2 dot4(s, p')) << 32 | s read as
// a float64: since 2 s.p' = 510 (sx + sy + sz) - 2 s.p its high word is
// |s|^2 - 2 s.p + 2^18 = D^2 - |p|^2 + 2^18, in (0, 2^20) for every seed, so
// the double is a non-negative denormal ordered as the integer (D^2, s) is
// for this voxel, and one v_min_f64 keeps the better of two keys; a missing
// seed's high word stays above 0x7E000000 (a large finite double) and always
// loses.  One unsigned byte dot product and one shift-add per candidate, for
// every n up to 256; the final pass recovers D^2 = high - 2^18 + |p|^2.
//
// Steps k = 4 kb >= 4: a brick's candidates are whole bricks at brick offsets
// kb (i, j, l), so the bricks with equal coordinates modulo kb form a
// sublattice on which the pass is a 3x3x3 neighbourhood.  A workgroup takes a
// 2x2x2 tile of one sublattice (eight wavefronts, one brick each) and stages
// the 4x4x4 tile-plus-halo bricks once, so a brick is read from memory by
// eight workgroups instead of by each of its 27 neighbours.  Candidates
// outside the grid are skipped with a wave-uniform choice among unrolled
// bodies for 2 or 3 distinct offsets per axis.  In the first passes, where
// most of the grid holds no seed yet, staged bricks without any seed are
// skipped as well (a bit mask in LDS read into scalar registers).
// Steps 2 and 1 stage an (8 + 2k)^3 block of voxels (eight bricks plus a
// k-voxel halo; x rows padded to 12 entries so that the 16 lanes of a
// quarter wavefront never share an LDS bank) and read their candidates at
// compile-time LDS offsets.  The k = 1 pass writes the final seeds, D^2 and c
// in the caller's linear layout.
#include "common.hpp"

namespace rtsdf {

constexpr uint32_t kNoSeed = 0xFFFFFFFFu;
constexpr uint32_t kKeyBias = 1u << 18;     // keeps the key's high word positive
constexpr uint32_t kNoSeedW = 0x7F000000u;  // w of a missing seed: its key always loses
constexpr uint32_t kKeyNone = 0x7E000000u;  // high words at or above this carry no seed

// the voxel's complemented coordinates 255 - x | (255 - y) << 8 | (255 - z) << 16
__device__ __forceinline__ uint32_t jfa_pc(int x, int y, int z)
{
    return ((uint32_t)x | ((uint32_t)y << 8) | ((uint32_t)z << 16)) ^ 0x00FFFFFFu;
}

// staged form of a seed (a seed's top byte is 0, so s ^ 0xFFFFFF complements its three coordinates)
__device__ __forceinline__ uint2 jfa_stage(uint32_t s)
{
    const uint32_t c = s ^ 0x00FFFFFFu;
    const uint32_t w = __builtin_amdgcn_udot4(c, c, kKeyBias - 3u * 255u * 255u, false);
    return make_uint2(s, s == kNoSeed ? kNoSeedW : w);
}

__device__ __forceinline__ double jfa_key(uint32_t pc, uint2 e)
{
    const uint32_t q = __builtin_amdgcn_udot4(e.x, pc, 0u, false);  // s . p' <= 3 * 255^2
    const uint32_t hi = (q << 1) + e.y;
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)e.x);
}

__device__ __forceinline__ uint32_t key_hi(double k) { return (uint32_t)(__builtin_bit_cast(uint64_t, k) >> 32); }

// the packed seed of the best key (kNoSeed if no candidate had one)
__device__ __forceinline__ uint32_t key_seed(double k)
{
    return key_hi(k) >= kKeyNone ? kNoSeed : (uint32_t)__builtin_bit_cast(uint64_t, k);
}

__device__ __forceinline__ uint32_t pack_linear(int32_t s, int logn)
{
    if (s < 0) return kNoSeed;
    const uint32_t m = (1u << logn) - 1u;
    const uint32_t u = (uint32_t)s;
    return (u & m) | (((u >> logn) & m) << 8) | ((u >> (2 * logn)) << 16);
}

__device__ __forceinline__ int32_t unpack_linear(uint32_t p, int logn)
{
    if (p == kNoSeed) return -1;
    return (int32_t)((p & 0xFFu) | (((p >> 8) & 0xFFu) << logn) | ((p >> 16) << (2 * logn)));
}

// Spread consecutive workgroups of one XCD over a contiguous range (the
// dispatcher deals workgroups to the 8 XCDs round-robin; each XCD has its own
// L2, so workgroups that read the same bricks should land on the same one).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblocks)
{
    if ((nblocks & 7u) != 0) return bid;
    return (bid & 7u) * (nblocks >> 3) + (bid >> 3);
}

// linear caller layout -> packed brick layout
__device__ __forceinline__ void jfa_to_bricks_body(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                                   int logn, int64_t e)
{
    const int B = n >> 2;
    const int b = (int)(e >> 6), l = (int)(e & 63);
    const int bx = b % B, by = (b / B) % B, bz = b / (B * B);
    const int x = bx * 4 + (l & 3), y = by * 4 + ((l >> 2) & 3), z = bz * 4 + (l >> 4);
    dst[e] = (int32_t)pack_linear(src[x + n * (y + n * z)], logn);
}

__global__ void __launch_bounds__(256) jfa_to_bricks(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                                     int n, int logn)
{
    jfa_to_bricks_body(src, dst, n, logn, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------- far passes ----

// Staged tile of a far pass: 4x4x4 brick positions (q = px + 4 py + 16 pz) of
// 64 pairs each, and a 64-bit mask of the positions holding a seed.
struct FarTile {
    uint2 e[64][64];
    uint32_t occ[2];
};

// The candidates of one brick: NX * NY * NZ staged positions starting at the
// wavefront's base position (its own position, moved back by one along every
// axis where the lower neighbour is in the grid).  CULL skips positions
// without any seed.
template <int NX, int NY, int NZ, bool CULL>
__device__ __forceinline__ double jfa_far_cands(const FarTile &T, int base, int lane, uint32_t p8, uint64_t occ)
{
    double best = __builtin_bit_cast(double, 0x7FE0000000000000ull);
#pragma unroll
    for (int o = 0; o < NX * NY * NZ; ++o) {
        const int d = (o % NX) + 4 * ((o / NX) % NY) + 16 * (o / (NX * NY));
        if (CULL && !((occ >> (base + d)) & 1ull)) continue;
        best = __builtin_fmin(best, jfa_key(p8, (&T.e[0][0])[(base + d) * 64 + lane]));
    }
    return best;
}

// One pass with step k = 4 kb >= 4 for workgroup `blk` of `nblk` (n^3 / 512
// workgroups of 512 lanes).  LINEAR_IN: the source is the caller's linear
// index array (first pass only).
template <bool LINEAR_IN, bool CULL>
__device__ __forceinline__ void jfa_far_body(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                             int logn, int logkb, uint32_t blk, uint32_t nblk)
{
    __shared__ FarTile T;
    const int logB = logn - 2;
    const int logBs = logB - logkb;  // sublattice bricks per axis: Bs >= 2 (kb <= B / 2)
    const int logTs = logBs - 1;     // 2x2x2 tiles per axis
    const int Bs = 1 << logBs;
    const uint32_t g = xcd_remap(blk, nblk);
    const uint32_t tm = (1u << logTs) - 1u;
    const int tx = (int)(g & tm), ty = (int)((g >> logTs) & tm), tz = (int)((g >> (2 * logTs)) & tm);
    const uint32_t r = g >> (3 * logTs);  // sublattice (residue of the brick coordinates modulo kb)
    const uint32_t km = (1u << logkb) - 1u;
    const int rx = (int)(r & km), ry = (int)((r >> logkb) & km), rz = (int)(r >> (2 * logkb));
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    // stage: wavefront w takes positions 8 w .. 8 w + 7.  Every read is issued before any is used (positions
    // outside the grid read a clamped brick and are then replaced by "no seed"), so a wavefront waits for
    // memory once.
    uint32_t v[8];
    bool in[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int q = wave * 8 + i;
        const int sx = 2 * tx - 1 + (q & 3), sy = 2 * ty - 1 + ((q >> 2) & 3), sz = 2 * tz - 1 + (q >> 4);
        in[i] = (unsigned)sx < (unsigned)Bs && (unsigned)sy < (unsigned)Bs && (unsigned)sz < (unsigned)Bs;
        const int cx = min(max(sx, 0), Bs - 1), cy = min(max(sy, 0), Bs - 1), cz = min(max(sz, 0), Bs - 1);
        const int bx = rx + (cx << logkb), by = ry + (cy << logkb), bz = rz + (cz << logkb);
        if (!LINEAR_IN) {
            v[i] = (uint32_t)src[(((bz << logB | by) << logB | bx) << 6) | lane];
        } else {
            const int x = bx * 4 + lx, y = by * 4 + ly, z = bz * 4 + lz;
            v[i] = (uint32_t)src[x + (y << logn) + (z << (2 * logn))];
        }
    }
    uint32_t occ_bits = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t s = !in[i] ? kNoSeed : LINEAR_IN ? pack_linear((int32_t)v[i], logn) : v[i];
        T.e[wave * 8 + i][lane] = jfa_stage(s);
        if (CULL && __ballot(s != kNoSeed) != 0) occ_bits |= 1u << i;
    }
    if (CULL && lane == 0) reinterpret_cast<uint8_t *>(T.occ)[wave] = (uint8_t)occ_bits;
    __syncthreads();
    uint64_t occ = 0;
    if (CULL) {
        const uint2 o2 = *reinterpret_cast<const uint2 *>(T.occ);
        occ = ((uint64_t)__builtin_amdgcn_readfirstlane(o2.y) << 32) | __builtin_amdgcn_readfirstlane(o2.x);
    }
    // this wavefront's brick: tile position (1 + wx, 1 + wy, 1 + wz), sublattice coordinate 2 t + w
    const int wx = wave & 1, wy = (wave >> 1) & 1, wz = wave >> 2;
    const int cx = 2 * tx + wx, cy = 2 * ty + wy, cz = 2 * tz + wz;
    const int bx = rx + (cx << logkb), by = ry + (cy << logkb), bz = rz + (cz << logkb);
    const uint32_t p8 = jfa_pc(bx * 4 + lx, by * 4 + ly, bz * 4 + lz);
    // per axis: both neighbours in the grid (3 candidates from own - 1), or one (2: from own - 1 if only the
    // lower one is, else from own)
    const bool lox = cx > 0, hix = cx + 1 < Bs, loy = cy > 0, hiy = cy + 1 < Bs, loz = cz > 0, hiz = cz + 1 < Bs;
    const int base = (1 + wx - (lox ? 1 : 0)) + 4 * (1 + wy - (loy ? 1 : 0)) + 16 * (1 + wz - (loz ? 1 : 0));
    double best;
    switch ((lox && hix ? 0 : 1) | (loy && hiy ? 0 : 2) | (loz && hiz ? 0 : 4)) {
    case 0: best = jfa_far_cands<3, 3, 3, CULL>(T, base, lane, p8, occ); break;
    case 1: best = jfa_far_cands<2, 3, 3, CULL>(T, base, lane, p8, occ); break;
    case 2: best = jfa_far_cands<3, 2, 3, CULL>(T, base, lane, p8, occ); break;
    case 3: best = jfa_far_cands<2, 2, 3, CULL>(T, base, lane, p8, occ); break;
    case 4: best = jfa_far_cands<3, 3, 2, CULL>(T, base, lane, p8, occ); break;
    case 5: best = jfa_far_cands<2, 3, 2, CULL>(T, base, lane, p8, occ); break;
    case 6: best = jfa_far_cands<3, 2, 2, CULL>(T, base, lane, p8, occ); break;
    default: best = jfa_far_cands<2, 2, 2, CULL>(T, base, lane, p8, occ); break;
    }
    dst[(((bz << logB | by) << logB | bx) << 6) | lane] = (int32_t)key_seed(best);
}

template <bool LINEAR_IN, bool CULL>
__global__ void __launch_bounds__(512) jfa_far(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                               int logn, int logkb)
{
    jfa_far_body<LINEAR_IN, CULL>(src, dst, n, logn, logkb, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------ near passes ----

// One pass with step K in {1, 2}: eight bricks (an 8^3 block) per workgroup,
// staged with a K-voxel halo in LDS (x rows of 12 entries).  FINAL writes
// the caller's outputs.
template <int K, bool FINAL>
__device__ __forceinline__ void jfa_near_body(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                              int logn, int32_t *__restrict__ dist2, float *__restrict__ sdf, float h,
                                              float beta, uint32_t blk_id, uint32_t nblk)
{
    constexpr int T = 8 + 2 * K;  // staged extent per axis
    constexpr int TX = 12;        // x row pitch (lx + 12 ly covers 16 distinct banks of 8 bytes)
    __shared__ uint2 tile[TX * T * T];
    // n is a power of two: block and brick coordinates are bit fields (shifts and masks, no divisions)
    const int logB = logn - 2, logTB = logn - 3, TB = 1 << logTB;  // 8^3 blocks per axis
    const int blk = (int)xcd_remap(blk_id, nblk);
    const int tx0 = (blk & (TB - 1)) * 8, ty0 = ((blk >> logTB) & (TB - 1)) * 8, tz0 = (blk >> (2 * logTB)) * 8;
    // staging: x slot = lane % 16 of the row, 32 rows (y, z) per sweep; all of a lane's reads are issued
    // before any is used (coordinates outside the grid read a clamped voxel, replaced by "no seed" after)
    constexpr int NS = (T * T + 31) / 32;  // sweeps
    const int xs = threadIdx.x & 15, r0 = threadIdx.x >> 4;
    const int x = tx0 - K + xs;
    const bool xin = xs < T && (unsigned)x < (unsigned)n;
    const int xc = min(max(x, 0), n - 1);
    uint32_t v[NS];
    bool in[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int row = r0 + 32 * i;
        const int yy = row % T, zz = row / T;
        const int y = ty0 - K + yy, z = tz0 - K + zz;
        in[i] = xin && row < T * T && (unsigned)y < (unsigned)n && (unsigned)z < (unsigned)n;
        const int yc = min(max(y, 0), n - 1), zc = min(max(z, 0), n - 1);
        const int b = (xc >> 2) | ((yc >> 2) << logB) | ((zc >> 2) << (2 * logB));
        v[i] = (uint32_t)src[(b << 6) | (xc & 3) | ((yc & 3) << 2) | ((zc & 3) << 4)];
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int row = r0 + 32 * i;
        if (xs < T && row < T * T) tile[xs + TX * row] = jfa_stage(in[i] ? v[i] : kNoSeed);
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lx = (wave & 1) * 4 + (lane & 3), ly = ((wave >> 1) & 1) * 4 + ((lane >> 2) & 3),
              lz = (wave >> 2) * 4 + (lane >> 4);
    const int px = tx0 + lx, py = ty0 + ly, pz = tz0 + lz;
    const uint32_t p8 = jfa_pc(px, py, pz);
    const int c = (lx + K) + TX * ((ly + K) + T * (lz + K));
    double best = __builtin_bit_cast(double, 0x7FE0000000000000ull);
#pragma unroll
    for (int o = 0; o < 27; ++o) {
        const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
        best = __builtin_fmin(best, jfa_key(p8, tile[c + K * (ox + TX * (oy + T * oz))]));
    }
    const uint32_t s = key_seed(best);
    if (!FINAL) {
        const int b = (px >> 2) | ((py >> 2) << logB) | ((pz >> 2) << (2 * logB));
        dst[(b << 6) | (px & 3) | ((py & 3) << 2) | ((pz & 3) << 4)] = (int32_t)s;
    } else {
        const int idx = px | (py << logn) | (pz << (2 * logn));  // n <= 256: below 2^24
        if (s == kNoSeed) {
            dst[idx] = -1;
            dist2[idx] = INT32_MAX;
            sdf[idx] = __builtin_inff();
        } else {
            const int d2 = (int)(key_hi(best) - kKeyBias) + px * px + py * py + pz * pz;
            dst[idx] = unpack_linear(s, logn);
            dist2[idx] = d2;
            sdf[idx] = rn_sub(rn_mul(h, rn_sqrt((float)d2)), beta);
        }
    }
}

template <int K, bool FINAL>
__global__ void __launch_bounds__(512) jfa_near(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                                int logn, int32_t *__restrict__ dist2, float *__restrict__ sdf,
                                                float h, float beta)
{
    jfa_near_body<K, FINAL>(src, dst, n, logn, dist2, sdf, h, beta, blockIdx.x, gridDim.x);
}

// Passes at the start of a schedule skip staged bricks without seeds: in the
// first three passes of n/2, ..., 1 most of the grid holds none yet.
constexpr int kCullPasses = 3;

static int launch_far(bool linear_in, bool cull, const int32_t *src, int32_t *dst, int n, int logn, int k,
                      hipStream_t s)
{
    const unsigned blocks = (unsigned)((int64_t)n * n * n / 512);
    const int logkb = ilog2(k / 4);
    if (linear_in) {
        if (cull) jfa_far<true, true><<<dim3(blocks), dim3(512), 0, s>>>(src, dst, n, logn, logkb);
        else jfa_far<true, false><<<dim3(blocks), dim3(512), 0, s>>>(src, dst, n, logn, logkb);
    } else {
        if (cull) jfa_far<false, true><<<dim3(blocks), dim3(512), 0, s>>>(src, dst, n, logn, logkb);
        else jfa_far<false, false><<<dim3(blocks), dim3(512), 0, s>>>(src, dst, n, logn, logkb);
    }
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

static int launch_near(int k, const int32_t *src, int32_t *dst, int n, int logn, hipStream_t s)
{
    const unsigned blocks = (unsigned)((int64_t)n * n * n / 512);
    if (k == 2)
        jfa_near<2, false><<<dim3(blocks), dim3(512), 0, s>>>(src, dst, n, logn, nullptr, nullptr, 0.f, 0.f);
    else
        jfa_near<1, false><<<dim3(blocks), dim3(512), 0, s>>>(src, dst, n, logn, nullptr, nullptr, 0.f, 0.f);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

static int jfa_run(const rtsdf_grid &g, int32_t *seeds, int32_t *scratch, float beta, int32_t *dist2, float *sdf,
                   const int32_t *steps, int m, hipStream_t s)
{
    const int n = g.n, logn = ilog2(n);
    const int64_t nvox = (int64_t)n * n * n;
    const unsigned blocks = (unsigned)(nvox / 512);
    // Passes 0 .. m-2 go brick layout to brick layout; the final pass (step 1) must read `scratch` and write the
    // caller's linear layout to `seeds` (and `dist2`, `sdf`).  When the first step is a far one it reads the
    // linear input directly, and the brick passes alternate between `dist2` (written only by the final pass,
    // and distinct from `seeds` and `scratch` since that pass reads one and writes the other) and `scratch`,
    // chosen so that the last one lands in `scratch`.  Otherwise the input is converted into `scratch` first,
    // and copied once more when the number of brick passes would leave the last one in the wrong buffer.
    const int npass = m - 1;
    const int32_t *cur = seeds;
    int rc = RTSDF_OK;
    if (npass >= 1 && steps[0] >= 4) {
        for (int i = 0; i < npass && rc == RTSDF_OK; ++i) {
            const int k = steps[i];
            int32_t *dst = (npass - 1 - i) % 2 == 0 ? scratch : dist2;
            rc = k >= 4 ? launch_far(i == 0, i < kCullPasses, cur, dst, n, logn, k, s)
                        : launch_near(k, cur, dst, n, logn, s);
            cur = dst;
        }
    } else {
        int32_t *bufs[2] = {seeds, scratch};
        int next = 0;  // index into bufs of the next destination
        jfa_to_bricks<<<dim3((unsigned)(nvox / 256)), dim3(256), 0, s>>>(seeds, scratch, n, logn);
        RTSDF_CHECK_LAUNCH();
        cur = scratch;
        if (npass % 2 == 1) {
            RTSDF_TRY(hipMemcpyAsync(seeds, scratch, sizeof(int32_t) * nvox, hipMemcpyDeviceToDevice, s));
            cur = seeds;
            next = 1;
        }
        for (int i = 0; i < npass && rc == RTSDF_OK; ++i) {
            const int k = steps[i];
            int32_t *dst = bufs[next];
            rc = k >= 4 ? launch_far(false, i < kCullPasses, cur, dst, n, logn, k, s)
                        : launch_near(k, cur, dst, n, logn, s);
            cur = dst;
            next ^= 1;
        }
    }
    if (rc != RTSDF_OK) return rc;
    // cur == scratch here by construction
    jfa_near<1, true><<<dim3(blocks), dim3(512), 0, s>>>(cur, seeds, n, logn, dist2, sdf, g.h, beta);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

}  // namespace rtsdf

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
    return jfa_run(coarse, seeds, scratch, beta, dist2, coarse_sdf, steps, nsteps, s);
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
