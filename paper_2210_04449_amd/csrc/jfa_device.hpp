// 3D jump flooding and the coarse SDF (paper Sec. 2.1; the jump flooding of
// Rong & Tan extended to three dimensions).
//
// Pass k (k = n/2, ..., 1) gives every voxel the best of its own seed and the
// seeds of the 26 voxels at offsets k (i, j, l), i, j, l in {-1, 0, 1}: the
// smallest squared distance, ties to the lowest linear seed index.  After the
// last pass the coarse SDF is c = h sqrt(D^2) - beta.
//
// Layout between passes (internal): the grid is cut into 4x4x4 bricks; brick
// b = bx + B (by + B bz) (B = n / 4) stores its 64 voxels contiguously (lane =
// lx + 4 ly + 16 lz), so every candidate read of a wavefront (one lane per
// voxel of a brick) is one coalesced 256-byte block.  A seed is packed as
// x | y << 8 | z << 16 (0xFFFFFFFF = none); packed order equals linear-index
// order, so ties compare the packed word directly.
//
// Candidate key: the 64-bit word (hi << 32 | low), read as a float64, where hi
// orders the candidates by D^2 and low increases with the packed seed.  Its
// exponent field is zero (hi < 2^20), so it is a non-negative denormal whose
// order is the integer order, and one v_min_f64 keeps the better of two keys.
// A missing seed gets bits 0x7F000000 in the high word (a large finite
// double) and always loses.  Two key forms, both from byte dot products:
// * 7-bit (far passes, n <= 128): hi = D^2.  The voxel constant C holds
//   128 - x, 128 - y, 128 - z in its bytes, so u = S + C holds (s - x) + 128
//   etc. in [1, 255] per byte without carries: u is the key's low word
//   (S = u - C), u ^ 0x808080 the signed byte differences, and one
//   v_dot4_i32_i8 squares and sums them.
// * byte-dot (every pass at n = 256, the near passes at every n): hi =
//   |S|^2 - 2 S.p + 2^18 = D^2 - |p|^2 + 2^18 for the voxel p, low = S: two
//   v_dot4_u32_u8 and one 24-bit multiply-add, or, with w(S) = |S|^2 staged
//   beside each seed, one of each (near passes at n <= 128 stage a pair that
//   needs the dot product alone: jfa_pair_small).
//
// Steps k >= 4 read whole neighbour bricks straight from global memory (an
// axis offset that would leave the grid is not read, or reads the brick with
// offset 0 on that axis, a candidate the set already holds), one brick per
// wavefront or, sharing the candidate bricks they have in common, two or four
// bricks of one residue class per wavefront.  Steps 2 and 1 stage an
// (8 + 2k)^3 block of voxels (eight bricks plus halo) in LDS; candidates then
// sit at compile-time LDS offsets and out-of-grid halo entries are empty.  The
// k = 1 pass writes the final seeds, D^2 and c in the caller's linear layout.
#pragma once

#include "common.hpp"

namespace rtsdf {

constexpr uint32_t kNoSeed = 0xFFFFFFFFu;

typedef short jfa_short2 __attribute__((ext_vector_type(2)));

// Voxel-side constants.  a: the 7-bit key's C = (128 - x) | (128 - y) << 8 | (128 - z) << 16 (n <= 128);
// p = x | y << 8 | z << 16 and pp = |p|^2 for the byte-dot key; neg2 = -2, a kernel argument (a constant
// multiplier would be strength-reduced to a shift and a subtraction instead of one 24-bit multiply-add).
struct JfaPos {
    uint32_t a, p;
    int32_t pp, neg2;
};

__device__ __forceinline__ JfaPos jfa_pos(int x, int y, int z, int neg2)
{
    JfaPos P;
    P.a = (uint32_t)(128 - x) | ((uint32_t)(128 - y) << 8) | ((uint32_t)(128 - z) << 16);
    P.p = (uint32_t)x | ((uint32_t)y << 8) | ((uint32_t)z << 16);
    P.pp = x * x + y * y + z * z;
    P.neg2 = neg2;
    return P;
}

// 7-bit key (n <= 128): high word D^2 from the signed byte differences, low word u = S + C.
__device__ __forceinline__ double jfa_key7(JfaPos P, uint32_t s)
{
    const uint32_t low = s + P.a;
    const int d = (int)(low ^ 0x00808080u);
    // the missing-seed bits have zero low 24 bits and D^2 < 2^24, so adding them is or-ing them
    const uint32_t hi = (uint32_t)__builtin_amdgcn_sdot4(d, d, (int)(s & 0x7F000000u), false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)low);
}

// Byte-dot key (n <= 256): high word |S|^2 - 2 S.p + 2^18 = D^2 - |p|^2 + 2^18 (in [2^18 - 3 * 255^2,
// 2^18 + 3 * 255^2], the same order as D^2 for one voxel) plus the missing-seed bits, low word the seed.  w(S)
// = |S|^2 + missing bits depends on the seed alone, so staged seeds carry it; the 2^18 enters as -2^17 in
// the accumulator of S.p (S.p - 2^17 in [-2^17, 2^16): a 24-bit operand of the multiply-add by -2).
__device__ __forceinline__ uint32_t jfa_w(uint32_t s)
{
    return __builtin_amdgcn_udot4(s, s, s & 0x7F000000u, false);
}

__device__ __forceinline__ double jfa_keyd_w(JfaPos P, uint32_t s, uint32_t w)
{
    const int sp = (int)__builtin_amdgcn_udot4(s, P.p, 0xFFFE0000u, false);  // S.p - 2^17 (wraps)
    const uint32_t hi = (uint32_t)(__mul24(sp, P.neg2) + (int)w);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)s);
}

__device__ __forceinline__ double jfa_keyd(JfaPos P, uint32_t s) { return jfa_keyd_w(P, s, jfa_w(s)); }

__device__ __forceinline__ uint32_t key_hi(double k) { return (uint32_t)(__builtin_bit_cast(uint64_t, k) >> 32); }

// the packed seed of the best key (kNoSeed if no candidate had one); BYTEDOT: which key formula made it
template <bool BYTEDOT>
__device__ __forceinline__ uint32_t key_seed(JfaPos P, double k)
{
    if (key_hi(k) >= 0x7F000000u) return kNoSeed;
    const uint32_t low = (uint32_t)__builtin_bit_cast(uint64_t, k);
    return BYTEDOT ? low : low - P.a;
}

// D^2 of a byte-dot key with a seed
__device__ __forceinline__ uint32_t keyd_d2(JfaPos P, double k) { return key_hi(k) - 0x40000u + (uint32_t)P.pp; }

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
// L2, so neighbouring bricks should land on the same one).
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

// The distinct offsets along one axis of a pass with step k = 4 kb >= 4 (brick coordinate c, in units of
// the stride st).  An offset that would leave the grid is replaced by 0: the brick read is then the candidate
// whose offset on that axis is 0, which the set already holds, and a duplicate cannot change the minimum.  So
// an axis where one side leaves the grid (at most one can, unless kb = B/2, where exactly one does) has two
// distinct offsets, {0, the side that stays}, and an axis where neither does has three.
template <int N>
__device__ __forceinline__ void jfa_axis(int c, int kb, int st, int (&d)[N])
{
    if (N == 3) {
        d[0] = -st;
        d[1] = 0;
        d[N - 1] = st;
    } else {
        d[0] = 0;
        d[N - 1] = c >= kb ? -st : st;
    }
}

// The candidates of brick b: NX * NY * NZ distinct neighbour bricks, every read in the grid.
template <bool WIDE, bool LINEAR_IN, int NX, int NY, int NZ>
__device__ __forceinline__ void jfa_far_brick(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                              int logn, int kb, int b, int lane, int neg2)
{
    constexpr int NCAND = NX * NY * NZ;
    const int logB = logn - 2, B = 1 << logB;
    const int bx = b & (B - 1), by = (b >> logB) & (B - 1), bz = b >> (2 * logB);
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const JfaPos P = jfa_pos(bx * 4 + lx, by * 4 + ly, bz * 4 + lz, neg2);
    double best = __builtin_bit_cast(double, 0x7FE0000000000000ull);
    uint32_t cand[NCAND];
    if (!LINEAR_IN) {
        int dx[NX], dy[NY], dz[NZ];
        jfa_axis(bx, kb, kb, dx);
        jfa_axis(by, kb, kb << logB, dy);
        jfa_axis(bz, kb, kb << (2 * logB), dz);
        // raw buffer loads: the lane's byte offset is one vector register shared by all the reads, the brick's
        // byte offset a scalar (every read lies in the n^3-word buffer; gfx9 descriptor word 3)
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t *>(src), (short)0, (n * n * n) * 4, 0x00020000);
#pragma unroll
        for (int o = 0; o < NCAND; ++o) {
            const int off = (b + dx[o % NX] + dy[(o / NX) % NY] + dz[o / (NX * NY)]) << 8;
            cand[o] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, lane * 4, off, 0);
        }
    } else {
        int dx[NX], dy[NY], dz[NZ];
        jfa_axis(bx, kb, kb, dx);
        jfa_axis(by, kb, kb, dy);
        jfa_axis(bz, kb, kb, dz);
#pragma unroll
        for (int o = 0; o < NCAND; ++o) {
            const int x = (bx + dx[o % NX]) * 4 + lx, y = (by + dy[(o / NX) % NY]) * 4 + ly;
            const int z = (bz + dz[o / (NX * NY)]) * 4 + lz;
            cand[o] = pack_linear(src[x + (y << logn) + (z << (2 * logn))], logn);
        }
    }
#pragma unroll
    for (int o = 0; o < NCAND; ++o) best = __builtin_fmin(best, WIDE ? jfa_keyd(P, cand[o]) : jfa_key7(P, cand[o]));
    dst[(int64_t)b * 64 + lane] = (int32_t)key_seed<WIDE>(P, best);
}

// The brick a far-pass wavefront takes, from its place v in dispatch order (after the XCD remap, so that
// each XCD takes one contiguous eighth of v).  Slab order (coset = 0): brick v, so an XCD walks a slab of
// whole z-layers, and at large steps the z-neighbours it reads sit in other XCDs' slabs (each brick is then
// fetched into up to three L2s).  Coset order (coset = 1, step kb >= 2 bricks): the candidates of a brick
// all lie in its residue class (bx, by, bz) mod kb, so v runs over one class after another (the class index
// in the high bits, the brick's position within the class, x fastest, in the low bits): every brick is read
// by the XCD that owns its class only, and within a class a wavefront's reads are the previous, current and
// next layer of the class.  Both orders visit every brick once.
__device__ __forceinline__ int far_brick(uint32_t v, int logB, int kb, int coset)
{
    if (!coset || kb < 2) return (int)v;
    const int lk = __builtin_ctz((unsigned)kb), m = logB - lk;  // kb^3 classes of (2^m)^3 bricks
    const int mm = (1 << m) - 1;
    const int w = (int)v & ((1 << (3 * m)) - 1), r = (int)(v >> (3 * m));
    const int cx = w & mm, cy = (w >> m) & mm, cz = w >> (2 * m);
    const int rx = r & (kb - 1), ry = (r >> lk) & (kb - 1), rz = r >> (2 * lk);
    return (rx | (cx << lk)) | ((ry | (cy << lk)) << logB) | ((rz | (cz << lk)) << (2 * logB));
}

// One pass with step k >= 4 (a multiple of the brick size) for the four
// bricks of workgroup `blk` of `nblk`.  LINEAR_IN: the source is the caller's
// linear index array (first pass only).  Each wavefront (one brick) takes the
// unrolled body for its own distinct-offset counts per axis: a wave-uniform
// branch, so every body keeps all its reads in flight together.
template <bool WIDE, bool LINEAR_IN>
__device__ __forceinline__ void jfa_far_body(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                             int logn, int kb, uint32_t blk, uint32_t nblk, int neg2, int coset)
{
    const int logB = logn - 2, B = 1 << logB;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int b = far_brick(xcd_remap(blk, nblk) * 4 + wave, logB, kb, coset);
    const int bx = b & (B - 1), by = (b >> logB) & (B - 1), bz = b >> (2 * logB);
    const auto two = [&](int c) { return c < kb || c + kb >= B; };  // one side leaves the grid
    switch ((two(bx) ? 1 : 0) | (two(by) ? 2 : 0) | (two(bz) ? 4 : 0)) {
    case 0: jfa_far_brick<WIDE, LINEAR_IN, 3, 3, 3>(src, dst, n, logn, kb, b, lane, neg2); break;
    case 1: jfa_far_brick<WIDE, LINEAR_IN, 2, 3, 3>(src, dst, n, logn, kb, b, lane, neg2); break;
    case 2: jfa_far_brick<WIDE, LINEAR_IN, 3, 2, 3>(src, dst, n, logn, kb, b, lane, neg2); break;
    case 3: jfa_far_brick<WIDE, LINEAR_IN, 2, 2, 3>(src, dst, n, logn, kb, b, lane, neg2); break;
    case 4: jfa_far_brick<WIDE, LINEAR_IN, 3, 3, 2>(src, dst, n, logn, kb, b, lane, neg2); break;
    case 5: jfa_far_brick<WIDE, LINEAR_IN, 2, 3, 2>(src, dst, n, logn, kb, b, lane, neg2); break;
    case 6: jfa_far_brick<WIDE, LINEAR_IN, 3, 2, 2>(src, dst, n, logn, kb, b, lane, neg2); break;
    default: jfa_far_brick<WIDE, LINEAR_IN, 2, 2, 2>(src, dst, n, logn, kb, b, lane, neg2); break;
    }
}

// Two bricks per wavefront: b0 at an even coordinate cx of its residue class along x (coset order, or any
// brick pair (2i, 2i + 1) at step 4) and b1 = b0 + kb, the next brick of the class.  Their candidate columns
// along x are cx - 1, cx, cx + 1 and cx, cx + 1, cx + 2 (in class units), so the wavefront reads the (up to)
// four distinct columns once and keys each against the bricks that take it: 4 x 3 x 3 = 36 reads for two bricks
// instead of 54.  XL: column cx - 1 lies in the grid (cx > 0); XR: column cx + 2 does; a column outside is not
// read (for the y and z axes, as for one brick, an offset that leaves the grid is replaced by 0, a duplicate).
// Each lane keys one voxel of each brick: the same lane position in both.
template <bool WIDE, bool XL, bool XR, int NY, int NZ>
__device__ __forceinline__ void jfa_far_pair(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                             int logn, int kb, int b0, int lane, int neg2)
{
    constexpr int NX = 2 + (XL ? 1 : 0) + (XR ? 1 : 0), NCAND = NX * NY * NZ;
    const int logB = logn - 2, B = 1 << logB;
    const int bx = b0 & (B - 1), by = (b0 >> logB) & (B - 1), bz = b0 >> (2 * logB);
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const JfaPos P0 = jfa_pos(bx * 4 + lx, by * 4 + ly, bz * 4 + lz, neg2);
    const JfaPos P1 = jfa_pos((bx + kb) * 4 + lx, by * 4 + ly, bz * 4 + lz, neg2);
    int dx[NX], dy[NY], dz[NZ];
    {
        int i = 0;
        if (XL) dx[i++] = -kb;
        dx[i++] = 0;
        dx[i++] = kb;
        if (XR) dx[i++] = 2 * kb;
    }
    jfa_axis(by, kb, kb << logB, dy);
    jfa_axis(bz, kb, kb << (2 * logB), dz);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t *>(src), (short)0, (n * n * n) * 4, 0x00020000);
    uint32_t cand[NCAND];
#pragma unroll
    for (int o = 0; o < NCAND; ++o) {
        const int off = (b0 + dx[o % NX] + dy[(o / NX) % NY] + dz[o / (NX * NY)]) << 8;
        cand[o] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, lane * 4, off, 0);
    }
    double best0 = __builtin_bit_cast(double, 0x7FE0000000000000ull), best1 = best0;
    constexpr int X0 = XL ? 1 : 0;  // the slot of column cx
#pragma unroll
    for (int o = 0; o < NCAND; ++o) {
        const int xs = o % NX;
        if (xs <= X0 + 1) best0 = __builtin_fmin(best0, WIDE ? jfa_keyd(P0, cand[o]) : jfa_key7(P0, cand[o]));
        if (xs >= X0) best1 = __builtin_fmin(best1, WIDE ? jfa_keyd(P1, cand[o]) : jfa_key7(P1, cand[o]));
    }
    dst[(int64_t)b0 * 64 + lane] = (int32_t)key_seed<WIDE>(P0, best0);
    dst[(int64_t)(b0 + kb) * 64 + lane] = (int32_t)key_seed<WIDE>(P1, best1);
}

// One pass with step k >= 4 in brick pairs: the four wavefronts of workgroup `blk` of `nblk` take pairs
// 4 blk' + w (blk' after the XCD remap) of the coset order (far_brick of 2 v and 2 v + 1: one class after another,
// so an XCD owns whole classes).
template <bool WIDE>
__device__ __forceinline__ void jfa_far_pair_body(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                                  int logn, int kb, uint32_t blk, uint32_t nblk, int neg2)
{
    const int logB = logn - 2, B = 1 << logB;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int b0 = far_brick((xcd_remap(blk, nblk) * 4 + wave) * 2, logB, kb, 1);
    const int bx = b0 & (B - 1), by = (b0 >> logB) & (B - 1), bz = b0 >> (2 * logB);
    const int lk = __builtin_ctz((unsigned)kb);
    const int cx = bx >> lk, side = B >> lk;  // class coordinate and class side along x
    const auto two = [&](int c) { return c < kb || c + kb >= B; };  // one side leaves the grid
    const int xc = (cx > 0 ? 1 : 0) | (cx + 2 < side ? 2 : 0);
    switch (xc | (two(by) ? 4 : 0) | (two(bz) ? 8 : 0)) {
#define RTSDF_PAIR_CASE(C, XL, XR, NY, NZ) \
    case C: jfa_far_pair<WIDE, XL, XR, NY, NZ>(src, dst, n, logn, kb, b0, lane, neg2); break;
    RTSDF_PAIR_CASE(0, false, false, 3, 3)
    RTSDF_PAIR_CASE(1, true, false, 3, 3)
    RTSDF_PAIR_CASE(2, false, true, 3, 3)
    RTSDF_PAIR_CASE(3, true, true, 3, 3)
    RTSDF_PAIR_CASE(4, false, false, 2, 3)
    RTSDF_PAIR_CASE(5, true, false, 2, 3)
    RTSDF_PAIR_CASE(6, false, true, 2, 3)
    RTSDF_PAIR_CASE(7, true, true, 2, 3)
    RTSDF_PAIR_CASE(8, false, false, 3, 2)
    RTSDF_PAIR_CASE(9, true, false, 3, 2)
    RTSDF_PAIR_CASE(10, false, true, 3, 2)
    RTSDF_PAIR_CASE(11, true, true, 3, 2)
    RTSDF_PAIR_CASE(12, false, false, 2, 2)
    RTSDF_PAIR_CASE(13, true, false, 2, 2)
    RTSDF_PAIR_CASE(14, false, true, 2, 2)
    default: jfa_far_pair<WIDE, true, true, 2, 2>(src, dst, n, logn, kb, b0, lane, neg2); break;
#undef RTSDF_PAIR_CASE
    }
}

// Four bricks per wavefront: the 2 x 2 block at even class coordinates (cx, cy) and (cx + 1, cy), (cx, cy + 1),
// (cx + 1, cy + 1) of one residue class (steps of kb bricks along x and y).  As for a pair, along x and along y
// the (up to) four distinct columns are read once and keyed against the bricks that take them: 4 x 4 x 3 = 48
// reads for four bricks instead of 108.  XL / XR / YL / YR: the columns cx - 1 / cx + 2 / cy - 1 / cy + 2 lie in
// the grid.  Each lane keys one voxel of each brick: the same lane position in all four.
template <bool WIDE, bool XL, bool XR, bool YL, bool YR, int NZ>
__device__ __forceinline__ void jfa_far_quad(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                             int logn, int kb, int b0, int lane, int neg2)
{
    constexpr int NX = 2 + (XL ? 1 : 0) + (XR ? 1 : 0), NY = 2 + (YL ? 1 : 0) + (YR ? 1 : 0);
    constexpr int NCAND = NX * NY * NZ;
    const int logB = logn - 2, B = 1 << logB;
    const int bx = b0 & (B - 1), by = (b0 >> logB) & (B - 1), bz = b0 >> (2 * logB);
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    JfaPos P[4];  // brick i + 2 j: (bx + i kb, by + j kb)
#pragma unroll
    for (int q = 0; q < 4; ++q)
        P[q] = jfa_pos((bx + (q & 1) * kb) * 4 + lx, (by + (q >> 1) * kb) * 4 + ly, bz * 4 + lz, neg2);
    const int sy = kb << logB;
    int dx[NX], dy[NY], dz[NZ];
    {
        int i = 0;
        if (XL) dx[i++] = -kb;
        dx[i++] = 0;
        dx[i++] = kb;
        if (XR) dx[i++] = 2 * kb;
        i = 0;
        if (YL) dy[i++] = -sy;
        dy[i++] = 0;
        dy[i++] = sy;
        if (YR) dy[i++] = 2 * sy;
    }
    jfa_axis(bz, kb, kb << (2 * logB), dz);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t *>(src), (short)0, (n * n * n) * 4, 0x00020000);
    uint32_t cand[NCAND];
#pragma unroll
    for (int o = 0; o < NCAND; ++o) {
        const int off = (b0 + dx[o % NX] + dy[(o / NX) % NY] + dz[o / (NX * NY)]) << 8;
        cand[o] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, lane * 4, off, 0);
    }
    double best[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) best[q] = __builtin_bit_cast(double, 0x7FE0000000000000ull);
    constexpr int X0 = XL ? 1 : 0, Y0 = YL ? 1 : 0;  // the slots of columns cx and cy
#pragma unroll
    for (int o = 0; o < NCAND; ++o) {
        const int xs = o % NX, ys = (o / NX) % NY;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = q & 1, j = q >> 1;
            if (xs >= X0 - 1 + i && xs <= X0 + 1 + i && ys >= Y0 - 1 + j && ys <= Y0 + 1 + j)
                best[q] = __builtin_fmin(best[q], WIDE ? jfa_keyd(P[q], cand[o]) : jfa_key7(P[q], cand[o]));
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        dst[(int64_t)(b0 + (q & 1) * kb + (q >> 1) * sy) * 64 + lane] = (int32_t)key_seed<WIDE>(P[q], best[q]);
}

// The (even, even) brick of quad v in coset order: within a class of side 2^m bricks, v's low bits give cx / 2
// and cy / 2 (m - 1 bits each), then cz (m bits), then the class; the classes and an XCD's range as for one brick.
__device__ __forceinline__ int quad_brick(uint32_t v, int logB, int kb)
{
    const int lk = __builtin_ctz((unsigned)kb), m = logB - lk;
    const int h = m - 1, hm = (1 << h) - 1;
    const int qx = (int)v & hm, qy = (int)(v >> h) & hm, cz = (int)(v >> (2 * h)) & ((1 << m) - 1);
    const int r = (int)(v >> (2 * h + m));
    const int rx = r & (kb - 1), ry = (r >> lk) & (kb - 1), rz = r >> (2 * lk);
    return (rx | (qx << (lk + 1))) | ((ry | (qy << (lk + 1))) << logB) | ((rz | (cz << lk)) << (2 * logB));
}

// One pass with step k >= 4 in 2 x 2 brick quads: the W wavefronts of workgroup `blk` of `nblk` take quads
// W blk' + w (blk' after the XCD remap; W = 1 for the single-scene passes, 4 in the batched kernel).
template <bool WIDE>
__device__ __forceinline__ void jfa_far_quad_body(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                                  int logn, int kb, uint32_t blk, uint32_t nblk, int neg2)
{
    const int logB = logn - 2, B = 1 << logB;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int b0 = quad_brick(xcd_remap(blk, nblk) * (blockDim.x >> 6) + wave, logB, kb);
    const int bx = b0 & (B - 1), by = (b0 >> logB) & (B - 1), bz = b0 >> (2 * logB);
    const int lk = __builtin_ctz((unsigned)kb);
    const int cx = bx >> lk, cy = by >> lk, side = B >> lk;
    const bool two_z = bz < kb || bz + kb >= B;  // one side leaves the grid
    const int c = (cx > 0 ? 1 : 0) | (cx + 2 < side ? 2 : 0) | (cy > 0 ? 4 : 0) | (cy + 2 < side ? 8 : 0) |
                  (two_z ? 16 : 0);
    switch (c) {
#define RTSDF_QUAD_CASE(C)                                                                                       \
    case C:                                                                                                      \
        jfa_far_quad<WIDE, (C & 1) != 0, (C & 2) != 0, (C & 4) != 0, (C & 8) != 0, (C & 16) ? 2 : 3>(             \
            src, dst, n, logn, kb, b0, lane, neg2);                                                              \
        break;
    RTSDF_QUAD_CASE(0) RTSDF_QUAD_CASE(1) RTSDF_QUAD_CASE(2) RTSDF_QUAD_CASE(3)
    RTSDF_QUAD_CASE(4) RTSDF_QUAD_CASE(5) RTSDF_QUAD_CASE(6) RTSDF_QUAD_CASE(7)
    RTSDF_QUAD_CASE(8) RTSDF_QUAD_CASE(9) RTSDF_QUAD_CASE(10) RTSDF_QUAD_CASE(11)
    RTSDF_QUAD_CASE(12) RTSDF_QUAD_CASE(13) RTSDF_QUAD_CASE(14) RTSDF_QUAD_CASE(15)
    RTSDF_QUAD_CASE(16) RTSDF_QUAD_CASE(17) RTSDF_QUAD_CASE(18) RTSDF_QUAD_CASE(19)
    RTSDF_QUAD_CASE(20) RTSDF_QUAD_CASE(21) RTSDF_QUAD_CASE(22) RTSDF_QUAD_CASE(23)
    RTSDF_QUAD_CASE(24) RTSDF_QUAD_CASE(25) RTSDF_QUAD_CASE(26) RTSDF_QUAD_CASE(27)
    RTSDF_QUAD_CASE(28) RTSDF_QUAD_CASE(29) RTSDF_QUAD_CASE(30)
    default:
        jfa_far_quad<WIDE, true, true, true, true, 2>(src, dst, n, logn, kb, b0, lane, neg2);
        break;
#undef RTSDF_QUAD_CASE
    }
}

// The first pass of plain jump flooding (step n/2) from the caller's linear seeds.  At that step one side of
// every axis leaves the grid, so a voxel's distinct candidates are its own seed and the seeds at p XOR n/2 on
// any subset of the axes: the same eight voxels for all eight members of such an orbit, and brick b's
// candidates sit at the same lane in the bricks b XOR B/2 on those axes.  A workgroup of eight wavefronts
// takes one orbit of bricks: each wavefront stages its brick once in LDS, and every lane keys the eight staged
// candidates of its voxel (instead of each wavefront reading all eight bricks from memory).
template <bool WIDE>
__device__ __forceinline__ void jfa_first_orbit_body(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                                     int n, int logn, int neg2, uint32_t blk_id, uint32_t nblk)
{
    __shared__ uint32_t tile[8][kWave];
    const int logB = logn - 2, logH = logB - 1, H = 1 << logH;  // orbits: H^3 workgroups, H = B / 2
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = (int)xcd_remap(blk_id, nblk);
    const int gx = g & (H - 1), gy = (g >> logH) & (H - 1), gz = g >> (2 * logH);
    // this wavefront's brick: the orbit member (wave bit 0: +B/2 in x, bit 1: in y, bit 2: in z)
    const int bx = gx + ((wave & 1) << logH), by = gy + (((wave >> 1) & 1) << logH), bz = gz + ((wave >> 2) << logH);
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int x = bx * 4 + lx, y = by * 4 + ly, z = bz * 4 + lz;
    tile[wave][lane] = pack_linear(src[x + (y << logn) + (z << (2 * logn))], logn);
    __syncthreads();
    const JfaPos P = jfa_pos(x, y, z, neg2);
    double best = __builtin_bit_cast(double, 0x7FE0000000000000ull);
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const uint32_t c = tile[wave ^ o][lane];
        best = __builtin_fmin(best, WIDE ? jfa_keyd(P, c) : jfa_key7(P, c));
    }
    const int b = bx | (by << logB) | (bz << (2 * logB));
    dst[((int64_t)b << 6) | lane] = (int32_t)key_seed<WIDE>(P, best);
}

// The same first pass for four orbits next to each other along x (n >= 32, so H = n / 8 >= 4): orbit
// coordinates (4 gq + t, gy, gz), t = 0..3.  Member m of the four orbits are four bricks next to each other
// along x, so the workgroup reads each of their rows of 16 voxels as one 64-byte run of the caller's linear
// seeds (instead of four 16-byte pieces), stages the 32 bricks in LDS, and wavefront m keys the voxel of its
// lane in the four bricks of member m.
template <bool WIDE>
__device__ __forceinline__ void jfa_first_orbit4_body(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                                      int n, int logn, int neg2, uint32_t blk_id, uint32_t nblk)
{
    __shared__ uint32_t tile[8][4][kWave];  // [member][orbit t][lane]
    const int logB = logn - 2, logH = logB - 1, H = 1 << logH, logQ = logH - 2;  // H / 4 groups along x
    const int g = (int)xcd_remap(blk_id, nblk);
    const int gx0 = (g & ((1 << logQ) - 1)) * 4, gy = (g >> logQ) & (H - 1), gz = g >> (logQ + logH);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = (int)threadIdx.x + 512 * r;  // 2048 voxels: 16 along x, 16 rows, 8 members
        const int xx = e & 15, row = (e >> 4) & 15, m = e >> 8;
        const int x = (gx0 + ((m & 1) << logH)) * 4 + xx;
        const int y = (gy + (((m >> 1) & 1) << logH)) * 4 + (row & 3);
        const int z = (gz + ((m >> 2) << logH)) * 4 + (row >> 2);
        tile[m][xx >> 2][(xx & 3) | ((row & 3) << 2) | ((row >> 2) << 4)] =
            pack_linear(src[x + (y << logn) + (z << (2 * logn))], logn);
    }
    __syncthreads();
    const int m = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int by = gy + (((m >> 1) & 1) << logH), bz = gz + ((m >> 2) << logH);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int bx = gx0 + t + ((m & 1) << logH);
        const JfaPos P = jfa_pos(bx * 4 + lx, by * 4 + ly, bz * 4 + lz, neg2);
        double best = __builtin_bit_cast(double, 0x7FE0000000000000ull);
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const uint32_t c = tile[m ^ o][t][lane];
            best = __builtin_fmin(best, WIDE ? jfa_keyd(P, c) : jfa_key7(P, c));
        }
        const int b = bx | (by << logB) | (bz << (2 * logB));
        dst[((int64_t)b << 6) | lane] = (int32_t)key_seed<WIDE>(P, best);
    }
}

// The halo shell of a near pass's LDS tile: every entry (u, v, w) of the T^3 tile (T = 8 + 2K) outside the
// block's eight bricks, in (w, v, u) order, packed as u | v << 4 | w << 8 | (tile index u + PX (v + T w)) << 12.
// A table built at compile time: a lane reads its entry instead of taking j apart by divisions.
template <int K, int PX>
struct ShellTable {
    static constexpr int T = 8 + 2 * K, N = T * T * T - 512;
    uint32_t e[N];
    constexpr ShellTable() : e()
    {
        int j = 0;
        for (int w = 0; w < T; ++w)
            for (int v = 0; v < T; ++v)
                for (int u = 0; u < T; ++u)
                    if (!(u >= K && u < K + 8 && v >= K && v < K + 8 && w >= K && w < K + 8))
                        e[j++] = (uint32_t)(u | v << 4 | w << 8 | (u + PX * (v + T * w)) << 12);
    }
};

namespace {  // one copy per translation unit (the JFA's own unit and the batch kernels' unit)
template <int K, int PX>
struct Shell {
    static __constant__ const ShellTable<K, PX> tab;
};
template <int K, int PX>
__constant__ const ShellTable<K, PX> Shell<K, PX>::tab = ShellTable<K, PX>();
}  // namespace

// Near-pass key for n <= 128 (every coordinate below 128): the staged pair is (2S, W) with W = |S|^2 - 510 sum(S)
// + 2^18 (in [2^18 - 3 * 127 * 383, 2^18]), and with q = 255 - p per byte one byte dot product gives
// hi = (2S).q + W = 510 sum(S) - 2 S.p + |S|^2 - 510 sum(S) + 2^18 = D^2 - |p|^2 + 2^18, the byte-dot key's high
// word, so a candidate costs the dot product and the min.  The low word 2S orders seeds as S does (no byte of S
// carries when doubled); the seed is low >> 1.  A missing seed (0xFFFFFFFF) gets the bits 0x7F000000 in W, so
// its hi stays at or above them (below 2^32: W < 0x7F000000 + 2^20, the dot product below 2^18) and it loses.
__device__ __forceinline__ uint2 jfa_pair_small(uint32_t s)
{
    const uint32_t sum = __builtin_amdgcn_udot4(s, 0x00010101u, 0u, false);
    const uint32_t sq = __builtin_amdgcn_udot4(s, s, (s & 0x7F000000u) | 0x40000u, false);
    return make_uint2(s << 1, (uint32_t)__mul24((int)sum, -510) + sq);
}

__device__ __forceinline__ double jfa_key_small(uint32_t q, uint2 e)
{
    return __builtin_bit_cast(double, ((uint64_t)__builtin_amdgcn_udot4(e.x, q, e.y, false) << 32) | (uint64_t)e.x);
}

// One pass with step K in {1, 2}: eight bricks (an 8^3 block) per workgroup of 512 threads, staged with a
// K-voxel halo in LDS.  FINAL writes the caller's outputs.  SMALL (n <= 128, with PAIRS): the two-instruction
// key above.
template <int K, bool PAIRS, bool FINAL, bool SMALL = false>
__device__ __forceinline__ void jfa_near_body(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int n,
                                              int logn, int32_t *__restrict__ dist2, float *__restrict__ sdf, float h,
                                              float beta, uint32_t blk_id, uint32_t nblk, int neg2)
{
    static_assert(!SMALL || PAIRS, "the small-grid key stages pairs");
    constexpr int T = 8 + 2 * K;
    // Entry (u, v, w) of the tile sits at u + PX (v + T w).  The 16 lanes that one LDS read serves together
    // (a 4 x 4 row block of a brick) reach entries u + PX v, u, v < 4: with 8-byte pairs they fall on distinct
    // banks for a row pitch PX of 12 entries, not for T = 10 (the step-1 tile), which is padded to 12.
    constexpr int PX = PAIRS && T == 10 ? 12 : T;
    // PAIRS: each entry staged as a pair ((s, w(s)), or (2s, W) for SMALL); else the seed alone (w formed per
    // candidate)
    __shared__ uint32_t tile[(PAIRS ? 2 : 1) * PX * T * T];
    uint2 *tile2 = reinterpret_cast<uint2 *>(tile);
    // n is a power of two: block and brick coordinates are bit fields (shifts and masks, no divisions)
    const int logB = logn - 2, logTB = logn - 3, TB = 1 << logTB;  // 8^3 blocks per axis
    const int blk = (int)xcd_remap(blk_id, nblk);
    const int tx0 = (blk & (TB - 1)) * 8, ty0 = ((blk >> logTB) & (TB - 1)) * 8, tz0 = (blk >> (2 * logTB)) * 8;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lx = (wave & 1) * 4 + (lane & 3), ly = ((wave >> 1) & 1) * 4 + ((lane >> 2) & 3),
              lz = (wave >> 2) * 4 + (lane >> 4);
    const int c = (lx + K) + PX * ((ly + K) + T * (lz + K));
    const auto stage = [&](int i, uint32_t v) {
        if (SMALL) tile2[i] = jfa_pair_small(v);
        else if (PAIRS) tile2[i] = make_uint2(v, jfa_w(v));
        else tile[i] = v;
    };
    // All reads first, then all LDS writes, so a wavefront has every staging read in flight at once.  The block's
    // eight bricks: wavefront w reads brick w, each lane its own voxel (one coalesced 256-byte read per
    // wavefront).  The K-voxel shell around them (ShellTable), voxel by voxel, out-of-grid entries empty.
    constexpr int NH = ShellTable<K, PX>::N, R = (NH + 511) / 512;
    const int b0 = ((tx0 + lx) >> 2) | (((ty0 + ly) >> 2) << logB) | (((tz0 + lz) >> 2) << (2 * logB));
    const uint32_t inner = (uint32_t)src[(b0 << 6) | lane];
    uint32_t val[R];
    int at[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = (int)threadIdx.x + 512 * r;
        val[r] = kNoSeed;
        at[r] = -1;
        if (r < R - 1 || j < NH) {
            const uint32_t e = Shell<K, PX>::tab.e[j];
            const int x = tx0 - K + (int)(e & 15u), y = ty0 - K + (int)((e >> 4) & 15u),
                      z = tz0 - K + (int)((e >> 8) & 15u);
            at[r] = (int)(e >> 12);
            if ((unsigned)x < (unsigned)n && (unsigned)y < (unsigned)n && (unsigned)z < (unsigned)n) {
                const int b = (x >> 2) | ((y >> 2) << logB) | ((z >> 2) << (2 * logB));
                val[r] = (uint32_t)src[(b << 6) | (x & 3) | ((y & 3) << 2) | ((z & 3) << 4)];
            }
        }
    }
    stage(c, inner);
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (at[r] >= 0) stage(at[r], val[r]);
    __syncthreads();
    const int x = tx0 + lx, y = ty0 + ly, z = tz0 + lz;
    const JfaPos P = jfa_pos(x, y, z, neg2);
    const uint32_t q = 0x00FFFFFFu - P.p;  // 255 - p per byte
    double best = __builtin_bit_cast(double, 0x7FE0000000000000ull);
#pragma unroll
    for (int o = 0; o < 27; ++o) {
        const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
        const int e = c + K * (ox + PX * (oy + T * oz));
        best = __builtin_fmin(best, SMALL   ? jfa_key_small(q, tile2[e])
                                    : PAIRS ? jfa_keyd_w(P, tile2[e].x, tile2[e].y)
                                            : jfa_keyd(P, tile[e]));
    }
    // the seed of the best key (kNoSeed if none): its low word, halved for the small-grid key
    const uint32_t low = (uint32_t)__builtin_bit_cast(uint64_t, best);
    const uint32_t s = SMALL ? (key_hi(best) >= 0x7F000000u ? kNoSeed : low >> 1) : key_seed<true>(P, best);
    if (!FINAL) {
        dst[(b0 << 6) | lane] = (int32_t)s;
    } else {
        const int idx = x | (y << logn) | (z << (2 * logn));  // n <= 256: below 2^24
        if (s == kNoSeed) {
            dst[idx] = -1;
            dist2[idx] = INT32_MAX;
            sdf[idx] = __builtin_inff();
        } else {
            const int d2 = (int)keyd_d2(P, best);
            dst[idx] = unpack_linear(s, logn);
            dist2[idx] = d2;
            sdf[idx] = rn_sub(rn_mul(h, rn_sqrt((float)d2)), beta);
        }
    }
}

}  // namespace rtsdf
