// Rebuilding the hierarchy on the device (linear BVH).
//
// Refitting keeps the topology built at creation; when geometry moves far
// from where it was, boxes overlap more and more and tracing slows (20x after
// 48 frames of continuous motion on the moving-scene workload).  A rebuild
// from scratch on the host costs seconds for a million triangles; the kernels here build
// a new hierarchy on the device every frame instead, in the node format the
// tracer reads, over the scene's references (split pieces of large triangles
// keep their subdivision paths, so a rebuild re-derives each piece's box from
// the current vertices):
//
//   1. reference boxes from the current vertices, and the bounds of their
//      centres (atomic min/max on order-preserving integer images of floats);
//   2. 30-bit Morton codes of the centres in those bounds;
//   3. radix sort of (code, reference) pairs (below: least-significant digit
//      first, 8-bit digits, stable); equal codes keep the reference order,
//      so (code, position) keys are distinct;
//   4. the binary radix tree over the sorted keys (Karras, "Maximizing
//      Parallelism in the Construction of BVHs, Octrees, and k-d Trees",
//      HPG 2012): internal node i finds its key range from the common-prefix
//      lengths of its neighbours and splits where the prefix changes; one
//      reference per leaf; node 0 is the root;
//   5. boxes bottom-up: one thread per leaf climbs, the second thread to
//      arrive at a node writes its two child boxes and goes on.  A node's
//      leaves are a contiguous run of the sorted order, so the climb runs in
//      two passes: workgroups of kChunk threads own kChunk consecutive leaves
//      and finish every node whose run lies inside their chunk (counters and
//      boxes in LDS, workgroup-scope ordering); the few nodes whose run
//      crosses a chunk border (about 10 per chunk) are finished by a second
//      pass that climbs from a queue of the children the first pass
//      completed, with device-scope ordering.  Ordering across workgroups
//      costs an L2 write-back and invalidate per fence on this GPU (the eight
//      L2 caches are not coherent with each other within a kernel): 7.0 ms
//      when every leaf's climb paid it, 0.1 ms for the crossing nodes alone;
//   6. the triangle records and affine maps in leaf order.
// The tree depth is at most 30 + ceil(log2 n) (each level consumes one bit of
// the distinct 30-bit code + position key), which sizes the traversal stack.
// A refit of a rebuilt scene reuses steps 1 and 5 on the same tree.
//
// Every step is a kernel launch with a launch shape fixed by the reference
// count (no host synchronisation, allocation or memset), so a rebuild can be
// captured in a graph.
//
// The closest hit a ray finds is the minimum over all references of a value
// computed from the reference alone, so a rebuilt scene traces like the
// original one; only where two candidates lie within float rounding of each
// other (a ray through an edge) can the order of the tests, which follows
// the hierarchy, pick the other one.
#include "common.hpp"

namespace rtsdf {

// float <-> unsigned keeping the order of all finite values
__device__ __forceinline__ unsigned ordered_bits(float f)
{
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(unsigned u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// step 1: reference boxes (padded) and centre bounds; bounds[0..2] min, [3..5] max (ordered integers).  A
// grid-stride loop over a bounded number of workgroups, the bounds reduced in registers, across the wavefront
// and across the workgroup, then one atomic per workgroup and bound (one per wavefront contended on the same
// six words: 1.1 ms for a million references).
constexpr int kRefBoxBlocks = 1024;

__global__ void __launch_bounds__(256) lbvh_ref_boxes(const float *__restrict__ v, const int32_t *__restrict__ f,
                                                      const int32_t *__restrict__ ref_tri,
                                                      const int32_t *__restrict__ ref_path, int nref, float pad,
                                                      float *__restrict__ box, unsigned *__restrict__ bounds)
{
    __shared__ unsigned part[6][256 / kWave];
    unsigned mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0u, 0u, 0u};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nref; i += gridDim.x * blockDim.x) {
        const int t = ref_tri[i];
        float a[3], b[3], cc[3];
        for (int k = 0; k < 3; ++k) {
            a[k] = v[3 * f[3 * t] + k];
            b[k] = v[3 * f[3 * t + 1] + k];
            cc[k] = v[3 * f[3 * t + 2] + k];
        }
        follow_path(a, b, cc, ref_path[i]);
        for (int k = 0; k < 3; ++k) {
            const float lo = nextafterf(fminf(a[k], fminf(b[k], cc[k])) - pad, -__builtin_inff());
            const float hi = nextafterf(fmaxf(a[k], fmaxf(b[k], cc[k])) + pad, __builtin_inff());
            box[6 * i + k] = lo;
            box[6 * i + 3 + k] = hi;
            const unsigned c = ordered_bits(0.5f * (lo + hi));
            mn[k] = min(mn[k], c);
            mx[k] = max(mx[k], c);
        }
    }
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int k = 0; k < 3; ++k) {
        for (int off = 32; off > 0; off >>= 1) {
            mn[k] = min(mn[k], (unsigned)__shfl_xor((int)mn[k], off));
            mx[k] = max(mx[k], (unsigned)__shfl_xor((int)mx[k], off));
        }
        if (lane == 0) {
            part[k][wave] = mn[k];
            part[3 + k][wave] = mx[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        unsigned r = part[k][0];
        for (int w = 1; w < (int)blockDim.x / kWave; ++w) r = k < 3 ? min(r, part[k][w]) : max(r, part[k][w]);
        if (k < 3) atomicMin(&bounds[k], r);
        else atomicMax(&bounds[k], r);
    }
}

__device__ __forceinline__ uint32_t morton30(float x, float y, float z)
{
    const uint32_t X = (uint32_t)fminf(fmaxf(x * 1024.0f, 0.0f), 1023.0f);
    const uint32_t Y = (uint32_t)fminf(fmaxf(y * 1024.0f, 0.0f), 1023.0f);
    const uint32_t Z = (uint32_t)fminf(fmaxf(z * 1024.0f, 0.0f), 1023.0f);
    return morton3(X, Y, Z);
}

// step 2
__global__ void __launch_bounds__(256) lbvh_codes(const float *__restrict__ box, int nref,
                                                  const unsigned *__restrict__ bounds, uint32_t *__restrict__ code)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nref) return;
    float q[3];
    for (int k = 0; k < 3; ++k) {
        const float lo = from_ordered(bounds[k]), hi = from_ordered(bounds[3 + k]);
        const float ext = hi - lo;
        const float c = 0.5f * (box[6 * i + k] + box[6 * i + 3 + k]);
        q[k] = ext > 0.0f ? (c - lo) / ext : 0.5f;
    }
    code[i] = morton30(q[0], q[1], q[2]);
}

// ---------------------------------------------------------------- sort ----
//
// Least-significant-digit radix sort of (key, value) pairs, 8-bit digits,
// stable.  Each pass over the n pairs:
//   rsort_count    tile t (kSortTile consecutive pairs, 4 wavefronts of 1024
//                  each) counts its digits; counts go to hist[digit][tile];
//   rsort_scan     one workgroup: exclusive prefix of hist in that order, so
//                  hist[d][t] becomes the output position of the first pair
//                  of tile t with digit d;
//   rsort_scatter  tile t counts again per wavefront, turns the counts into
//                  per-wavefront starting positions for every digit, and each
//                  wavefront walks its 1024 pairs in order, 64 at a time: the
//                  lanes holding one digit find each other with eight ballots
//                  (one per digit bit), a lane's rank among them is the count
//                  of lower lanes, and the group's lowest lane advances the
//                  digit's position.  Pairs with equal digits therefore keep
//                  their order: within a wavefront by the walk, across
//                  wavefronts and tiles by the prefix.
// The first pass takes the values as the identity (value = input position).
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                                    // pairs per lane per tile
constexpr int kSortChunk = kWave * kSortItems;                    // pairs per wavefront
constexpr int kSortTile = kSortThreads * kSortItems;              // pairs per tile
constexpr int kSortBins = 256;

__global__ void __launch_bounds__(kSortThreads) rsort_count(const uint32_t *__restrict__ keys, int n, int shift,
                                                            uint32_t *__restrict__ hist, int ntiles)
{
    __shared__ uint32_t h[kSortThreads / kWave][kSortBins];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int b = lane; b < kSortBins; b += kWave) h[wave][b] = 0u;
    __syncthreads();
    const int base = blockIdx.x * kSortTile + wave * kSortChunk;
#pragma unroll 4
    for (int i = 0; i < kSortItems; ++i) {
        const int idx = base + i * kWave + lane;
        if (idx < n) atomicAdd(&h[wave][(keys[idx] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    const int d = threadIdx.x;  // kSortThreads == kSortBins
    hist[d * ntiles + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// exclusive prefix of hist[0 .. total) in place (one workgroup of 1024 lanes): rounds of 4096 consecutive
// counts, four per lane (one 16-byte load and store), lane sums scanned within each wavefront by shuffles and
// across the 16 wavefronts through LDS; the running total of earlier rounds is carried along
__global__ void __launch_bounds__(1024) rsort_scan(uint32_t *__restrict__ hist, int total)
{
    __shared__ uint32_t wsum[1024 / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), wave = t >> 6;
    uint32_t carry = 0;
    for (int base = 0; base < total; base += 4 * 1024) {
        const int i0 = base + 4 * t;
        uint32_t v[4] = {0u, 0u, 0u, 0u};
        if (i0 + 3 < total) {
            const uint4 q = *reinterpret_cast<const uint4 *>(hist + i0);
            v[0] = q.x;
            v[1] = q.y;
            v[2] = q.z;
            v[3] = q.w;
        } else {
            for (int k = 0; k < 4; ++k)
                if (i0 + k < total) v[k] = hist[i0 + k];
        }
        const uint32_t s = v[0] + v[1] + v[2] + v[3];
        uint32_t x = s;  // inclusive scan of the lane sums within the wavefront
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == kWave - 1) wsum[wave] = x;
        __syncthreads();
        uint32_t before = 0, round = 0;
        for (int k = 0; k < 1024 / kWave; ++k) {
            const uint32_t w = wsum[k];
            before += k < wave ? w : 0u;
            round += w;
        }
        uint32_t e = carry + before + x - s;  // exclusive prefix of the lane's first count
        uint32_t o[4];
        for (int k = 0; k < 4; ++k) {
            o[k] = e;
            e += v[k];
        }
        if (i0 + 3 < total) {
            *reinterpret_cast<uint4 *>(hist + i0) = make_uint4(o[0], o[1], o[2], o[3]);
        } else {
            for (int k = 0; k < 4; ++k)
                if (i0 + k < total) hist[i0 + k] = o[k];
        }
        carry += round;
        __syncthreads();  // wsum is rewritten next round
    }
}

template <bool IDENTITY>
__global__ void __launch_bounds__(kSortThreads) rsort_scatter(const uint32_t *__restrict__ kin,
                                                              const int32_t *__restrict__ vin,
                                                              uint32_t *__restrict__ kout, int32_t *__restrict__ vout,
                                                              int n, int shift, const uint32_t *__restrict__ offs,
                                                              int ntiles)
{
    __shared__ uint32_t pos[kSortThreads / kWave][kSortBins];  // per wavefront: counts, then next positions
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int b = lane; b < kSortBins; b += kWave) pos[wave][b] = 0u;
    __syncthreads();
    const int base = blockIdx.x * kSortTile + wave * kSortChunk;
    uint32_t key[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int idx = base + i * kWave + lane;
        key[i] = idx < n ? kin[idx] : 0u;
        if (idx < n) atomicAdd(&pos[wave][(key[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;  // one digit per lane
        uint32_t p = offs[d * ntiles + blockIdx.x];
        const uint32_t c0 = pos[0][d], c1 = pos[1][d], c2 = pos[2][d];
        pos[0][d] = p;
        p += c0;
        pos[1][d] = p;
        p += c1;
        pos[2][d] = p;
        pos[3][d] = p + c2;
    }
    __syncthreads();
    const uint64_t lower = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int idx = base + i * kWave + lane;
        const bool valid = idx < n;
        const uint32_t d = (key[i] >> shift) & 0xFFu;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lower);
        const uint32_t at = pos[wave][d];
        if (valid) {
            kout[at + rank] = key[i];
            vout[at + rank] = IDENTITY ? idx : vin[idx];
            if (rank == 0) pos[wave][d] = at + (uint32_t)__popcll(peers);
        }
        // the next group of 64 reads the advanced positions
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

static int rsort_tiles(int n) { return (n + kSortTile - 1) / kSortTile; }
static size_t rsort_hist_words(int n) { return (size_t)kSortBins * rsort_tiles(n); }

// Sort n pairs with `bits`-bit keys (1 <= bits <= 32) starting in (k0, v0) -- with IDENTITY_IN the values
// are taken as 0 .. n - 1 and v0 is not read; the result lands in (k0, v0) after an even number of passes and
// in (k1, v1) after an odd one, returned through out_k / out_v.
static int rsort_run(uint32_t *k0, int32_t *v0, uint32_t *k1, int32_t *v1, uint32_t *hist, int n, int bits,
                     bool identity_in, uint32_t **out_k, int32_t **out_v, hipStream_t s)
{
    const int ntiles = rsort_tiles(n);
    uint32_t *ka = k0, *kb = k1;
    int32_t *va = v0, *vb = v1;
    for (int shift = 0, pass = 0; shift < bits; shift += 8, ++pass) {
        rsort_count<<<dim3(ntiles), dim3(kSortThreads), 0, s>>>(ka, n, shift, hist, ntiles);
        RTSDF_CHECK_LAUNCH();
        rsort_scan<<<dim3(1), dim3(1024), 0, s>>>(hist, kSortBins * ntiles);
        RTSDF_CHECK_LAUNCH();
        if (pass == 0 && identity_in)
            rsort_scatter<true><<<dim3(ntiles), dim3(kSortThreads), 0, s>>>(ka, nullptr, kb, vb, n, shift, hist, ntiles);
        else
            rsort_scatter<false><<<dim3(ntiles), dim3(kSortThreads), 0, s>>>(ka, va, kb, vb, n, shift, hist, ntiles);
        RTSDF_CHECK_LAUNCH();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    *out_k = ka;
    *out_v = va;
    return RTSDF_OK;
}

// common-prefix length of the keys (code, position) at positions i and j; -1 outside [0, n)
__device__ __forceinline__ int lbvh_delta(const uint32_t *__restrict__ code, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const uint32_t a = code[i], b = code[j];
    if (a != b) return __clz(a ^ b) - 2;  // 30-bit codes in 32-bit words
    return 30 + __clz((uint32_t)i ^ (uint32_t)j);
}

// step 4: internal node i of the radix tree over n sorted keys.  A child whose leaf run holds at most
// max_leaf references is referenced as one leaf of that run (the run is consecutive in the sorted order); the
// internal nodes below it stay in the array, unreferenced, so the bottom-up box passes climb through them as
// before (their parent pointers follow the full radix tree).
__global__ void __launch_bounds__(256) lbvh_internal(const uint32_t *__restrict__ code, int n, int max_leaf,
                                                     BvhNode *nodes, int32_t *__restrict__ leaf_parent,
                                                     int2 *__restrict__ range)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = lbvh_delta(code, n, i, i + 1) - lbvh_delta(code, n, i, i - 1) >= 0 ? 1 : -1;
    const int dmin = lbvh_delta(code, n, i, i - d);
    int lmax = 2;
    while (lbvh_delta(code, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (lbvh_delta(code, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = lbvh_delta(code, n, i, j);
    int s = 0;
    for (int t = (l + 1) >> 1;; t = (t + 1) >> 1) {
        if (lbvh_delta(code, n, i, i + (s + t) * d) > dnode) s += t;
        if (t == 1) break;
    }
    const int gamma = i + s * d + min(d, 0);
    const int lo = min(i, j), hi = max(i, j);
    range[i] = make_int2(lo, hi);
    const bool left_leaf = lo == gamma, right_leaf = hi == gamma + 1;
    BvhNode &nd = nodes[i];
    const int nl = gamma - lo + 1, nr = hi - gamma;  // references under each child
    const int c0 = nl <= max_leaf ? leaf_code(lo, nl) : gamma;
    const int c1 = nr <= max_leaf ? leaf_code(gamma + 1, nr) : gamma + 1;
    nd.meta.x = c0;
    nd.meta.y = c1;
    nd.meta.w = 0;
    if (left_leaf) leaf_parent[gamma] = i;
    else nodes[gamma].meta.z = i;
    if (right_leaf) leaf_parent[gamma + 1] = i;
    else nodes[gamma + 1].meta.z = i;
    if (i == 0) nd.meta.z = -1;
}

// step 5, first pass.  Workgroup b owns leaves [c0, c1) = [b kChunk, min(n, (b + 1) kChunk)); an internal
// node whose leaf run [lo, hi] lies inside the chunk has its index in [c0, c1) (a node's index is one end of
// its run), which addresses its counter and box in LDS.  A climb that reaches a node whose run crosses the
// chunk border stops and queues the child it finished.
constexpr int kChunk = 1024;
constexpr int kMaxRebuildLeaf = 8;  // references per leaf of a rebuilt hierarchy at most

__device__ __forceinline__ void leaf_ref_box(const float *__restrict__ box, const int32_t *__restrict__ ids, int k,
                                             float lo[3], float hi[3])
{
    const float *b = box + 6 * ids[k];
    for (int a = 0; a < 3; ++a) {
        lo[a] = b[a];
        hi[a] = b[3 + a];
    }
}

// the box of a leaf child (code c): the union of its references' boxes
__device__ __forceinline__ void leaf_box(const float *__restrict__ box, const int32_t *__restrict__ ids, int c,
                                         float lo[3], float hi[3])
{
    const int first = leaf_first(c), cnt = leaf_count(c);
    leaf_ref_box(box, ids, first, lo, hi);
    for (int k = first + 1; k < first + cnt; ++k) {
        float l[3], h[3];
        leaf_ref_box(box, ids, k, l, h);
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], l[a]);
            hi[a] = fmaxf(hi[a], h[a]);
        }
    }
}

__global__ void __launch_bounds__(kChunk) lbvh_boxes_local(BvhNode *nodes, const int32_t *__restrict__ leaf_parent,
                                                          const int2 *__restrict__ range,
                                                          const int32_t *__restrict__ ids,
                                                          const float *__restrict__ box, int n,
                                                          int32_t *__restrict__ counter, int32_t *__restrict__ queue,
                                                          int32_t *qcount)
{
    __shared__ int cnt[kChunk];
    __shared__ float lbox[6][kChunk];
    const int c0 = blockIdx.x * kChunk, c1 = min(n, c0 + kChunk);
    const int t = threadIdx.x, k = c0 + t;
    cnt[t] = 0;
    if (k < n - 1) counter[k] = 0;  // the second pass's counters, one per internal node
    __syncthreads();
    if (k >= n) return;
    float lo[3], hi[3];
    leaf_ref_box(box, ids, k, lo, hi);
    int child = leaf_code(k, 1);
    int node = leaf_parent[k];
    while (node >= 0) {
        const int2 r = range[node];
        if (r.x < c0 || r.y >= c1) {
            queue[atomicAdd(qcount, 1)] = child;
            return;
        }
        // publish the finished child's box (an internal child's: in LDS), then arrive
        if (child >= 0)
            for (int a = 0; a < 3; ++a) {
                lbox[a][child - c0] = lo[a];
                lbox[3 + a][child - c0] = hi[a];
            }
        if (__hip_atomic_fetch_add(&cnt[node - c0], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == 0)
            return;  // the sibling's thread is still climbing; it goes on from here
        BvhNode *nd = &nodes[node];
        const int c[2] = {nd->meta.x, nd->meta.y};
        const float own_lo[3] = {lo[0], lo[1], lo[2]}, own_hi[3] = {hi[0], hi[1], hi[2]};
        for (int s = 0; s < 2; ++s) {
            float l[3], h[3];
            if (c[s] == child) {
                for (int a = 0; a < 3; ++a) l[a] = own_lo[a], h[a] = own_hi[a];
            } else if (c[s] < 0) {
                leaf_box(box, ids, c[s], l, h);
            } else {
                for (int a = 0; a < 3; ++a) {
                    l[a] = lbox[a][c[s] - c0];
                    h[a] = lbox[3 + a][c[s] - c0];
                }
            }
            set_slot(nd, s, l, h);
            if (c[s] != child)
                for (int a = 0; a < 3; ++a) {
                    lo[a] = fminf(lo[a], l[a]);
                    hi[a] = fmaxf(hi[a], h[a]);
                }
        }
        child = node;
        node = nd->meta.z;
    }
}

// step 5, second pass: threads climb from the queued children through the nodes that cross chunk borders
// (their counters were cleared by the first pass); the arrival counter orders the boxes at device scope
__global__ void __launch_bounds__(256) lbvh_boxes_top(BvhNode *nodes, const int32_t *__restrict__ leaf_parent,
                                                      const int32_t *__restrict__ ids, const float *__restrict__ box,
                                                      int32_t *counter, const int32_t *__restrict__ queue,
                                                      const int32_t *__restrict__ qcount)
{
    const int nq = *qcount;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        const int first = queue[q];
        int node = first < 0 ? leaf_parent[leaf_first(first)] : nodes[first].meta.z;
        while (node >= 0) {
            if (__hip_atomic_fetch_add(&counter[node], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 0)
                break;  // the other child is not done; its thread goes on
            BvhNode *nd = &nodes[node];
            const int c[2] = {nd->meta.x, nd->meta.y};
            for (int s = 0; s < 2; ++s) {
                float lo[3], hi[3];
                if (c[s] < 0) {
                    leaf_box(box, ids, c[s], lo, hi);
                } else {
                    const BvhNode *ch = &nodes[c[s]];
                    float l2[3], h2[3];
                    get_slot(ch, 0, lo, hi);
                    get_slot(ch, 1, l2, h2);
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = fminf(lo[a], l2[a]);
                        hi[a] = fmaxf(hi[a], h2[a]);
                    }
                }
                set_slot(nd, s, lo, hi);
            }
            node = nd->meta.z;
        }
    }
}

// step 6: triangle records in leaf order (whole triangle, global id, the piece's path)
__global__ void __launch_bounds__(256) lbvh_records(const float *__restrict__ v, const int32_t *__restrict__ f,
                                                    const int32_t *__restrict__ ref_tri,
                                                    const int32_t *__restrict__ ref_path,
                                                    const int32_t *__restrict__ ids, int n, float4 *__restrict__ tris,
                                                    int4 *__restrict__ leaf_faces)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int r = ids[k], t = ref_tri[r], path = ref_path[r];
    const int vid[3] = {f[3 * t], f[3 * t + 1], f[3 * t + 2]};
    for (int q = 0; q < 3; ++q) {
        const float *p = v + 3 * vid[q];
        tris[3 * k + q] = make_float4(p[0], p[1], p[2], q == 0 ? __int_as_float(t) : (q == 1 ? __int_as_float(path)
                                                                                           : 0.f));
    }
    leaf_faces[k] = make_int4(vid[0], vid[1], vid[2], t);
}

__global__ void lbvh_init_bounds(unsigned *bounds, int32_t *qcount)
{
    const int k = threadIdx.x;
    if (k < 3) bounds[k] = 0xffffffffu;
    else if (k < 6) bounds[k] = 0u;
    else if (k == 6) *qcount = 0;
}

}  // namespace rtsdf

// device buffers of a rebuildable scene (allocated by rtsdf_scene_enable_rebuild)
struct rtsdf_lbvh {
    int32_t *ref_tri = nullptr, *ref_path = nullptr;  // [nref] the references, in creation order
    float *box = nullptr;                              // [nref][6]
    unsigned *bounds = nullptr;                        // [6]
    uint32_t *code = nullptr, *code_sorted = nullptr;  // [nref]
    int32_t *id = nullptr, *id_sorted = nullptr;       // [nref]
    int32_t *leaf_parent = nullptr;                    // [nref]
    int2 *range = nullptr;                             // [nref - 1] leaf run of each internal node
    int32_t *queue = nullptr, *qcount = nullptr;       // [nref], [1] children handed to the top pass
    uint32_t *hist = nullptr;                          // radix-sort digit counts: [256][tiles]
};

static void lbvh_free(rtsdf_lbvh *L)
{
    if (!L) return;
    for (void *p : {(void *)L->ref_tri, (void *)L->ref_path, (void *)L->box, (void *)L->bounds, (void *)L->code,
                    (void *)L->code_sorted, (void *)L->id, (void *)L->id_sorted, (void *)L->leaf_parent, (void *)L->range, (void *)L->queue,
                    (void *)L->qcount, (void *)L->hist})
        (void)hipFree(p);
    delete L;
}

namespace rtsdf {

// steps 1 and 5 on the current tree (refit), or 1-6 (rebuild)
static int lbvh_run(rtsdf_scene *sc, bool rebuild, hipStream_t s)
{
    rtsdf_lbvh *L = sc->lbvh;
    const int n = sc->nref;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    lbvh_init_bounds<<<dim3(1), dim3(64), 0, s>>>(L->bounds, L->qcount);
    RTSDF_CHECK_LAUNCH();
    lbvh_ref_boxes<<<dim3(std::min(blocks, (unsigned)kRefBoxBlocks)), dim3(256), 0, s>>>(
        sc->vertices, sc->faces, L->ref_tri, L->ref_path, n, sc->pad, L->box, L->bounds);
    RTSDF_CHECK_LAUNCH();
    if (rebuild) {
        lbvh_codes<<<dim3(blocks), dim3(256), 0, s>>>(L->box, n, L->bounds, L->code_sorted);
        RTSDF_CHECK_LAUNCH();
        // four 8-bit passes from code_sorted: the sorted pairs land back in (code_sorted, id_sorted)
        uint32_t *ok_ = nullptr;
        int32_t *ov_ = nullptr;
        const int rc = rsort_run(L->code_sorted, L->id_sorted, L->code, L->id, L->hist, n, 30, true, &ok_, &ov_, s);
        if (rc != RTSDF_OK) return rc;
        if (ok_ != L->code_sorted || ov_ != L->id_sorted) return RTSDF_EHIP;  // (an even number of passes)
        lbvh_internal<<<dim3((unsigned)((n - 1 + 255) / 256)), dim3(256), 0, s>>>(L->code_sorted, n, sc->max_leaf,
                                                                                  sc->nodes, L->leaf_parent, L->range);
        RTSDF_CHECK_LAUNCH();
        lbvh_records<<<dim3(blocks), dim3(256), 0, s>>>(sc->vertices, sc->faces, L->ref_tri, L->ref_path,
                                                         L->id_sorted, n, sc->tris, sc->leaf_faces);
        RTSDF_CHECK_LAUNCH();
    } else {
        refit_tris<<<dim3(blocks), dim3(256), 0, s>>>(sc->vertices, sc->leaf_faces, sc->tris, n);
        RTSDF_CHECK_LAUNCH();
    }
    tri_maps<<<dim3(blocks), dim3(256), 0, s>>>(sc->tris, sc->tmap, n);
    RTSDF_CHECK_LAUNCH();
    lbvh_boxes_local<<<dim3((unsigned)((n + kChunk - 1) / kChunk)), dim3(kChunk), 0, s>>>(
        sc->nodes, L->leaf_parent, L->range, L->id_sorted, L->box, n, sc->refit_counter, L->queue, L->qcount);
    RTSDF_CHECK_LAUNCH();
    lbvh_boxes_top<<<dim3(64), dim3(256), 0, s>>>(sc->nodes, L->leaf_parent, L->id_sorted, L->box,
                                                   sc->refit_counter, L->queue, L->qcount);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

}  // namespace rtsdf

extern "C" int rtsdf_scene_enable_rebuild(rtsdf_scene *sc, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!sc || sc->ninst > 0) return RTSDF_EINVAL;
    if (sc->lbvh) return RTSDF_OK;
    const int n = sc->nref;
    if (n < 2) return RTSDF_EINVAL;  // a one-reference scene has nothing to rebuild
    int bits = 0;
    while ((1ll << bits) < (int64_t)n) ++bits;
    const int depth = 30 + bits + 1;  // leaves included
    if (depth + 1 > 64) return RTSDF_EINVAL;
    hipStream_t s = as_stream(stream);
    // the references in leaf order now; their (triangle, path) identities are what every rebuild sorts
    std::vector<float4> htri((size_t)3 * n);
    RTSDF_TRY(hipMemcpyAsync(htri.data(), sc->tris, sizeof(float4) * htri.size(), hipMemcpyDeviceToHost, s));
    RTSDF_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> rt(n), rp(n);
    for (int i = 0; i < n; ++i) {
        rt[i] = __builtin_bit_cast(int32_t, htri[3 * i].w);
        rp[i] = __builtin_bit_cast(int32_t, htri[3 * i + 1].w);
    }
    auto *L = new rtsdf_lbvh();
    int64_t bytes = 0;
    auto alloc = [&](void **p, size_t b) -> bool {
        if (hipMalloc(p, b ? b : 16) != hipSuccess) return false;
        bytes += (int64_t)b;
        return true;
    };
    BvhNode *nodes = nullptr;
    int32_t *counter = nullptr;
    bool ok = alloc((void **)&L->ref_tri, sizeof(int32_t) * n) && alloc((void **)&L->ref_path, sizeof(int32_t) * n) &&
              alloc((void **)&L->box, sizeof(float) * 6 * n) && alloc((void **)&L->bounds, sizeof(unsigned) * 6) &&
              alloc((void **)&L->code, sizeof(uint32_t) * n) && alloc((void **)&L->code_sorted, sizeof(uint32_t) * n) &&
              alloc((void **)&L->id, sizeof(int32_t) * n) && alloc((void **)&L->id_sorted, sizeof(int32_t) * n) &&
              alloc((void **)&L->leaf_parent, sizeof(int32_t) * n) && alloc((void **)&L->range, sizeof(int2) * n) &&
              alloc((void **)&L->queue, sizeof(int32_t) * n) && alloc((void **)&L->qcount, sizeof(int32_t)) &&
              alloc((void **)&nodes, sizeof(BvhNode) * (n - 1)) && alloc((void **)&counter, sizeof(int32_t) * (n - 1));
    ok = ok && alloc((void **)&L->hist, sizeof(uint32_t) * rsort_hist_words(n));
    ok = ok && hipMemcpyAsync(L->ref_tri, rt.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s) == hipSuccess &&
         hipMemcpyAsync(L->ref_path, rp.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s) == hipSuccess &&
         hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        lbvh_free(L);
        (void)hipFree(nodes);
        (void)hipFree(counter);
        return RTSDF_ENOMEM;
    }
    // the rebuilt tree replaces the creation hierarchy (and the refit tables and 4-wide copy that went with it)
    wide_free(sc);
    (void)hipFree(sc->nodes);
    (void)hipFree(sc->refit_counter);
    sc->nodes = nodes;
    sc->refit_counter = counter;
    sc->nnodes = n - 1;
    sc->nstart = 0;
    sc->max_depth = depth;
    sc->max_leaf = std::max(1, std::min(sc->leaf_size, kMaxRebuildLeaf));
    sc->bytes += bytes;
    sc->lbvh = L;
    return lbvh_run(sc, true, s);
}

extern "C" int rtsdf_scene_rebuild(rtsdf_scene *scene, const float *vertices, rtsdf_stream stream)
{
    using namespace rtsdf;
    if (!scene || !scene->lbvh || (scene->nv > 0 && !vertices)) return RTSDF_EINVAL;
    hipStream_t s = as_stream(stream);
    if (scene->nv > 0 && vertices != scene->vertices)
        RTSDF_TRY(hipMemcpyAsync(scene->vertices, vertices, sizeof(float) * 3 * scene->nv, hipMemcpyDeviceToDevice, s));
    return lbvh_run(scene, true, s);
}

extern "C" size_t rtsdf_sort_pairs_workspace_size(int32_t n)
{
    using namespace rtsdf;
    if (n <= 0) return 0;
    return (size_t)n * (sizeof(uint32_t) + sizeof(int32_t)) + rsort_hist_words(n) * sizeof(uint32_t) + 256;
}

extern "C" int rtsdf_sort_pairs(uint32_t *keys, int32_t *values, int32_t n, int32_t bits, void *workspace,
                                rtsdf_stream stream)
{
    using namespace rtsdf;
    if (n < 0 || bits < 1 || bits > 32 || (n > 0 && (!keys || !values || !workspace))) return RTSDF_EINVAL;
    if (n <= 1) return RTSDF_OK;
    hipStream_t s = as_stream(stream);
    char *w = static_cast<char *>(workspace);
    uint32_t *k1 = reinterpret_cast<uint32_t *>(w);
    int32_t *v1 = reinterpret_cast<int32_t *>(w + (size_t)n * sizeof(uint32_t));
    // the scan moves 16-byte groups of counts: align them (the size has 256 bytes of slack)
    uint32_t *hist = reinterpret_cast<uint32_t *>((reinterpret_cast<uintptr_t>(w + (size_t)n * 8) + 15) &
                                                  ~(uintptr_t)15);
    uint32_t *ok_ = nullptr;
    int32_t *ov_ = nullptr;
    const int rc = rsort_run(keys, values, k1, v1, hist, n, bits, false, &ok_, &ov_, s);
    if (rc != RTSDF_OK) return rc;
    if (ok_ != keys) {  // an odd number of passes ends in the workspace
        RTSDF_TRY(hipMemcpyAsync(keys, ok_, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
        RTSDF_TRY(hipMemcpyAsync(values, ov_, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    return RTSDF_OK;
}
