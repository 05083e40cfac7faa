/*
 * rtsdf_oracle.c -- plain CPU oracle of the RTSDF SDF-generation path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library: it is written separately from the paper (Tan, Chua,
 * Koh, Bhojan, "RTSDF: Generating Signed Distance Fields in Real Time for
 * Soft Shadow Rendering", PG 2020 short paper) and from the published
 * algorithms it cites.
 *
 * Everything is straightforward loops in double precision, except where the
 * result itself is defined as a float32 value (the coarse SDF and the ray
 * origins/directions, which both sides must produce bit-identically); those
 * are computed with float operations, each rounded separately (this file is
 * compiled with -ffp-contract=off), and then widened to double.
 *
 * Sections of the paper referred to below:
 *   Sec. 2      two-level design: coarse SDF by jump flooding, fine SDF by
 *               ray tracing near surfaces, soft shadows from the fine SDF.
 *   Sec. 2.1    voxelization by orthographic projection along x, y and z with
 *               depth culling disabled; 3D jump flooding with occupied voxels
 *               as seeds; coarse distance minus a bias beta.
 *   Sec. 2.2    selection of fine texels with coarse distance within d; rays
 *               towards random points on a sphere; per-frame minimum hit
 *               distance r_t; Eq. (1) temporal update with decay alpha;
 *               sign from accumulated front/back hit counts.
 *   Sec. 2.3    sphere-traced soft shadows through the fine SDF.
 * Readings where the paper is silent are stated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Voxelization (Sec. 2.1).                                                  */
/*                                                                           */
/* The paper rasterizes the scene three times with an orthographic camera    */
/* looking along x, y and z, depth writes off, so every triangle produces    */
/* fragments, and marks the voxel under each fragment.  Reading used here    */
/* (the raster rule itself is not given): vertex coordinates are snapped to  */
/* 1/256 of a voxel; for each triangle and each axis, a voxel column is      */
/* covered when its centre lies inside or on the boundary of the projected   */
/* triangle; the covered voxel is the one containing the triangle's depth    */
/* at the column centre (floor of the exact rational depth), a depth exactly */
/* on the far face of the domain goes to the last layer, depths outside the  */
/* domain are dropped, and edge-on projections (zero area) are skipped.      */
/* ------------------------------------------------------------------------ */

static int64_t floor_div_i64(int64_t num, int64_t den) /* den > 0 */
{
    int64_t q = num / den;
    if ((num % den) != 0 && num < 0) q -= 1;
    return q;
}

/* twice the signed area of (u, v, p) in the projection plane */
static int64_t edge_fn(const int64_t u[2], const int64_t v[2], const int64_t p[2])
{
    return (v[0] - u[0]) * (p[1] - u[1]) - (v[1] - u[1]) * (p[0] - u[0]);
}

int oracle_voxelize(const float *v, int nv, const int *f, int nt,
                    const float lo[3], float h, int n, int *seeds)
{
    if (n <= 0 || h <= 0.0f) return ORC_EINVAL;
    const double side = (double)n * (double)h;
    int64_t *X = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)(nv > 0 ? nv : 1));
    if (!X) return ORC_EINVAL;
    for (int i = 0; i < nv; ++i) {
        for (int a = 0; a < 3; ++a) {
            double rel = (double)v[3 * i + a] - (double)lo[a];
            if (!(rel >= -side && rel <= 2.0 * side)) { free(X); return ORC_EINVAL; }
            X[3 * i + a] = (int64_t)rint(rel / (double)h * 256.0);
        }
    }
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k)
            if (f[3 * t + k] < 0 || f[3 * t + k] >= nv) { free(X); return ORC_EINVAL; }

    const size_t nvox = (size_t)n * n * n;
    for (size_t i = 0; i < nvox; ++i) seeds[i] = -1;

    for (int t = 0; t < nt; ++t) {
        for (int a = 0; a < 3; ++a) {
            const int e1 = (a + 1) % 3, e2 = (a + 2) % 3;
            int64_t P[3][2], Z[3];
            for (int k = 0; k < 3; ++k) {
                const int64_t *x = &X[3 * f[3 * t + k]];
                P[k][0] = x[e1];
                P[k][1] = x[e2];
                Z[k] = x[a];
            }
            int64_t area2 = edge_fn(P[0], P[1], P[2]);
            if (area2 == 0) continue;
            if (area2 < 0) { /* make the projected triangle counter-clockwise */
                int64_t tp[2] = {P[1][0], P[1][1]}, tz = Z[1];
                P[1][0] = P[2][0]; P[1][1] = P[2][1]; Z[1] = Z[2];
                P[2][0] = tp[0]; P[2][1] = tp[1]; Z[2] = tz;
                area2 = -area2;
            }
            /* columns whose centre can lie in the triangle's bounding box
               (one extra column on each side; the edge test decides) */
            int64_t mn[2], mx[2];
            for (int c = 0; c < 2; ++c) {
                mn[c] = P[0][c] < P[1][c] ? P[0][c] : P[1][c];
                if (P[2][c] < mn[c]) mn[c] = P[2][c];
                mx[c] = P[0][c] > P[1][c] ? P[0][c] : P[1][c];
                if (P[2][c] > mx[c]) mx[c] = P[2][c];
            }
            const int64_t ilo = floor_div_i64(mn[0], 256) - 1, ihi = floor_div_i64(mx[0], 256) + 1;
            const int64_t jlo = floor_div_i64(mn[1], 256) - 1, jhi = floor_div_i64(mx[1], 256) + 1;
            for (int j = 0; j < n; ++j) {
                if (j < jlo || j > jhi) continue;
                for (int i = 0; i < n; ++i) {
                    if (i < ilo || i > ihi) continue;
                    const int64_t c[2] = {256 * (int64_t)i + 128, 256 * (int64_t)j + 128};
                    const int64_t w0 = edge_fn(P[1], P[2], c);
                    const int64_t w1 = edge_fn(P[2], P[0], c);
                    const int64_t w2 = edge_fn(P[0], P[1], c);
                    if (w0 < 0 || w1 < 0 || w2 < 0) continue;
                    const int64_t num = w0 * Z[0] + w1 * Z[1] + w2 * Z[2];
                    const int64_t den = area2 * 256;
                    int64_t L;
                    if (num == (int64_t)n * den) L = n - 1;
                    else {
                        L = floor_div_i64(num, den);
                        if (L < 0 || L >= n) continue;
                    }
                    int q[3];
                    q[a] = (int)L;
                    q[e1] = i;
                    q[e2] = j;
                    const size_t idx = (size_t)q[0] + (size_t)n * ((size_t)q[1] + (size_t)n * q[2]);
                    seeds[idx] = (int)idx;
                }
            }
        }
    }
    free(X);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Jump flooding in 3D (Sec. 2.1; Rong & Tan's jump flooding extended to     */
/* three dimensions).  Each voxel keeps the nearest seed found so far; pass  */
/* k looks at the seeds of the 26 voxels at offsets k*(i, j, l),             */
/* i, j, l in {-1, 0, 1}, plus its own, for k = n/2, n/4, ..., 1.  Each pass */
/* reads only the previous pass's field.  Ties in squared distance go to    */
/* the seed with the lowest linear index.                                    */
/* ------------------------------------------------------------------------ */

static int64_t seed_d2(int n, int p, int s)
{
    const int px = p % n, py = (p / n) % n, pz = p / (n * n);
    const int sx = s % n, sy = (s / n) % n, sz = s / (n * n);
    const int64_t dx = px - sx, dy = py - sy, dz = pz - sz;
    return dx * dx + dy * dy + dz * dz;
}

void oracle_jfa_pass(int n, int k, const int *in, int *out)
{
    const int total = n * n * n;
#pragma omp parallel for schedule(static)
    for (int p = 0; p < total; ++p) {
        const int px = p % n, py = (p / n) % n, pz = p / (n * n);
        int best = -1;
        int64_t best_d2 = 0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    const int qx = px + k * ox, qy = py + k * oy, qz = pz + k * oz;
                    if (qx < 0 || qy < 0 || qz < 0 || qx >= n || qy >= n || qz >= n) continue;
                    const int s = in[qx + n * (qy + n * qz)];
                    if (s < 0) continue;
                    const int64_t d2 = seed_d2(n, p, s);
                    if (best < 0 || d2 < best_d2 || (d2 == best_d2 && s < best)) {
                        best = s;
                        best_d2 = d2;
                    }
                }
        out[p] = best;
    }
}

/* Jump flooding with an explicit pass schedule: the passes of oracle_jfa_pass
 * with steps steps[0], steps[1], ... in order, each reading the previous
 * pass's output (Sec. 2.1; the extra-pass variants JFA+1, JFA+2 and 1+JFA of
 * Rong and Tan are schedules of this form). */
int oracle_jfa_steps(int n, const int *seeds_in, const int *steps, int nsteps, int *seeds_out)
{
    if (n <= 0 || nsteps < 0) return ORC_EINVAL;
    const size_t total = (size_t)n * n * n;
    int *a = (int *)malloc(sizeof(int) * total), *b = (int *)malloc(sizeof(int) * total);
    if (!a || !b) { free(a); free(b); return ORC_EINVAL; }
    memcpy(a, seeds_in, sizeof(int) * total);
    for (int i = 0; i < nsteps; ++i) {
        if (steps[i] < 1) { free(a); free(b); return ORC_EINVAL; }
        oracle_jfa_pass(n, steps[i], a, b);
        int *t = a; a = b; b = t;
    }
    memcpy(seeds_out, a, sizeof(int) * total);
    free(a);
    free(b);
    return ORC_OK;
}

int oracle_jfa(int n, const int *seeds_in, int *seeds_out)
{
    if (n <= 0 || (n & (n - 1)) != 0) return ORC_EINVAL;
    const size_t total = (size_t)n * n * n;
    int *a = (int *)malloc(sizeof(int) * total), *b = (int *)malloc(sizeof(int) * total);
    if (!a || !b) { free(a); free(b); return ORC_EINVAL; }
    memcpy(a, seeds_in, sizeof(int) * total);
    for (int k = n / 2; k >= 1; k /= 2) {
        oracle_jfa_pass(n, k, a, b);
        int *t = a; a = b; b = t;
    }
    memcpy(seeds_out, a, sizeof(int) * total);
    free(a);
    free(b);
    return ORC_OK;
}

/* Coarse SDF (Sec. 2.1): distance to the nearest seed voxel minus the bias
 * beta.  Stored as float: c = h * sqrt(D^2) - beta with float operations
 * each rounded once (sqrt correctly rounded).  No seed at all: D^2 is
 * INT32_MAX and c = +inf. */
void oracle_coarse(int n, const int *seeds, float h, float beta, int *dist2, float *c)
{
    const int total = n * n * n;
    for (int p = 0; p < total; ++p) {
        if (seeds[p] < 0) {
            dist2[p] = INT32_MAX;
            c[p] = INFINITY;
            continue;
        }
        const int64_t d2 = seed_d2(n, p, seeds[p]);
        dist2[p] = (int)d2;
        volatile float r = sqrtf((float)d2);
        volatile float m = h * r;
        c[p] = m - beta;
    }
}

/* ------------------------------------------------------------------------ */
/* Selection (Sec. 2.2; Eq. (1) case split).  A fine texel is traced when    */
/* the coarse SDF at its coarse voxel is within d:  c <= d  with             */
/* c = h_c sqrt(D^2) - beta, i.e. D^2 <= K, K = floor(((d + beta)/h_c)^2)    */
/* evaluated exactly in integers.  The fine texel j reads the coarse voxel   */
/* containing its centre (j / r per axis with r = n_f / n_c).  The queue     */
/* lists the selected texels' linear indices in ascending Morton order of    */
/* their fine coordinates (bit b of x, y, z goes to bit 3b, 3b+1, 3b+2).     */
/* ------------------------------------------------------------------------ */

int oracle_select_threshold(float hc, float beta, float d)
{
    const double q = ((double)d + (double)beta) / (double)hc;
    if (q < 0) return -1;
    const double k = floor(q * q);
    return k > (double)INT32_MAX ? INT32_MAX : (int)k;
}

static uint64_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    uint64_t m = 0;
    for (int b = 0; b < 21; ++b) {
        m |= (uint64_t)((x >> b) & 1u) << (3 * b);
        m |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
        m |= (uint64_t)((z >> b) & 1u) << (3 * b + 2);
    }
    return m;
}

typedef struct { uint64_t key; int idx; } keyed_t;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed_t *x = (const keyed_t *)a, *y = (const keyed_t *)b;
    return (x->key > y->key) - (x->key < y->key);
}

int oracle_select(int nc, const int *dist2, int nf, int K,
                  unsigned char *mask, int *queue, int cap, int *count)
{
    if (nc <= 0 || nf <= 0 || nf % nc != 0) return ORC_EINVAL;
    const int r = nf / nc;
    const size_t total = (size_t)nf * nf * nf;
    size_t cnt = 0;
    for (size_t j = 0; j < total; ++j) {
        const int x = (int)(j % nf), y = (int)((j / nf) % nf), z = (int)(j / ((size_t)nf * nf));
        const int cidx = x / r + nc * (y / r + nc * (z / r));
        mask[j] = (unsigned char)(dist2[cidx] <= K);
        cnt += mask[j];
    }
    *count = (int)cnt;
    keyed_t *list = (keyed_t *)malloc(sizeof(keyed_t) * (cnt ? cnt : 1));
    if (!list) return ORC_EINVAL;
    size_t w = 0;
    for (size_t j = 0; j < total; ++j) {
        if (!mask[j]) continue;
        const int x = (int)(j % nf), y = (int)((j / nf) % nf), z = (int)(j / ((size_t)nf * nf));
        list[w].key = morton3((uint32_t)x, (uint32_t)y, (uint32_t)z);
        list[w].idx = (int)j;
        ++w;
    }
    qsort(list, cnt, sizeof(keyed_t), cmp_keyed);
    const size_t lim = cnt < (size_t)cap ? cnt : (size_t)cap;
    for (size_t i = 0; i < lim; ++i) queue[i] = list[i].idx;
    free(list);
    return cnt > (size_t)cap ? -4 : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Trilinear coarse sampling (a smoother reading of the coarse value c that  */
/* Sec. 2.2 compares with d and stores for unselected texels; the blocky    */
/* look of the point-sampled coarse SDF is what Sec. 2.1 remarks on).  The   */
/* coarse values are samples at voxel centres; the fine texel centre j sits  */
/* at coarse coordinate u = (j + 1/2)/r - 1/2 per axis (r = nf/nc), clamped  */
/* to [0, nc - 1] (constant extension beyond the outermost centres).  The    */
/* value is linear interpolation along x between the corner pairs, then     */
/* along y, then along z, each step a + t (b - a) in float32 (the selection  */
/* decision c <= d is a float32 comparison on both sides, so the value must  */
/* be the same float); an infinite corner (an empty coarse field) gives      */
/* +inf.                                                                     */
/* ------------------------------------------------------------------------ */

static float lerpf_plain(float a, float b, float t)
{
    const float diff = b - a;
    const float step = t * diff;
    return a + step;
}

static void clamp_axis(int j, int r, int nc, int *i0, int *i1, float *t)
{
    double u = ((double)j + 0.5) / (double)r - 0.5;
    if (u < 0.0) u = 0.0;
    if (u > (double)(nc - 1)) u = (double)(nc - 1);
    *i0 = (int)floor(u);
    *i1 = *i0 + 1 < nc ? *i0 + 1 : nc - 1;
    *t = (float)(u - (double)*i0); /* a multiple of 1/(2r): exact in float */
}

int oracle_coarse_trilinear(int nc, const float *c, int nf, float *out)
{
    if (nc <= 0 || nf <= 0 || nf % nc != 0) return ORC_EINVAL;
    const int r = nf / nc;
    const int64_t total = (int64_t)nf * nf * nf;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < total; ++j) {
        const int jx = (int)(j % nf), jy = (int)((j / nf) % nf), jz = (int)(j / ((int64_t)nf * nf));
        int x[2], y[2], z[2];
        float tx, ty, tz;
        clamp_axis(jx, r, nc, &x[0], &x[1], &tx);
        clamp_axis(jy, r, nc, &y[0], &y[1], &ty);
        clamp_axis(jz, r, nc, &z[0], &z[1], &tz);
        float v[2][2][2]; /* v[dz][dy][dx] */
        int any_inf = 0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int e = 0; e < 2; ++e) {
                    v[a][b][e] = c[x[e] + (int64_t)nc * (y[b] + (int64_t)nc * z[a])];
                    if (isinf(v[a][b][e])) any_inf = 1;
                }
        if (any_inf) {
            out[j] = INFINITY;
            continue;
        }
        float vy[2][2]; /* after x: vy[dz][dy] */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) vy[a][b] = lerpf_plain(v[a][b][0], v[a][b][1], tx);
        float vz[2]; /* after y */
        for (int a = 0; a < 2; ++a) vz[a] = lerpf_plain(vy[a][0], vy[a][1], ty);
        out[j] = lerpf_plain(vz[0], vz[1], tz);
    }
    return ORC_OK;
}

/* Selection on a field given at the texels themselves: texel j is selected  */
/* when field[j] <= d (float32 comparison); queue in ascending Morton order  */
/* as for oracle_select.                                                     */
int oracle_select_field(int n, const float *field, float d, unsigned char *mask, int *queue, int cap, int *count)
{
    if (n <= 0 || cap < 0) return ORC_EINVAL;
    const size_t total = (size_t)n * n * n;
    size_t cnt = 0;
    for (size_t j = 0; j < total; ++j) {
        mask[j] = (unsigned char)(field[j] <= d);
        cnt += mask[j];
    }
    *count = (int)cnt;
    keyed_t *list = (keyed_t *)malloc(sizeof(keyed_t) * (cnt ? cnt : 1));
    if (!list) return ORC_EINVAL;
    size_t w = 0;
    for (size_t j = 0; j < total; ++j) {
        if (!mask[j]) continue;
        const int x = (int)(j % n), y = (int)((j / n) % n), z = (int)(j / ((size_t)n * n));
        list[w].key = morton3((uint32_t)x, (uint32_t)y, (uint32_t)z);
        list[w].idx = (int)j;
        ++w;
    }
    qsort(list, cnt, sizeof(keyed_t), cmp_keyed);
    const size_t lim = cnt < (size_t)cap ? cnt : (size_t)cap;
    for (size_t i = 0; i < lim; ++i) queue[i] = list[i].idx;
    free(list);
    return cnt > (size_t)cap ? -4 : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Random sphere directions (Sec. 2.2: rays towards random points on the     */
/* surface of a sphere).  Random bits: Philox4x64 with 10 rounds (Salmon,   */
/* Moraes, Dror, Shaw, SC'11), key (seed, 0), counter (texel, frame*2^32 +   */
/* ray, scene, attempt).  Each 32-bit half h gives the float                 */
/* x = (2*(h >> 9) + 1 - 2^23) * 2^-23 in (-1, 1); consecutive halves form   */
/* pairs (x1, x2); the first pair with s = x1^2 + x2^2 < 1 is mapped to the  */
/* sphere by Marsaglia's 1972 method:                                        */
/*   w = (2 x1 sqrt(1 - s), 2 x2 sqrt(1 - s), 1 - 2 s).                      */
/* After 8 attempts (32 pairs) without success, w = (0, 0, 1).               */
/* ------------------------------------------------------------------------ */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    const unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, x0, &hi0, &lo0);
        mulhilo64(M1, x2, &hi1, &lo1);
        const uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static float uniform_pm1(uint32_t h)
{
    const int32_t m = (int32_t)((h >> 9) << 1) + 1 - 8388608;
    return (float)m * 0x1p-23f;
}

/* returns the attempt that succeeded (0..7) or 8 for the fallback */
int oracle_direction(uint64_t seed, uint64_t texel, uint32_t frame, uint32_t ray,
                     uint32_t scene, float out[3])
{
    const uint64_t key[2] = {seed, 0};
    for (uint32_t attempt = 0; attempt < 8; ++attempt) {
        const uint64_t ctr[4] = {texel, ((uint64_t)frame << 32) | ray, scene, attempt};
        uint64_t w[4];
        oracle_philox4x64_10(ctr, key, w);
        uint32_t h[8];
        for (int i = 0; i < 4; ++i) {
            h[2 * i] = (uint32_t)w[i];
            h[2 * i + 1] = (uint32_t)(w[i] >> 32);
        }
        for (int p = 0; p < 4; ++p) {
            volatile float x1 = uniform_pm1(h[2 * p]);
            volatile float x2 = uniform_pm1(h[2 * p + 1]);
            volatile float a = x1 * x1;
            volatile float b = x2 * x2;
            volatile float s = a + b;
            if (s < 1.0f) {
                volatile float om = 1.0f - s;
                volatile float q = sqrtf(om);
                volatile float t1 = 2.0f * x1;
                volatile float t2 = 2.0f * x2;
                volatile float ts = 2.0f * s;
                out[0] = t1 * q;
                out[1] = t2 * q;
                out[2] = 1.0f - ts;
                return (int)attempt;
            }
        }
    }
    out[0] = 0.0f;
    out[1] = 0.0f;
    out[2] = 1.0f;
    return 8;
}

/* Texel centre in world units, each coordinate lo + (i + 1/2) h in float. */
static void texel_origin(int nf, const float lo[3], float h, int j, float o[3])
{
    const int idx[3] = {j % nf, (j / nf) % nf, j / (nf * nf)};
    for (int a = 0; a < 3; ++a) {
        volatile float c = (float)idx[a] + 0.5f;
        volatile float m = c * h;
        o[a] = lo[a] + m;
    }
}

void oracle_texel_origin(int nf, const float lo[3], float h, int j, float o[3])
{
    texel_origin(nf, lo, h, j, o);
}

/* ------------------------------------------------------------------------ */
/* Closest hit (Sec. 2.2: the distance each ray travels to its closest hit). */
/* Ray/triangle test of Moller and Trumbore (1997) in double precision:      */
/* hit iff the determinant is non-zero, u, v >= 0, u + v <= 1 and t > 0.     */
/* The closest hit is the smallest (t, triangle index).  A hit is on the     */
/* front face when the ray runs against the geometric normal                 */
/* (v1 - v0) x (v2 - v0).                                                    */
/*                                                                           */
/* A ray is flagged ambiguous when a float32 evaluation could legitimately   */
/* pick a different closest triangle: some triangle whose plane is crossed   */
/* no farther than the closest hit (plus a margin) is crossed within 1e-6 of */
/* one of its edges, another triangle is hit within that margin of the      */
/* closest hit (two surfaces meeting there), or the closest hit grazes its   */
/* triangle (|cos| < 1e-2).                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lo[3], hi[3];
    int left, right;  /* children (internal) */
    int start, count; /* triangle range in the permutation (leaf: count > 0) */
} onode_t;

typedef struct oracle_scene {
    int nv, nt;
    double *v;   /* [nv][3] */
    int *f;      /* [nt][3] */
    int *perm;   /* triangle order of the hierarchy */
    onode_t *nodes;
    int nnodes;
    int use_bvh;
} oracle_scene;

static void tri_bounds(const oracle_scene *s, int t, double lo[3], double hi[3])
{
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int k = 0; k < 3; ++k) {
        const double *p = &s->v[3 * s->f[3 * t + k]];
        for (int a = 0; a < 3; ++a) {
            if (p[a] < lo[a]) lo[a] = p[a];
            if (p[a] > hi[a]) hi[a] = p[a];
        }
    }
}

static const double *g_centroids; /* qsort context (build is single-threaded): [nt][3] centroids */
static int g_centroid_axis;        /* and the axis being sorted on */

static int cmp_centroid(const void *a, const void *b)
{
    const double x = g_centroids[3 * *(const int *)a + g_centroid_axis];
    const double y = g_centroids[3 * *(const int *)b + g_centroid_axis];
    if (x < y) return -1;
    if (x > y) return 1;
    return (*(const int *)a > *(const int *)b) - (*(const int *)a < *(const int *)b);
}

/* Median-split bounding volume hierarchy.  Only an acceleration: the        */
/* closest hit it returns is the same as testing every triangle, because     */
/* boxes are padded by 1e-5 (plus a relative margin), far more than any      */
/* rounding in the box test, and a box is skipped only when it starts beyond */
/* the closest hit found so far (plus the ambiguity margin).                 */
static int build_rec(oracle_scene *s, double *cent, int start, int count, int *cap)
{
    if (s->nnodes >= *cap) {
        *cap *= 2;
        s->nodes = (onode_t *)realloc(s->nodes, sizeof(onode_t) * (size_t)(*cap));
    }
    const int id = s->nnodes++;
    onode_t nd;
    for (int a = 0; a < 3; ++a) { nd.lo[a] = INFINITY; nd.hi[a] = -INFINITY; }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = start; i < start + count; ++i) {
        double tl[3], th[3];
        tri_bounds(s, s->perm[i], tl, th);
        for (int a = 0; a < 3; ++a) {
            if (tl[a] < nd.lo[a]) nd.lo[a] = tl[a];
            if (th[a] > nd.hi[a]) nd.hi[a] = th[a];
            const double c = cent[3 * s->perm[i] + a];
            if (c < clo[a]) clo[a] = c;
            if (c > chi[a]) chi[a] = c;
        }
    }
    for (int a = 0; a < 3; ++a) {
        const double pad = 1e-5 + 1e-7 * (fabs(nd.lo[a]) + fabs(nd.hi[a]));
        nd.lo[a] -= pad;
        nd.hi[a] += pad;
    }
    nd.left = nd.right = -1;
    nd.start = start;
    nd.count = count;
    if (count <= 4) {
        s->nodes[id] = nd;
        return id;
    }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
        if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    g_centroids = cent;
    g_centroid_axis = axis;
    qsort(&s->perm[start], (size_t)count, sizeof(int), cmp_centroid);
    const int half = count / 2;
    nd.count = 0;
    s->nodes[id] = nd;
    const int l = build_rec(s, cent, start, half, cap);
    const int r = build_rec(s, cent, start + half, count - half, cap);
    s->nodes[id].left = l;
    s->nodes[id].right = r;
    return id;
}

static oracle_scene *scene_create_common(oracle_scene *s, const int *f, int nt, int use_bvh);

oracle_scene *oracle_scene_create(const float *v, int nv, const int *f, int nt, int use_bvh)
{
    oracle_scene *s = (oracle_scene *)calloc(1, sizeof(oracle_scene));
    s->nv = nv;
    s->v = (double *)malloc(sizeof(double) * 3 * (size_t)(nv > 0 ? nv : 1));
    for (int i = 0; i < 3 * nv; ++i) s->v[i] = (double)v[i];
    return scene_create_common(s, f, nt, use_bvh);
}

/* Same with double-precision vertices (finite-difference checks). */
oracle_scene *oracle_scene_create_f64(const double *v, int nv, const int *f, int nt, int use_bvh)
{
    oracle_scene *s = (oracle_scene *)calloc(1, sizeof(oracle_scene));
    s->nv = nv;
    s->v = (double *)malloc(sizeof(double) * 3 * (size_t)(nv > 0 ? nv : 1));
    memcpy(s->v, v, sizeof(double) * 3 * (size_t)nv);
    return scene_create_common(s, f, nt, use_bvh);
}

static oracle_scene *scene_create_common(oracle_scene *s, const int *f, int nt, int use_bvh)
{
    s->nt = nt;
    s->f = (int *)malloc(sizeof(int) * 3 * (size_t)(nt > 0 ? nt : 1));
    s->perm = (int *)malloc(sizeof(int) * (size_t)(nt > 0 ? nt : 1));
    memcpy(s->f, f, sizeof(int) * 3 * (size_t)nt);
    for (int t = 0; t < nt; ++t) s->perm[t] = t;
    s->use_bvh = use_bvh && nt > 0;
    if (s->use_bvh) {
        double *cent = (double *)malloc(sizeof(double) * 3 * (size_t)nt);
        for (int t = 0; t < nt; ++t)
            for (int a = 0; a < 3; ++a)
                cent[3 * t + a] = (s->v[3 * s->f[3 * t] + a] + s->v[3 * s->f[3 * t + 1] + a] + s->v[3 * s->f[3 * t + 2] + a]) / 3.0;
        int cap = 2 * nt + 1;
        s->nodes = (onode_t *)malloc(sizeof(onode_t) * (size_t)cap);
        build_rec(s, cent, 0, nt, &cap);
        free(cent);
    }
    return s;
}

void oracle_scene_destroy(oracle_scene *s)
{
    if (!s) return;
    free(s->v);
    free(s->f);
    free(s->perm);
    free(s->nodes);
    free(s);
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Moller-Trumbore.  Returns 1 on a hit; always reports the plane parameter
 * and barycentrics when the determinant is non-zero (for the ambiguity
 * test).  *valid tells whether the plane is crossed at all. */
static int mt_intersect(const double o[3], const double d[3], const double *v0, const double *v1,
                        const double *v2, double *t, double *u, double *w, int *valid)
{
    double e1[3], e2[3], p[3], s[3], q[3];
    for (int a = 0; a < 3; ++a) { e1[a] = v1[a] - v0[a]; e2[a] = v2[a] - v0[a]; s[a] = o[a] - v0[a]; }
    cross3(d, e2, p);
    const double det = dot3(e1, p);
    *valid = 0;
    if (det == 0.0) return 0;
    const double inv = 1.0 / det;
    *u = dot3(s, p) * inv;
    cross3(s, e1, q);
    *w = dot3(d, q) * inv;
    *t = dot3(e2, q) * inv;
    *valid = 1;
    if (*u < 0.0 || *w < 0.0 || *u + *w > 1.0) return 0;
    return *t > 0.0;
}

typedef struct {
    double t;
    int tri;
    int front;
    int ambiguous;
    double b[3]; /* barycentrics of the closest hit for vertices 0, 1, 2 */
} ohit_t;

/* distance-based edge proximity of a plane crossing at barycentrics (u, w) */
static int near_edge(const double *v0, const double *v1, const double *v2, double u, double w)
{
    double e[3][3];
    for (int a = 0; a < 3; ++a) {
        e[0][a] = v1[a] - v0[a];
        e[1][a] = v2[a] - v1[a];
        e[2][a] = v0[a] - v2[a];
    }
    double n[3];
    cross3(e[0], e[2], n);
    const double area2 = sqrt(dot3(n, n));
    /* barycentric b_k is (distance to the opposite edge) / (height onto it) */
    const double bary[3] = {1.0 - u - w, u, w};
    const int opp[3] = {1, 2, 0}; /* edge opposite vertex k */
    for (int k = 0; k < 3; ++k) {
        const double len = sqrt(dot3(e[opp[k]], e[opp[k]]));
        const double height = len > 0 ? area2 / len : 0.0;
        if (fabs(bary[k]) * height <= 1e-6) return 1;
    }
    return 0;
}

static void test_tri(const oracle_scene *s, int t, const double o[3], const double d[3], ohit_t *best)
{
    const double *v0 = &s->v[3 * s->f[3 * t]], *v1 = &s->v[3 * s->f[3 * t + 1]], *v2 = &s->v[3 * s->f[3 * t + 2]];
    double tt, u, w;
    int valid;
    const int hit = mt_intersect(o, d, v0, v1, v2, &tt, &u, &w, &valid);
    if (hit && (tt < best->t || (tt == best->t && t < best->tri))) {
        best->t = tt;
        best->tri = t;
        best->b[0] = 1.0 - u - w;
        best->b[1] = u;
        best->b[2] = w;
    }
}

/* second sweep over candidates for the ambiguity flag: a crossing near an   */
/* edge, or a second triangle hit no farther than the margin past the best   */
static void amb_tri(const oracle_scene *s, int t, const double o[3], const double d[3], double tlim, int best_tri,
                    int *amb)
{
    const double *v0 = &s->v[3 * s->f[3 * t]], *v1 = &s->v[3 * s->f[3 * t + 1]], *v2 = &s->v[3 * s->f[3 * t + 2]];
    double tt, u, w;
    int valid;
    const int hit = mt_intersect(o, d, v0, v1, v2, &tt, &u, &w, &valid);
    if (!valid || !(tt > -1e-6) || tt > tlim) return;
    if (hit && t != best_tri) {
        *amb = 1;
        return;
    }
    const double tol = -1e-3; /* only crossings close to the triangle matter */
    if (u < tol || w < tol || u + w > 1.0 - tol) return;
    if (near_edge(v0, v1, v2, u, w)) *amb = 1;
}

static int box_hit(const onode_t *nd, const double o[3], const double d[3], double tmax)
{
    double t0 = 0.0, t1 = tmax;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < nd->lo[a] || o[a] > nd->hi[a]) return 0;
            continue;
        }
        double ta = (nd->lo[a] - o[a]) / d[a], tb = (nd->hi[a] - o[a]) / d[a];
        if (ta > tb) { double x = ta; ta = tb; tb = x; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

static void visit(const oracle_scene *s, const double o[3], const double d[3], ohit_t *best,
                  double margin, int amb_pass, double tlim, int *amb)
{
    if (!s->use_bvh) {
        for (int t = 0; t < s->nt; ++t) {
            if (amb_pass) amb_tri(s, t, o, d, tlim, best->tri, amb);
            else test_tri(s, t, o, d, best);
        }
        return;
    }
    int stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const onode_t *nd = &s->nodes[stack[--sp]];
        const double lim = amb_pass ? tlim : (best->t * (1.0 + margin) + margin);
        if (!box_hit(nd, o, d, lim)) continue;
        if (nd->count > 0) {
            for (int i = nd->start; i < nd->start + nd->count; ++i) {
                if (amb_pass) amb_tri(s, s->perm[i], o, d, tlim, best->tri, amb);
                else test_tri(s, s->perm[i], o, d, best);
            }
        } else {
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
        }
    }
}

static void closest_hit(const oracle_scene *s, const double o[3], const double d[3], ohit_t *best)
{
    best->t = INFINITY;
    best->tri = -1;
    best->front = 0;
    best->ambiguous = 0;
    visit(s, o, d, best, 1e-9, 0, 0.0, NULL);
    const double tlim = (isinf(best->t) ? 1e30 : best->t * (1.0 + 1e-6) + 1e-6);
    int amb = 0;
    visit(s, o, d, best, 0.0, 1, tlim, &amb);
    if (best->tri >= 0) {
        const int t = best->tri;
        const double *v0 = &s->v[3 * s->f[3 * t]], *v1 = &s->v[3 * s->f[3 * t + 1]], *v2 = &s->v[3 * s->f[3 * t + 2]];
        double e1[3], e2[3], n[3];
        for (int a = 0; a < 3; ++a) { e1[a] = v1[a] - v0[a]; e2[a] = v2[a] - v0[a]; }
        cross3(e1, e2, n);
        const double dn = dot3(d, n);
        best->front = dn < 0.0;
        const double cosv = fabs(dn) / (sqrt(dot3(n, n)) * sqrt(dot3(d, d)));
        if (cosv < 1e-2) amb = 1;
    }
    best->ambiguous = amb;
}

/* Closest hits of a batch of rays (double precision): for tests. */
void oracle_closest_hits(const oracle_scene *s, int nr, const double *orig, const double *dir,
                         double *t, int *tri, int *front, int *amb)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < nr; ++i) {
        ohit_t h;
        closest_hit(s, &orig[3 * i], &dir[3 * i], &h);
        t[i] = h.t;
        tri[i] = h.tri;
        front[i] = h.front;
        amb[i] = h.ambiguous;
    }
}

/* ------------------------------------------------------------------------ */
/* One frame of fine-SDF tracing and temporal accumulation (Sec. 2.2,        */
/* Eq. (1)).  Reading used for the points the equation leaves open:          */
/*  * the state keeps an unsigned distance u; the sign is applied to the    */
/*    output only:  u_t = min(alpha u_{t-1} + (1 - alpha) max(c_t, 0), r_t)  */
/*    with u = +inf before the first traced frame (alpha = 1 makes this the  */
/*    running minimum of all hit distances);                                 */
/*  * r_t is the smallest closest-hit distance t |w| among the texel's rays */
/*    this frame (+inf if none hits); ties go to the lowest ray index;       */
/*  * front and back counts add the closest hit of every ray;               */
/*  * f_t = u_t if finite, else c_t; negated when back > front;             */
/*  * the argmin record (frame, ray, triangle) belongs to u_t when it came   */
/*    from a ray; it is kept on ties (earliest wins) and cleared when the    */
/*    decayed term wins with alpha < 1;                                      */
/*  * texels not selected this frame output c_t and their state resets.    */
/* ``texels`` optionally restricts the work to a subset (the state arrays    */
/* are still full-size); pass NULL / ntex < 0 for every texel.              */
/* ------------------------------------------------------------------------ */

/* Eq. (1) for a selected texel, on the unsigned state:
 *   u_t = min(alpha * u_{t-1} + (1 - alpha) * max(c_t, 0), r_t).
 * *src tells where u_t came from: 1 = this frame's rays (r_t strictly
 * smaller), 0 = the previous state unchanged (alpha = 1), 2 = the decayed
 * mixture (alpha < 1; the value no longer belongs to one ray). */
double oracle_eq1(double alpha, double u_prev, float c, double rt, int *src)
{
    const double cm = c > 0.0f ? (double)c : 0.0;
    /* alpha = 0 keeps no memory: the alpha u term is its limit 0, also for u = +inf (no history yet),
     * where the product itself would be 0 * inf */
    const double decayed = alpha == 1.0 ? u_prev : (alpha == 0.0 ? cm : alpha * u_prev + (1.0 - alpha) * cm);
    if (rt < decayed) { *src = 1; return rt; }
    *src = (alpha == 1.0) ? 0 : 2;
    return decayed;
}

/* Output value of a selected texel: the accumulated distance if any ray has
 * hit so far, else the coarse value; negative when more closest hits were
 * back faces than front faces (Sec. 2.2). */
/* Output value of a texel.  A texel whose state holds no traced distance    */
/* takes c.  Sign policy 0 (Sec. 2.2): negative when more closest hits were  */
/* back faces than front faces.  Policy 1, for open or thin surfaces that    */
/* the vote cannot sign: the unsigned distance minus a shell half-thickness, */
/* i.e. every surface read as a closed slab of that half-thickness.          */
double oracle_fine_value(double u, float c, int nfront, int nback, int sign_policy, double shell)
{
    if (isinf(u)) return (double)c;
    if (sign_policy == 1) return u - shell;
    return nback > nfront ? -u : u;
}

/* Two distances closer than this (relative) may compare either way once     */
/* evaluated in float32: the texel's argmin record is then not unique.       */
#define TIE_REL 3e-5

static int near_tie(double a, double b)
{
    if (!isfinite(a) || !isfinite(b)) return 0;
    const double m = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
    return fabs(a - b) <= TIE_REL * m;
}

/* texel_amb (bits sticky while the texel stays selected) marks what a       */
/* float32 evaluation could legitimately get differently: bit 0 (AMB_RAY),  */
/* one of the texel's rays was ambiguous (above), so its front/back counts  */
/* and sign are not unique; bit 1 (AMB_TIE), a frame's two smallest ray     */
/* distances, or its r_t and the value it was compared with in Eq. (1), are  */
/* within TIE_REL of each other, so the argmin record is not unique.        */
/* arg_amb marks texels whose argmin ray itself is ambiguous (their distance */
/* may differ beyond rounding and their argmin record is not unique).       */
/* Everything else about a selected texel is unique.                         */
#define AMB_RAY 1
#define AMB_TIE 2
int oracle_trace_frame(const oracle_scene *s,
                       int nc, const float *coarse_sdf,
                       int nf, const float lo[3], float hf,
                       const unsigned char *mask, const int *texels, int ntex,
                       int rays, uint32_t frame, uint64_t seed, uint32_t scene, double alpha,
                       double *u, int *nfront, int *nback,
                       int *arg_frame, int *arg_ray, int *arg_tri, unsigned char *arg_amb,
                       unsigned char *texel_amb,
                       double *fine, double *rmin_out, int sign_policy, double shell)
{
    if (nc <= 0 || nf <= 0 || nf % nc != 0 || rays <= 0) return ORC_EINVAL;
    const int r = nf / nc;
    const long total = (long)nf * nf * nf;
    const long count = texels ? ntex : total;
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < count; ++i) {
        const int j = texels ? texels[i] : (int)i;
        const int x = j % nf, y = (j / nf) % nf, z = j / (nf * nf);
        const float c = coarse_sdf[x / r + nc * (y / r + nc * (z / r))];
        if (!mask[j]) {
            u[j] = INFINITY;
            nfront[j] = nback[j] = 0;
            arg_frame[j] = arg_ray[j] = arg_tri[j] = -1;
            arg_amb[j] = 0;
            texel_amb[j] = 0;
            fine[j] = (double)c;
            if (rmin_out) rmin_out[j] = INFINITY;
            continue;
        }
        float of[3];
        texel_origin(nf, lo, hf, j, of);
        const double o[3] = {of[0], of[1], of[2]};
        double rt = INFINITY, rt2 = INFINITY; /* smallest and second smallest ray distance */
        int best_ray = -1, best_tri = -1, best_amb = 0;
        for (int k = 0; k < rays; ++k) {
            float wf[3];
            oracle_direction(seed, (uint64_t)j, frame, (uint32_t)k, scene, wf);
            const double w[3] = {wf[0], wf[1], wf[2]};
            ohit_t h;
            closest_hit(s, o, w, &h);
            if (h.ambiguous) texel_amb[j] |= AMB_RAY;
            if (h.tri < 0) continue;
            if (h.front) nfront[j] += 1;
            else nback[j] += 1;
            const double dist = h.t * sqrt(dot3(w, w));
            if (dist < rt) {
                rt2 = rt;
                rt = dist;
                best_ray = k;
                best_tri = h.tri;
                best_amb = h.ambiguous;
            } else if (dist < rt2) {
                rt2 = dist;
            }
        }
        if (rmin_out) rmin_out[j] = rt;
        if (near_tie(rt, rt2)) texel_amb[j] |= AMB_TIE;
        {
            /* the value r_t is compared with in Eq. (1) */
            int src0;
            const double decayed = oracle_eq1(alpha, u[j], c, INFINITY, &src0);
            if (near_tie(rt, decayed)) texel_amb[j] |= AMB_TIE;
        }
        int src;
        u[j] = oracle_eq1(alpha, u[j], c, rt, &src);
        if (src == 1) {
            arg_frame[j] = (int)frame;
            arg_ray[j] = best_ray;
            arg_tri[j] = best_tri;
            arg_amb[j] = (unsigned char)best_amb;
        } else if (src == 2) {
            arg_frame[j] = arg_ray[j] = arg_tri[j] = -1;
            arg_amb[j] = 0;
        }
        fine[j] = oracle_fine_value(u[j], c, nfront[j], nback[j], sign_policy, shell);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Gradient of the fine SDF with respect to vertex positions (not in the     */
/* paper; the derivative of its ray-traced distance).  A texel whose value   */
/* came from a ray with direction w hitting triangle (v0, v1, v2) at         */
/* barycentrics b has f = sign * t |w| with t the ray parameter; moving      */
/* vertex i by delta moves the hit point's plane by b_i (n . delta) along    */
/* the normal n, so dt/dv_i = b_i n / (n . w).  The sign, the selection, the */
/* flooding and the identity of the argmin ray are piecewise constant and    */
/* contribute nothing.                                                       */
/* grad_v[3*vertex + a] += grad_f[j] * sign_j * |w| * b_i * n_a / (n . w).   */
/* ------------------------------------------------------------------------ */
int oracle_fine_grad(const oracle_scene *s, int nf, const float lo[3], float hf,
                     uint64_t seed, uint32_t scene, const double *fine,
                     const int *arg_frame, const int *arg_ray, const int *arg_tri,
                     const double *grad_f, double *grad_v, int sign_policy)
{
    const long total = (long)nf * nf * nf;
    for (long j = 0; j < total; ++j) {
        const int t = arg_tri[j];
        if (t < 0 || grad_f[j] == 0.0) continue;
        float of[3], wf[3];
        texel_origin(nf, lo, hf, (int)j, of);
        oracle_direction(seed, (uint64_t)j, (uint32_t)arg_frame[j], (uint32_t)arg_ray[j], scene, wf);
        const double o[3] = {of[0], of[1], of[2]}, w[3] = {wf[0], wf[1], wf[2]};
        const int iv[3] = {s->f[3 * t], s->f[3 * t + 1], s->f[3 * t + 2]};
        const double *v0 = &s->v[3 * iv[0]], *v1 = &s->v[3 * iv[1]], *v2 = &s->v[3 * iv[2]];
        double tt, u, w2;
        int valid;
        mt_intersect(o, w, v0, v1, v2, &tt, &u, &w2, &valid);
        if (!valid) continue;
        double e1[3], e2[3], n[3];
        for (int a = 0; a < 3; ++a) { e1[a] = v1[a] - v0[a]; e2[a] = v2[a] - v0[a]; }
        cross3(e1, e2, n);
        const double nw = dot3(n, w);
        const double sgn = sign_policy == 0 && fine[j] < 0 ? -1.0 : 1.0;
        const double scale = grad_f[j] * sgn * sqrt(dot3(w, w)) / nw;
        const double b[3] = {1.0 - u - w2, u, w2};
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) grad_v[3 * iv[k] + a] += scale * b[k] * n[a];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact unsigned distance from points to the mesh (the quantity the traced  */
/* fine SDF of Sec. 2.2 approaches from above: every hit is on the mesh).    */
/* Plain definition: the minimum over all triangles of the distance to the   */
/* triangle, which is the distance to the plane when the point's projection  */
/* lies in the closed triangle, else the distance to the nearest of its      */
/* three edges (closest point of a segment by clamped projection).           */
/* Zero-area triangles have only their edges.  Ties go to the lowest index.  */
/* ------------------------------------------------------------------------ */
static double seg_dist2_d(const double p[3], const double a[3], const double b[3])
{
    double e[3], ap[3];
    for (int k = 0; k < 3; ++k) { e[k] = b[k] - a[k]; ap[k] = p[k] - a[k]; }
    const double ee = dot3(e, e);
    double t = ee > 0 ? dot3(ap, e) / ee : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double d2 = 0;
    for (int k = 0; k < 3; ++k) {
        const double q = a[k] + t * e[k] - p[k];
        d2 += q * q;
    }
    return d2;
}

static double tri_dist2_d(const double p[3], const double a[3], const double b[3], const double c[3])
{
    double ab[3], ac[3], ap[3], n[3];
    for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; ap[k] = p[k] - a[k]; }
    cross3(ab, ac, n);
    const double nn = dot3(n, n);
    if (nn > 0) {
        const double h = dot3(ap, n) / nn;
        double q[3];
        for (int k = 0; k < 3; ++k) q[k] = p[k] - h * n[k];
        /* q inside the closed triangle: each edge sees q on the inner side */
        const double *v[3] = {a, b, c};
        int inside = 1;
        for (int e = 0; e < 3 && inside; ++e) {
            const double *u0 = v[e], *u1 = v[(e + 1) % 3];
            double ed[3], uq[3], cr[3];
            for (int k = 0; k < 3; ++k) { ed[k] = u1[k] - u0[k]; uq[k] = q[k] - u0[k]; }
            cross3(ed, uq, cr);
            if (dot3(cr, n) < 0) inside = 0;
        }
        if (inside) {
            const double d = dot3(ap, n);
            return d * d / nn;
        }
    }
    double d2 = seg_dist2_d(p, a, b);
    const double d2b = seg_dist2_d(p, b, c), d2c = seg_dist2_d(p, c, a);
    if (d2b < d2) d2 = d2b;
    if (d2c < d2) d2 = d2c;
    return d2;
}

void oracle_point_distance(const oracle_scene *s, int n, const double *pts, double *dist, int *tri)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; ++i) {
        double best = INFINITY;
        int bid = -1;
        for (int t = 0; t < s->nt; ++t) {
            const double d2 = tri_dist2_d(&pts[3 * i], &s->v[3 * s->f[3 * t]], &s->v[3 * s->f[3 * t + 1]],
                                          &s->v[3 * s->f[3 * t + 2]]);
            if (d2 < best) {
                best = d2;
                bid = t;
            }
        }
        dist[i] = bid >= 0 ? sqrt(best) : INFINITY;
        if (tri) tri[i] = bid;
    }
}

/* ------------------------------------------------------------------------ */
/* World positions of rigid parts (a scene given as parts in object space    */
/* and one object-to-world transform per part, rows r_a = (r_a0, r_a1,       */
/* r_a2, t_a)).  Defined in float32 with the operation order                 */
/* ((r_a0 x + r_a1 y) + r_a2 z) + t_a, each operation rounded once, because */
/* voxelization and selection downstream must see the same float positions  */
/* on both sides.  part[v] < 0 leaves a vertex where it is.                  */
/* ------------------------------------------------------------------------ */
void oracle_instance_world(int nv, const float *obj, const int *part, const float *T, float *out)
{
    for (int v = 0; v < nv; ++v) {
        const float x = obj[3 * v], y = obj[3 * v + 1], z = obj[3 * v + 2];
        if (part[v] < 0) {
            out[3 * v] = x;
            out[3 * v + 1] = y;
            out[3 * v + 2] = z;
            continue;
        }
        const float *m = &T[12 * part[v]];
        for (int a = 0; a < 3; ++a) {
            volatile float px = m[4 * a] * x;
            volatile float py = m[4 * a + 1] * y;
            volatile float pz = m[4 * a + 2] * z;
            volatile float s1 = px + py;
            volatile float s2 = s1 + pz;
            volatile float s3 = s2 + m[4 * a + 3];
            out[3 * v + a] = s3;
        }
    }
}

/* Directions for many keys (same rule as oracle_direction). */
void oracle_directions(int n, const int *texel, const uint32_t *frame, const int *ray, uint64_t seed,
                       uint32_t scene, float *out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) oracle_direction(seed, (uint64_t)texel[i], frame[i], (uint32_t)ray[i], scene, &out[3 * i]);
}

/* ------------------------------------------------------------------------ */
/* Soft shadows (Sec. 2.3): march from p towards the light through the fine  */
/* SDF, sampled linearly (trilinear between texel centres) rather than at   */
/* the nearest texel; stop after max_steps samples, when the sample falls    */
/* below eps (fully shadowed), when t exceeds max_dist or the point leaves   */
/* the grid; the step is the sample value capped at max_step (and at least   */
/* eps); the penumbra term is the running minimum of k s / t.  The march is  */
/* defined in float arithmetic with this exact operation order (each        */
/* operation rounded once), because its stopping decisions must be taken in */
/* the same precision on both sides:                                         */
/*   q = p + t l;  g = (q - lo) / h - 1/2 per axis (outside if g < -1/2 or   */
/*   g > n - 1/2); g clamped to [0, n-1]; i = min(floor(g), n-2); f = g - i; */
/*   lerp(a, b, f) = a + f (b - a), along x, then y, then z;                 */
/*   vis = min(vis, (k s) / t);  t = t + max(min(s, max_step), eps).         */
/*                                                                           */
/* Two options of Sec. 2.3:                                                  */
/*  * jitter: the march starts at t = eps + jitter[p] * jitter_scale, i.e.   */
/*    the origin is moved towards the light by a per-point random amount     */
/*    (the caller draws jitter in [0, 1), per frame, and filters over time). */
/*  * triangulation (penumbra = 1; Aaltonen 2018, cited for the banding      */
/*    fix): consecutive samples s_prev at t_prev and s at t are two empty    */
/*    spheres along the ray; the nearest occluder is estimated on the circle */
/*    where they intersect, at distance y back from the current point and    */
/*    radius d from the ray:                                                 */
/*      D = t - t_prev,  y = ((D D + s s) - s_prev s_prev) / (D + D),        */
/*      y clamped to [0, s],  d = sqrt(max(s s - y y, 0)),                    */
/*      vis = min(vis, (k d) / (t - y))  if t - y > 0.                       */
/*    With D = s_prev (an unclamped sphere-tracing step) y = s^2/(2 s_prev), */
/*    the published form.  The first sample has no predecessor and uses the  */
/*    cone term k s / t.                                                     */
/* ------------------------------------------------------------------------ */
static int shadow_axis(float q, float lo, float h, int n, int *i, float *f)
{
    volatile float a = q - lo;
    volatile float b = a / h;
    volatile float g = b - 0.5f;
    if (g < -0.5f || g > (float)n - 0.5f) return 0;
    float gc = g < 0.0f ? 0.0f : g;
    if (gc > (float)(n - 1)) gc = (float)(n - 1);
    int ii = (int)floorf(gc);
    if (ii > n - 2) ii = n - 2;
    *i = ii;
    volatile float ff = gc - (float)ii;
    *f = ff;
    return 1;
}

static float lerpf_(float a, float b, float f)
{
    volatile float d = b - a;
    volatile float m = f * d;
    volatile float r = a + m;
    return r;
}

void oracle_shadow(int n, const float lo[3], float h, const float *sdf, int np, const float *pts, const float l[3],
                   float k, float eps, int max_steps, float max_step, float max_dist, int penumbra,
                   const float *jitter, float jitter_scale, float *vis_out)
{
#pragma omp parallel for schedule(static)
    for (int p = 0; p < np; ++p) {
        float vis = 1.0f, t = eps;
        if (jitter) {
            volatile float off = jitter[p] * jitter_scale;
            volatile float t0 = eps + off;
            t = t0;
        }
        int have_prev = 0;
        float t_prev = 0.0f, s_prev = 0.0f;
        for (int step = 0; step < max_steps; ++step) {
            if (t > max_dist) break;
            float q[3];
            int idx[3];
            float fr[3];
            int inside = 1;
            for (int a = 0; a < 3; ++a) {
                volatile float m = t * l[a];
                volatile float qq = pts[3 * p + a] + m;
                q[a] = qq;
                if (!shadow_axis(q[a], lo[a], h, n, &idx[a], &fr[a])) inside = 0;
            }
            if (!inside) break;
            const long b = idx[0] + (long)n * (idx[1] + (long)n * idx[2]);
            const long sy = n, sz = (long)n * n;
            const float c00 = lerpf_(sdf[b], sdf[b + 1], fr[0]);
            const float c10 = lerpf_(sdf[b + sy], sdf[b + sy + 1], fr[0]);
            const float c01 = lerpf_(sdf[b + sz], sdf[b + sz + 1], fr[0]);
            const float c11 = lerpf_(sdf[b + sy + sz], sdf[b + sy + sz + 1], fr[0]);
            const float s = lerpf_(lerpf_(c00, c10, fr[1]), lerpf_(c01, c11, fr[1]), fr[2]);
            if (s < eps) {
                vis = 0.0f;
                break;
            }
            if (penumbra == 1 && have_prev) {
                volatile float D = t - t_prev;
                volatile float DD = D * D;
                volatile float ss = s * s;
                volatile float sum = DD + ss;
                volatile float pp = s_prev * s_prev;
                volatile float num = sum - pp;
                volatile float den = D + D;
                volatile float y = num / den;
                float yc = y > 0.0f ? y : 0.0f;
                if (yc > s) yc = s;
                volatile float yy = yc * yc;
                volatile float r = ss - yy;
                const float d = sqrtf(r > 0.0f ? r : 0.0f);
                volatile float w = t - yc;
                if (w > 0.0f) {
                    volatile float kd = k * d;
                    volatile float pen = kd / w;
                    if (pen < vis) vis = pen;
                }
            } else {
                volatile float ks = k * s;
                volatile float pen = ks / t;
                if (pen < vis) vis = pen;
            }
            have_prev = 1;
            t_prev = t;
            s_prev = s;
            float st = s < max_step ? s : max_step;
            if (st < eps) st = eps;
            volatile float tn = t + st;
            t = tn;
        }
        vis_out[p] = vis > 0.0f ? vis : 0.0f;
    }
}
