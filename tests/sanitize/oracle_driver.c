/*
 * Test driver that runs every entry point of the oracle (oracle/rtsdf_oracle.c)
 * once on a small mesh, for builds under the address, undefined-behaviour and
 * thread sanitizers (tests/test_oracle_sanitizers.py).  It checks return codes
 * only; the numbers are pinned by the other oracle tests.
 *
 * usage: oracle_driver mesh.bin
 *   mesh.bin = int32 nv, int32 nt, float32 vertices[nv][3], int32 faces[nt][3]
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct oracle_scene oracle_scene;
int oracle_num_threads(void);
int oracle_voxelize(const float *v, int nv, const int *f, int nt, const float lo[3], float h, int n, int *seeds);
int oracle_jfa(int n, const int *seeds_in, int *seeds_out);
int oracle_jfa_steps(int n, const int *seeds_in, const int *steps, int nsteps, int *seeds_out);
void oracle_coarse(int n, const int *seeds, float h, float beta, int *dist2, float *c);
int oracle_select_threshold(float hc, float beta, float d);
int oracle_select(int nc, const int *dist2, int nf, int K, unsigned char *mask, int *queue, int cap, int *count);
int oracle_coarse_trilinear(int nc, const float *c, int nf, float *out);
int oracle_select_field(int n, const float *field, float d, unsigned char *mask, int *queue, int cap, int *count);
oracle_scene *oracle_scene_create(const float *v, int nv, const int *f, int nt, int use_bvh);
void oracle_scene_destroy(oracle_scene *s);
void oracle_closest_hits(const oracle_scene *s, int nr, const double *orig, const double *dir, double *t, int *tri,
                         int *front, int *amb);
int oracle_trace_frame(const oracle_scene *s, int nc, const float *coarse_sdf, int nf, const float lo[3], float hf,
                       const unsigned char *mask, const int *texels, int ntex, int rays, uint32_t frame,
                       uint64_t seed, uint32_t scene, double alpha, double *u, int *nfront, int *nback,
                       int *arg_frame, int *arg_ray, int *arg_tri, unsigned char *arg_amb,
                       unsigned char *texel_amb, double *fine, double *rmin_out, int sign_policy, double shell);
int oracle_fine_grad(const oracle_scene *s, int nf, const float lo[3], float hf, uint64_t seed, uint32_t scene,
                     const double *fine, const int *arg_frame, const int *arg_ray, const int *arg_tri,
                     const double *grad_f, double *grad_v, int sign_policy);
void oracle_point_distance(const oracle_scene *s, int n, const double *pts, double *dist, int *tri);
void oracle_directions(int n, const int *texel, const uint32_t *frame, const int *ray, uint64_t seed, uint32_t scene,
                       float *out);
void oracle_shadow(int n, const float lo[3], float h, const float *sdf, int np, const float *pts, const float l[3],
                   float k, float eps, int max_steps, float max_step, float max_dist, int penumbra,
                   const float *jitter, float jitter_scale, float *vis_out);
void oracle_instance_world(int nv, const float *obj, const int *part, const float *T, float *out);

#define CHECK(x)                                                        \
    do {                                                                \
        if ((x) != 0) {                                                 \
            fprintf(stderr, "driver: %s failed at line %d\n", #x, __LINE__); \
            return 2;                                                   \
        }                                                               \
    } while (0)

static void *xcalloc(size_t n, size_t sz)
{
    void *p = calloc(n ? n : 1, sz);
    if (!p) {
        fprintf(stderr, "driver: out of memory\n");
        exit(3);
    }
    return p;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 1;
    FILE *fp = fopen(argv[1], "rb");
    if (!fp) return 1;
    int32_t nv = 0, nt = 0;
    if (fread(&nv, 4, 1, fp) != 1 || fread(&nt, 4, 1, fp) != 1 || nv <= 0 || nt <= 0) return 1;
    float *v = xcalloc((size_t)nv * 3, sizeof(float));
    int *f = xcalloc((size_t)nt * 3, sizeof(int));
    if (fread(v, sizeof(float), (size_t)nv * 3, fp) != (size_t)nv * 3) return 1;
    if (fread(f, sizeof(int), (size_t)nt * 3, fp) != (size_t)nt * 3) return 1;
    fclose(fp);

    const int nc = 16, nf = 32, rays = 4;
    const float lo[3] = {0, 0, 0}, hc = 1.0f / nc, hf = 1.0f / nf, beta = 0.5f * hc, d = 2.0f * hc;
    const size_t n3 = (size_t)nc * nc * nc, f3 = (size_t)nf * nf * nf;
    int *s0 = xcalloc(n3, sizeof(int)), *s1 = xcalloc(n3, sizeof(int)), *d2 = xcalloc(n3, sizeof(int));
    float *c = xcalloc(n3, sizeof(float));
    CHECK(oracle_voxelize(v, nv, f, nt, lo, hc, nc, s0));
    CHECK(oracle_jfa(nc, s0, s1));
    const int steps[] = {1, 8, 4, 2, 1, 2, 1};
    CHECK(oracle_jfa_steps(nc, s0, steps, 7, s1));
    CHECK(oracle_jfa(nc, s0, s1));
    oracle_coarse(nc, s1, hc, beta, d2, c);
    unsigned char *mask = xcalloc(f3, 1);
    int *queue = xcalloc(f3, sizeof(int));
    int count = 0;
    CHECK(oracle_select(nc, d2, nf, oracle_select_threshold(hc, beta, d), mask, queue, (int)f3, &count));
    float *cf = xcalloc(f3, sizeof(float));
    unsigned char *mask2 = xcalloc(f3, 1);
    int count2 = 0;
    CHECK(oracle_coarse_trilinear(nc, c, nf, cf));
    CHECK(oracle_select_field(nf, cf, d, mask2, queue, (int)f3, &count2));
    CHECK(oracle_select(nc, d2, nf, oracle_select_threshold(hc, beta, d), mask, queue, (int)f3, &count));

    for (int use_bvh = 0; use_bvh <= 1; ++use_bvh) {
        oracle_scene *sc = oracle_scene_create(v, nv, f, nt, use_bvh);
        if (!sc) return 2;
        double *u = xcalloc(f3, sizeof(double)), *fine = xcalloc(f3, sizeof(double)), *rmin = xcalloc(f3, sizeof(double));
        int *nfr = xcalloc(f3, sizeof(int)), *nbk = xcalloc(f3, sizeof(int));
        int *af = xcalloc(f3, sizeof(int)), *ar = xcalloc(f3, sizeof(int)), *at = xcalloc(f3, sizeof(int));
        unsigned char *aa = xcalloc(f3, 1), *ta = xcalloc(f3, 1);
        for (size_t j = 0; j < f3; ++j) {
            u[j] = INFINITY;
            af[j] = ar[j] = at[j] = -1;
        }
        for (uint32_t fr = 0; fr < 2; ++fr)
            CHECK(oracle_trace_frame(sc, nc, c, nf, lo, hf, mask, NULL, -1, rays, fr, 0, 0, 0.9, u, nfr, nbk, af, ar,
                                     at, aa, ta, fine, rmin, 0, 0.0));
        CHECK(oracle_trace_frame(sc, nc, c, nf, lo, hf, mask, queue, count < 64 ? count : 64, rays, 2, 0, 0, 1.0, u,
                                 nfr, nbk, af, ar, at, aa, ta, fine, rmin, 1, 0.01));
        double *gf = xcalloc(f3, sizeof(double)), *gv = xcalloc((size_t)nv * 3, sizeof(double));
        for (size_t j = 0; j < f3; ++j) gf[j] = mask[j] ? 1.0 : 0.0;
        CHECK(oracle_fine_grad(sc, nf, lo, hf, 0, 0, fine, af, ar, at, gf, gv, 0));
        const int np = 257;
        double *pts = xcalloc((size_t)np * 3, sizeof(double)), *dirs = xcalloc((size_t)np * 3, sizeof(double));
        double *dist = xcalloc(np, sizeof(double)), *tt = xcalloc(np, sizeof(double));
        int *tri = xcalloc(np, sizeof(int)), *fro = xcalloc(np, sizeof(int)), *amb = xcalloc(np, sizeof(int));
        for (int i = 0; i < np; ++i)
            for (int a = 0; a < 3; ++a) {
                pts[3 * i + a] = (double)((i * 37 + a * 11) % 101) / 100.0;
                dirs[3 * i + a] = (double)((i * 13 + a * 29) % 7) - 3.0;
            }
        oracle_point_distance(sc, np, pts, dist, tri);
        oracle_closest_hits(sc, np, pts, dirs, tt, tri, fro, amb);
        free(pts); free(dirs); free(dist); free(tt); free(tri); free(fro); free(amb);
        free(gf); free(gv);
        free(u); free(fine); free(rmin); free(nfr); free(nbk); free(af); free(ar); free(at); free(aa); free(ta);
        oracle_scene_destroy(sc);
    }

    const int nq = 100;
    int *tex = xcalloc(nq, sizeof(int)), *ray = xcalloc(nq, sizeof(int));
    uint32_t *frm = xcalloc(nq, sizeof(uint32_t));
    float *dout = xcalloc((size_t)nq * 3, sizeof(float));
    for (int i = 0; i < nq; ++i) {
        tex[i] = i * 31;
        ray[i] = i % 16;
        frm[i] = (uint32_t)(i / 7);
    }
    oracle_directions(nq, tex, frm, ray, 0, 0, dout);
    float *fs = xcalloc(f3, sizeof(float)), *pts = xcalloc((size_t)nq * 3, sizeof(float));
    float *jit = xcalloc(nq, sizeof(float)), *vis = xcalloc(nq, sizeof(float));
    for (size_t j = 0; j < f3; ++j) fs[j] = cf[j];
    for (int i = 0; i < nq; ++i) {
        pts[3 * i] = (float)(i % 10) / 10.0f;
        pts[3 * i + 1] = 0.2f;
        pts[3 * i + 2] = (float)(i / 10) / 10.0f;
        jit[i] = (float)i / (float)nq;
    }
    const float l[3] = {0.3f, 0.9f, 0.3f};
    oracle_shadow(nf, lo, hf, fs, nq, pts, l, 8.0f, hf, 64, 2 * hf, 1.0f, 0, NULL, 0.0f, vis);
    oracle_shadow(nf, lo, hf, fs, nq, pts, l, 8.0f, hf, 64, 2 * hf, 1.0f, 1, jit, 2 * hf, vis);
    int *part = xcalloc(nv, sizeof(int));
    float T[24] = {0};
    for (int p = 0; p < 2; ++p) T[12 * p] = T[12 * p + 5] = T[12 * p + 10] = 1.0f;
    T[12 + 3] = 0.01f;
    for (int i = 0; i < nv; ++i) part[i] = i % 2;
    float *wv = xcalloc((size_t)nv * 3, sizeof(float));
    oracle_instance_world(nv, v, part, T, wv);
    printf("driver ok: %d threads, %d selected, %d field-selected\n", oracle_num_threads(), count, count2);
    free(tex); free(ray); free(frm); free(dout); free(fs); free(pts); free(jit); free(vis); free(part); free(wv);
    free(s0); free(s1); free(d2); free(c); free(mask); free(queue); free(cf); free(mask2);
    free(v); free(f);
    return 0;
}
