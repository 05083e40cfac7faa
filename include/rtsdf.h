/*
 * rtsdf.h -- C ABI of the MI355X (gfx950) SDF-generation library.
 *
 * The library implements the data-parallel path of RTSDF (Tan, Chua, Koh,
 * Bhojan, "RTSDF: Generating Signed Distance Fields in Real Time for Soft
 * Shadow Rendering", Pacific Graphics 2020 short paper):
 *
 *   1. rtsdf_voxelize          mark the coarse voxels touched by the mesh
 *                              (Sec. 2.1, orthographic projections along
 *                              x, y and z with depth culling off);
 *   2. rtsdf_jfa               3D jump flooding from those voxels with steps
 *                              n/2, n/4, ..., 1 and the coarse SDF
 *                              c = distance - beta (Sec. 2.1);
 *   3. rtsdf_select            fine texels whose coarse value is within d,
 *                              compacted into a queue (Sec. 2.2, the case
 *                              split of Eq. (1));
 *   4. rtsdf_trace_accumulate  per selected texel, rays towards random points
 *                              on a sphere, closest hits against a bounding
 *                              volume hierarchy, the per-frame minimum r_t,
 *                              the temporal update of Eq. (1) and the
 *                              front/back sign vote (Sec. 2.2);
 *   5. rtsdf_shadow            soft-shadow visibility by sphere tracing the
 *                              fine SDF towards a directional light (Sec. 2.3).
 *
 * plus the vertex gradient of the fine SDF (rtsdf_trace_backward), many
 * scenes per launch (rtsdf_batch_*), and a captured per-frame graph
 * (rtsdf_frame_graph_*).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  * All array arguments are DEVICE pointers owned by the caller, unless a
 *    parameter says "host".  The library never frees them.
 *  * The library allocates device memory only inside rtsdf_scene_create and
 *    rtsdf_batch_create / rtsdf_frame_graph_create (released by the matching
 *    destroy call).
 *  * Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 *    stream) and do not synchronise, except *_create and rtsdf_sync_status.
 *  * Arguments that can be checked on the host are checked before anything
 *    is launched; a failure returns RTSDF_EINVAL and launches nothing.
 *    Conditions only the device can see (a face index out of range, a vertex
 *    outside the allowed box, a full queue) set bits of a per-device error
 *    word, which rtsdf_sync_status returns and clears.
 *  * Grids are cubes: `n` cells per axis, cell i along an axis spans
 *    [lo + i h, lo + (i + 1) h); arrays over a grid are n^3 elements, x
 *    fastest (index x + n (y + n z)).
 *  * Lengths (h, beta, d, distances) are in world units.
 *  * Calls that share an output or a workspace must not run concurrently.
 *    Read-only inputs may be shared: traces of one scene on several streams
 *    are safe with separate workspaces and outputs (a scene holds no
 *    per-trace scratch).  Calls that modify a scene (refit, rebuild,
 *    set_transforms, set_sign, set_tuning) must not overlap its traces.
 */
#ifndef RTSDF_H
#define RTSDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *rtsdf_stream; /* hipStream_t */

typedef struct rtsdf_grid {
    float lo[3]; /* world position of the grid's lower corner */
    float h;     /* cell size */
    int32_t n;   /* cells per axis */
} rtsdf_grid;

enum {
    RTSDF_OK = 0,
    RTSDF_EINVAL = -1,    /* bad argument (checked on the host) */
    RTSDF_ENOMEM = -2,    /* a *_create call could not allocate */
    RTSDF_EHIP = -3,      /* a HIP runtime call failed */
    RTSDF_EDEVICE = -4    /* rtsdf_sync_status: device-side error bits set */
};

/* device error bits (returned through *bits of rtsdf_sync_status) */
enum {
    RTSDF_ERR_FACE_INDEX = 1,  /* a face index outside [0, nv) */
    RTSDF_ERR_VERTEX_RANGE = 2,/* a vertex farther than one domain side outside the grid */
    RTSDF_ERR_QUEUE_FULL = 4,  /* rtsdf_select: more selected texels than queue_cap */
    RTSDF_ERR_BATCH = 8,       /* rtsdf_batch_step: inconsistent batch tables */
    RTSDF_ERR_TRANSFORM = 16,  /* rtsdf_scene_set_transforms: a transform that is not rigid */
    RTSDF_ERR_FRAME = 32       /* a tracer read a frame index >= 2^23 through frame_ptr (that frame was not traced) */
};

const char *rtsdf_status_string(int status);
int rtsdf_version(void); /* 100 * major + minor */

/* Synchronise `stream`, then read and clear the device error word of the
 * current device.  Returns RTSDF_OK if no bit was set, else RTSDF_EDEVICE
 * with the bits in *bits (may be NULL). */
int rtsdf_sync_status(rtsdf_stream stream, uint32_t *bits);

/* Device-to-device copy of `bytes` bytes on `stream` (lets bindings copy
 * library-owned buffers, e.g. a batch's outputs, into their own memory). */
int rtsdf_copy(void *dst, const void *src, size_t bytes, rtsdf_stream stream);

/* ------------------------------------------------------------------------ */
/* 1. Voxelization (Sec. 2.1).                                               */
/*                                                                           */
/* vertices  float32 [nv][3] world positions.                                */
/* faces     int32 [nt][3] vertex indices.                                   */
/* coarse    the coarse grid; n a power of two in [8, 256].                  */
/* seeds     int32 [n^3] output: the voxel's own linear index if occupied,   */
/*           else -1.                                                        */
/*                                                                           */
/* Rule (the paper rasterizes; this is the exact rule used): vertex          */
/* coordinates are snapped to 1/256 of a voxel (round half to even of        */
/* (v - lo) / h * 256 in double precision).  For each triangle and each axis */
/* a, every voxel column along a whose centre lies inside or on the boundary */
/* of the triangle's projection marks the voxel containing the triangle's    */
/* depth at that centre (floor of the exact rational depth; a depth exactly  */
/* on the far face goes to the last layer; depths outside the grid and       */
/* zero-area projections are skipped).  Every vertex must lie within the     */
/* grid grown by one side length on each side (else ERR_VERTEX_RANGE and the */
/* triangle is skipped).  The result does not depend on triangle order.     */
/* ------------------------------------------------------------------------ */
int rtsdf_voxelize(const float *vertices, int32_t nv, const int32_t *faces, int32_t nt,
                   rtsdf_grid coarse, int32_t *seeds, rtsdf_stream stream);

/* ------------------------------------------------------------------------ */
/* 2. Jump flooding and coarse SDF (Sec. 2.1).                               */
/*                                                                           */
/* seeds     int32 [n^3] in: rtsdf_voxelize's output (own index or -1);      */
/*           out: the nearest seed found by jump flooding (linear index, -1  */
/*           only if the grid has no seed at all).  Passes k = n/2, ..., 1;  */
/*           pass k takes, per voxel, the best of its own seed and those of  */
/*           the 26 voxels at offsets k (i, j, l), i, j, l in {-1, 0, 1}     */
/*           inside the grid, by squared distance, ties to the lowest index. */
/* scratch   int32 [n^3] workspace (contents destroyed).                     */
/* beta      bias subtracted from the distance (world units).                */
/* dist2     int32 [n^3] out: squared distance in voxels to the seed         */
/*           (INT32_MAX if none); also a work buffer during the passes.     */
/*           seeds, scratch and dist2 must be three distinct arrays         */
/*           (EINVAL if two of the pointers are equal).                      */
/* coarse_sdf float32 [n^3] out: h * sqrt(dist2) - beta, each float          */
/*           operation rounded once (+inf if no seed).                       */
/* n must be a power of two in [8, 256].                                     */
/* ------------------------------------------------------------------------ */
int rtsdf_jfa(rtsdf_grid coarse, int32_t *seeds, int32_t *scratch, float beta,
              int32_t *dist2, float *coarse_sdf, rtsdf_stream stream);

/* The same with a caller-chosen pass schedule: steps (host, [nsteps]) lists
 * the step of every pass in order; each step a power of two in [1, n/2], the
 * last one 1, 1 <= nsteps <= 64.  Besides n/2, ..., 1 this runs the
 * error-reducing variants of jump flooding (Rong and Tan 2006, the method
 * Sec. 2.1 builds on): "JFA+1" (n/2, ..., 1, 1), "JFA+2" (n/2, ..., 1, 2, 1)
 * and "1+JFA" (1, n/2, ..., 1).  Extra passes never increase a voxel's
 * distance.  Other arguments as rtsdf_jfa; rtsdf_jfa is this call with
 * n/2, ..., 1.  A schedule that starts with a step below 4 converts the
 * input to the internal layout first, and adds one device-to-device copy of
 * n^3 int32 when its passes would end in the wrong buffer. */
int rtsdf_jfa_steps(rtsdf_grid coarse, int32_t *seeds, int32_t *scratch, const int32_t *steps, int32_t nsteps,
                    float beta, int32_t *dist2, float *coarse_sdf, rtsdf_stream stream);

/* Tuning of the jump flooding per grid size (the results are the same; only
 * speed differs).
 * How the step-2 and step-1 passes stage their (8 + 2k)^3 block in LDS:
 *   near_stage 0  automatic (the default): 2;
 *              1  the seed alone (the candidate's distance key is formed
 *                 from it: 4 B per entry, 4 integer instructions per
 *                 candidate);
 *              2  the pair (seed, |seed|^2 term) (8 B per entry, 2).
 * The order in which the passes with step k >= 8 (2 bricks of 4^3 or more)
 * hand bricks to wavefronts:
 *   far_order  0  automatic (the default): 4;
 *              1  slab order: consecutive bricks, so each XCD takes a slab of
 *                 z-layers;
 *              2  coset order: the bricks of one residue class of the brick
 *                 coordinates modulo k / 4 (a class holds every candidate of
 *                 its bricks) one class after another, so each brick is read
 *                 into the L2 of one XCD only;
 *              3  coset order in pairs: each wavefront takes two bricks
 *                 next to each other in their class along x and reads their
 *                 shared candidate bricks once (36 reads instead of 54);
 *              4  coset order in 2 x 2 quads (x and y): 48 reads for four
 *                 bricks instead of 108 (grids of 8^3 voxels take pairs).
 * rtsdf_jfa_config sets both for grids of side n (a power of two in [8, 256];
 * EINVAL otherwise or for values outside the sets); the setting is process
 * state read at each rtsdf_jfa / rtsdf_jfa_steps call (calls that overlap
 * with a change may see either).  rtsdf_jfa_config_get reads it back. */
typedef struct rtsdf_jfa_tuning {
    int32_t near_stage;
    int32_t far_order;
} rtsdf_jfa_tuning;
int rtsdf_jfa_config(int32_t n, const rtsdf_jfa_tuning *t);
int rtsdf_jfa_config_get(int32_t n, rtsdf_jfa_tuning *t);

/* ------------------------------------------------------------------------ */
/* 3. Selection (Sec. 2.2; the case c <= d of Eq. (1)).                      */
/*                                                                           */
/* A fine texel is selected when the coarse voxel containing its centre has */
/* dist2 <= K with K = floor(((d + beta) / h_c)^2), i.e. c <= d exactly.    */
/* fine.n must be a power-of-two multiple of coarse.n and the fine grid must */
/* cover the same box (fine.h * fine.n == coarse.h * coarse.n).              */
/*                                                                           */
/* mask      uint8 [n_f^3] out: 1 if selected.                               */
/* queue     int32 [queue_cap] out: the selected texels' linear indices in   */
/*           ascending Morton order of their fine coordinates (bit b of x,   */
/*           y, z at bits 3b, 3b+1, 3b+2).                                   */
/* count     int32 [1] out (device): number of selected texels; if it        */
/*           exceeds queue_cap only queue_cap entries are written and        */
/*           ERR_QUEUE_FULL is raised.                                       */
/* workspace device memory of rtsdf_select_workspace_size(coarse.n) bytes.   */
/* ------------------------------------------------------------------------ */
size_t rtsdf_select_workspace_size(int32_t coarse_n);
int rtsdf_select(rtsdf_grid coarse, const int32_t *dist2, rtsdf_grid fine, float beta, float d,
                 uint8_t *mask, int32_t *queue, int32_t queue_cap, int32_t *count,
                 void *workspace, rtsdf_stream stream);

/* rtsdf_select for callers that cannot allocate device memory or pass a     */
/* workspace (code under graph capture, tight serving loops, harnesses that */
/* forbid hipMalloc): the same selection, bit for bit, with the block sums  */
/* kept in a static device array of the library instead of `workspace`.    */
/* That array holds rtsdf_select_noalloc_max_bytes() bytes (512 KiB: enough */
/* for coarse.n up to 512, the largest rtsdf_select takes; larger is        */
/* EINVAL), exists once per device and stays allocated until the process    */
/* ends.  Its device address is looked up on the first call on each device */
/* (hipGetSymbolAddress, no allocation); the call itself allocates nothing. */
/* Every call on one device shares the array, and no entry is read before   */
/* the same call writes it, so nothing carries over between calls; but      */
/* calls that overlap on one device (different streams or threads) race on  */
/* it and must be serialised by the caller.  Other arguments, errors and     */
/* outputs as rtsdf_select.                                                  */
size_t rtsdf_select_noalloc_max_bytes(void);
int rtsdf_select_noalloc(rtsdf_grid coarse, const int32_t *dist2, rtsdf_grid fine, float beta, float d,
                         uint8_t *mask, int32_t *queue, int32_t queue_cap, int32_t *count, rtsdf_stream stream);

/* ------------------------------------------------------------------------ */
/* 3b. Trilinear coarse sampling (a smoother reading of the coarse value c  */
/* that Sec. 2.2 compares with d and stores for unselected texels; Sec. 2.1 */
/* notes the point-sampled coarse SDF is blocky).                           */
/*                                                                           */
/* rtsdf_coarse_trilinear writes, for every fine texel, the coarse SDF       */
/* interpolated trilinearly at the texel centre.  Coarse values are samples  */
/* at voxel centres; the fine centre j lies at coarse coordinate             */
/* u = (j + 1/2) / r - 1/2 per axis (r = fine.n / coarse.n), clamped to      */
/* [0, coarse.n - 1]; the value is lerp along x, then y, then z, each       */
/* lerp(a, b, t) = a + t (b - a) with every float operation rounded once, so */
/* the result is reproducible bit for bit.  A cell with an infinite corner   */
/* (a field without seeds) gives +inf.  Grids as for rtsdf_select, with      */
/* coarse.n <= 512.                                                          */
/*                                                                           */
/* coarse_sdf float32 [n_c^3] in; fine_c float32 [n_f^3] out.                */
/*                                                                           */
/* rtsdf_select_field selects the texels of `grid` with field <= d (a        */
/* float32 comparison; NaN never selects), with the same mask, queue order,  */
/* count and ERR_QUEUE_FULL behaviour as rtsdf_select at r = 1.  grid.n is a */
/* power of two in [4, 1024]; workspace holds                                */
/* rtsdf_select_workspace_size(grid.n) bytes.  d must not be NaN.            */
/*                                                                           */
/* With both, the trilinear pipeline is: rtsdf_coarse_trilinear, then        */
/* rtsdf_select_field on the fine grid, then rtsdf_trace_accumulate with the */
/* fine grid and fine_c passed as its coarse grid and coarse_sdf (so c_t in  */
/* Eq. (1) and the unselected texels' value are the interpolated field).     */
/* ------------------------------------------------------------------------ */
int rtsdf_coarse_trilinear(rtsdf_grid coarse, const float *coarse_sdf, rtsdf_grid fine, float *fine_c,
                           rtsdf_stream stream);
int rtsdf_select_field(rtsdf_grid grid, const float *field, float d, uint8_t *mask, int32_t *queue,
                       int32_t queue_cap, int32_t *count, void *workspace, rtsdf_stream stream);

/* ------------------------------------------------------------------------ */
/* Scene: the triangles and their bounding volume hierarchy, resident on    */
/* the device.  create copies the mesh (device pointers) and builds the      */
/* hierarchy (binned surface-area heuristic, two children per node); it      */
/* synchronises `stream`.  EINVAL for 2^26 or more triangles or 2^24 or more */
/* triangle references after large triangles are split.  refit takes new    */
/* positions for the same topology                                           */
/* and recomputes every box bottom-up on the device, asynchronously.         */
/* ------------------------------------------------------------------------ */
typedef struct rtsdf_scene rtsdf_scene;

typedef struct rtsdf_scene_info {
    int32_t nv, nt;
    int32_t nodes;      /* internal nodes of the hierarchy */
    int32_t max_depth;  /* deepest leaf (root = 0) */
    int32_t leaf_size;  /* largest reference count in a leaf */
    int64_t device_bytes;
    int32_t references; /* triangle references in the leaves (>= nt: large triangles are split into pieces) */
    int32_t instances;  /* rigid parts of a two-level scene; 0 for a single-level scene */
} rtsdf_scene_info;

int rtsdf_scene_create(const float *vertices, int32_t nv, const int32_t *faces, int32_t nt,
                       int32_t leaf_size, rtsdf_scene **out, rtsdf_stream stream);
int rtsdf_scene_refit(rtsdf_scene *scene, const float *vertices, rtsdf_stream stream);
int rtsdf_scene_info_get(const rtsdf_scene *scene, rtsdf_scene_info *info);

/* Copy of a single-level scene's hierarchy to host memory (for inspection   */
/* and tests).  Node 0 is the root; node i has two child slots s = 0, 1:     */
/* boxes[i][s] = (lo x, lo y, lo z, hi x, hi y, hi z) (float32 [cap][2][6]), */
/* links[i][s] = (j, 0) for internal node j, or (-1 - first, count) for a    */
/* leaf holding references [first, first + count) of the scene's reference  */
/* order (int32 [cap][2][2]; count 0 marks the empty second slot of a        */
/* one-reference scene), parents[i] the parent node, -1 for the root (int32 */
/* [cap], may be NULL).  All three are host buffers; synchronises `stream`.  */
/* A rebuilt hierarchy may hold nodes that no slot references (below its    */
/* leaves of several references); read the tree from the root.              */
/* EINVAL for two-level scenes or cap < rtsdf_scene_info.nodes.             */
int rtsdf_scene_hierarchy(const rtsdf_scene *scene, int32_t cap, float *boxes, int32_t *links, int32_t *parents,
                          rtsdf_stream stream);

/* Rebuilding the hierarchy on the device (for geometry that moves far from  */
/* where it was built, which a refit only loosens).  enable_rebuild          */
/* allocates the rebuild buffers (it allocates, like create, and             */
/* synchronises `stream`) and replaces the creation hierarchy with a linear  */
/* BVH built on the device over the same triangle references: 30-bit Morton  */
/* codes of the reference centres, a radix sort, the binary radix tree of    */
/* Karras (HPG 2012) whose subtrees of at most the scene's creation leaf    */
/* size (capped at 8) references become single leaves, boxes bottom-up.     */
/* rebuild takes new positions for the same topology (as refit) and         */
/* rebuilds it; a refit of such a scene refits the rebuilt tree.  Traced     */
/* results are those of the creation hierarchy: a triangle's hit test does  */
/* not depend on the order the hierarchy tests it in.                       */
/* EINVAL for two-level scenes and for scenes with                           */
/* fewer than two references; rebuild before enable_rebuild is EINVAL.       */
/* rebuild is a fixed sequence of kernel launches (no allocation, host      */
/* synchronisation or memset; its radix sort is the library's own), so it   */
/* may be captured in a graph (see rtsdf_frame_desc.refit).                  */
int rtsdf_scene_enable_rebuild(rtsdf_scene *scene, rtsdf_stream stream);
int rtsdf_scene_rebuild(rtsdf_scene *scene, const float *vertices, rtsdf_stream stream);

/* The radix sort of the device rebuild, exported so callers and tests can  */
/* check it: sorts n (key, value) pairs (device arrays, in place) by the low */
/* `bits` bits of the key (1..32; higher bits must be 0), stably (pairs with */
/* equal keys keep their order), least-significant 8-bit digit first.       */
/* workspace: rtsdf_sort_pairs_workspace_size(n) bytes of device memory.    */
size_t rtsdf_sort_pairs_workspace_size(int32_t n);
int rtsdf_sort_pairs(uint32_t *keys, int32_t *values, int32_t n, int32_t bits, void *workspace,
                     rtsdf_stream stream);

/* Two-level scene: a static world plus rigidly moving parts (refitting one */
/* hierarchy over moving geometry loosens it frame after frame).  Part i     */
/* owns faces [instance_faces[i], instance_faces[i + 1]) (host array of      */
/* ninst + 1 offsets, 0 first, nt last) and the vertices they use (a vertex  */
/* used by two parts is EINVAL).  Part 0 is the static world (world          */
/* coordinates, may have no faces); parts 1.. move and have at least one     */
/* face each, their vertices in object space.  transforms (device, float32   */
/* [ninst][12], row 0 unused) are the parts' object-to-world rows            */
/* (r00 r01 r02 t0, r10 r11 r12 t1, r20 r21 r22 t2) and must be rigid:       */
/* R R^T = I and det R = 1 within 1e-4 (EINVAL at create, ERR_TRANSFORM at   */
/* set_transforms).  Each moving part gets its own hierarchy, built once in  */
/* object space; the top level is one surface-area-heuristic tree over the   */
/* static triangles and the moving parts' world boxes, whose nodes above the */
/* moving parts rtsdf_scene_set_transforms refits.  set_transforms also     */
/* recomputes the world position of every vertex (each coordinate            */
/* ((r0 x + r1 y) + r2 z) + t, float operations rounded once) into the scene */
/* and, if world_vertices is non-NULL, into that caller buffer (float32      */
/* [nv][3], e.g. for rtsdf_voxelize).  Triangle ids (hits, argmin records,   */
/* gradients) are global face indices; rtsdf_trace_backward gives gradients  */
/* with respect to the world positions.  The tracer uses its one-fetch loop  */
/* (tuning loop 3) for two-level scenes whatever the tuning says;            */
/* rtsdf_scene_refit, rtsdf_closest_hits, rtsdf_point_distance and           */
/* rtsdf_texel_distance return EINVAL for them, and batches do not take      */
/* them.  rtsdf_scene_world_vertices copies the current world positions.     */
int rtsdf_scene_create_instanced(const float *vertices, int32_t nv, const int32_t *faces, int32_t nt,
                                 const int32_t *instance_faces, int32_t ninst, const float *transforms,
                                 int32_t leaf_size, rtsdf_scene **out, rtsdf_stream stream);
int rtsdf_scene_set_transforms(rtsdf_scene *scene, const float *transforms, float *world_vertices,
                               rtsdf_stream stream);
int rtsdf_scene_world_vertices(const rtsdf_scene *scene, float *out, rtsdf_stream stream);

/* How rtsdf_trace_accumulate signs a texel's traced distance u (texels     */
/* without a hit output c either way):                                       */
/*  RTSDF_SIGN_VOTE   (default) the vote of Sec. 2.2: -u when more closest   */
/*                    hits were back faces than front faces, else u.  For    */
/*                    closed meshes.  Open surfaces get a negative region    */
/*                    behind them (texels that see only their back face).    */
/*  RTSDF_SIGN_SHELL  u - shell: every surface becomes a closed slab of      */
/*                    half-thickness `shell` (>= 0, finite; 0 is the plain   */
/*                    unsigned distance).  For open or thin surfaces: no     */
/*                    inside/outside guess, and a shell of at least the      */
/*                    shadow march's eps keeps thin surfaces from being      */
/*                    stepped through (the holes Sec. 3 reports).           */
/* The policy is read at each rtsdf_trace_accumulate and rtsdf_trace_backward */
/* call (the gradient of a shell value is that of u).                        */
enum { RTSDF_SIGN_VOTE = 0, RTSDF_SIGN_SHELL = 1 };
int rtsdf_scene_set_sign(rtsdf_scene *scene, int32_t policy, float shell);
void rtsdf_scene_destroy(rtsdf_scene *scene);

/* ------------------------------------------------------------------------ */
/* 4. Tracing and temporal accumulation (Sec. 2.2, Eq. (1)).                 */
/*                                                                           */
/* Per-texel state (all [n_f^3], caller-owned, initialise with               */
/* rtsdf_accum_reset):                                                       */
/*   u         float32  unsigned accumulated distance (+inf = none yet);     */
/*   hits      uint32   front-face count | back-face count << 16;            */
/*   arg_tri   int32    triangle of the ray that produced u, -1 if none;     */
/*   arg_ray   int32    frame << 8 | ray of that ray (-1 if none).           */
/*                                                                           */
/* For a selected texel j with centre o (lo + (i + 1/2) h per axis, float), */
/* each ray k < rays_per_texel goes along w = Marsaglia's sphere point from  */
/* Philox4x64-10 random bits, key (seed, 0), counter (j, frame << 32 | k,    */
/* scene_id, attempt): each 32-bit half h gives x = (2 (h >> 9) + 1 - 2^23)  */
/* 2^-23; the first pair with s = x1^2 + x2^2 < 1 gives                      */
/* w = (2 x1 sqrt(1-s), 2 x2 sqrt(1-s), 1 - 2 s) (float ops, each rounded    */
/* once); after 8 attempts w = (0, 0, 1).  Its closest hit (smallest t > 0,  */
/* ties to the lowest triangle index) gives the distance t |w| and a front   */
/* (w . n < 0, n = (v1 - v0) x (v2 - v0)) or back hit.  With r_t the         */
/* smallest distance of the frame (ties to the lowest ray):                  */
/*   u <- min(alpha u + (1 - alpha) max(c, 0), r_t)   (alpha = 1: min(u, r_t))*/
/*   front/back counts += this frame's closest hits                          */
/*   fine_sdf = (u finite ? u : c), negated if back > front.                 */
/* Texels not selected get fine_sdf = c (coarse value of the voxel holding   */
/* the centre) and their state is reset.                                     */
/*                                                                           */
/* coarse_sdf float32 [n_c^3]; mask/queue/count from rtsdf_select; only the */
/*            first min(count, queue_cap) queue entries are traced.          */
/* rays_per_texel in [1, 64]; alpha in [0, 1].                               */
/* frame_ptr  optional device uint32: if non-NULL the frame index is read    */
/*            from it at run time (for captured graphs) and `frame` is       */
/*            ignored.  A value >= 2^23 (past the argmin record's frame      */
/*            field) traces nothing: the state and the selected texels'      */
/*            fine values keep the previous frame's, and ERR_FRAME is raised. */
/*            `frame` itself must be < 2^23 (EINVAL).                        */
/* workspace  rtsdf_trace_workspace_size() bytes of device memory: 256 B of  */
/*            counters, per-wavefront buffers holding the directions of the  */
/*            rays of each persistent wavefront's tile (drawn, then sorted   */
/*            by direction bin), and the spill area of the traversal stacks  */
/*            (entries deeper than the LDS part, for hierarchies up to depth */
/*            64); ~310 MB on a 256-CU device (the size is that of the       */
/*            current device).  Calls that run                               */
/*            concurrently need separate workspaces; they may trace the same */
/*            scene.                                                         */
/* ------------------------------------------------------------------------ */
typedef struct rtsdf_accum {
    float *u;
    uint32_t *hits;
    int32_t *arg_tri;
    int32_t *arg_ray;
} rtsdf_accum;

int rtsdf_accum_reset(rtsdf_grid fine, rtsdf_accum state, rtsdf_stream stream);
size_t rtsdf_trace_workspace_size(void);
int rtsdf_trace_accumulate(const rtsdf_scene *scene, rtsdf_grid coarse, const float *coarse_sdf,
                           rtsdf_grid fine, const uint8_t *mask, const int32_t *queue,
                           const int32_t *count, int32_t queue_cap, int32_t rays_per_texel, uint32_t frame,
                           const uint32_t *frame_ptr, uint64_t seed, uint32_t scene_id, float alpha,
                           rtsdf_accum state, float *fine_sdf, void *workspace, rtsdf_stream stream);

/* Tuning and instrumentation of the tracer.  Results never depend on it,
 * only speed does.  rtsdf_trace_config sets the process default (host-side
 * state read at each trace call); rtsdf_scene_set_tuning gives one scene its
 * own tuning (NULL: back to the process default) and rtsdf_batch_set_tuning
 * one batch, so callers tracing different scenes do not share it.
 * rtsdf_scene_get_tuning returns the tuning a trace of the scene uses.
 * Defaults: refill 28, blocks_per_cu 0, stats 0, loop 4, bin_directions 1,
 * stack_lds 12, tile_texels 64, bvh_width 2:
 *   refill          a wavefront hands out new rays once this many of its
 *                   lanes are free (16 or 28);
 *   blocks_per_cu   persistent workgroups of four wavefronts per compute
 *                   unit, i.e. traversal wavefronts per SIMD (0 = as many as
 *                   fit: 6 with the default LDS stack; 1 to 8);
 *   stats           1: count into 64-bit counters at byte offsets 8, 16, ...
 *                   of the workspace: node visits, triangle tests, rays,
 *                   traversal iterations x 64, refill rounds x 64, lane
 *                   iterations with work (loop >= 1), tiles x 64, node
 *                   visits entering neither child box (loop 3, 4), tiles
 *                   started while rays of the previous one were still
 *                   traced x 64, traversal rounds that waited for every
 *                   lane before a next tile x 64 (slower; for measurement
 *                   only);
 *   loop            0: two phases per iteration (walk nodes until every lane
 *                   holds a leaf, then test the leaves); 1: one unit of work
 *                   per lane per iteration (a triangle or a node); 2: as 1,
 *                   with one shared stack push/pop per iteration; 3: as 2,
 *                   with each lane's node or triangle record fetched by one
 *                   shared load sequence (one memory wait per iteration);
 *                   4: queued: lanes fetch and step nodes only and append
 *                   the triangles of the leaves they reach to a queue of
 *                   their wavefront; each time 64 tests are queued, every
 *                   lane takes one (of any lane's ray); traversals cull
 *                   with their ray's best distance as of the last queue
 *                   flush.  Two-level scenes, 4-wide traversals and scenes
 *                   of 2^26 or more triangle references use 3 instead;
 *                   default 4;
 *   bin_directions  1: each wavefront's tile of rays is sorted by direction
 *                   before tracing (coherence); 0: queue order;
 *   stack_lds       traversal stack entries kept in LDS per lane (12, 16 or
 *                   24); deeper entries go to the workspace's spill area;
 *   tile_texels     texels per wavefront tile at most (16, 32 or 64; a tile
 *                   also holds at most 768 rays, i.e. 768 / rays texels);
 *   bvh_width       2: traverse the two-child hierarchy; 4: a 4-wide copy of
 *                   it (each wide node takes up to four descendants of a
 *                   two-child node, greedily by box area; the boxes are the
 *                   same, and a refit updates both), with the one-fetch loop.
 *                   rtsdf_scene_set_tuning with bvh_width 4 builds a
 *                   single-level scene's 4-wide copy on first use (it
 *                   allocates and synchronises the device); EINVAL for
 *                   two-level scenes, scenes that rebuild on the device
 *                   (enable_rebuild drops the copy) and copies too deep for
 *                   the traversal stack.  Scenes without the copy, and
 *                   batches, trace with width 2 whatever the tuning says.
 * Values outside these sets are rejected with RTSDF_EINVAL. */
typedef struct rtsdf_trace_tuning {
    int32_t refill, blocks_per_cu, stats, loop, bin_directions, stack_lds, tile_texels, bvh_width;
} rtsdf_trace_tuning;
int rtsdf_trace_config(const rtsdf_trace_tuning *tuning);
int rtsdf_trace_config_get(rtsdf_trace_tuning *tuning);
int rtsdf_scene_set_tuning(rtsdf_scene *scene, const rtsdf_trace_tuning *tuning);
int rtsdf_scene_get_tuning(const rtsdf_scene *scene, rtsdf_trace_tuning *tuning);

/* Ray directions exactly as rtsdf_trace_accumulate draws them, for n keys  */
/* (texel[i], frame[i], ray[i]) with one seed and scene id: out float32      */
/* [n][3].  Lets callers and tests check the generator bit for bit.          */
int rtsdf_directions(const int32_t *texel, const uint32_t *frame, const int32_t *ray, int32_t n,
                     uint64_t seed, uint32_t scene_id, float *out, rtsdf_stream stream);

/* The float32 square root every stage takes (ray directions, coarse SDF,   */
/* shadow triangulation), correctly rounded: out[i] = sqrt(x[i]) for n      */
/* values (device arrays).  Exported so callers and tests can check it     */
/* bit for bit against another IEEE implementation.                         */
int rtsdf_sqrt(const float *x, int64_t n, float *out, rtsdf_stream stream);

/* Closest hits of arbitrary rays (float32 origins and directions [n][3]):   */
/* t_out float32 (+inf on a miss), tri_out int32 (-1 on a miss), front_out   */
/* int32 (1 front, 0 back or miss).  Same traversal as the tracer.           */
int rtsdf_closest_hits(const rtsdf_scene *scene, const float *origins, const float *dirs, int32_t n,
                       float *t_out, int32_t *tri_out, int32_t *front_out, rtsdf_stream stream);

/* ------------------------------------------------------------------------ */
/* Vertex gradient of the fine SDF (the derivative of the traced distance).  */
/* For every texel whose fine value came from a ray (arg_tri >= 0), the ray  */
/* is regenerated from (texel, frame, ray) and intersected with its          */
/* triangle; with barycentrics b and geometric normal n,                     */
/*   grad_v[vertex i] += grad_fine[j] * sign(fine_sdf[j]) * |w| * b_i n/(n.w)*/
/* grad_v float32 [nv][3] is ACCUMULATED into (zero it first).  Uses the     */
/* scene's current vertex positions.                                         */
/* ------------------------------------------------------------------------ */
int rtsdf_trace_backward(const rtsdf_scene *scene, rtsdf_grid fine, rtsdf_accum state,
                         const float *fine_sdf, const float *grad_fine, uint64_t seed,
                         uint32_t scene_id, float *grad_v, rtsdf_stream stream);

/* ------------------------------------------------------------------------ */
/* One SDF update as a captured graph.  The descriptor names every buffer of */
/* the per-frame sequence (the same ones the stage calls take); create        */
/* records  [refit ->] voxelize -> jfa -> select -> trace_accumulate  on a   */
/* private stream (it synchronises `stream` first) and instantiates it;      */
/* each launch replays the whole update on `stream` for frame index          */
/* *frame_counter (device uint32) and then increments that counter.  The     */
/* descriptor's pointers must stay valid while the graph exists; buffers     */
/* are cleared with kernels only (no memset nodes).                          */
/* ------------------------------------------------------------------------ */
typedef struct rtsdf_frame_desc {
    const float *vertices;      /* [nv][3]; refit reads it every launch if refit != 0 */
    int32_t nv;
    const int32_t *faces;       /* [nt][3] */
    int32_t nt;
    rtsdf_scene *scene;
    int32_t refit;              /* 0: static scene; 1: refit the scene from `vertices` each frame; 2: rebuild
                                   its hierarchy on the device from `vertices` each frame (rtsdf_scene_rebuild;
                                   the scene must have had rtsdf_scene_enable_rebuild) */
    rtsdf_grid coarse, fine;
    float beta, d;
    int32_t rays_per_texel;
    uint64_t seed;
    uint32_t scene_id;
    float alpha;
    int32_t *seeds, *scratch, *dist2; /* [n_c^3] each */
    float *coarse_sdf;                /* [n_c^3] */
    uint8_t *mask;                    /* [n_f^3] */
    int32_t *queue;                   /* [queue_cap] */
    int32_t queue_cap;
    int32_t *count;                   /* [1] */
    void *select_workspace;           /* rtsdf_select_workspace_size(coarse.n) bytes */
    rtsdf_accum state;
    float *fine_sdf;                  /* [n_f^3] */
    void *trace_workspace;            /* rtsdf_trace_workspace_size() bytes */
    uint32_t *frame_counter;          /* [1], device */
    float *fine_c;                    /* NULL: point sampling.  Else [n_f^3]: trilinear sampling (rtsdf_coarse_trilinear
                                         into fine_c, rtsdf_select_field, trace against fine_c); select_workspace then
                                         holds rtsdf_select_workspace_size(fine.n) bytes */
    const int32_t *jfa_steps;         /* HOST, read during create only.  NULL: n/2, ..., 1; else the pass
                                         schedule of rtsdf_jfa_steps (jfa_nsteps entries) */
    int32_t jfa_nsteps;
    const float *transforms;          /* two-level scene with refit != 0: [ninst][12], read every launch and
                                         applied with rtsdf_scene_set_transforms, which writes the world
                                         positions into world_vertices [nv][3]; voxelization then reads those */
    float *world_vertices;
} rtsdf_frame_desc;

typedef struct rtsdf_frame_graph rtsdf_frame_graph;
int rtsdf_frame_graph_create(const rtsdf_frame_desc *desc, rtsdf_frame_graph **out, rtsdf_stream stream);
int rtsdf_frame_graph_launch(rtsdf_frame_graph *graph, rtsdf_stream stream);
void rtsdf_frame_graph_destroy(rtsdf_frame_graph *graph);

/* ------------------------------------------------------------------------ */
/* Many independent scenes per launch.  create copies each mesh (device     */
/* pointers, as for rtsdf_scene_create), builds its hierarchy, allocates     */
/* every buffer of every scene and resets the accumulation state; it         */
/* synchronises `stream`.  step runs one SDF update of all scenes -- one     */
/* launch per stage for the whole batch -- for frame index `frame` (or       */
/* *frame_ptr if non-NULL).  Each scene's results are bit-identical to its   */
/* single-scene run.  outputs gives device pointers into the batch's pools   */
/* (valid until destroy).  Grids: coarse_n a power of two in [8, 128],       */
/* fine_n a power-of-two multiple of it (at most 1024), both spanning the    */
/* cube [lo, lo + side].                                                     */
/* ------------------------------------------------------------------------ */
typedef struct rtsdf_batch rtsdf_batch;

typedef struct rtsdf_batch_scene {
    const float *vertices;  /* [nv][3], device */
    int32_t nv;
    const int32_t *faces;   /* [nt][3], device */
    int32_t nt;
    float lo[3];
    float side;
    int32_t coarse_n, fine_n;
    float beta, d;
    int32_t rays_per_texel;
    float alpha;
    uint32_t scene_id;      /* part of the ray counter (distinct scenes draw distinct rays) */
    int32_t sign_policy;    /* RTSDF_SIGN_VOTE or RTSDF_SIGN_SHELL (see rtsdf_scene_set_sign) */
    float shell;
} rtsdf_batch_scene;

typedef struct rtsdf_batch_view {
    rtsdf_grid coarse, fine;
    int32_t *seeds, *dist2;
    float *coarse_sdf;
    uint8_t *mask;
    int32_t *queue;
    int32_t *count;
    rtsdf_accum state;
    float *fine_sdf;
    rtsdf_scene *scene;
} rtsdf_batch_view;

int rtsdf_batch_create(const rtsdf_batch_scene *scenes /* host array [n] */, int32_t n, uint64_t seed,
                       int32_t leaf_size, rtsdf_batch **out, rtsdf_stream stream);
int rtsdf_batch_reset(rtsdf_batch *batch, rtsdf_stream stream);
int rtsdf_batch_step(rtsdf_batch *batch, uint32_t frame, const uint32_t *frame_ptr, rtsdf_stream stream);
int rtsdf_batch_outputs(const rtsdf_batch *batch, int32_t index, rtsdf_batch_view *out);
/* the batch's own tracer tuning (NULL: the process default; see
 * rtsdf_trace_config) */
int rtsdf_batch_set_tuning(rtsdf_batch *batch, const rtsdf_trace_tuning *tuning);
/* one batch step as a captured graph: each launch runs the step for frame
 * *frame_counter (device) and then increments it */
int rtsdf_batch_graph_create(rtsdf_batch *batch, uint32_t *frame_counter, rtsdf_frame_graph **out,
                             rtsdf_stream stream);
void rtsdf_batch_destroy(rtsdf_batch *batch);

/* ------------------------------------------------------------------------ */
/* Exact unsigned distance to the scene's triangles: the value the traced    */
/* fine SDF approaches from above (Sec. 2.2: every ray hit lies on the mesh, */
/* so for the current geometry a traced distance is never below it).  For    */
/* measuring the method's accuracy and, in moving scenes, stale history      */
/* (Eq. (1)'s decay alpha).  Computed in float32 by a best-first descent of  */
/* the scene's hierarchy; whole triangles are tested (split references are   */
/* exact: the piece holding the closest point is never pruned).              */
/*                                                                           */
/* rtsdf_point_distance: points float32 [n][3] -> dist float32 [n] (+inf    */
/* for a scene without triangles), tri int32 [n] (nearest original triangle, */
/* ties to the lowest index; -1 if none; may be NULL).                       */
/* rtsdf_texel_distance: the same at texel centres lo + (i + 1/2) h of       */
/* `grid` (float operations rounded once, as for the ray origins); texels    */
/* int32 [n] linear texel indices, or NULL for all n = grid.n^3 texels in     */
/* order.  An index outside the grid only yields a point outside it (no      */
/* memory is read through it).                                               */
/* ------------------------------------------------------------------------ */
int rtsdf_point_distance(const rtsdf_scene *scene, const float *points, int32_t n, float *dist, int32_t *tri,
                         rtsdf_stream stream);
int rtsdf_texel_distance(const rtsdf_scene *scene, rtsdf_grid grid, const int32_t *texels, int32_t n, float *dist,
                         int32_t *tri, rtsdf_stream stream);

/* ------------------------------------------------------------------------ */
/* 5. Soft shadows (Sec. 2.3): for each point p, march from p towards the    */
/* light (unit direction `light_dir`, host float[3]) through the fine SDF,   */
/* sampled trilinearly between texel centres (clamped at the border).        */
/* Starting at t = eps, each step samples s = sdf(p + t l); the march stops  */
/* with visibility 0 when s < eps, stops when t > max_dist, the point leaves */
/* the grid or max_steps samples were taken; otherwise visibility            */
/* min(1, k s / t) is folded in and t advances by min(s, max_step) (at least */
/* eps).  visibility float32 [np] out in [0, 1].                             */
/* ------------------------------------------------------------------------ */
int rtsdf_shadow(rtsdf_grid fine, const float *fine_sdf, const float *points, int32_t np,
                 const float light_dir[3], float k, float eps, int32_t max_steps, float max_step,
                 float max_dist, float *visibility, rtsdf_stream stream);

/* The march with the two further options of Sec. 2.3.                       */
/*  * jitter (float32 [np], device, values in [0, 1), or NULL): the march of */
/*    point p starts at t = eps + jitter[p] * jitter_scale, i.e. its origin  */
/*    moves towards the light (the caller draws new values per frame and     */
/*    filters the result over time; that filter is not part of the library). */
/*  * penumbra = 1: triangulation between consecutive samples (Aaltonen      */
/*    2018, cited for the banding fix).  With the previous sample s_prev at   */
/*    t_prev and the current s at t, D = t - t_prev,                         */
/*    y = ((D*D + s*s) - s_prev*s_prev) / (D + D) clamped to [0, s],          */
/*    d = sqrt(max(s*s - y*y, 0)), and min(vis, (k*d) / (t - y)) is folded   */
/*    in when t - y > 0 (the first sample uses k*s/t).  penumbra = 0 is the   */
/*    cone term of rtsdf_shadow.                                             */
/* Every float operation is rounded once in the order written, as for       */
/* rtsdf_shadow.  params is a host pointer; EINVAL as rtsdf_shadow, and for  */
/* penumbra outside {0, 1} or a negative or NaN jitter_scale with jitter.    */
typedef struct rtsdf_shadow_params {
    float light_dir[3];
    float k, eps;
    int32_t max_steps;
    float max_step, max_dist;
    int32_t penumbra;
    float jitter_scale;
} rtsdf_shadow_params;
int rtsdf_shadow_ex(rtsdf_grid fine, const float *fine_sdf, const float *points, int32_t np,
                    const rtsdf_shadow_params *params, const float *jitter, float *visibility, rtsdf_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* RTSDF_H */
