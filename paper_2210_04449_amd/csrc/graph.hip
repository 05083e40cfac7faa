// One SDF update as a captured HIP graph.
//
// The whole per-frame sequence (optional refit of the scene from the vertex
// buffer, voxelize, jump flooding, selection, tracing with temporal
// accumulation) is recorded once on a private capture stream and replayed
// with a single hipGraphLaunch.  The frame index lives in device memory: the
// tracer reads it through its frame pointer and a one-thread kernel at the end
// of the graph advances it, so replays need no host-side parameter updates.
// Only kernels are recorded (buffers are cleared with fill kernels, never
// with memset nodes).
#include "common.hpp"

struct rtsdf_frame_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    rtsdf_frame_desc desc{};
    rtsdf_batch *batch = nullptr;      // batch graphs
    uint32_t *batch_frame = nullptr;
};

namespace rtsdf {

__global__ void advance_frame(uint32_t *frame) { *frame += 1u; }

static int record_frame(const rtsdf_frame_graph &G, hipStream_t s)
{
    if (G.batch) {
        const int rc = rtsdf_batch_step(G.batch, 0, G.batch_frame, s);
        if (rc != RTSDF_OK) return rc;
        advance_frame<<<dim3(1), dim3(1), 0, s>>>(G.batch_frame);
        RTSDF_CHECK_LAUNCH();
        return RTSDF_OK;
    }
    const rtsdf_frame_desc &D = G.desc;
    int rc;
    const float *verts = D.vertices;
    if (D.refit && D.transforms) {  // a two-level scene moves its parts
        rc = rtsdf_scene_set_transforms(D.scene, D.transforms, D.world_vertices, s);
        if (rc != RTSDF_OK) return rc;
        verts = D.world_vertices;
    } else if (D.refit == 2) {
        rc = rtsdf_scene_rebuild(D.scene, D.vertices, s);
        if (rc != RTSDF_OK) return rc;
    } else if (D.refit) {
        rc = rtsdf_scene_refit(D.scene, D.vertices, s);
        if (rc != RTSDF_OK) return rc;
    }
    rc = rtsdf_voxelize(verts, D.nv, D.faces, D.nt, D.coarse, D.seeds, s);
    if (rc != RTSDF_OK) return rc;
    rc = D.jfa_steps ? rtsdf_jfa_steps(D.coarse, D.seeds, D.scratch, D.jfa_steps, D.jfa_nsteps, D.beta, D.dist2,
                                       D.coarse_sdf, s)
                     : rtsdf_jfa(D.coarse, D.seeds, D.scratch, D.beta, D.dist2, D.coarse_sdf, s);
    if (rc != RTSDF_OK) return rc;
    // point sampling reads the containing coarse voxel; trilinear sampling
    // interpolates the coarse field at the fine centres and then works on the
    // fine grid alone
    rtsdf_grid cgrid = D.coarse;
    const float *cfield = D.coarse_sdf;
    if (D.fine_c) {
        rc = rtsdf_coarse_trilinear(D.coarse, D.coarse_sdf, D.fine, D.fine_c, s);
        if (rc != RTSDF_OK) return rc;
        rc = rtsdf_select_field(D.fine, D.fine_c, D.d, D.mask, D.queue, D.queue_cap, D.count, D.select_workspace, s);
        cgrid = D.fine;
        cfield = D.fine_c;
    } else {
        rc = rtsdf_select(D.coarse, D.dist2, D.fine, D.beta, D.d, D.mask, D.queue, D.queue_cap, D.count,
                          D.select_workspace, s);
    }
    if (rc != RTSDF_OK) return rc;
    rc = rtsdf_trace_accumulate(D.scene, cgrid, cfield, D.fine, D.mask, D.queue, D.count, D.queue_cap,
                                D.rays_per_texel, 0, D.frame_counter, D.seed, D.scene_id, D.alpha, D.state, D.fine_sdf,
                                D.trace_workspace, s);
    if (rc != RTSDF_OK) return rc;
    advance_frame<<<dim3(1), dim3(1), 0, s>>>(D.frame_counter);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

}  // namespace rtsdf

static int capture_graph(rtsdf_frame_graph *g, rtsdf_stream stream)
{
    using namespace rtsdf;
    hipStream_t cs = nullptr;
    RTSDF_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    // order the capture after whatever the caller queued before
    if (hipStreamSynchronize(as_stream(stream)) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return RTSDF_EHIP;
    }
    int rc = RTSDF_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = RTSDF_EHIP;
    } else {
        rc = record_frame(*g, cs);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        if (rc == RTSDF_OK && e != hipSuccess) rc = RTSDF_EHIP;
        g->graph = graph;
        if (rc == RTSDF_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
            rc = RTSDF_EHIP;
    }
    (void)hipStreamDestroy(cs);
    return rc;
}

extern "C" int rtsdf_frame_graph_create(const rtsdf_frame_desc *desc, rtsdf_frame_graph **out, rtsdf_stream stream)
{
    if (!desc || !out || !desc->frame_counter || !desc->scene) return RTSDF_EINVAL;
    if (desc->refit && desc->transforms && !desc->world_vertices) return RTSDF_EINVAL;
    if (desc->refit < 0 || desc->refit > 2 || (desc->refit == 2 && desc->transforms)) return RTSDF_EINVAL;
    *out = nullptr;
    auto *g = new rtsdf_frame_graph();
    g->desc = *desc;
    const int rc = capture_graph(g, stream);
    g->desc.jfa_steps = nullptr;  // the caller's host schedule is valid during this call only
    if (rc != RTSDF_OK) {
        rtsdf_frame_graph_destroy(g);
        return rc;
    }
    *out = g;
    return RTSDF_OK;
}

extern "C" int rtsdf_batch_graph_create(rtsdf_batch *batch, uint32_t *frame_counter, rtsdf_frame_graph **out,
                                        rtsdf_stream stream)
{
    if (!batch || !frame_counter || !out) return RTSDF_EINVAL;
    *out = nullptr;
    auto *g = new rtsdf_frame_graph();
    g->batch = batch;
    g->batch_frame = frame_counter;
    const int rc = capture_graph(g, stream);
    if (rc != RTSDF_OK) {
        rtsdf_frame_graph_destroy(g);
        return rc;
    }
    *out = g;
    return RTSDF_OK;
}

extern "C" int rtsdf_frame_graph_launch(rtsdf_frame_graph *g, rtsdf_stream stream)
{
    if (!g || !g->exec) return RTSDF_EINVAL;
    if (hipGraphLaunch(g->exec, rtsdf::as_stream(stream)) != hipSuccess) return RTSDF_EHIP;
    return RTSDF_OK;
}

extern "C" void rtsdf_frame_graph_destroy(rtsdf_frame_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}
