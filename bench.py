#!/usr/bin/env python
"""Benchmark of one SDF update (voxelize + jump flooding + selection + ray
tracing with temporal accumulation) on one MI355X.

Workload (default): the room-scale scene -- an axis-aligned room plus 300
random boxes, icospheres and tori (~216k triangles, fp32) -- with a 128^3
coarse grid and a 256^3 fine grid, beta = 0.5 and d = 3 coarse voxels, and 16
rays per selected texel per frame.  Inputs are seeded and synthetic and resident
in HBM before timing; the hierarchy is built once before timing (static scene).

Prints one JSON line: ms per update (the metric), per-stage times, fine-texel
rays/s, the jump-flooding effective HBM bandwidth, the roofline of the
dominant kernel (the tracer) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per SDF update (JFA+trace) at 128³/256³; fine-texel rays/s; JFA HBM GB/s"

# Peaks of one MI355X (gfx950): 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz issue
# 39.3e12 non-packed 32-bit VALU lane operations per second; HBM3E 8 TB/s.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0

# Algorithmic VALU lane-operations of the tracer per unit of work:
OPS_NODE = 39   # one two-child node: 2 x (6 slab FMAs + 12 min/max + 1 compare) + ordering
OPS_NODE4 = 103  # one 4-wide node: 4 x 19.5 (the same slab test per child) + a 5-comparator sort (5 x 5)
OPS_TRI = 33    # triangle-frame test: 18 FMAs (plane + 2 barycentric rows), 1/q, t, 2 barycentrics, margin, compares
OPS_RAY = 360   # Philox4x64-10 (10 rounds), Marsaglia mapping, ray set-up, accumulation


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="room", choices=["room", "tiny", "diff", "dynamic", "batched"])
    ap.add_argument("--graph", type=int, default=1, choices=[0, 1],
                    help="also time the whole update as one captured HIP graph")
    ap.add_argument("--autotune", action="store_true", help="pick the tracer tuning by measurement first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--refill", type=int, default=28, choices=[16, 28])
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--loop", type=int, default=4, choices=[0, 1, 2, 3, 4])
    ap.add_argument("--bin", type=int, default=1, choices=[0, 1])
    ap.add_argument("--stack-lds", type=int, default=12, choices=[12, 16, 24])
    ap.add_argument("--tile-texels", type=int, default=64, choices=[16, 32, 64])
    ap.add_argument("--bvh-width", type=int, default=2, choices=[2, 4],
                    help="trace the two-child hierarchy or its 4-wide copy (static and refitted scenes)")
    ap.add_argument("--leaf-size", type=int, default=4)
    ap.add_argument("--jfa", default="jfa", choices=["jfa", "jfa+1", "jfa+2", "1+jfa"],
                    help="jump-flooding pass schedule (the extra-pass variants reduce its errors)")
    ap.add_argument("--study", default=None, choices=["alpha", "refit", "motion"],
                    help="instead of the benchmark: decay alpha against stale history on the moving scene, or one "
                         "refitted hierarchy against a two-level scene over a continuous animation")
    ap.add_argument("--alphas", type=float, nargs="+", default=[1.0, 0.95, 0.9, 0.75, 0.5])
    ap.add_argument("--study-frames", type=int, default=24)
    ap.add_argument("--alpha", type=float, default=None, help="override the workload's decay alpha")
    ap.add_argument("--refit", action="store_true",
                    help="dynamic workload: refit the hierarchy every update instead of rebuilding it on the device "
                         "(the default for moving geometry)")
    ap.add_argument("--device-build", action="store_true",
                    help="build the hierarchy on the device (as moving scenes do) also for a static scene")
    ap.add_argument("--parts", action="store_true",
                    help="dynamic workload as a two-level scene of rigid parts instead of one refitted hierarchy")
    ap.add_argument("--no-shadow", action="store_true", help="skip timing the soft-shadow consumer")
    ap.add_argument("--no-extras", action="store_true",
                    help="room workload: skip the batched and differentiable comparison records")
    ap.add_argument("--sampling", default="point", choices=["point", "trilinear"],
                    help="how a fine texel reads the coarse SDF for selection and c_t")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 256 MiB device-to-device (scale for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(w, gpu_count: int, target_s: float, sampling: str = "point"):
    """Oracle on the same inputs: coarse stages in full, tracing on a seeded
    sample of the selected texels (one frame), extrapolated to one update."""
    import numpy as np

    import oracle

    lo = np.zeros(3, np.float32)
    hc, hf = np.float32(1.0 / w.nc), np.float32(1.0 / w.nf)
    t0 = time.perf_counter()
    s0 = oracle.voxelize(w.mesh.vertices, w.mesh.faces, lo, hc, w.nc)
    s = oracle.jfa(w.nc, s0)
    d2, c = oracle.coarse(w.nc, s, hc, w.beta)
    if sampling == "trilinear":
        c = oracle.coarse_trilinear(w.nc, c, w.nf)
        mask, queue = oracle.select_field(w.nf, c, w.d)
        nc = w.nf
    else:
        K = oracle.select_threshold(hc, w.beta, w.d)
        mask, queue = oracle.select(w.nc, d2, w.nf, K)
        nc = w.nc
    t_coarse = time.perf_counter() - t0
    sc = oracle.Scene(w.mesh.vertices, w.mesh.faces)
    st = oracle.TraceState(w.nf)
    rng = np.random.default_rng(0)
    # calibrate on a small sample, then size the main sample to ~target_s
    probe = np.sort(rng.choice(queue, min(len(queue), 4096), replace=False)).astype(np.int32)
    sc.trace_frame(nc, c, w.nf, lo, hf, mask, w.rays, 0, 0, w.scene_seed, w.alpha, st, probe[:256])  # warm-up
    t1 = time.perf_counter()
    sc.trace_frame(nc, c, w.nf, lo, hf, mask, w.rays, 0, 0, w.scene_seed, w.alpha, st, probe)
    per_texel = (time.perf_counter() - t1) / len(probe)
    n = int(min(len(queue), max(4096, (target_s - t_coarse) / max(per_texel, 1e-9))))
    sample = np.sort(rng.choice(queue, n, replace=False)).astype(np.int32)
    t2 = time.perf_counter()
    sc.trace_frame(nc, c, w.nf, lo, hf, mask, w.rays, 1, 0, w.scene_seed, w.alpha, st, sample)
    t_trace = time.perf_counter() - t2
    est_ms = (t_coarse + t_trace * len(queue) / n) * 1e3
    return {
        "value": round(est_ms, 1),
        "unit": "ms",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"voxelize+JFA+select in full ({t_coarse:.2f} s); trace of {n} of {len(queue)} selected texels "
                  f"x {w.rays} rays ({t_trace:.2f} s), extrapolated to all texels",
        "rays_per_s": round(n * w.rays / t_trace, 1),
        "selected_texels_match_gpu": int(len(queue)) == gpu_count,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the SDF update of one scene "
              "runs on one GPU; many scenes split across GPUs by scene)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2210_04449_amd.rtsdf as R
    from paper_2210_04449_amd.pipeline import Pipeline
    from synth.scenes import workload

    if args.study == "alpha":
        return run_alpha_study(args)
    if args.study == "refit":
        return run_refit_study(args)
    if args.study == "motion":
        return run_motion_study(args)
    if args.config == "batched":
        return run_batched(args)
    if args.config == "diff":
        return run_diff(args)
    w = workload(args.config)
    tuning = dict(refill=args.refill, blocks_per_cu=args.blocks_per_cu, stats=0, loop=args.loop,
                  bin_directions=args.bin, stack_lds=args.stack_lds, tile_texels=args.tile_texels,
                  bvh_width=args.bvh_width)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    use_parts = args.parts and args.config == "dynamic"
    kw = dict(seed=0, scene_id=w.scene_seed, alpha=w.alpha if args.alpha is None else args.alpha,
              leaf_size=args.leaf_size, jfa_variant=args.jfa, sampling=args.sampling)
    if args.refit:
        kw["rebuild"] = False
    if args.device_build:
        kw["rebuild"] = True
    dyn_frames = dyn_T = None
    # moving scenes move continuously: one geometry per update (warm-up, timed updates, the instrumented frame and
    # the graph replays), generated up front
    nfr = args.warmup + args.steps + 2 + max(2, args.steps // 2)
    if use_parts:
        # the moving primitives as rigid parts of a two-level scene; 8 transform sets cycled
        dyn = w.extra["scene"]
        pv, pf, offs, _ = dyn.parts()
        dyn_T = [torch.from_numpy(dyn.part_transforms(f)).to(dev) for f in range(nfr)]
        p = Pipeline(torch.from_numpy(pv).to(dev), torch.from_numpy(pf).to(dev), w.nc, w.nf, w.beta, w.d, w.rays,
                     parts=(offs, dyn_T[0]), **kw)
    else:
        p = Pipeline(torch.from_numpy(w.mesh.vertices).to(dev), torch.from_numpy(w.mesh.faces).to(dev), w.nc, w.nf,
                     w.beta, w.d, w.rays, **kw)
        if args.config == "dynamic":
            # the animated subset moves rigidly
            dyn = w.extra["scene"]
            dyn_frames = [torch.from_numpy(dyn.mesh(f).vertices).to(dev) for f in range(nfr)]
    if args.bvh_width == 4 and (use_parts or p.rebuild or args.config == "dynamic"):
        tuning["bvh_width"] = 2  # the 4-wide copy serves static and refitted single-level scenes
    p.scene.set_tuning(**tuning)  # this scene's tracer tuning (builds the 4-wide copy if asked for)
    info = p.scene.info()
    stream = torch.cuda.current_stream()

    def update(f):
        if dyn_frames is not None:
            p.set_vertices(dyn_frames[f % len(dyn_frames)])
        if dyn_T is not None:
            p.set_transforms(dyn_T[f % len(dyn_T)])

    if args.autotune:
        from paper_2210_04449_amd import autotune
        tuned = autotune.tune(p)
        tuning.update(tuned["tuning"])
        print(f"[autotune] {tuned['key']}: {tuned['tuning']} {tuned['ms']:.3f} ms, {len(tuned['trials'])} trials"
              f"{' (cached)' if tuned['cached'] else ''}; jfa {tuned.get('jfa')}", file=sys.stderr, flush=True)
    for f in range(args.warmup):
        update(f)
        p.step(f)
    torch.cuda.synchronize()
    selected = p.selected()
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        f = args.warmup + i
        e = ev[i]
        e[0].record(stream)
        update(f)
        p.voxelize()
        e[1].record(stream)
        p.jfa()
        e[2].record(stream)
        p.select()
        e[3].record(stream)
        p.trace(f)
        e[4].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / K
    names = ["voxelize", "jfa", "select", "trace"]
    stage = {n: sum(ev[i][j].elapsed_time(ev[i][j + 1]) for i in range(K)) / K for j, n in enumerate(names)}
    per_step = sorted(ev[i][0].elapsed_time(ev[i][4]) for i in range(K))
    gpu_ms = sum(per_step) / K

    def pct(q):
        return per_step[min(K - 1, int(round(q * (K - 1))))]
    rays = selected * w.rays
    trace_s = stage["trace"] / 1e3

    # instrumented frame (untimed): node visits and triangle tests per ray
    def counters(t):
        p.scene.set_tuning(**{**t, "stats": 1})
        p.trace(args.warmup + K)
        torch.cuda.synchronize()
        c = p.trace_ws[8:88].view(torch.int64).cpu().tolist()
        p.scene.set_tuning(**tuning)
        return c
    ctr = counters(tuning)
    # algorithmic work: the visits and tests of a traversal that culls with its ray's current best distance
    # (the one-fetch loop); the queued loop's extra ones, culled against the best as of the last flush, are
    # overhead and are reported beside them
    alg = counters({**tuning, "loop": 3}) if tuning["loop"] == 4 else ctr
    nodes_per_ray = alg[0] / max(alg[2], 1)
    tris_per_ray = alg[1] / max(alg[2], 1)
    ops_node = OPS_NODE4 if tuning["bvh_width"] == 4 else OPS_NODE
    ops = rays * (OPS_RAY + nodes_per_ray * ops_node + tris_per_ray * OPS_TRI)
    achieved = ops / trace_s / 1e12

    graph_ms = None
    if args.graph:  # a captured update also rebuilds or refits the hierarchy of a moving scene
        g = p.make_graph(first_frame=args.warmup + K + 1, refit=dyn_frames is not None or dyn_T is not None)
        g.launch()  # warm-up replay
        torch.cuda.synchronize()
        gs, ge = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(2, K // 2)
        gs.record(stream)
        for i in range(reps):
            if dyn_frames is not None:  # the graph refits from the vertex buffer
                p.vertices.copy_(dyn_frames[(args.warmup + K + 1 + i) % len(dyn_frames)])
            if dyn_T is not None:  # the graph applies the transform buffer
                p.transforms.copy_(dyn_T[(args.warmup + K + 1 + i) % len(dyn_T)])
            g.launch()
        ge.record(stream)
        torch.cuda.synchronize()
        graph_ms = gs.elapsed_time(ge) / reps
        g.close()

    shadow = None if args.no_shadow else time_shadow(R, p, w, stream)
    acc = accuracy(R, p)

    # HBM bytes per trace launch from the committed PMC summary of this workload, when it was taken on the
    # current kernel sources (else null)
    from paper_2210_04449_amd.prof_summary import traffic_from_summary
    inst = "true" if use_parts else "false"
    if tuning["bvh_width"] == 4:
        tname = f"trace_persistent<{tuning['stack_lds']},{tuning['refill']},3,false,false,false,true>"
    else:
        tname = f"trace_persistent<{tuning['stack_lds']},{tuning['refill']},{tuning['loop']},false,false,{inst},false>"
    tr = traffic_from_summary(os.path.join(ROOT, "profiles", f"pmc_{w.name}_{w.nc}_{w.nf}.txt"), tname)
    traffic = None if tr is None else int(tr["fetch_bytes"] + tr["write_bytes"])

    n3 = w.nc ** 3
    import math
    jfa_passes = len(p.jfa_steps) if p.jfa_steps else int(math.log2(w.nc))
    jfa_bytes = 8 * n3 * jfa_passes + 12 * n3
    jfa_gbs = jfa_bytes / (stage["jfa"] / 1e3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(ms_per_step, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {w.mesh.nt} triangles, coarse {w.nc}^3 / fine {w.nf}^3, beta {w.beta_vox} "
                        f"and d {w.d_vox} coarse voxels, {w.rays} rays/texel/frame, alpha {p.alpha}",
            "triangles": w.mesh.nt,
            "coarse": w.nc,
            "fine": w.nf,
            "rays_per_texel": w.rays,
            "sampling": args.sampling,
        },
        "gpu_ms_per_step": round(gpu_ms, 3),
        "gpu_ms_p10_p50_p90": [round(pct(0.1), 3), round(pct(0.5), 3), round(pct(0.9), 3)],
        "graph_ms_per_step": None if graph_ms is None else round(graph_ms, 3),
        "stages_ms": {k: round(v, 4) for k, v in stage.items()},
        "selected_texels": selected,
        "rays_per_step": rays,
        "rays_per_s": round(rays / trace_s, 1),
        "jfa": {"gbps": round(jfa_gbs, 1), "frac_hbm": round(jfa_gbs / HBM_PEAK_GBS, 4),
                "algorithmic_bytes": jfa_bytes, "schedule": args.jfa,
                # 0 = automatic: seed pairs in LDS, far passes in 2 x 2 brick quads of a residue class
                "near_stage": R.rtsdf_jfa_config_get(w.nc), "far_order": R.rtsdf_jfa_config_get(w.nc, "far_order")},
        "trace_stats": {"nodes_per_ray": round(nodes_per_ray, 2), "tris_per_ray": round(tris_per_ray, 2),
                        "run_nodes_per_ray": round(ctr[0] / max(ctr[2], 1), 2),
                        "run_tris_per_ray": round(ctr[1] / max(ctr[2], 1), 2),
                        "rays_counted": ctr[2], "wave_iterations": ctr[3] // 64, "refill_rounds": ctr[4] // 64,
                        "tiles": ctr[6] // 64, "tiles_started_early": ctr[8] // 64, "drain_rounds": ctr[9] // 64,
                        "empty_node_fraction": round(ctr[7] / max(ctr[0], 1), 4) if tuning["loop"] in (3, 4) else None,
                        "lane_work_fraction": round(ctr[5] / max(ctr[3], 1), 4) if tuning["loop"] >= 1 else None,
                        "bvh_nodes": info.nodes, "bvh_references": info.references, "bvh_max_depth": info.max_depth,
                        "bvh_max_leaf": info.leaf_size, "leaf_size": args.leaf_size},
        "trace_tuning": tuning,
        "shadow": shadow,
        "accuracy": acc,
        "roofline": {
            "kernel": "trace_persistent",
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "TOP/s",
            "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        },
    }
    if dyn_frames is not None:
        how = "refit" if args.refit else "device rebuild"
        out["config"]["dynamic"] = (f"20% of primitives move rigidly and continuously (a new vertex set every "
                                    f"update); {how} of the hierarchy each update")
    if use_parts:
        out["config"]["dynamic"] = ("20% of primitives move rigidly and continuously, as parts of a two-level scene; "
                                    "top-level refit and world positions each update")
    if not args.no_cpu_baseline and args.config != "dynamic":
        out["cpu_baseline"] = cpu_baseline(w, selected, args.cpu_seconds, args.sampling)
    if args.config == "room" and not args.no_extras:
        # the batched and differentiable forms against their plain single-scene forward, a few steps each
        p.close()
        del p
        torch.cuda.empty_cache()
        b = batched_record(args, 4, 1)
        out["batched"] = {"workload": b["config"]["workload"], "triangles": b["config"]["triangles"],
                          **{k: v for k, v in b.items() if k not in ("config", "batch_ms_per_step")},
                          "batch_ms_per_step": round(b["batch_ms_per_step"], 3)}
        torch.cuda.empty_cache()
        d = diff_record(args, 8, 1)
        out["diff"] = {"workload": d["config"]["workload"],
                       **{k: v for k, v in d.items() if k not in ("config", "forward_backward_ms_value")}}
    print(json.dumps(out), flush=True)


def time_shadow(R, p, w, stream, npts: int = 1920 * 1080):
    """Soft shadows (Sec. 2.3) from the fine SDF the updates produced, for one 1080p frame of shading points:
    points drawn (seeded) from the texel centres within one to three fine texels of a surface, in texel order, a fixed
    light; cone and triangulated penumbra, jittered starts; occluders searched up to 0.3 of the domain side
    (the room is closed, so an unbounded march from inside would always end on a wall).  Outside the timed
    update."""
    import torch

    h = 1.0 / w.nf
    f = p.fine_sdf
    near = torch.nonzero((f >= h) & (f <= 3 * h)).flatten()
    if near.numel() == 0:
        return None
    g = torch.Generator(device=f.device).manual_seed(1)
    # in texel order, as a frame's shading points are coherent in screen space and hence in space
    pick = near[torch.randint(0, near.numel(), (npts,), device=f.device, generator=g)].sort().values
    nf = w.nf
    ijk = torch.stack([pick % nf, (pick // nf) % nf, pick // (nf * nf)], 1).to(torch.float32)
    pts = ((ijk + 0.5) * h).contiguous()
    jit = torch.rand(npts, device=f.device, generator=g)
    light = [0.3, 0.9, 0.2]
    nrm = sum(x * x for x in light) ** 0.5
    light = [x / nrm for x in light]
    vis = torch.empty(npts, dtype=torch.float32, device=f.device)
    out = {"points": npts, "max_steps": 96, "eps_texels": 1, "max_step_texels": 2, "max_dist": 0.3}
    for name, pen in (("cone", 0), ("triangulated", 1)):
        def run():
            R.rtsdf_shadow_ex(p.fine, f, pts, light, 8.0, h, 96, 2 * h, 0.3, vis, penumbra=pen, jitter=jit,
                              jitter_scale=2 * h)
        run()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(5):
            run()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 5
        out[f"{name}_ms"] = round(ms, 4)
        out[f"{name}_points_per_s"] = round(npts / ms * 1e3, 1)
        out[f"{name}_mean_visibility"] = round(float(vis.mean().item()), 4)
    return out


def accuracy(R, p, tol_texels: float = 0.25):
    """Traced state u against the exact distance to the current geometry, over the selected texels.

    For static geometry Eq. (1) keeps u >= min(exact, max(c, 0)): every hit is on the mesh, and the decayed
    term never drops below the smaller of the previous u and max(c, 0).  With alpha < 1, u is pulled towards
    max(c, 0), which lies below the exact distance (the coarse field is biased down by beta), so "below exact"
    mixes that pull with stale history.  Stale history proper is u below min(exact, max(c, 0)): only geometry
    that has moved away can leave it ("ghost")."""
    import torch

    n = p.selected()
    if n == 0:
        return None
    q = p.queue[:n]
    exact = torch.empty(n, dtype=torch.float32, device=q.device)
    # distance queries take single-level scenes: a two-level scene is asked through its world mesh
    dscene = R.Scene(p.vertices, p.faces) if p.parts else p.scene
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    R.rtsdf_texel_distance(dscene, p.fine, q, exact)
    b.record()
    ql = q.long()
    u = p.state.u[ql]
    cgrid, cfield = p.trace_field()
    if cgrid.n == p.nf:
        c = cfield[ql]
    else:
        r = p.nf // cgrid.n
        nf, ncg = p.nf, cgrid.n
        c = cfield[(ql % nf) // r + ncg * (((ql // nf) % nf) // r + ncg * ((ql // (nf * nf)) // r))]
    fin = torch.isfinite(u)
    u, exact, c = u[fin].double(), exact[fin].double(), c[fin].double()
    gap = u - exact
    h = 1.0 / p.nf
    floor_ = torch.minimum(exact, c.clamp(min=0))
    ghost = (floor_ - u) > tol_texels * h
    qs = torch.quantile(gap[torch.randperm(gap.numel(), device=gap.device)[:1 << 20]],
                        torch.tensor([0.5, 0.95, 0.99], dtype=torch.float64, device=gap.device)).tolist()
    torch.cuda.synchronize()
    if dscene is not p.scene:
        dscene.close()
    return {
        "texels": n,
        "finite_fraction": round(fin.float().mean().item(), 5),
        "traced_minus_exact_texels": {"mean": round(gap.mean().item() / h, 4), "p50": round(qs[0] / h, 4),
                                      "p95": round(qs[1] / h, 4), "p99": round(qs[2] / h, 4),
                                      "max": round(gap.max().item() / h, 3)},
        "abs_err_mean_texels": round(gap.abs().mean().item() / h, 4),
        "below_exact_fraction": round((gap < -tol_texels * h).double().mean().item(), 6),
        "ghost_fraction": round(ghost.double().mean().item(), 6),
        "ghost_mean_texels": round(((floor_ - u).clamp(min=0)).mean().item() / h, 5),
        "exact_distance_ms": round(a.elapsed_time(b), 3),
    }


def run_alpha_study(args):
    """Decay alpha of Eq. (1) against stale history on the moving-scene workload: the same continuous motion
    replayed for each alpha, then the traced state compared with the exact distance to the final geometry;
    the same frames on the motionless scene give each alpha's error without motion."""
    import torch

    import paper_2210_04449_amd.rtsdf as R
    from paper_2210_04449_amd.pipeline import Pipeline
    from synth.scenes import workload

    w = workload("dynamic")
    dyn = w.extra["scene"]
    dev = torch.device("cuda:0")
    frames = args.study_frames
    verts = [torch.from_numpy(dyn.mesh(f).vertices).to(dev) for f in range(frames)]
    p = Pipeline(verts[0].clone(), torch.from_numpy(w.mesh.faces).to(dev), w.nc, w.nf, w.beta, w.d, w.rays,
                 scene_id=w.scene_seed, alpha=1.0, leaf_size=args.leaf_size)
    rows = []
    for alpha in args.alphas:
        p.alpha = float(alpha)
        for moving in (True, False):
            p.reset()
            for f in range(frames):
                p.set_vertices(verts[f] if moving else verts[-1])
                p.step(f)
            torch.cuda.synchronize()
            acc = accuracy(R, p)
            rows.append({"alpha": alpha, "moving": moving, **acc})
            print(f"[alpha {alpha} moving {moving}] ghost {acc['ghost_fraction']:.4f}, "
                  f"below exact {acc['below_exact_fraction']:.4f}, "
                  f"|traced-exact| mean {acc['abs_err_mean_texels']:.3f} texels", file=sys.stderr, flush=True)
    print(json.dumps({"study": "alpha vs stale history", "workload": w.name, "frames": frames,
                      "fine": w.nf, "rays_per_texel": w.rays, "motion": "20% of primitives rigid, continuous",
                      "units": "fine texels", "rows": rows}), flush=True)


def run_refit_study(args):
    """One refitted hierarchy, one rebuilt on the device every frame, and a two-level scene of rigid parts on the
    moving-scene workload, over a continuous animation: per-update time (geometry update + the whole SDF update)
    frame by frame."""
    import torch

    import paper_2210_04449_amd.rtsdf as R
    from paper_2210_04449_amd.pipeline import Pipeline
    from synth.scenes import workload

    w = workload("dynamic")
    dyn = w.extra["scene"]
    dev = torch.device("cuda:0")
    frames = args.study_frames
    stream = torch.cuda.current_stream()
    pv, pf, offs, _ = dyn.parts()
    rows = {}
    verts = [torch.from_numpy(dyn.mesh(f).vertices).to(dev) for f in range(frames)]
    for kind in ("refit", "rebuild", "parts"):
        if kind in ("refit", "rebuild"):
            p = Pipeline(verts[0].clone(), torch.from_numpy(w.mesh.faces).to(dev), w.nc, w.nf, w.beta, w.d, w.rays,
                         scene_id=w.scene_seed, alpha=w.alpha, leaf_size=args.leaf_size, rebuild=kind == "rebuild")
            move = lambda f: p.set_vertices(verts[f])  # noqa: E731
        else:
            Ts = [torch.from_numpy(dyn.part_transforms(f)).to(dev) for f in range(frames)]
            p = Pipeline(torch.from_numpy(pv).to(dev), torch.from_numpy(pf).to(dev), w.nc, w.nf, w.beta, w.d, w.rays,
                         scene_id=w.scene_seed, alpha=w.alpha, leaf_size=args.leaf_size, parts=(offs, Ts[0]))
            move = lambda f: p.set_transforms(Ts[f])  # noqa: E731
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(frames)]
        for f in range(frames):
            ev[f][0].record(stream)
            move(f)
            p.voxelize()
            p.jfa()
            p.select()
            ev[f][1].record(stream)
            p.trace(f)
            ev[f][2].record(stream)
        torch.cuda.synchronize()
        total = [a.elapsed_time(c) for a, _, c in ev]
        trace = [b.elapsed_time(c) for _, b, c in ev]
        rows[kind] = {"ms_per_update": [round(x, 2) for x in total], "trace_ms": [round(x, 2) for x in trace],
                      "mean_ms": round(sum(total) / frames, 2), "first4_ms": round(sum(total[:4]) / 4, 2),
                      "last4_ms": round(sum(total[-4:]) / 4, 2), "triangles": int(p.faces.shape[0]),
                      "selected_last": p.selected()}
        print(f"[{kind}] mean {rows[kind]['mean_ms']} ms, first 4 {rows[kind]['first4_ms']}, "
              f"last 4 {rows[kind]['last4_ms']}", file=sys.stderr, flush=True)
        p.close()
        del p
        torch.cuda.empty_cache()
    print(json.dumps({"study": "refit vs rebuild vs two-level", "workload": w.name, "frames": frames, "fine": w.nf,
                      "rays_per_texel": w.rays, "motion": "20% of primitives rigid, continuous", "rows": rows}),
          flush=True)


def run_motion_study(args):
    """The moving-scene workload with the library's default handling of moving geometry (the hierarchy rebuilt on
    the device at every update, inside the captured frame graph), over a continuous animation of
    --study-frames updates: the time of every update, to show it stays flat."""
    import torch

    from paper_2210_04449_amd.pipeline import Pipeline
    from synth.scenes import workload

    w = workload("dynamic")
    dyn = w.extra["scene"]
    dev = torch.device("cuda:0")
    frames = args.study_frames
    verts = [torch.from_numpy(dyn.mesh(f).vertices).to(dev) for f in range(frames)]
    print(f"[motion] {frames} vertex sets generated", file=sys.stderr, flush=True)
    p = Pipeline(verts[0].clone(), torch.from_numpy(w.mesh.faces).to(dev), w.nc, w.nf, w.beta, w.d, w.rays,
                 scene_id=w.scene_seed, alpha=w.alpha, leaf_size=args.leaf_size)
    g = p.make_graph(first_frame=0, refit=True)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(frames)]
    for f in range(frames):
        p.vertices.copy_(verts[f])
        ev[f][0].record(stream)
        g.launch()
        ev[f][1].record(stream)
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in ev]
    g.close()
    first4, last4 = sum(ms[:4]) / 4, sum(ms[-4:]) / 4
    print(json.dumps({"study": "continuous motion, default hierarchy handling (device rebuild in the frame graph)",
                      "workload": w.name, "frames": frames, "triangles": w.mesh.nt, "fine": w.nf,
                      "rays_per_texel": w.rays, "motion": "20% of primitives rigid, continuous",
                      "ms_per_update": [round(x, 2) for x in ms], "first4_ms": round(first4, 2),
                      "last4_ms": round(last4, 2), "max_over_first4": round(max(ms) / first4, 3),
                      "mean_ms": round(sum(ms) / frames, 2)}), flush=True)


def _base_record(args, value_ms, config):
    return {
        "metric": METRIC, "value": round(value_ms, 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(value_ms, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": config,
    }


def run_batched(args):
    rec = batched_record(args, args.steps, args.warmup)
    out = _base_record(args, rec.pop("batch_ms_per_step"), rec.pop("config"))
    out.update(rec)
    print(json.dumps(out), flush=True)


def batched_record(args, steps: int, warmup: int) -> dict:
    """64 seeded scenes of uneven size in one launch per stage, captured as one graph, against the same
    scenes run one by one through the single-scene path."""
    import torch

    import paper_2210_04449_amd.rtsdf as R
    from paper_2210_04449_amd.pipeline import Pipeline
    from synth.scenes import batched_scenes

    ws = batched_scenes(64)
    dev = torch.device("cuda:0")
    meshes = [(torch.from_numpy(w.mesh.vertices).to(dev), torch.from_numpy(w.mesh.faces).to(dev)) for w in ws]
    B = R.Batch([dict(vertices=v, faces=f, coarse_n=w.nc, fine_n=w.nf, beta=w.beta, d=w.d, rays=w.rays,
                      alpha=w.alpha, scene_id=w.scene_seed) for w, (v, f) in zip(ws, meshes)], seed=0)
    if args.autotune:
        from paper_2210_04449_amd import autotune
        autotune.tune(B)
    elif args.config == "batched" and args.refill != 28:
        B.set_tuning(refill=args.refill)
    g = B.make_graph(first_frame=0)
    for _ in range(warmup):
        g.launch()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    s0.record(stream)
    for _ in range(steps):
        g.launch()
    s1.record(stream)
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) * 1e3 / steps
    rays = sum(B.tensors(i)["count"].item() * w.rays for i, w in enumerate(ws))
    # the same scenes one at a time (eager single-scene path)
    single_ms = 0.0
    for w, (v, f) in zip(ws, meshes):
        p = Pipeline(v, f, w.nc, w.nf, w.beta, w.d, w.rays, scene_id=w.scene_seed, alpha=w.alpha)
        p.step(0)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for fr in range(1, 3):
            p.step(fr)
        b.record(stream)
        torch.cuda.synchronize()
        single_ms += a.elapsed_time(b) / 2
        p.close()
        del p
    g.close()
    B.close()
    return {"config": {
        "workload": "batched: 64 seeded scenes, triangles log-uniform 1k-100k, coarse in {32,64,128}, fine 2x, "
                    "beta 0.5 / d 2 coarse voxels, 8 rays/texel, one graph-captured step",
        "scenes": len(ws), "triangles": int(sum(w.mesh.nt for w in ws))},
        "batch_ms_per_step": batch_ms, "steps": steps,
        "batch_gpu_ms_per_step": round(s0.elapsed_time(s1) / steps, 3),
        "sum_single_scene_ms": round(single_ms, 3), "speedup_vs_single": round(single_ms / batch_ms, 3),
        "rays_per_step": int(rays), "rays_per_s": round(rays / (batch_ms / 1e3), 1)}


def run_diff(args):
    rec = diff_record(args, args.steps, args.warmup)
    out = _base_record(args, rec.pop("forward_backward_ms_value"), rec.pop("config"))
    out.update(rec)
    print(json.dumps(out), flush=True)


def diff_record(args, steps: int, warmup: int) -> dict:
    """Differentiable config: forward (all frames) and backward to vertex positions, against the plain forward."""
    import torch

    from paper_2210_04449_amd.autograd import fine_sdf
    from paper_2210_04449_amd.pipeline import Pipeline
    from synth.scenes import workload

    w = workload("diff")
    dev = torch.device("cuda:0")
    v0 = torch.from_numpy(w.mesh.vertices).to(dev)
    p = Pipeline(v0, torch.from_numpy(w.mesh.faces).to(dev), w.nc, w.nf, w.beta, w.d, w.rays, scene_id=w.scene_seed)
    j = torch.arange(w.nf ** 3, device=dev)
    P = torch.stack([j % w.nf, (j // w.nf) % w.nf, j // w.nf ** 2], 1).float().add_(0.5).div_(w.nf)
    target = (P - 0.5).norm(dim=1) - 0.3
    frames = range(w.frames)
    stream = torch.cuda.current_stream()

    def plain():
        p.set_vertices(v0)
        p.reset()
        for f in frames:
            p.step(f)

    def fwd_bwd():
        v = v0.clone().requires_grad_(True)
        f = fine_sdf(v, p, frames)
        loss = ((f - target) ** 2).sum()
        loss.backward()
        return v.grad

    for _ in range(warmup):
        plain()
        fwd_bwd()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    reps = max(1, steps // 4)
    ev[0].record(stream)
    for _ in range(reps):
        plain()
    ev[1].record(stream)
    for _ in range(reps):
        g = fwd_bwd()
    ev[2].record(stream)
    torch.cuda.synchronize()
    plain_ms = ev[0].elapsed_time(ev[1]) / reps
    fb_ms = ev[1].elapsed_time(ev[2]) / reps
    p.close()
    return {"config": {
        "workload": f"diff: perturbed geodesic sphere {w.mesh.nt} triangles, coarse {w.nc}^3 / fine {w.nf}^3, "
                    f"{w.rays} rays x {w.frames} frames; loss sum (f - sphere SDF)^2; forward + backward",
        "triangles": w.mesh.nt},
        "forward_backward_ms_value": fb_ms, "reps": reps,
        "plain_forward_ms": round(plain_ms, 3), "forward_backward_ms": round(fb_ms, 3),
        "backward_overhead_ms": round(fb_ms - plain_ms, 3),
        "backward_vs_forward": round(fb_ms / plain_ms, 4),
        "grad_norm": float(g.norm().item())}


if __name__ == "__main__":
    main()
