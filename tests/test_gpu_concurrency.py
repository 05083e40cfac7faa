"""Concurrency and per-scene state of the tracer boundary, on the GPU.

* One scene traced on two streams at once (separate workspaces and outputs)
  gives exactly the results of the same traces run one after the other: the
  spill area of the traversal stacks lives in each call's workspace, not in
  the scene.  The room's hierarchy is deeper than the LDS part of the stack,
  so the spill area is in use.
* A scene's own tuning (rtsdf_scene_set_tuning) is what its traces use, the
  process default is untouched, and results equal the default's bitwise.
* A device frame counter at 2^23 - 1 traces normally; at 2^23 (past the
  argmin record's frame field) the tracer traces nothing, leaves the state
  and fine values as they were and raises ERR_FRAME.
"""
import sys

import numpy as np
import pytest
import torch

from synth.scenes import workload

pytestmark = pytest.mark.gpu


def say(*a):
    print("[concurrency]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    return R


def make_pipe(name, **kw):
    from paper_2210_04449_amd.pipeline import Pipeline
    w = workload(name)
    dev = torch.device("cuda:0")
    p = Pipeline(torch.from_numpy(w.mesh.vertices).to(dev), torch.from_numpy(w.mesh.faces).to(dev), w.nc, w.nf,
                 w.beta, w.d, w.rays, seed=0, scene_id=w.scene_seed, **kw)
    return w, p


def outputs(R, p):
    return {"fine": p.fine_sdf.clone(), **{k: v.clone() for k, v in p.state.tensors().items()}}


def trace_into(R, p, frame, state, fine, ws, stream):
    R.rtsdf_trace_accumulate(p.scene, *p.trace_field(), p.fine, p.mask, p.queue, p.count, p.rays, frame, p.seed,
                             p.scene_id, p.alpha, state, fine, ws, stream=stream)


def test_one_scene_two_streams_equals_sequential(R):
    w, p = make_pipe("room")
    assert p.scene.info().max_depth + 1 > 12, "the test needs a hierarchy deeper than the LDS stack part"
    p.voxelize()
    p.jfa()
    p.select()
    torch.cuda.synchronize()
    say("room selected", p.selected(), "depth", p.scene.info().max_depth)
    frames = (5, 9)
    # sequential reference: each frame from a fresh state, one after the other on the current stream
    ref = []
    for fr in frames:
        st = R.AccumState(p.fine)
        fine = torch.empty_like(p.fine_sdf)
        trace_into(R, p, fr, st, fine, p.trace_ws, None)
        torch.cuda.synchronize()
        ref.append((fine.clone(), {k: v.clone() for k, v in st.tensors().items()}))
    # concurrent: the two frames on two streams, same scene, own workspaces
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [torch.empty(R.rtsdf_trace_workspace_size(), dtype=torch.uint8, device=p.device) for _ in frames]
    states = [R.AccumState(p.fine) for _ in frames]
    fines = [torch.empty_like(p.fine_sdf) for _ in frames]
    torch.cuda.synchronize()
    for i, fr in enumerate(frames):
        with torch.cuda.stream(streams[i]):
            trace_into(R, p, fr, states[i], fines[i], wss[i], streams[i])
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    for i in range(len(frames)):
        assert torch.equal(fines[i], ref[i][0]), i
        for k, v in states[i].tensors().items():
            assert torch.equal(v, ref[i][1][k]), (i, k)
    say("two streams identical to sequential")
    p.close()


def test_scene_tuning_is_per_scene_and_keeps_results(R):
    w, p = make_pipe("tiny")
    default = R.rtsdf_trace_config_get().as_dict()
    for f in range(3):
        p.step(f)
    torch.cuda.synchronize()
    ref = outputs(R, p)
    assert p.scene.tuning().as_dict() == default
    for t in (dict(tile_texels=16, blocks_per_cu=3), dict(tile_texels=32, refill=16, stack_lds=16),
              dict(blocks_per_cu=5, bin_directions=0, loop=2)):
        say("scene tuning", t)
        p.scene.set_tuning(**t)
        got = p.scene.tuning().as_dict()
        assert all(got[k] == v for k, v in t.items())
        assert R.rtsdf_trace_config_get().as_dict() == default  # the process default is untouched
        p.reset()
        for f in range(3):
            p.step(f)
        torch.cuda.synchronize()
        out = outputs(R, p)
        for k in ref:
            assert torch.equal(out[k], ref[k]), (t, k)
        p.scene.clear_tuning()
    assert p.scene.tuning().as_dict() == default
    p.close()


def test_frame_counter_past_argmin_range_raises_and_traces_nothing(R):
    w, p = make_pipe("tiny")
    p.voxelize()
    p.jfa()
    p.select()
    counter = torch.full((1,), (1 << 23) - 1, dtype=torch.int32, device=p.device)
    p.trace(0, frame_ptr=counter)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    sel = p.mask.bool()
    ar = p.state.arg_ray[sel]
    traced = ar >= 0
    assert int(traced.sum()) > 0
    assert bool(((ar[traced] >> 8) == (1 << 23) - 1).all())  # the last representable frame is recorded
    before = outputs(R, p)
    counter.fill_(1 << 23)
    p.trace(0, frame_ptr=counter)
    torch.cuda.synchronize()
    bits = R.rtsdf_sync_status()
    assert bits & R.ERR_FRAME, bits
    after = outputs(R, p)
    for k in before:
        assert torch.equal(after[k], before[k]), k
    say("frame 2^23 refused on the device")
    p.close()
