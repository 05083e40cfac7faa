"""rtsdf_select_noalloc (selection with the library's static per-device
scratch instead of a caller workspace) against rtsdf_select, through the C ABI:
mask, queue and count must be identical bit for bit.  Two calls in a row, the
second on a smaller grid, so the second call runs over scratch the first one
left behind; a third call repeats the first size after the smaller one.
Inputs are real coarse fields (voxelize + jump flooding of the seeded room and
tiny scenes), so the selected set has the shape of the benchmark's."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2210_04449_amd.rtsdf as R
    return R


def say(*a):
    print("[no_alloc]", *a, flush=True)


def coarse_field(R, name):
    from synth.scenes import workload
    w = workload(name)
    dev = torch.device("cuda:0")
    v = torch.from_numpy(w.mesh.vertices).to(dev)
    f = torch.from_numpy(w.mesh.faces).to(dev)
    cg, fg = R.Grid.make(w.nc), R.Grid.make(w.nf)
    n3 = w.nc ** 3
    seeds = torch.empty(n3, dtype=torch.int32, device=dev)
    scratch = torch.empty_like(seeds)
    d2 = torch.empty_like(seeds)
    c = torch.empty(n3, dtype=torch.float32, device=dev)
    R.rtsdf_voxelize(v, f, cg, seeds)
    R.rtsdf_jfa(cg, seeds, scratch, w.beta, d2, c)
    return w, cg, fg, d2


def run_select(R, noalloc, cg, fg, d2, beta, d, cap):
    L = R.lib()
    dev = d2.device
    mask = torch.full((fg.n ** 3,), 7, dtype=torch.uint8, device=dev)
    queue = torch.full((cap,), -5, dtype=torch.int32, device=dev)
    count = torch.full((1,), -9, dtype=torch.int32, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    if noalloc:
        st = L.rtsdf_select_noalloc(cg, C.c_void_p(d2.data_ptr()), fg, C.c_float(beta), C.c_float(d),
                                    C.c_void_p(mask.data_ptr()), C.c_void_p(queue.data_ptr()), cap,
                                    C.c_void_p(count.data_ptr()), C.c_void_p(s))
    else:
        ws = torch.empty(R.rtsdf_select_workspace_size(cg.n), dtype=torch.uint8, device=dev)
        st = L.rtsdf_select(cg, C.c_void_p(d2.data_ptr()), fg, C.c_float(beta), C.c_float(d),
                            C.c_void_p(mask.data_ptr()), C.c_void_p(queue.data_ptr()), cap,
                            C.c_void_p(count.data_ptr()), C.c_void_p(ws.data_ptr()), C.c_void_p(s))
    assert st == R.OK, st
    assert R.rtsdf_sync_status() == 0
    n = int(count.item())
    return mask.cpu().numpy(), queue[:n].cpu().numpy(), n


def test_select_noalloc_matches_select_twice_smaller_second(R):
    fields = {name: coarse_field(R, name) for name in ("room", "tiny")}
    for name in ("room", "tiny", "room"):
        w, cg, fg, d2 = fields[name]
        cap = fg.n ** 3
        say(name, "coarse", cg.n, "fine", fg.n)
        ref = run_select(R, False, cg, fg, d2, w.beta, w.d, cap)
        got = run_select(R, True, cg, fg, d2, w.beta, w.d, cap)
        assert got[2] == ref[2] and ref[2] > 0, (got[2], ref[2])
        assert np.array_equal(got[0], ref[0])
        assert np.array_equal(got[1], ref[1])
        say(name, "selected", ref[2], "identical")
