"""Hierarchies rebuilt on the device (linear BVH over the scene's references).

The closest hit of a ray is a minimum over references of values computed from
each reference alone (a triangle's decision does not depend on the bound the
traversal holds when it tests it), so a rebuilt scene traces exactly like the
scene built on the host, static or after the vertices moved (rebuild against
refit), and a refit of a rebuilt tree too.  Leaves of the rebuilt tree hold up
to the scene's leaf size of consecutive references.  The moving scene is also
checked against the oracle, and bad calls are refused.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth.scenes import DynamicScene, workload

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    return R


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def same(a, b):
    """Every state field and the fine SDF identical."""
    diff = ((a.fine_sdf != b.fine_sdf) | (a.state.u != b.state.u) | (a.state.hits != b.state.hits)
            | (a.state.arg_tri != b.state.arg_tri) | (a.state.arg_ray != b.state.arg_ray))
    n = int(diff.sum())
    if n:
        fa, fb = a.fine_sdf[diff].abs(), b.fine_sdf[diff].abs()
        print("texels differing:", n, "max |f| difference", float((fa - fb).abs().max()))
    return n == 0


@pytest.mark.parametrize("case", ["tiny", "room"])
def test_rebuilt_scene_traces_like_the_host_build(R, case):
    say("rebuild static", case)
    from paper_2210_04449_amd.pipeline import Pipeline
    w = workload(case)
    frames = range(3) if case == "tiny" else range(1)
    mk = lambda rb: Pipeline(cu(w.mesh.vertices), cu(w.mesh.faces), w.nc, w.nf, w.beta, w.d, w.rays,  # noqa: E731
                             scene_id=w.scene_seed, rebuild=rb)
    a, b = mk(False), mk(True)
    ia, ib = a.scene.info(), b.scene.info()
    assert ib.references == ia.references and ib.nodes == ia.references - 1 and ib.leaf_size == a.leaf_size == 4
    bits = int(np.ceil(np.log2(ia.references)))
    assert ib.max_depth == 30 + bits + 1
    for f in frames:
        a.step(f)
        b.step(f)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    assert same(a, b)


def test_rebuild_refit_and_oracle_on_a_moving_scene(R):
    say("rebuild moving")
    from paper_2210_04449_amd.pipeline import Pipeline
    dyn = DynamicScene(7, n_prims=30, detail="low")
    nc, nf, rays, alpha = 32, 64, 4, 0.9
    beta, d = np.float32(0.5 / nc), np.float32(2.0 / nc)
    m0 = dyn.mesh(0)
    mk = lambda rb: Pipeline(cu(m0.vertices), cu(m0.faces), nc, nf, float(beta), float(d), rays,  # noqa: E731
                             scene_id=9, alpha=alpha, rebuild=rb)
    refit, rebuilt = mk(False), mk(True)
    # a rebuilt scene whose later frames only refit its own tree
    refit_of_rebuilt = mk(True)
    refit_of_rebuilt.rebuild = False
    st = oracle.TraceState(nf)
    for f in range(6):
        m = dyn.mesh(f)
        for p in (refit, rebuilt, refit_of_rebuilt):
            p.set_vertices(cu(m.vertices))
            p.step(f)
        ref = oracle.run_frames(m.vertices, m.faces, nc, nf, beta, d, rays, [f], seed=0, scene=9, alpha=alpha,
                                state=st)
    torch.cuda.synchronize()
    assert R.rtsdf_sync_status() == 0
    assert same(refit, rebuilt) and same(refit, refit_of_rebuilt)
    from test_gpu_parity import compare_trace
    print(compare_trace(rebuilt, ref))


def test_rebuild_refusals(R):
    say("rebuild refusals")
    from synth.scenes import rigid_parts
    w = workload("tiny")
    sc = R.Scene(cu(w.mesh.vertices), cu(w.mesh.faces))
    with pytest.raises(R.RtsdfError):
        sc.rebuild(cu(w.mesh.vertices))  # not enabled
    sc.enable_rebuild()
    sc.enable_rebuild()  # a second call keeps the buffers
    sc.rebuild(cu(w.mesh.vertices))
    torch.cuda.synchronize()
    sc.close()
    v, f, offs, T = rigid_parts()
    ps = R.Scene.instanced(cu(v), cu(f), offs, cu(T))
    with pytest.raises(R.RtsdfError):
        ps.enable_rebuild()
    ps.close()
    empty = R.Scene(torch.zeros((3, 3), device="cuda"), torch.zeros((0, 3), dtype=torch.int32, device="cuda"))
    with pytest.raises(R.RtsdfError):
        empty.enable_rebuild()  # no reference: nothing to rebuild
    empty.close()


def check_tree(boxes, links, parents, nref):
    """A valid binary tree over references 0..nref-1, read from the root (a rebuilt hierarchy may hold
    internal nodes no slot references: the radix-tree nodes below a leaf of several references), whose every
    internal slot is exactly the union of that child's two slots (tight boxes, not only conservative ones).
    Returns the leaf slots' first references, counts and boxes."""
    n = len(parents)
    assert parents[0] == -1
    internal = links[:, :, 0] >= 0
    child = np.where(internal, links[:, :, 0], 0)
    reach = np.zeros(n, bool)
    reach[0] = True
    stack = [0]
    while stack:
        i = stack.pop()
        for s in range(2):
            if internal[i, s]:
                c = child[i, s]
                assert not reach[c], "a node referenced twice"
                reach[c] = True
                stack.append(c)
    live = internal & reach[:, None]  # internal slots of reachable nodes
    # every reachable node other than the root is the child of exactly one slot, and its parent link names it
    owner = np.repeat(np.arange(n), 2).reshape(n, 2)
    assert (parents[child[live]] == owner[live]).all()
    # internal slots: union of the child's slots
    kids = boxes[child]                                      # [n, 2, 2, 6]
    union = np.concatenate([kids[..., :3].min(axis=2), kids[..., 3:].max(axis=2)], axis=-1)
    assert np.array_equal(boxes[live], union[live])
    # leaves of reachable nodes: each reference in exactly one leaf
    leaf = ~internal & (links[:, :, 1] > 0) & reach[:, None]
    first, cnt = -1 - links[:, :, 0][leaf], links[:, :, 1][leaf]
    cover = np.zeros(nref, np.int64)
    for fi, c in zip(first, cnt):
        cover[fi:fi + c] += 1
    assert (cover == 1).all()
    return first, cnt, boxes[leaf]


def sub_multiset(a, b):
    """Every row of a occurs in b at least as often as in a (rows compared bit for bit)."""
    view = lambda x: np.ascontiguousarray(x).view(np.dtype((np.void, x.dtype.itemsize * x.shape[1]))).ravel()  # noqa: E731
    ua, ca = np.unique(view(a), return_counts=True)
    ub, cb = np.unique(view(b), return_counts=True)
    pos = np.searchsorted(ub, ua)
    pos = np.minimum(pos, len(ub) - 1)
    return bool((ub[pos] == ua).all() and (cb[pos] >= ca).all())


@pytest.mark.parametrize("case", ["moving", "room"])
def test_rebuilt_boxes_are_exact(R, case):
    """The rebuilt tree (several chunks of the two-pass box climb, and the pass across chunks) against a
    host-built tree of one reference per leaf refitted on the device: same reference boxes, both trees tight."""
    say("rebuild boxes", case)
    if case == "moving":
        dyn = DynamicScene(7, n_prims=30, detail="low")
        meshes = [dyn.mesh(0), dyn.mesh(3)]
    else:
        meshes = [workload("room").mesh]
    v0, faces = cu(meshes[0].vertices), cu(meshes[0].faces)
    host = R.Scene(v0, faces, leaf_size=1)
    dev = R.Scene(v0, faces, leaf_size=1)
    dev.enable_rebuild()
    dev4 = R.Scene(v0, faces, leaf_size=4)  # the same rebuild with leaves of up to four references
    dev4.enable_rebuild()
    nref = dev.info().references
    assert host.info().references == nref and nref > 4 * 1024 and dev4.info().leaf_size == 4
    for i, m in enumerate(meshes):
        v = cu(m.vertices)
        host.refit(v)
        dev.rebuild(v)
        dev4.rebuild(v)
        torch.cuda.synchronize()
        assert R.rtsdf_sync_status() == 0
        hb, hl, hp = host.hierarchy()
        db, dl, dp = dev.hierarchy()
        assert len(db) == nref - 1
        _, hc, hleaf = check_tree(hb, hl, hp, nref)
        dfirst, dc, dleaf = check_tree(db, dl, dp, nref)
        assert (dc == 1).all() and (hc == 1).sum() >= 1000  # the host SAH also makes two-reference leaves
        # leaves of several references: each box is the union of its references' boxes (both rebuilds sort
        # the same codes stably, so reference k is the same in both)
        b4, l4, p4 = dev4.hierarchy()
        f4, c4, leaf4 = check_tree(b4, l4, p4, nref)
        assert c4.max() == 4 and (c4 > 1).sum() > nref // 8
        ref_box = np.empty((nref, 6), np.float32)
        ref_box[dfirst] = dleaf
        for fi, c, bx in zip(f4, c4, leaf4):
            rb = ref_box[fi:fi + c]
            assert np.array_equal(bx, np.concatenate([rb[:, :3].min(axis=0), rb[:, 3:].max(axis=0)]))
        # the same reference boxes (the references are the same, in another order): the host tree's
        # one-reference leaves are among the rebuilt tree's leaves, and both roots bound the same set
        assert sub_multiset(hleaf[hc == 1], dleaf), i
        root = lambda b: np.concatenate([b[0, :, :3].min(axis=0), b[0, :, 3:].max(axis=0)])  # noqa: E731
        assert np.array_equal(root(hb), root(db)), i
        if i == 0:
            # a refit of the rebuilt tree keeps its topology and its boxes
            dev.refit(v)
            torch.cuda.synchronize()
            rb, rl, rp = dev.hierarchy()
            assert np.array_equal(rl, dl) and np.array_equal(rp, dp) and np.array_equal(rb, db)
    # a buffer smaller than the hierarchy is refused
    n = dev.info().nodes
    buf = np.zeros((n - 1, 2, 6), np.float32)
    lnk = np.zeros((n - 1, 2, 2), np.int32)
    assert R._lib.rtsdf_scene_hierarchy(dev.handle, n - 1, buf.ctypes.data, lnk.ctypes.data, None, None) == R.EINVAL
    host.close()
    dev.close()
    dev4.close()
