"""CPU checks of the C ABI: the built library loads, exports every function the
header declares, and rejects bad arguments on the host (no GPU call is made for
those: validation happens before any launch)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtsdf.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rtsdf_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def R():
    from paper_2210_04449_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    import paper_2210_04449_amd.rtsdf as R
    return R


def test_header_declares_the_five_stages():
    names = declared()
    for n in ("rtsdf_voxelize", "rtsdf_jfa", "rtsdf_select", "rtsdf_trace_accumulate", "rtsdf_shadow"):
        assert n in names


def test_every_declared_symbol_is_exported(R):
    out = subprocess.run(["nm", "-D", "--defined-only", R.LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (rtsdf_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    # nothing torch-typed crosses the boundary: the library does not link torch
    deps = subprocess.run(["ldd", R.LIB], capture_output=True, text=True).stdout
    assert "torch" not in deps


def test_status_strings(R):
    L = R.lib()
    assert L.rtsdf_status_string(0) == b"ok"
    assert L.rtsdf_status_string(-1) == b"invalid argument"
    assert R.rtsdf_version() >= 100


def test_host_validation(R):
    L = R.lib()
    g = R.Grid.make(32)
    bad_n = R.Grid.make(33)
    dummy = C.c_void_p(16)  # never dereferenced: every call below fails validation first
    assert L.rtsdf_voxelize(dummy, 3, dummy, 1, bad_n, dummy, None) == R.EINVAL
    assert L.rtsdf_voxelize(dummy, 3, dummy, 1, R.Grid.make(512), dummy, None) == R.EINVAL
    assert L.rtsdf_voxelize(dummy, 3, dummy, 1, g, None, None) == R.EINVAL
    assert L.rtsdf_jfa(g, dummy, dummy, 0.0, dummy, dummy, None) == R.EINVAL  # seeds == scratch
    assert L.rtsdf_jfa(R.Grid.make(4), dummy, C.c_void_p(32), 0.0, dummy, dummy, None) == R.EINVAL
    other, d2p = C.c_void_p(32), C.c_void_p(48)
    for bad in ([], [8, 4, 2], [3, 1], [32, 1], [0, 1], [16, -4, 1]):
        arr = (C.c_int32 * max(len(bad), 1))(*bad)
        assert L.rtsdf_jfa_steps(g, dummy, other, arr, len(bad), 0.0, d2p, dummy, None) == R.EINVAL, bad
    ok = (C.c_int32 * 2)(16, 1)
    assert L.rtsdf_jfa_steps(g, dummy, other, None, 2, 0.0, d2p, dummy, None) == R.EINVAL  # no schedule
    assert L.rtsdf_jfa_steps(g, dummy, dummy, ok, 2, 0.0, d2p, dummy, None) == R.EINVAL  # seeds == scratch
    # dist2 is also a work buffer: it may be neither seeds nor scratch
    assert L.rtsdf_jfa_steps(g, dummy, other, ok, 2, 0.0, dummy, dummy, None) == R.EINVAL
    assert L.rtsdf_jfa_steps(g, dummy, other, ok, 2, 0.0, other, dummy, None) == R.EINVAL
    assert R.jfa_schedule(32, "jfa+2") == [16, 8, 4, 2, 1, 2, 1] and R.jfa_schedule(16, "1+jfa") == [1, 8, 4, 2, 1]
    fine = R.Grid.make(64)
    assert L.rtsdf_select(g, dummy, R.Grid.make(48), 0.0, 0.1, dummy, dummy, 10, dummy, dummy, None) == R.EINVAL
    # fine grid must cover the same box as the coarse one
    assert L.rtsdf_select(g, dummy, R.Grid.make(64, 1 / 32), 0.0, 0.1, dummy, dummy, 10, dummy, dummy, None) == R.EINVAL
    # trilinear sampling: same box, power-of-two multiple, fine.n <= 1024; field selection grid in [4, 1024]
    assert L.rtsdf_coarse_trilinear(g, dummy, R.Grid.make(48), dummy, None) == R.EINVAL
    assert L.rtsdf_coarse_trilinear(g, dummy, R.Grid.make(64, 1 / 32), dummy, None) == R.EINVAL
    assert L.rtsdf_coarse_trilinear(fine, dummy, g, dummy, None) == R.EINVAL  # fine coarser than coarse
    assert L.rtsdf_coarse_trilinear(g, None, fine, dummy, None) == R.EINVAL
    assert L.rtsdf_select_field(R.Grid.make(2), dummy, 0.1, dummy, dummy, 10, dummy, dummy, None) == R.EINVAL
    assert L.rtsdf_select_field(R.Grid.make(2048), dummy, 0.1, dummy, dummy, 10, dummy, dummy, None) == R.EINVAL
    assert L.rtsdf_select_field(fine, dummy, float("nan"), dummy, dummy, 10, dummy, dummy, None) == R.EINVAL
    assert L.rtsdf_select_field(fine, dummy, 0.1, dummy, None, 10, dummy, dummy, None) == R.EINVAL  # no queue
    assert L.rtsdf_select_field(fine, None, 0.1, dummy, dummy, 10, dummy, dummy, None) == R.EINVAL
    acc = R.Accum(16, 16, 16, 16)
    assert L.rtsdf_trace_accumulate(dummy, g, dummy, fine, dummy, dummy, dummy, 10, 0, 0, None, 0, 0, 1.0, acc,
                                    dummy, dummy, None) == R.EINVAL  # zero rays
    assert L.rtsdf_trace_accumulate(dummy, g, dummy, fine, dummy, dummy, dummy, 10, 65, 0, None, 0, 0, 1.0, acc,
                                    dummy, dummy, None) == R.EINVAL
    assert L.rtsdf_trace_accumulate(dummy, g, dummy, fine, dummy, dummy, dummy, 10, 4, 0, None, 0, 0, 1.5, acc,
                                    dummy, dummy, None) == R.EINVAL
    ld = (C.c_float * 3)(0, 1, 0)
    assert L.rtsdf_shadow(fine, dummy, dummy, 4, ld, 8.0, 0.0, 16, 0.1, 1.0, dummy, None) == R.EINVAL  # eps 0
    sp = R.ShadowParams(ld, 8.0, 0.01, 16, 0.1, 1.0, 2, 0.0)  # penumbra 2
    assert L.rtsdf_shadow_ex(fine, dummy, dummy, 4, C.byref(sp), None, dummy, None) == R.EINVAL
    sp.penumbra, sp.jitter_scale = 1, -1.0  # negative jitter scale with a jitter array
    assert L.rtsdf_shadow_ex(fine, dummy, dummy, 4, C.byref(sp), dummy, dummy, None) == R.EINVAL
    assert L.rtsdf_shadow_ex(fine, dummy, dummy, 4, None, None, dummy, None) == R.EINVAL
    for bad in (dict(refill=8), dict(loop=5), dict(loop=-1), dict(stack_lds=20), dict(bin_directions=5), dict(blocks_per_cu=-1),
                dict(blocks_per_cu=9), dict(tile_texels=48), dict(tile_texels=0), dict(bvh_width=3),
                dict(bvh_width=8)):
        t = R.TraceTuning(**{**R.rtsdf_trace_config_get().as_dict(), **bad})
        assert L.rtsdf_trace_config(C.byref(t)) == R.EINVAL
        assert L.rtsdf_scene_set_tuning(dummy, C.byref(t)) == R.EINVAL  # rejected before the scene is read
        assert L.rtsdf_batch_set_tuning(dummy, C.byref(t)) == R.EINVAL
    assert L.rtsdf_trace_config(None) == R.EINVAL
    jt = R.JfaTuning(1, 0)
    for n, stage, order in ((4, 1, 0), (512, 1, 0), (48, 1, 0), (64, 3, 0), (64, -1, 0), (64, 1, 5), (64, 1, -1)):
        jt.near_stage, jt.far_order = stage, order
        assert L.rtsdf_jfa_config(n, C.byref(jt)) == R.EINVAL, (n, stage, order)
    assert L.rtsdf_jfa_config(64, None) == R.EINVAL and L.rtsdf_jfa_config_get(64, None) == R.EINVAL
    assert R.rtsdf_jfa_config_get(64) == 0 and R.rtsdf_jfa_config_get(64, "far_order") == 0  # automatic by default
    assert R.rtsdf_jfa_config(64, 1) == 0 and R.rtsdf_jfa_config_get(64) == 1 and R.rtsdf_jfa_config_get(128) == 0
    assert R.rtsdf_jfa_config(64, far_order=2) == 0 and R.rtsdf_jfa_config_get(64, "far_order") == 2
    assert R.rtsdf_jfa_config_get(64) == 1  # setting one field keeps the other
    assert R.rtsdf_jfa_config(64, 0, 0) == (1, 2)
    assert R.rtsdf_jfa_config_get(64) == 0 and R.rtsdf_jfa_config_get(64, "far_order") == 0
    assert L.rtsdf_sqrt(None, 4, dummy, None) == R.EINVAL and L.rtsdf_sqrt(dummy, -1, dummy, None) == R.EINVAL
    assert L.rtsdf_sqrt(None, 0, None, None) == R.OK  # nothing to do
    good = R.rtsdf_trace_config_get()
    assert L.rtsdf_scene_set_tuning(None, C.byref(good)) == R.EINVAL
    assert L.rtsdf_scene_get_tuning(None, C.byref(good)) == R.EINVAL
    assert L.rtsdf_batch_set_tuning(None, C.byref(good)) == R.EINVAL
    # the allocation-free selection validates like rtsdf_select (and needs no workspace)
    assert L.rtsdf_select_noalloc(g, dummy, R.Grid.make(48), 0.0, 0.1, dummy, dummy, 10, dummy, None) == R.EINVAL
    assert L.rtsdf_select_noalloc(R.Grid.make(1024), dummy, R.Grid.make(1024), 0.0, 0.1, dummy, dummy, 10, dummy,
                                  None) == R.EINVAL  # coarse grid beyond the static scratch
    assert L.rtsdf_select_noalloc(g, None, fine, 0.0, 0.1, dummy, dummy, 10, dummy, None) == R.EINVAL
    assert L.rtsdf_select_noalloc(g, dummy, fine, 0.0, float("nan"), dummy, dummy, 10, dummy, None) == R.EINVAL
    assert R.lib().rtsdf_select_noalloc_max_bytes() >= R.rtsdf_select_workspace_size(512)
    assert L.rtsdf_scene_set_sign(None, 0, 0.0) == R.EINVAL
    offs = (C.c_int32 * 3)(0, 1, 2)
    h = C.c_void_p()
    # host checks of a two-level scene: no parts, offsets not ending at nt, an empty moving part (all rejected
    # before any device access)
    assert L.rtsdf_scene_create_instanced(dummy, 3, dummy, 2, offs, 0, dummy, 2, C.byref(h), None) == R.EINVAL
    assert L.rtsdf_scene_create_instanced(dummy, 3, dummy, 3, offs, 2, dummy, 2, C.byref(h), None) == R.EINVAL
    bad = (C.c_int32 * 3)(0, 2, 2)  # the moving part 1 has no face
    assert L.rtsdf_scene_create_instanced(dummy, 3, dummy, 2, bad, 2, dummy, 2, C.byref(h), None) == R.EINVAL
    assert L.rtsdf_scene_set_transforms(None, dummy, None, None) == R.EINVAL
    assert L.rtsdf_scene_hierarchy(None, 10, dummy, dummy, None, None) == R.EINVAL
    assert L.rtsdf_scene_enable_rebuild(None, None) == R.EINVAL
    assert L.rtsdf_scene_rebuild(None, dummy, None) == R.EINVAL
    default = R.rtsdf_trace_config_get().as_dict()
    prev = R.rtsdf_trace_config(refill=16, stack_lds=24)
    assert prev.as_dict() == default and R.rtsdf_trace_config_get().refill == 16
    R.rtsdf_trace_config(**default)
    assert R.rtsdf_select_workspace_size(128) >= (128 ** 3 // 1024) * 4


def test_struct_layouts_match_header(R, tmp_path):
    # compile a C probe against include/rtsdf.h and compare sizes / offsets
    structs = {
        "rtsdf_grid": (R.Grid, ["lo", "h", "n"]),
        "rtsdf_accum": (R.Accum, ["u", "hits", "arg_tri", "arg_ray"]),
        "rtsdf_scene_info": (R.SceneInfo, ["nv", "nt", "nodes", "max_depth", "leaf_size", "device_bytes", "references",
                                            "instances"]),
        "rtsdf_trace_tuning": (R.TraceTuning, ["refill", "blocks_per_cu", "stats", "loop", "bin_directions",
                                               "stack_lds", "tile_texels", "bvh_width"]),
        "rtsdf_frame_desc": (R.FrameDesc, [f for f, _ in R.FrameDesc._fields_]),
        "rtsdf_batch_scene": (R.BatchScene, [f for f, _ in R.BatchScene._fields_]),
        "rtsdf_batch_view": (R.BatchView, [f for f, _ in R.BatchView._fields_]),
        "rtsdf_shadow_params": (R.ShadowParams, [f for f, _ in R.ShadowParams._fields_]),
    }
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "rtsdf.h"', "int main(void) {"]
    for cname, (_, fields) in structs.items():
        src.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fields:
            src.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src.append("  return 0; }")
    c = tmp_path / "probe.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, (cls, fields) in structs.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for f in fields:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)
