"""The oracle (plain C, test infrastructure) built with gcc's address and
undefined-behaviour sanitizers, and separately with the thread sanitizer, and
run through every entry point on the tiny scene (tests/sanitize/oracle_driver.c).
Any invalid access, leak, undefined operation or data race between its OpenMP
threads fails the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", "rtsdf_oracle.c"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")]
BASE = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def mesh_file(tmp_path_factory):
    from synth.scenes import tiny_scene
    m = tiny_scene()
    p = tmp_path_factory.mktemp("san") / "mesh.bin"
    with open(p, "wb") as f:
        np.array([m.nv, m.nt], np.int32).tofile(f)
        np.ascontiguousarray(m.vertices, np.float32).tofile(f)
        np.ascontiguousarray(m.faces, np.int32).tofile(f)
    return str(p)


def build_and_run(tmp_path, mesh_file, flags, env):
    exe = str(tmp_path / "driver")
    subprocess.run(BASE + flags + SRC + ["-lm", "-o", exe], check=True, capture_output=True, text=True)
    res = subprocess.run([exe, mesh_file], capture_output=True, text=True, timeout=600,
                         env={**os.environ, "OMP_NUM_THREADS": "4", **env})
    return res


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_ub_sanitizers(tmp_path, mesh_file):
    res = build_and_run(tmp_path, mesh_file, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                        {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"})
    print(res.stdout, res.stderr[-4000:])
    assert res.returncode == 0, res.stderr[-4000:]
    assert "driver ok" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr


# The thread sanitizer needs an OpenMP runtime that tells it about its barriers: gcc's libgomp does not (every
# region boundary then reads as a race), LLVM's libomp does through its Archer tool.
LLVM = "/opt/rocm/llvm"
CLANG, ARCHER = os.path.join(LLVM, "bin", "clang"), os.path.join(LLVM, "lib", "libarcher.so")
TSAN_ENV = {"OMP_TOOL_LIBRARIES": ARCHER, "TSAN_OPTIONS": "ignore_noninstrumented_modules=1:halt_on_error=1"}


def tsan_build(srcs, exe):
    subprocess.run([CLANG, "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fsanitize=thread", *srcs,
                    "-lm", "-o", exe, f"-Wl,-rpath,{LLVM}/lib"], check=True, capture_output=True, text=True)


@pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(ARCHER)), reason="needs LLVM clang + Archer")
def test_oracle_under_thread_sanitizer(tmp_path, mesh_file):
    # control: the same build flags must catch a planted race (an unsynchronised shared sum)
    ctl = tmp_path / "race.c"
    ctl.write_text("#include <stdio.h>\nint main(void){long s=0;\n#pragma omp parallel for\n"
                   "for(int i=0;i<100000;++i) s+=i;\nprintf(\"%ld\\n\",s);return 0;}\n")
    tsan_build([str(ctl)], str(tmp_path / "race"))
    r = subprocess.run([str(tmp_path / "race")], capture_output=True, text=True, timeout=120,
                       env={**os.environ, "OMP_NUM_THREADS": "4", **TSAN_ENV})
    assert r.returncode != 0 and "data race" in r.stderr
    exe = str(tmp_path / "driver_tsan")
    tsan_build(SRC, exe)
    res = subprocess.run([exe, mesh_file], capture_output=True, text=True, timeout=600,
                         env={**os.environ, "OMP_NUM_THREADS": "4", **TSAN_ENV})
    print(res.stdout, res.stderr[-4000:])
    assert res.returncode == 0, res.stderr[-4000:]
    assert "driver ok" in res.stdout and "ThreadSanitizer" not in res.stderr
