"""Sanitizer builds of the host code (CPU only).

The planner, engine, C-ABI and serving sources are compiled with g++ under
AddressSanitizer + UndefinedBehaviorSanitizer (errors fatal, leak check on)
and, separately, under ThreadSanitizer, linked with the library's HIP objects,
and driven by tests/sanitize/driver.cpp through the C-ABI on host-only
contexts: dense planning of the n=30 workload and of random circuits of every
gate kind, light-cone sets at n=500, plan records, invalid input, and the
serving loop with a simulated executor under concurrent submit, poll, cancel,
statistics and shutdown.  A sanitizer report or a wrong return code fails the
test.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_10239_amd", "csrc")
HOST_SOURCES = ["planner.cpp", "engine.cpp", "api.cpp", "serve.cpp"]
HIP_OBJECTS = ["kernels.o", "density.o", "coef.o", "noalloc.o", "block.o"]
VARIANTS = {
    "asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
    "tsan": ["-fsanitize=thread"],
}


def _hip_objects():
    bdir = os.path.join(ROOT, "paper_2112_10239_amd", "_build")
    objs = [os.path.join(bdir, o) for o in HIP_OBJECTS]
    if not all(os.path.exists(o) for o in objs):
        from paper_2112_10239_amd import build as b

        b.build()
    return objs


def _compile(args):
    cmd, out = args
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stderr[-4000:]}"
    return out


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    objs = _hip_objects()
    out = {}
    jobs = []
    inc = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    for name, flags in VARIANTS.items():
        d = tmp_path_factory.mktemp(name)
        srcs = [os.path.join(CSRC, s) for s in HOST_SOURCES] + [os.path.join(ROOT, "tests", "sanitize", "driver.cpp")]
        for s in srcs:
            o = str(d / (os.path.basename(s) + ".o"))
            jobs.append(((["g++", "-O1", "-g", "-std=c++17", "-w", *flags, *inc, "-c", s, "-o", o], o), name))
        out[name] = (d, flags)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 2)) as ex:
        built = list(ex.map(lambda j: (j[1], _compile(j[0])), jobs))
    exes = {}
    for name, (d, flags) in out.items():
        mine = [o for n, o in built if n == name]
        exe = str(d / f"driver_{name}")
        _compile((["g++", *flags, *mine, *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
                   "-lpthread", "-o", exe], exe))
        exes[name] = exe
    return exes


def _run(exe, *args, env_extra=None):
    env = dict(os.environ, **(env_extra or {}))
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=300, env=env)
    text = r.stdout + r.stderr
    return r.returncode, text


def test_asan_ubsan_host_code(drivers):
    rc, text = _run(drivers["asan"], env_extra={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"})
    assert rc == 0, text[-6000:]
    assert "driver: 0 failures" in text
    assert "ERROR: AddressSanitizer" not in text and "runtime error" not in text


def test_tsan_serving_loop(drivers):
    rc, text = _run(drivers["tsan"], "serving", env_extra={"TSAN_OPTIONS": "halt_on_error=1"})
    assert rc == 0, text[-6000:]
    assert "driver: 0 failures" in text and "completed" in text
    assert "WARNING: ThreadSanitizer" not in text
