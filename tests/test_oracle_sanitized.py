"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (host code only):
oracle.c is built with -fsanitize=address,undefined into a temporary directory, and a child
process loads that build and runs periodic, bounded, large-cell, grid and structure cases.  Any
sanitizer report fails the child (halt_on_error), and the child's results must equal the plain
build's."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import ctypes, json, os, sys
import numpy as np
sys.path.insert(0, %(root)r)
import oracle
oracle._LIB = %(lib)r
oracle.build = lambda force=False: oracle._LIB
from paper_1601_06429_amd import workloads as wl
out = {}
p = wl.uniform4096().pos
c = oracle.cells(p, 0.0, 1.0, query=np.arange(0, 4096, 37), nthreads=2)
out["periodic"] = [float(c.volume.sum()), int(c.nnb.sum())]
rng = np.random.default_rng(5)
b = rng.random((800, 3)) * [1.0, 2.0, 0.5]
c = oracle.cells(b, 0.0, [1.0, 2.0, 0.5], periodic=False, query=np.arange(0, 800, 7), nthreads=2)
out["bounded"] = [float(c.volume.sum()), int(c.nnb.sum()), int(c.flags.sum())]
m = 90
k = np.arange(m) + 0.5
phi = np.arccos(1 - 2 * k / m)
th = np.pi * (1 + 5 ** 0.5) * k
sph = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1) * 0.05
bg = rng.random((600, 3))
bg = bg[np.linalg.norm(bg - 0.5, axis=1) > 0.12]
q = np.concatenate([[[0.5, 0.5, 0.5]], 0.5 + sph, bg])
c = oracle.cells(q, 0.0, 1.0, query=[0, 1, 2], stride=256, nthreads=2)
out["large"] = [float(c.volume.sum()), int(c.nnb.sum())]
g = oracle.grid(p[:512], 0.0, 1.0, True, np.ones(512), (6, 5, 7), query=np.arange(0, 512, 9), nthreads=2)
out["grid"] = float(g.sum())
v, f = oracle.structure(p, 0.0, 1.0, 17)
out["structure"] = [len(v), len(f)]
print(json.dumps(out))
"""


def _run(lib, env):
    r = subprocess.run([sys.executable, "-c", CHILD % {"root": ROOT, "lib": lib}], capture_output=True, text=True,
                       env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return r.stdout.strip().splitlines()[-1]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    import oracle

    d = tempfile.mkdtemp(prefix="oracle_asan_")
    try:
        lib = os.path.join(d, "liboracle_asan.so")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
                               "-fno-omit-frame-pointer", "-shared", "-fPIC", "-o", lib,
                               os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
        asan_rt = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
        ubsan_rt = subprocess.check_output(["gcc", "-print-file-name=libubsan.so"], text=True).strip()
        env = dict(os.environ)
        env["LD_PRELOAD"] = ":".join(x for x in (asan_rt, ubsan_rt, env.get("LD_PRELOAD", "")) if x)
        env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
        env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
        env["OMP_NUM_THREADS"] = "2"
        sanitized = _run(lib, env)
        plain_env = dict(os.environ, OMP_NUM_THREADS="2")
        plain = _run(oracle.build(), plain_env)
        assert sanitized == plain
    finally:
        shutil.rmtree(d, ignore_errors=True)
