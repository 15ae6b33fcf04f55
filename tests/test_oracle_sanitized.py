"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, gcc): a build of oracle.c with both sanitizers runs the
entry points the tests use -- blocks of every pair class for the Laplace
and Helmholtz kernels and both layers, the quadrature rules, piecewise-linear
local matrices, Green matrices and the pivot-block inverse -- on a small
mesh in a subprocess; any report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
import numpy as np
import oracle
oracle.use_library(sys.argv[1])
from bem_inputs import octahedron_sphere
m = octahedron_sphere(4)
idx = np.arange(m.nt)
for kernel, kappa in ((0, 0.0), (1, 3.0)):
    for layer in (0, 1):
        G = oracle.block(m.v, m.tri, idx[:48], idx[:48], kernel=kernel, kappa=kappa, layer=layer,
                         q_reg=3, q_sing=3)
        assert np.all(np.isfinite(G)), (kernel, layer)
        L = oracle.p1_pairs(m.v, m.tri, idx[:16], idx[8:24], kernel=kernel, layer=layer,
                            kappa=kappa, q_reg=3, q_sing=3)
        assert np.all(np.isfinite(L))
for q in (1, 4, 9):
    x, w = oracle.gauss01(q)
    assert abs(w.sum() - 1.0) < 1e-14
for cs in (1, 2, 3):
    pts, w = oracle.ss_rule(cs, 3)
    assert np.all(np.isfinite(w))
rng = np.random.default_rng(0)
A = rng.standard_normal((6, 6)) + 6 * np.eye(6)
P = oracle.inverse(A)
assert np.allclose(P @ A, np.eye(6))
print("sanitized oracle ok")
"""


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = asan.stdout.strip()
    if asan.returncode or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = str(tmp_path / "liboracle_sanitized.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", lib,
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    env = dict(os.environ, LD_PRELOAD=path, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", SCRIPT, lib], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    report = r.stderr
    assert r.returncode == 0, report[-3000:]
    assert "sanitized oracle ok" in r.stdout
    assert "runtime error" not in report and "AddressSanitizer" not in report, report[-3000:]
