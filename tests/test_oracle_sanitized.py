"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): every entry point on small inputs, including the edge cases
(one point, coincident points, leaves of several points, far-field orders,
target vectors), in a child process with the sanitized build; any report
fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import numpy as np
import oracle, synth
rng = np.random.default_rng(0)
for n in (1, 2, 57):
    x = rng.uniform(-0.9, 0.9, (n, 3))
    if n > 2:
        x[:5] = x[0]
    mu = rng.standard_normal((n, 3))
    g = rng.standard_normal(n)
    for op, nu in (("A", mu), ("AT", g), ("G", mu)):
        oracle.direct(op, x, nu, 0.01)
    oracle.direct("P", x, g, 0.01, tvec=mu)
    oracle.direct("T", x, mu, 0.01, tvec=mu)
    for K in (1, 4):
        T = oracle.Tree(x, leaf_cap=K)
        T.export()
        T.reps(mu)
        T.reps(g)
        for order in (0, 1, 2):
            for op, nu in (("A", mu), ("AT", g), ("G", mu)):
                T.apply(op, nu, 0.01, 2.0, order=order, wsafe=bool(order % 2), with_stats=True)
        T.apply("P", g, 0.01, 2.0, tvec=mu)
        T.apply("T", mu, 0.01, 2.0, tvec=mu[: max(1, n // 2)], targets=x[: max(1, n // 2)])
        del T
    oracle.Tree(x, max_depth=2).apply("G", mu, 0.0, 0.5)
c = synth.fibonacci_sphere(300, 0)
xn, _, _ = oracle.normalize(c.points)
oracle.orient(xn, iters=3, order=2, wsafe=True)
oracle.winding_grad_x(xn, c.normals, np.ones(300), 0.002, backend="tree")
oracle.gradient_grad_x(xn, c.normals, c.normals, 0.002, backend="tree")
print("sanitized run done")
'''


def _gcc_lib(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    p = out.stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_sanitizers(tmp_path):
    asan = _gcc_lib("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = tmp_path / "liboracle_san.so"
    src = os.path.join(ROOT, "oracle", "wnnc_oracle.c")
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", src, "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ)
    env.update(WNNC_ORACLE_LIB=str(lib), LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24",
               PYTHONPATH=ROOT + os.pathsep + env.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
    assert "sanitized run done" in r.stdout
