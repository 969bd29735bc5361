"""The oracle built with the address and undefined-behaviour sanitizers (gcc,
host code only) runs its whole pipeline on small inputs without a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-ffp-contract=off", *san,
           os.path.join(ROOT, "oracle", "subsurf4d_oracle.c"), os.path.join(ROOT, "tests", "oracle_sanitize_main.c"),
           "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower() and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtime not installed")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "oracle sanitizer run ok" in r.stdout


_THREADS_SNIPPET = r"""
import hashlib, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle as orc
h = hashlib.sha256()
n = (17, 13, 11, 6)
rng = np.random.default_rng(5)
G = rng.uniform(0.05, 1.0, size=(4,) + orc.padded_shape(n))
w = np.zeros(orc.padded_shape(n))
w[1:-1, 1:-1, 1:-1, 1:-1] = rng.uniform(0.0, 1.0, size=orc.interior_shape(n))
coef, b = orc.assemble(n, G, w, 1.0, 1e-3, 0.5)
u, it, rr, st = orc.sor(n, coef, b, w, 1.6, 1e-12, 5000, orc.RB)
h.update(u.tobytes()); h.update(np.float64(rr).tobytes())
img = rng.uniform(0.0, 1.0, size=orc.interior_shape(n))
cs = np.array([(5.0, 6.0, 4.0, l) for l in range(n[3])], dtype=np.float64)
prep = orc.prepare(n, img, [tuple(c[:3]) + (int(c[3]),) for c in cs], orc.PrepareParams(ball_r=4.0))
h.update(prep["G"].tobytes())
print(orc.num_threads(), it, h.hexdigest())
"""


def test_oracle_threads_bitwise():
    """Race check of the oracle's OpenMP loops (ThreadSanitizer does not see
    the synchronisation of gcc's uninstrumented OpenMP runtime, so it reports
    the thread pool's reuse of shared stack variables): the red-black SOR,
    its residual and the preparation give the same bits with 1, 2 and 8
    threads.  A colour phase that read its own colour, or a reduction in
    thread order, would depend on the thread count."""
    import subprocess
    import sys

    outs = []
    for t in ("1", "2", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        r = subprocess.run([sys.executable, "-c", _THREADS_SNIPPET, ROOT], capture_output=True, text=True, env=env,
                           timeout=300)
        assert r.returncode == 0, r.stderr
        threads, it, digest = r.stdout.split()
        assert threads == t
        outs.append((it, digest))
    assert outs[0] == outs[1] == outs[2], outs
