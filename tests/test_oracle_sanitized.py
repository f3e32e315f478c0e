"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer runs
a few steps of every kind of workload without a report.

The sanitized library is loaded into a child Python process that preloads
gcc's libasan (leak detection off: the interpreter itself keeps memory until
exit); any out-of-bounds access, use after free or undefined operation in the
oracle ends that process with a report and a non-zero status.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, %(root)r)
from oracle import oracle as O
assert O.SANITIZE
O.build(force=True)
from paper_2002_00088_amd import workloads as W
cases = [
    ("periodic", W.single_periodic(seed=1, n=(12, 10, 8))),
    ("two_patch_circle_P5", W.two_patch(seed=2, ng=24, nl=16, P=5)),
    ("spherical_local", W.spherical(seed=3, ng=48, nr=40, nth=16, nph=32)),
    ("batched", W.batched(seed=4, ng=64, nlocal=8, nmin=16, nmax=24)),
    ("multimethod_two_vectors", W.multimethod(seed=5, ng=64, nl=24)),
    ("three_topology", W.three_topology(scale=0.5, steps=2)),
    ("test_four", W.test_four(scale=0.6, steps=2)),
]
for name, cfg in cases:
    for extra in ({}, {"buffer": 2}, {"pi_form": 1}, {"outer_bc": 1}):
        if extra and name not in ("two_patch_circle_P5",):
            continue
        c = dict(cfg, **extra)
        w = O.world_from_config(c)
        w.init_exact(0.0)
        w.step(c["dt"], 2 if name in ("periodic", "two_patch_circle_P5") else 1)
        w.exchange_ghosts(w.t)
        f, cov = w.flags()
        for pid in range(len(c["patches"])):
            w.diag(pid)
        w.close()
        print("ok", name, extra, flush=True)
"""


def test_oracle_under_address_and_ub_sanitizers():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's libasan is not installed")
    # the sanitizer runtime must come first; whatever the environment already
    # preloads stays preloaded after it
    pre = os.environ.get("LD_PRELOAD", "")
    env = dict(os.environ, PW_ORACLE_SANITIZE="1", LD_PRELOAD=asan + (":" + pre if pre else ""), OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", SCRIPT % {"root": ROOT}], env=env, capture_output=True, text=True,
                       timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert out.count("ok ") == 10, out[-2000:]
