"""Write the oracle's state after a prefix of steps of the full-size workloads
(tests/golden/prefix_<name>.npz), for the GPU parity tests at full size.

Calls only the CPU oracle (oracle/) and the seeded workload generators.  Stored
per run: the time, the counters, SHA-256 digests of the cover flags and cover ids
at the end, per patch and state vector the largest magnitude and the sum of
squares of every field over live cells, and the values of a seeded sample of
live cells (half drawn uniformly, half from the band next to the patch
interfaces, where the interpatch fills act).

    python tests/golden/make_prefix_golden.py [name ...]     (default: all)
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import world_from_config  # noqa: E402
from paper_2002_00088_amd import workloads as W  # noqa: E402

# name -> (workload config, steps): the two-patch workload over its whole run,
# the spherical one over a 50-step prefix, the batched and the scaled-down
# multimethod (256^3 + 8 x 96^3, two state vectors) over 3 steps
RUNS = {
    "two_patch_200": (lambda: W.two_patch(seed=2), 200),
    "spherical_50": (lambda: W.spherical(seed=3), 50),
    "batched_3": (lambda: W.batched(seed=4), 3),
    "multimethod_256_96_3": (lambda: W.multimethod(seed=5, ng=256, nl=96), 3),
}
N_GLOBAL = 4096  # sampled cells of the global patch
N_LOCAL = {"two_patch_200": 2048, "spherical_50": 4096, "batched_3": 256, "multimethod_256_96_3": 512}


def band(mask, width):
    """Cells of `mask` within `width` cells (Chebyshev) of a cell outside it or of the array edge."""
    from scipy import ndimage
    outside = np.pad(~mask, 1, constant_values=True)
    near = ndimage.maximum_filter(outside, size=2 * width + 1)[1:-1, 1:-1, 1:-1]
    return mask & near


def sample(rng, mask, nb, n):
    """n flat indices: half uniform over mask, half over the band nb (or mask)."""
    pool_u = np.flatnonzero(mask)
    pool_b = np.flatnonzero(nb) if nb.any() else pool_u
    a = rng.choice(pool_u, size=min(n // 2, pool_u.size), replace=False)
    b = rng.choice(pool_b, size=min(n - a.size, pool_b.size), replace=False)
    return np.unique(np.concatenate([a, b])).astype(np.int64)


def make(name):
    cfg_fn, steps = RUNS[name]
    cfg = cfg_fn()
    t0 = time.time()
    w = world_from_config(cfg)
    w.init_exact(0.0)
    for s in range(steps):
        w.step(cfg["dt"], 1)
        if (s + 1) % 10 == 0 or s + 1 == steps:
            print("%s: step %d/%d, %.0f s" % (name, s + 1, steps, time.time() - t0), flush=True)
    f, c = w.flags()
    rng = np.random.default_rng(2024)
    out = dict(time=np.float64(w.t), steps=np.int64(steps), dt=np.float64(cfg["dt"]),
               flags_sha256=np.bytes_(hashlib.sha256(f.tobytes()).hexdigest()),
               cover_sha256=np.bytes_(hashlib.sha256(c.astype(np.int32).tobytes()).hexdigest()))
    for k, v in w.counters().items():
        out["counter_" + k] = np.int64(v)
    nsv = len(cfg["wave_speed"])
    for pid, p in enumerate(cfg["patches"]):
        n = p["n"]
        if pid == 0 and len(cfg["patches"]) > 1:
            live = f == 0
            nb = band(live, 6)
            idx = sample(rng, live, nb, N_GLOBAL)
        else:
            live = np.ones((n[2], n[1], n[0]), dtype=bool)
            inner = np.zeros_like(live)
            inner[4:-4, 4:-4, 4:-4] = True
            idx = sample(rng, live, live & ~inner, N_LOCAL[name] if pid > 0 else N_GLOBAL)
        out["idx_%d" % pid] = idx
        for sv in range(nsv):
            if not p["sv_mask"] & (1 << sv):
                continue
            u = w.get_state(pid, sv).reshape(5, -1)
            lv = live.reshape(-1)
            out["max_%d_%d" % (pid, sv)] = np.abs(u[:, lv]).max(axis=1)
            out["sumsq_%d_%d" % (pid, sv)] = (u[:, lv] ** 2).sum(axis=1)
            out["val_%d_%d" % (pid, sv)] = u[:, idx]
    w.close()
    path = os.path.join(HERE, "prefix_%s.npz" % name)
    np.savez_compressed(path, **out)
    print("%s: wrote %s (%.0f KB), %.0f s" % (name, path, os.path.getsize(path) / 1024, time.time() - t0),
          flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(RUNS):
        make(nm)
