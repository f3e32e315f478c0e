"""Seeded synthetic workloads (patch layouts, exact-solution parameters, time steps).

This module only draws random numbers and lays out parameters.  It holds none
of the step's arithmetic (no maps, metric, stencils, interpolation or
transforms): the GPU library and the CPU oracle each receive the same plain
dictionaries and compute everything themselves.

Patch dictionaries use the keys of the library's patch description:
coord (0 Cartesian, 1 spherical), is_global, n (cells per numerical axis),
lo/hi (numerical box faces), periodic, euler (ZYZ angles), motion
(0 static, 1 linear, 2 circle), c0, vel, radius, speed, phase, sv_mask.
"""
import math

import numpy as np

CART, SPH = 0, 1
STATIC, LINEAR, CIRCLE = 0, 1, 2


def patch(n, lo, hi, coord=CART, is_global=0, periodic=(0, 0, 0), euler=(0.0, 0.0, 0.0), motion=STATIC,
          c0=(0.0, 0.0, 0.0), vel=(0.0, 0.0, 0.0), radius=0.0, speed=0.0, phase=0.0, sv_mask=1):
    return dict(n=[int(x) for x in n], lo=[float(x) for x in lo], hi=[float(x) for x in hi], coord=int(coord),
                is_global=int(is_global), periodic=[int(x) for x in periodic], euler=[float(x) for x in euler],
                motion=int(motion), c0=[float(x) for x in c0], vel=[float(x) for x in vel], radius=float(radius),
                speed=float(speed), phase=float(phase), sv_mask=int(sv_mask))


def random_euler(rng):
    """Uniformly random orientation as ZYZ angles."""
    return [float(rng.uniform(0, 2 * math.pi)), float(math.acos(rng.uniform(-1, 1))),
            float(rng.uniform(0, 2 * math.pi))]


def gauss_sum(rng, n, center_box, wmin=0.2, wmax=1.0, amin=0.5, amax=1.0):
    return dict(kind="gauss", amp=list(rng.uniform(amin, amax, n)),
                centers=rng.uniform(-center_box, center_box, (n, 3)).tolist(),
                widths=list(rng.uniform(wmin, wmax, n)))


def spacing_min(p):
    """Smallest physical cell spacing of a patch description (for the CFL choice)."""
    dx = [(p["hi"][a] - p["lo"][a]) / p["n"][a] for a in range(3)]
    if p["coord"] == CART:
        return min(dx)
    r_in = p["lo"][0]
    s_min = min(math.sin(p["lo"][1]), math.sin(p["hi"][1]))
    return min(dx[0], r_in * dx[1], r_in * s_min * dx[2])


def _finish(cfg, cfl=0.25):
    cfg.setdefault("ko_eps", 0.005)
    cfg.setdefault("buffer", 4)
    if "dt" not in cfg:
        cfg["dt"] = cfl * min(spacing_min(p) for p in cfg["patches"])
    return cfg


# --------------------------------------------------------------------------
# Configurations.  Sizes default to the full workloads; tests pass smaller n.
# --------------------------------------------------------------------------

def single_periodic(seed=1, n=32, steps=20):
    """One periodic Cartesian patch on [0,1)^3 with a plane wave of integer wave
    vector k in [1,3]^3 (wave speed 1, 4th-order FD, RK4, CFL 0.25)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 4, 3)
    nn = [n, n, n] if np.isscalar(n) else list(n)
    g = patch(nn, [0, 0, 0], [1, 1, 1], is_global=1, periodic=(1, 1, 1))
    ex = dict(kind="plane", A=1.0, B=0.0, kappa=[2 * math.pi * float(x) for x in k], psi=0.0)
    cfg = dict(name="periodic_%d" % nn[0], wave_speed=[1.0], interp_points=[6], patches=[g], exact=[ex],
               steps=steps, dt=0.25 / max(nn))
    return _finish(cfg)


def two_patch(seed=2, ng=128, nl=64, P=5, steps=200, motion=CIRCLE):
    """Global Cartesian [-8,8]^3 (ng^3) with analytic outer ghosts, plus a rotated
    Cartesian local patch of nl^3 cells at half the global spacing, moving on a
    circle of radius 2 at speed 0.1; one Gaussian pulse of width 0.5."""
    rng = np.random.default_rng(seed)
    L = 8.0
    dxg = 2 * L / ng
    half = nl * dxg / 4.0
    g = patch([ng] * 3, [-L] * 3, [L] * 3, is_global=1)
    eu = random_euler(rng)
    if motion == CIRCLE:
        loc = patch([nl] * 3, [-half] * 3, [half] * 3, euler=eu, motion=CIRCLE, radius=2.0, speed=0.1, phase=0.0)
    else:
        loc = patch([nl] * 3, [-half] * 3, [half] * 3, euler=eu, motion=motion, c0=(0.3, -0.2, 0.1),
                    vel=(0.1, 0.05, -0.02) if motion == LINEAR else (0, 0, 0))
    x0 = rng.uniform(-2, 2, 3)
    ex = dict(kind="gauss", amp=[1.0], centers=[list(x0)], widths=[0.5])
    cfg = dict(name="two_patch_%d_%d" % (ng, nl), wave_speed=[1.0], interp_points=[P], patches=[g, loc],
               exact=[ex], steps=steps)
    return _finish(cfg)


def quadrupole_pulse(rng, d=1.0, w=0.6):
    """Seeded l=2-type pulse: four Gaussians at +-d on two orthogonal, randomly
    oriented axes with alternating signs and seeded amplitudes."""
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    a = rng.uniform(0.5, 1.0, 2)
    centers = [list(d * q[:, 0]), list(-d * q[:, 0]), list(d * q[:, 1]), list(-d * q[:, 1])]
    return dict(kind="gauss", amp=[a[0], a[0], -a[1], -a[1]], centers=centers, widths=[w] * 4)


def spherical(seed=3, ng=256, nr=64, nth=64, nph=128, steps=500):
    """Global Cartesian [-8,8]^3 plus a static spherical local patch
    r in [0.5,6], theta in [pi/4,3pi/4], phi periodic, centred at the origin."""
    rng = np.random.default_rng(seed)
    L = 8.0
    g = patch([ng] * 3, [-L] * 3, [L] * 3, is_global=1)
    s = patch([nr, nth, nph], [0.5, math.pi / 4, 0.0], [6.0, 3 * math.pi / 4, 2 * math.pi], coord=SPH,
              periodic=(0, 0, 1))
    ex = quadrupole_pulse(rng)
    cfg = dict(name="spherical_%d" % ng, wave_speed=[1.0], interp_points=[6], patches=[g, s], exact=[ex],
               steps=steps)
    return _finish(cfg)


def _obb_corners(c, R, lo, hi):
    pts = []
    for m in range(8):
        y = np.array([hi[0] if m & 1 else lo[0], hi[1] if m & 2 else lo[1], hi[2] if m & 4 else lo[2]])
        pts.append(c + R @ y)
    return np.array(pts)


def _rot(eu):
    a, b, c = eu
    Z1 = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    Y = np.array([[math.cos(b), 0, math.sin(b)], [0, 1, 0], [-math.sin(b), 0, math.cos(b)]])
    Z2 = np.array([[math.cos(c), -math.sin(c), 0], [math.sin(c), math.cos(c), 0], [0, 0, 1]])
    return Z1 @ Y @ Z2


def _separated(A, B):
    """Separating-axis test between two convex bodies given as (corners, axes)."""
    (pa, ax_a), (pb, ax_b) = A, B
    axes = list(ax_a) + list(ax_b)
    for u in ax_a:
        for v in ax_b:
            c = np.cross(u, v)
            if np.linalg.norm(c) > 1e-9:
                axes.append(c / np.linalg.norm(c))
    for ax in axes:
        a = pa @ ax
        b = pb @ ax
        if a.max() < b.min() or b.max() < a.min():
            return True
    return False


def batched(seed=4, ng=256, nlocal=64, nmin=24, nmax=96, frac_cart=0.7, vmax=0.2, steps=23, margin=4,
            max_tries=3000):
    """Global Cartesian [-8,8]^3 plus `nlocal` moving local patches of uneven
    sizes: per-axis cells from [nmin,nmax], 70/30 Cartesian/spherical, random
    orientation, linear velocity |v| <= vmax, resolution 1-4x the global one.
    Placement: largest first, oriented-box separating-axis test with a margin of
    `margin` global cells plus the motion sweep; on failure the refinement ratio
    grows by 1.25 (cap 4), then the cell counts shrink by 0.8."""
    rng = np.random.default_rng(seed)
    L = 8.0
    dxg = 2 * L / ng
    g = patch([ng] * 3, [-L] * 3, [L] * 3, is_global=1)
    descs = []
    for _ in range(nlocal):
        n = rng.integers(nmin, nmax + 1, 3)
        coord = CART if rng.uniform() < frac_cart else SPH
        ratio = rng.uniform(1.0, 4.0)
        eu = random_euler(rng)
        vdir = rng.normal(size=3)
        vdir /= np.linalg.norm(vdir)
        vel = vdir * vmax * rng.uniform() ** (1.0 / 3.0)
        descs.append(dict(n=n, coord=coord, ratio=ratio, euler=eu, vel=vel))

    def geometry(d):
        dx = dxg / d["ratio"]
        n = d["n"]
        if d["coord"] == CART:
            half = n * dx / 2.0
            return dict(lo=-half, hi=half, dx=dx)
        r_in = max(n[1] * dx / 2.0, 6 * dx)
        return dict(lo=np.array([r_in, math.pi / 4, 0.0]), hi=np.array([r_in + n[0] * dx, 3 * math.pi / 4, 2 * math.pi]),
                    dx=dx)

    def extent(d):
        gm = geometry(d)
        if d["coord"] == CART:
            return float(np.linalg.norm(gm["hi"]))
        return float(gm["hi"][0])

    order = sorted(range(nlocal), key=lambda i: -extent(descs[i]))
    t_end = (steps + 1) * 0.25 * dxg / 4.0 * 4  # generous motion sweep
    placed = []
    locs = []
    for i in order:
        d = descs[i]
        ok = False
        for attempt in range(200):
            gm = geometry(d)
            R = _rot(d["euler"])
            ext = extent(d)
            pad = margin * dxg + np.linalg.norm(d["vel"]) * t_end
            room = L - ext - pad - 6 * dxg
            if room > 0:
                for _ in range(max_tries // 20):
                    c = rng.uniform(-room, room, 3)
                    if d["coord"] == CART:
                        body = (_obb_corners(c, R, gm["lo"] - pad, gm["hi"] + pad), [R[:, 0], R[:, 1], R[:, 2]])
                    else:
                        r = gm["hi"][0] + pad
                        body = (_obb_corners(c, np.eye(3), -np.full(3, r), np.full(3, r)), [np.eye(3)[k] for k in range(3)])
                    if all(_separated(body, other) for other in placed):
                        placed.append(body)
                        ok = True
                        break
            if ok:
                break
            if d["ratio"] < 4.0:
                d["ratio"] = min(4.0, d["ratio"] * 1.25)
            else:
                d["n"] = np.maximum(nmin, (0.8 * d["n"]).astype(int))
        if not ok:
            continue
        gm = geometry(d)
        if d["coord"] == CART:
            locs.append(patch(d["n"], gm["lo"], gm["hi"], euler=d["euler"], motion=LINEAR, c0=c, vel=d["vel"]))
        else:
            locs.append(patch(d["n"], gm["lo"], gm["hi"], coord=SPH, periodic=(0, 0, 1), euler=d["euler"],
                              motion=LINEAR, c0=c, vel=d["vel"]))
    ex = gauss_sum(rng, 16, 6.0)
    cfg = dict(name="batched_%d_%d" % (ng, len(locs)), wave_speed=[1.0], interp_points=[6], patches=[g] + locs,
               exact=[ex], steps=steps)
    return _finish(cfg)


def multimethod(seed=5, ng=512, nl=192, steps=100):
    """Global Cartesian [-16,16]^3 plus 8 Cartesian locals of nl^3 cells at half
    the global spacing on a jittered 2x2x2 lattice.  State vector A (speed 1)
    lives on every patch; state vector B (speed 0.5) on locals 1-4 only."""
    rng = np.random.default_rng(seed)
    L = 16.0
    dxg = 2 * L / ng
    half = nl * dxg / 4.0
    g = patch([ng] * 3, [-L] * 3, [L] * 3, is_global=1, sv_mask=1)
    locs = []
    k = 0
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                c = np.array([8.0 * sx, 8.0 * sy, 8.0 * sz]) * (L / 16.0) + rng.uniform(-1, 1, 3) * (L / 16.0)
                vdir = rng.normal(size=3)
                vel = vdir / np.linalg.norm(vdir) * 0.2 * rng.uniform() ** (1 / 3)
                mask = 3 if k < 4 else 1
                locs.append(patch([nl] * 3, [-half] * 3, [half] * 3, euler=random_euler(rng), motion=LINEAR, c0=c,
                                  vel=vel, sv_mask=mask))
                k += 1
    exA = gauss_sum(rng, 16, 12.0 * L / 16.0)
    exB = gauss_sum(rng, 16, 12.0 * L / 16.0)
    cfg = dict(name="multimethod_%d_%d" % (ng, nl), wave_speed=[1.0, 0.5], interp_points=[6, 6],
               patches=[g] + locs, exact=[exA, exB], steps=steps)
    return _finish(cfg)


def random_state(shape, seed):
    """Seeded smooth-ish random field values (inputs only)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, shape)


def live_cells(cfg, flags=None):
    """Cells evolved per step: all local interior cells plus live global cells."""
    n = 0
    for p in cfg["patches"][1:]:
        n += int(np.prod(p["n"])) * bin(p["sv_mask"]).count("1")
    g = cfg["patches"][0]
    if flags is None:
        n += int(np.prod(g["n"])) * bin(g["sv_mask"]).count("1")
    else:
        n += int((flags == 0).sum()) * bin(g["sv_mask"]).count("1")
    return n
