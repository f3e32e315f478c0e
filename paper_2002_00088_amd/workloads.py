"""Seeded synthetic workloads (patch layouts, exact-solution parameters, time steps).

This module only draws random numbers and lays out parameters.  It holds none
of the step's arithmetic (no maps, metric, stencils, interpolation or
transforms): the GPU library and the CPU oracle each receive the same plain
dictionaries and compute everything themselves.

Patch dictionaries use the keys of the library's patch description:
coord (0 Cartesian, 1 spherical, 2 cylindrical), is_global, n (cells per numerical axis),
lo/hi (numerical box faces), periodic, euler (ZYZ angles), motion
(0 static, 1 linear, 2 circle), c0, vel, radius, speed, phase, sv_mask, spin.
"""
import math

import numpy as np

CART, SPH, CYL = 0, 1, 2
STATIC, LINEAR, CIRCLE = 0, 1, 2


def patch(n, lo, hi, coord=CART, is_global=0, periodic=(0, 0, 0), euler=(0.0, 0.0, 0.0), motion=STATIC,
          c0=(0.0, 0.0, 0.0), vel=(0.0, 0.0, 0.0), radius=0.0, speed=0.0, phase=0.0, sv_mask=1,
          spin=(0.0, 0.0, 0.0)):
    """spin: angular velocity (background frame) of a rotation of the patch about
    its centre, R(t) = rotation by |spin| t about spin/|spin| composed with the
    Euler rotation."""
    return dict(n=[int(x) for x in n], lo=[float(x) for x in lo], hi=[float(x) for x in hi], coord=int(coord),
                is_global=int(is_global), periodic=[int(x) for x in periodic], euler=[float(x) for x in euler],
                motion=int(motion), c0=[float(x) for x in c0], vel=[float(x) for x in vel], radius=float(radius),
                speed=float(speed), phase=float(phase), sv_mask=int(sv_mask), spin=[float(x) for x in spin])


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
    if p["coord"] == CYL:
        return min(dx[0], r_in * dx[1], dx[2])
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


def test_two(motion="fixed", ng=40, P=6, cfl=0.6, t_end=20.0):
    """The paper's convergence test (Sec. 3.2, Test Two): global Cartesian cube
    [-20, 20]^3 with ng^3 cells, a Cartesian local cube [-10, 10]^3 at twice the
    resolution (2-to-1), plane wave phi = sin(2 pi (x - t)/20) + 2 (Eq.
    wave_solution) with analytic outer ghosts, CFL 0.6 on the local spacing, up to
    t = 20 (one wave period).  motion: "fixed" (centre (-1, -1, -1)), "rotating"
    (centre at the origin, spin 0.01 about z, counter-clockwise) or "translating"
    (from (-5, -5, 0) at velocity (0.1, 0.1, 0))."""
    g = patch([ng] * 3, [-20.0] * 3, [20.0] * 3, is_global=1)
    nl = ng
    if motion == "fixed":
        loc = patch([nl] * 3, [-10.0] * 3, [10.0] * 3, c0=(-1.0, -1.0, -1.0))
    elif motion == "rotating":
        loc = patch([nl] * 3, [-10.0] * 3, [10.0] * 3, spin=(0.0, 0.0, 0.01))
    elif motion == "translating":
        loc = patch([nl] * 3, [-10.0] * 3, [10.0] * 3, motion=LINEAR, c0=(-5.0, -5.0, 0.0), vel=(0.1, 0.1, 0.0))
    else:
        raise ValueError(motion)
    ex = dict(kind="plane", A=1.0, B=2.0, kappa=[2 * math.pi / 20.0, 0.0, 0.0], psi=0.0)
    dt0 = cfl * 20.0 / nl
    steps = int(math.ceil(t_end / dt0 - 1e-9))
    return dict(name="test_two_%s_%d" % (motion, ng), wave_speed=[1.0], interp_points=[P], patches=[g, loc],
                exact=[ex], ko_eps=0.005, buffer=4, dt=t_end / steps, steps=steps)


def three_topology(scale=1.0, steps=None, t_end=200.0, spin_sph=0.01, spin_cyl=-0.03, P=6):
    """The paper's three-topology test (Sec. 3.3, Test Three) at `scale` times
    its cell counts.  Global Cartesian 80 x 80 x 40 centred on the origin with
    160 x 160 x 40 cells; a spherical patch at (-22, 0, 0), r in [5, 20],
    theta in [pi/4, 3pi/4], phi periodic, 30 x 40 x 200 cells, spinning about
    its z axis at spin_sph; a cylindrical patch at (22, 0, 0) with the same r and
    phi ranges, z in [-10, 10], 30 x 200 x 20 cells, spinning at spin_cyl
    (clockwise).  Plane wave phi = sin(2 pi (x - t) / 20) + 2 (Sec. 3); CFL 0.25
    on the smallest spacing; `steps` defaults to reaching t_end."""
    def nn(v):
        return [max(4, int(round(x * scale))) for x in v]
    g = patch(nn([160, 160, 40]), [-40, -40, -20], [40, 40, 20], is_global=1)
    s = patch(nn([30, 40, 200]), [5.0, math.pi / 4, 0.0], [20.0, 3 * math.pi / 4, 2 * math.pi], coord=SPH,
              periodic=(0, 0, 1), c0=(-22.0, 0.0, 0.0), spin=(0.0, 0.0, spin_sph))
    c = patch(nn([30, 200, 20]), [5.0, 0.0, -10.0], [20.0, 2 * math.pi, 10.0], coord=CYL, periodic=(0, 1, 0),
              c0=(22.0, 0.0, 0.0), spin=(0.0, 0.0, spin_cyl))
    ex = dict(kind="plane", A=1.0, B=2.0, kappa=[2 * math.pi / 20.0, 0.0, 0.0], psi=0.0)
    cfg = _finish(dict(name="three_topology_%g" % scale, wave_speed=[1.0], interp_points=[P], patches=[g, s, c],
                       exact=[ex]))
    cfg["steps"] = steps if steps is not None else int(math.ceil(t_end / cfg["dt"]))
    return cfg


def test_four(scale=1.0, steps=None, t_end=200.0, P=6):
    """The paper's fourth test (Sec. 3.4, Test Four) at `scale` times its cell
    counts: a spherical global shell r in [5, 100], theta in [pi/4, 3pi/4], phi
    periodic, 100 x 100 x 300 cells; a Cartesian patch over the radial cutout,
    30 x 30 x 20 with 80 x 80 x 20 cells, spinning at 0.03 about z; a cylindrical
    patch r in [5, 25], z in [-10, 10], phi periodic, 40 x 200 x 20 cells (the
    paper gives no cell counts for it), starting at (45, 45, 0) and translating
    at -0.5 along x.  Plane wave phi = sin(2 pi (x - t)/20) + 2; dt = 0.05 / scale.
    Below scale 0.6 the global's radial ghosts would reach r <= 0."""
    def nn(v):
        return [max(4, int(round(x * scale))) for x in v]
    g = patch(nn([100, 100, 300]), [5.0, math.pi / 4, 0.0], [100.0, 3 * math.pi / 4, 2 * math.pi], coord=SPH,
              is_global=1, periodic=(0, 0, 1))
    q = patch(nn([80, 80, 20]), [-15.0, -15.0, -10.0], [15.0, 15.0, 10.0], spin=(0.0, 0.0, 0.03))
    c = patch(nn([40, 200, 20]), [5.0, 0.0, -10.0], [25.0, 2 * math.pi, 10.0], coord=CYL, periodic=(0, 1, 0),
              motion=LINEAR, c0=(45.0, 45.0, 0.0), vel=(-0.5, 0.0, 0.0))
    ex = dict(kind="plane", A=1.0, B=2.0, kappa=[2 * math.pi / 20.0, 0.0, 0.0], psi=0.0)
    dt = 0.05 / scale
    cfg = dict(name="test_four_%g" % scale, wave_speed=[1.0], interp_points=[P], patches=[g, q, c], exact=[ex],
               ko_eps=0.005, buffer=4, dt=dt)
    cfg["steps"] = steps if steps is not None else int(math.ceil(t_end / dt - 1e-9))
    return cfg


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


def _rot(eu):
    a, b, c = eu
    Z1 = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    Y = np.array([[math.cos(b), 0, math.sin(b)], [0, 1, 0], [-math.sin(b), 0, math.cos(b)]])
    Z2 = np.array([[math.cos(c), -math.sin(c), 0], [math.sin(c), math.cos(c), 0], [0, 0, 1]])
    return Z1 @ Y @ Z2


def _obb_overlap(c1, R1, h1, c2, R2, h2):
    """Separating-axis test of two oriented boxes (centre, axes as columns, half sizes)."""
    axes = [R1[:, i] for i in range(3)] + [R2[:, i] for i in range(3)]
    for i in range(3):
        for j in range(3):
            v = np.cross(R1[:, i], R2[:, j])
            nv = np.linalg.norm(v)
            if nv > 1e-9:
                axes.append(v / nv)
    d = c2 - c1
    for ax in axes:
        r1 = np.sum(h1 * np.abs(R1.T @ ax))
        r2 = np.sum(h2 * np.abs(R2.T @ ax))
        if abs(d @ ax) > r1 + r2:
            return False
    return True


def _sphere_obb_overlap(cs, r, c, R, h):
    q = np.clip(R.T @ (cs - c), -h, h)
    return np.linalg.norm(R @ q + c - cs) <= r


def _overlap(a, b):
    if a["kind"] == "sph" and b["kind"] == "sph":
        return np.linalg.norm(a["c"] - b["c"]) <= a["r"] + b["r"]
    if a["kind"] == "sph":
        return _sphere_obb_overlap(a["c"], a["r"], b["c"], b["R"], b["h"])
    if b["kind"] == "sph":
        return _sphere_obb_overlap(b["c"], b["r"], a["c"], a["R"], a["h"])
    return _obb_overlap(a["c"], a["R"], a["h"], b["c"], b["R"], b["h"])


def batched(seed=4, ng=256, nlocal=64, nmin=24, nmax=96, frac_cart=0.7, vmax=0.2, steps=23, pad_cells=4,
            edge_cells=8, tries=400):
    """Global Cartesian [-8,8]^3 plus `nlocal` moving local patches of uneven
    sizes: per-axis cells from [nmin,nmax], 70/30 Cartesian/spherical, random
    orientation, linear velocity |v| <= vmax, resolution 1-4x the global one
    (spherical patches 2-4x, radial spacing; r_in = n_r dr / 4, theta in
    [pi/4, 3pi/4], phi periodic).  Placement: largest first; each patch is an
    oriented box (a sphere for spherical patches) grown by `pad_cells` global cells
    plus its motion over the run, kept `edge_cells` from the domain edge and
    disjoint from every placed one.  When no spot is found in `tries` draws the
    refinement ratio grows by 1.25 (cap 4), then the cell counts shrink by 0.8."""
    rng = np.random.default_rng(seed)
    L = 8.0
    dxg = 2 * L / ng
    g = patch([ng] * 3, [-L] * 3, [L] * 3, is_global=1)
    descs = []
    for _ in range(nlocal):
        n = rng.integers(nmin, nmax + 1, 3)
        coord = CART if rng.uniform() < frac_cart else SPH
        ratio = rng.uniform(1.0, 4.0) if coord == CART else rng.uniform(2.0, 4.0)
        eu = random_euler(rng)
        vdir = rng.normal(size=3)
        vdir /= np.linalg.norm(vdir)
        vel = vdir * vmax * rng.uniform() ** (1.0 / 3.0)
        descs.append(dict(n=n, coord=coord, ratio=ratio, euler=eu, vel=vel))

    def geometry(d):
        dx = dxg / d["ratio"]
        n = d["n"]
        if d["coord"] == CART:
            return dict(lo=-n * dx / 2.0, hi=n * dx / 2.0)
        r_in = n[0] * dx / 4.0
        return dict(lo=np.array([r_in, math.pi / 4, 0.0]), hi=np.array([r_in + n[0] * dx, 3 * math.pi / 4, 2 * math.pi]))

    def bound(d):
        gm = geometry(d)
        return float(np.linalg.norm(gm["hi"])) if d["coord"] == CART else float(gm["hi"][0])

    order = sorted(range(nlocal), key=lambda i: -bound(descs[i]))
    t_run = (steps + 1) * 0.25 * dxg  # generous bound on the simulated time of a run
    placed = []
    locs = []
    for i in order:
        d = descs[i]
        body = None
        for attempt in range(40):
            gm = geometry(d)
            pad = pad_cells * dxg + np.linalg.norm(d["vel"]) * t_run
            rb = bound(d) + pad
            room = L - rb - edge_cells * dxg
            if room > 0:
                cands = rng.uniform(-room, room, (tries, 3))
                pc = np.array([b["c"] for b in placed]) if placed else np.zeros((0, 3))
                pr = np.array([b["rb"] for b in placed]) if placed else np.zeros(0)
                R = _rot(d["euler"])
                for c in cands:
                    near = np.nonzero(np.linalg.norm(pc - c, axis=1) <= pr + rb)[0] if len(pc) else []
                    if d["coord"] == CART:
                        cand = dict(kind="cart", c=c, R=R, h=gm["hi"] + pad, rb=rb)
                    else:
                        cand = dict(kind="sph", c=c, r=rb, rb=rb)
                    if all(not _overlap(cand, placed[k]) for k in near):
                        body = cand
                        break
            if body is not None:
                break
            if d["ratio"] < 4.0:
                d["ratio"] = min(4.0, d["ratio"] * 1.25)
            else:
                d["n"] = np.maximum(nmin, (0.8 * d["n"]).astype(int))
        if body is None:
            continue
        placed.append(body)
        gm = geometry(d)
        c = body["c"]
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
