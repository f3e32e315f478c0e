"""Pins of the oracle's interpatch exchange rules that need more than one patch:
the covered physical ghost cells of the global patch (Sec. 2.4.2, last
paragraph), the membership of several state vectors (Sec. 1.1), and the fill of
cells that become live at a step end.

Expected values come from closed forms written here (polynomials, which the
6-point Lagrange stencil reproduces exactly; plane waves; the one-form law of a
translating Cartesian frame), from a brute-force cover test with a rotation
matrix built here, and from polynomial fits through the stencil nodes
(numpy.polyfit), an interpolation route independent of the oracle's weights.
"""
import math

import numpy as np
import pytest

from oracle.oracle import CART, FLAG_LIVE, LINEAR, NG, OracleWorld, world_from_config
from paper_2002_00088_amd import workloads as W


def zyz(e):
    a, b, c = e
    Rz = lambda t: np.array([[math.cos(t), -math.sin(t), 0], [math.sin(t), math.cos(t), 0], [0, 0, 1]])
    Ry = np.array([[math.cos(b), 0, math.sin(b)], [0, 1, 0], [-math.sin(b), 0, math.cos(b)]])
    return Rz(a) @ Ry @ Rz(c)


def centers(p, ghosts):
    """Cell-centre coordinates (x, y, z) of a Cartesian patch, arrays [k][j][i]."""
    g = NG if ghosts else 0
    xs = []
    for a in range(3):
        dx = (p["hi"][a] - p["lo"][a]) / p["n"][a]
        xs.append(p["lo"][a] + (np.arange(-g, p["n"][a] + g) + 0.5) * dx)
    z, y, x = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return x, y, z


# a polynomial of total degree 5 in the background coordinates and its gradient
def poly(X, Y, Z):
    return (0.3 + 0.2 * X - 0.1 * Y + 0.05 * Z + 0.04 * X * X - 0.03 * X * Y + 0.02 * Y * Z * Z
            + 0.01 * X ** 3 - 0.002 * X * Y * Y * Z + 0.0007 * Y ** 5 - 0.0004 * X * X * Z ** 3)


def poly_grad(X, Y, Z):
    gx = 0.2 + 0.08 * X - 0.03 * Y + 0.03 * X * X - 0.002 * Y * Y * Z - 0.0008 * X * Z ** 3
    gy = -0.1 - 0.03 * X + 0.02 * Z * Z - 0.004 * X * Y * Z + 0.0035 * Y ** 4
    gz = 0.05 + 0.04 * Y * Z - 0.002 * X * Y * Y - 0.0012 * X * X * Z * Z
    return gx, gy, gz


def plane(ex, t, X, Y, Z, v=1.0):
    """Plane wave phi = A sin(k.X - v|k| t + psi) + B (Eq. wave_solution) and its one-form."""
    k = np.asarray(ex["kappa"])
    kn = np.linalg.norm(k)
    arg = k[0] * X + k[1] * Y + k[2] * Z - v * kn * t + ex["psi"]
    c = ex["A"] * np.cos(arg)
    return np.stack([ex["A"] * np.sin(arg) + ex["B"], -v * kn * c, k[0] * c, k[1] * c, k[2] * c])


PLANE = dict(kind="plane", A=0.7, B=1.5, kappa=[0.9, -0.4, 0.6], psi=0.3)


# --------------------------------------------------------------------------
# Covered physical ghost cells of the global patch (Sec. 2.4.2, last paragraph)
# --------------------------------------------------------------------------
def _face_world(eu, c0):
    g = W.patch([24] * 3, [-6] * 3, [6] * 3, is_global=1)
    loc = W.patch([16] * 3, [-2] * 3, [2] * 3, euler=eu, c0=c0)
    w = OracleWorld()
    w.add_patch(g)
    w.add_patch(loc)
    w.set_exact(0, PLANE)
    return w, g, loc


@pytest.mark.parametrize("eu,c0", [([0.4, 1.1, 2.3], (5.4, 0.3, -0.2)), ([1.9, 0.7, 0.2], (-4.9, 5.3, 0.4))])
def test_covered_physical_ghosts_interpolated(eu, c0):
    """A static local patch across the global patch's outer face (and, in the
    second case, across an edge).  The local patch carries a polynomial of
    degree 5, which the 6-point stencil reproduces exactly; the registered exact
    solution is a different function (a plane wave).  After a ghost exchange each
    physical ghost cell of the global patch inside the local patch must hold the
    polynomial (interpolated through the frame transform), unless its stencil
    leaves the local interior, where the boundary value (the plane wave) stays;
    every other outer ghost holds the plane wave."""
    w, g, loc = _face_world(eu, c0)
    R = zyz(eu)
    # local state: the polynomial in the local frame (Pi' = R^T grad phi, Pi_t = 0)
    xl, yl, zl = centers(loc, False)
    Xb = [c0[a] + R[a, 0] * xl + R[a, 1] * yl + R[a, 2] * zl for a in range(3)]
    gr = poly_grad(*Xb)
    sl = np.zeros((5,) + xl.shape)
    sl[0] = poly(*Xb)
    for j in range(3):
        sl[2 + j] = sum(R[a, j] * gr[a] for a in range(3))
    w.set_state(1, 0, sl)
    xg, yg, zg = centers(g, False)
    w.set_state(0, 0, plane(PLANE, 0.0, xg, yg, zg))
    w.exchange_ghosts(0.0)

    # brute-force cover of the physical ghost cells and interpolability
    X, Y, Z = centers(g, True)
    ghost = np.ones(X.shape, dtype=bool)
    ghost[NG:-NG, NG:-NG, NG:-NG] = False
    D = np.stack([X - c0[0], Y - c0[1], Z - c0[2]])
    xp = np.einsum("ab,a...->b...", R, D)  # R^T (X - c0)
    inside = np.all((xp >= -2.0) & (xp <= 2.0), axis=0) & ghost
    q = (xp + 2.0) / 0.25 - 0.5
    s = np.floor(q - 2.0)  # 6-point stencil start (Eq. Pijk: i_c - 2)
    valid = inside & np.all((s >= 0) & (s + 5 <= 15), axis=0)

    cov = w.cover_full()
    assert (((cov == 1) & ghost) == inside).all()
    assert ((cov[ghost] == -1) | (cov[ghost] == 1)).all()
    n_cov, n_val = int(inside.sum()), int(valid.sum())
    assert n_cov > 100 and n_val > 20 and n_cov - n_val > 20, (n_cov, n_val)
    c = w.counters()
    assert c["n_outer"] == n_cov and c["skip_outer"] == n_cov - n_val

    full = w.get_full(0)
    pw_val = plane(PLANE, 0.0, X, Y, Z)
    gx, gy, gz = poly_grad(X, Y, Z)
    pol = np.stack([poly(X, Y, Z), np.zeros_like(X), gx, gy, gz])
    for f in range(5):
        assert np.allclose(full[f][valid], pol[f][valid], rtol=0, atol=1e-12), f
        keep = ghost & ~valid
        assert np.allclose(full[f][keep], pw_val[f][keep], rtol=0, atol=1e-13), f


def test_sommerfeld_outer_ghosts_are_not_interpatch_targets():
    """The Sommerfeld variant evolves its outer ghosts: covered ones are not
    overwritten by the local patch (reading of this build for a variant the
    paper does not have)."""
    g = W.patch([24] * 3, [-6] * 3, [6] * 3, is_global=1)
    loc = W.patch([16] * 3, [-2] * 3, [2] * 3, euler=[0.4, 1.1, 2.3], c0=(5.4, 0.3, -0.2))
    w = OracleWorld(outer_bc=1)
    w.add_patch(g)
    w.add_patch(loc)
    w.set_exact(0, PLANE)
    w.init_exact(0.0)
    w.step(0.05, 1)
    c = w.counters()
    assert c["n_outer"] == 0 and c["skip_outer"] == 0


def test_covered_physical_ghosts_convergence():
    """Fourth-order convergence of a translating, rotated local patch that sits
    across the global patch's +x face (its covered outer ghosts are
    interpolated in every stage)."""
    errs = []
    T = 2.0
    for ng in (32, 64):
        L = 16.0
        dxg = 2 * L / ng
        nl = int(round(10.0 / (dxg / 2)))
        g = W.patch([ng] * 3, [-L] * 3, [L] * 3, is_global=1)
        loc = W.patch([nl] * 3, [-5.0] * 3, [5.0] * 3, euler=[0.3, 0.8, 1.9], motion=LINEAR, c0=(13.0, -0.5, 0.2),
                      vel=(0.1, 0.1, 0.0))
        ex = dict(kind="plane", A=1.0, B=2.0, kappa=[2 * math.pi / 16 * x for x in (1.0, 0.6, 0.3)], psi=0.4)
        cfg = dict(wave_speed=[1.0], interp_points=[6], patches=[g, loc], exact=[ex], ko_eps=0.005, buffer=4)
        w = world_from_config(cfg)
        w.init_exact(0.0)
        steps = int(round(T / (0.5 * dxg / 2)))
        w.step(T / steps, steps)
        c = w.counters()
        assert c["n_outer"] > 0 and c["skip_eff"] == 0 and c["skip_uncover"] == 0
        errs.append(w.diag(0)["int_rel_err"] + w.diag(1)["int_rel_err"])
    slope = math.log2(errs[0] / errs[1])
    assert 3.5 < slope < 4.8, (errs, slope)


# --------------------------------------------------------------------------
# Several state vectors (Sec. 1.1): each vector's evolution is independent of
# the others; membership decides the exchange partners.
# --------------------------------------------------------------------------
GAUSS = dict(kind="gauss", amp=[0.8, 0.6], centers=[[0.5, -0.3, 0.2], [-1.0, 0.8, -0.5]], widths=[0.9, 0.7])


def _sv_patches(mask_g, mask_1, mask_2):
    # a translating local patch that uncovers global cells within a few steps,
    # and a static one; both large enough (in global cells) to have effective ghosts
    g = W.patch([56] * 3, [-14] * 3, [14] * 3, is_global=1, sv_mask=mask_g)
    l1 = W.patch([28] * 3, [-3.5] * 3, [3.5] * 3, euler=[0.2, 0.15, 0.1], motion=LINEAR, c0=(-5.0, 0.2, 0.1),
                 vel=(0.15, -0.1, 0.05), sv_mask=mask_1)
    l2 = W.patch([24] * 3, [-3.0] * 3, [3.0] * 3, euler=[0.1, 0.2, 0.05], c0=(5.5, -0.4, 0.6), sv_mask=mask_2)
    return [g, l1, l2]


def _run(cfg, steps=6, dt=0.05):
    w = world_from_config(cfg)
    w.init_exact(0.0)
    w.step(dt, steps)
    return w


def test_two_vectors_equal_two_one_vector_worlds():
    """Vectors A (v = 1, P = 6, Gaussian pulses) and B (v = 0.5, P = 5, plane
    wave) on every patch: each equals, bitwise, a world that carries only it,
    and the swapped order gives the same results."""
    both = _run(dict(wave_speed=[1.0, 0.5], interp_points=[6, 5], patches=_sv_patches(3, 3, 3),
                     exact=[GAUSS, PLANE]))
    swap = _run(dict(wave_speed=[0.5, 1.0], interp_points=[5, 6], patches=_sv_patches(3, 3, 3),
                     exact=[PLANE, GAUSS]))
    a = _run(dict(wave_speed=[1.0], interp_points=[6], patches=_sv_patches(1, 1, 1), exact=[GAUSS]))
    b = _run(dict(wave_speed=[0.5], interp_points=[5], patches=_sv_patches(1, 1, 1), exact=[PLANE]))
    for pid in range(3):
        assert np.array_equal(both.get_state(pid, 0), a.get_state(pid, 0))
        assert np.array_equal(both.get_state(pid, 1), b.get_state(pid, 0))
        assert np.array_equal(swap.get_state(pid, 1), a.get_state(pid, 0))
        assert np.array_equal(swap.get_state(pid, 0), b.get_state(pid, 0))
    cb, ca, cbb = both.counters(), a.counters(), b.counters()
    for k in ("skip_local", "skip_eff", "skip_uncover", "n_uncover"):
        assert cb[k] == ca[k] + cbb[k], k
    assert ca["n_uncover"] > 0  # the translating patch uncovers cells


def test_vector_missing_on_a_local_patch():
    """B on the global patch and local 1 only.  A is unchanged, bitwise; B's
    effective ghosts under local 2 have no donor: each ghost fill counts them as
    skipped and gives them B's exact solution."""
    both = _run(dict(wave_speed=[1.0, 0.5], interp_points=[6, 5], patches=_sv_patches(3, 3, 1),
                     exact=[GAUSS, PLANE]), steps=2)
    a = _run(dict(wave_speed=[1.0], interp_points=[6], patches=_sv_patches(1, 1, 1), exact=[GAUSS]), steps=2)
    for pid in range(3):
        assert np.array_equal(both.get_state(pid, 0), a.get_state(pid, 0))
    f, cov = both.flags()
    n_under2 = int(((f == 1) & (cov == 2)).sum())
    assert n_under2 > 0
    sk0 = both.counters()["skip_eff"]
    t = both.t
    both.exchange_ghosts(t)
    assert both.counters()["skip_eff"] - sk0 == n_under2
    gp = both.patches[0]
    X, Y, Z = centers(gp, False)
    sel = (f == 1) & (cov == 2)
    full = both.get_full(0, 1)[:, NG:-NG, NG:-NG, NG:-NG]
    exp = plane(PLANE, t, X, Y, Z, v=0.5)
    for fld in range(5):
        assert np.allclose(full[fld][sel], exp[fld][sel], rtol=0, atol=1e-13)
    # B's effective ghosts under local 1 are interpolated, not exact
    sel1 = (f == 1) & (cov == 1)
    assert np.max(np.abs(full[0][sel1] - exp[0][sel1])) > 0


def test_vector_only_on_local_patches():
    """B on the two local patches only (the global patch does not carry it): the
    local ghost cells have no donor and hold B's exact solution in each
    patch's frame; nothing is counted as skipped for B."""
    pats = _sv_patches(1, 3, 3)
    pats[1]["motion"] = 0  # static frames: the exact one-form is R^T grad phi, Pi_t unchanged
    both = _run(dict(wave_speed=[1.0, 0.5], interp_points=[6, 5], patches=pats, exact=[GAUSS, PLANE]), steps=2)
    a = _run(dict(wave_speed=[1.0], interp_points=[6], patches=[dict(p, sv_mask=1) for p in pats], exact=[GAUSS]),
             steps=2)
    assert both.counters() == a.counters()
    t = both.t
    both.exchange_ghosts(t)
    for pid in (1, 2):
        p = both.patches[pid]
        R = zyz(p["euler"])
        x, y, z = centers(p, True)
        Xb = [p["c0"][a] + R[a, 0] * x + R[a, 1] * y + R[a, 2] * z for a in range(3)]
        e = plane(PLANE, t, *Xb, v=0.5)
        ep = np.stack([e[0], e[1]] + [sum(R[a, j] * e[2 + a] for a in range(3)) for j in range(3)])
        full = both.get_full(pid, 1)
        ghost = np.ones(x.shape, dtype=bool)
        ghost[NG:-NG, NG:-NG, NG:-NG] = False
        for fld in range(5):
            assert np.allclose(full[fld][ghost], ep[fld][ghost], rtol=0, atol=1e-13)


# --------------------------------------------------------------------------
# Cells that become live at a step end take u_{n+1} interpolated from the
# covering local patch at t_{n+1}.
# --------------------------------------------------------------------------
def _interp_polyfit(U, q, P):
    """Tensor-product interpolation of the 3-D array U[k][j][i] at fractional
    index q = (qi, qj, qk): polynomial fits of degree P-1 through the P nodes of
    the stencil that starts at floor(q - (P-2)/2), axis by axis."""
    s = [int(math.floor(q[a] - 0.5 * (P - 2))) for a in range(3)]
    box = U[s[2]:s[2] + P, s[1]:s[1] + P, s[0]:s[0] + P]
    nodes = np.arange(P, dtype=float)

    def along(vals, qa):
        c = np.polyfit(nodes, vals, P - 1)
        return np.polyval(c, qa)

    lay = np.array([[along(box[k, j, :], q[0] - s[0]) for j in range(P)] for k in range(P)])
    row = np.array([along(lay[k, :], q[1] - s[1]) for k in range(P)])
    return along(row, q[2] - s[2])


def test_uncover_fill_values():
    """A local patch translating at speed 0.45 uncovers global cells every few
    steps.  Each cell that becomes live holds the local patch's u_{n+1}
    interpolated at its centre (P = 6) and carried to the global frame by the
    one-form law of a translating frame: Pi_a = (R Pi')_a,
    Pi_t = Pi'_t - Pi'.(R^T v)."""
    eu, c0, vel = [0.2, 0.15, 0.1], np.array([-1.0, 0.2, 0.1]), np.array([0.35, -0.25, 0.12])
    g = W.patch([56] * 3, [-14] * 3, [14] * 3, is_global=1)
    loc = W.patch([28] * 3, [-3.5] * 3, [3.5] * 3, euler=eu, motion=LINEAR, c0=tuple(c0), vel=tuple(vel))
    cfg = dict(wave_speed=[1.0], interp_points=[6], patches=[g, loc], exact=[GAUSS], ko_eps=0.005, buffer=4)
    w = world_from_config(cfg)
    w.init_exact(0.0)
    R = zyz(eu)
    dt = 0.0625
    X, Y, Z = centers(g, False)
    checked = 0
    for _ in range(12):
        f0, _c = w.flags()
        w.step(dt, 1)
        f1, c1 = w.flags()
        new = (f0 != FLAG_LIVE) & (f1 == FLAG_LIVE)
        if not new.any():
            continue
        t = w.t
        ul = w.get_state(1)
        ug = w.get_state(0)
        for k, j, i in zip(*np.nonzero(new)):
            xp = R.T @ (np.array([X[k, j, i], Y[k, j, i], Z[k, j, i]]) - c0 - vel * t)
            q = (xp + 3.5) / 0.25 - 0.5
            vals = np.array([_interp_polyfit(ul[f], q, 6) for f in range(5)])
            exp = np.empty(5)
            exp[0] = vals[0]
            exp[1] = vals[1] - vals[2:] @ (R.T @ vel)
            exp[2:] = R @ vals[2:]
            scale = np.max(np.abs(ul), axis=(1, 2, 3))
            assert np.all(np.abs(ug[:, k, j, i] - exp) <= 1e-10 * scale), (k, j, i)
            checked += 1
    c = w.counters()
    assert c["n_uncover"] == checked and checked >= 10 and c["skip_uncover"] == 0
