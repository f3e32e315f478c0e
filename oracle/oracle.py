"""ctypes binding of the plain FP64 CPU oracle (``pw_oracle.c``).

Test infrastructure only: the test-suite, the smoke check and the CPU leg of
``bench.py`` use it.  The GPU library never imports it, and it never imports
the GPU library.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pw_oracle.c")
# PW_ORACLE_SANITIZE=1 selects a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (the process must preload libasan; see
# tests/test_oracle_sanitized.py)
SANITIZE = os.environ.get("PW_ORACLE_SANITIZE") == "1"
LIB = os.path.join(HERE, "liboracle_asan.so" if SANITIZE else "liboracle.so")

CART, SPH, CYL = 0, 1, 2
STATIC, LINEAR, CIRCLE = 0, 1, 2
FLAG_LIVE, FLAG_EFFGHOST, FLAG_DEACT = 0, 1, 2
NG = 3


def build(force=True):
    """Compile the oracle with gcc (plain C, OpenMP on outer loops only)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"] \
        if SANITIZE else []
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           "-Wall"] + san + ["-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        vp = C.c_void_p
        L.or_new.restype = vp
        L.or_new.argtypes = [C.c_int, dp, ip, C.c_double, C.c_int]
        L.or_set_form.argtypes = [vp, C.c_int]
        L.or_set_outer_bc.argtypes = [vp, C.c_int]
        L.or_rhs_outer.argtypes = [vp, C.c_int, dp]
        L.or_free.argtypes = [vp]
        L.or_add_patch.restype = C.c_int
        L.or_add_patch.argtypes = [vp, C.c_int, C.c_int, ip, dp, dp, ip, dp, C.c_int, dp, dp,
                                   C.c_double, C.c_double, C.c_double, C.c_uint]
        L.or_set_spin.restype = C.c_int
        L.or_set_spin.argtypes = [vp, C.c_int, dp]
        L.or_set_exact_plane.argtypes = [vp, C.c_int, C.c_double, C.c_double, dp, C.c_double]
        L.or_set_exact_gauss.argtypes = [vp, C.c_int, C.c_int, dp, dp, dp]
        L.or_set_state.argtypes = [vp, C.c_int, C.c_int, dp, C.c_double]
        L.or_get_state.argtypes = [vp, C.c_int, C.c_int, dp]
        L.or_get_full.argtypes = [vp, C.c_int, C.c_int, dp]
        L.or_set_full.argtypes = [vp, C.c_int, C.c_int, dp]
        L.or_init_exact.argtypes = [vp, C.c_double]
        L.or_prepare.argtypes = [vp]
        L.or_get_flags.argtypes = [vp, C.POINTER(C.c_uint8), C.POINTER(C.c_int32)]
        L.or_exchange_ghosts.argtypes = [vp, C.c_double]
        L.or_step.argtypes = [vp, C.c_double, C.c_int]
        L.or_time.restype = C.c_double
        L.or_time.argtypes = [vp]
        L.or_counters.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.or_cover_full.argtypes = [vp, C.POINTER(C.c_int32)]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_max_threads.restype = C.c_int
        L.or_diag.argtypes = [vp, C.c_int, C.c_int, dp]
        L.or_metric_at.argtypes = [vp, C.c_int, C.c_int, C.c_double, dp, dp, dp, dp]
        L.or_jac_at.argtypes = [vp, C.c_int, C.c_double, dp, dp]
        L.or_map_fwd.argtypes = [vp, C.c_int, C.c_double, dp, dp]
        L.or_map_inv.argtypes = [vp, C.c_int, C.c_double, dp, dp]
        L.or_rotation.argtypes = [vp, C.c_int, dp]
        L.or_lagrange.argtypes = [C.c_int, C.c_double, ip, dp]
        L.or_transform.argtypes = [vp, C.c_int, dp, C.c_int, dp, C.c_double, dp, dp]
        L.or_interp.argtypes = [vp, C.c_int, C.c_int, C.c_double, dp, dp, dp]
        L.or_exact_bg.argtypes = [vp, C.c_int, C.c_double, dp, dp]
        L.or_exact_patch.argtypes = [vp, C.c_int, C.c_int, C.c_double, dp, dp]
        L.or_rhs.argtypes = [vp, C.c_int, C.c_int, C.c_double, dp]
        L.or_stencil.restype = C.c_double
        L.or_stencil.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int))


class OracleWorld:
    """One global patch (id 0) plus local patches, FP64 throughout."""

    def __init__(self, wave_speed=(1.0,), interp_points=None, ko_eps=0.005, buffer=4, pi_form=0, outer_bc=0):
        self.L = lib()
        nsv = len(wave_speed)
        if interp_points is None:
            interp_points = [6] * nsv
        ws, wsp = _d(wave_speed)
        ip, ipp = _i(interp_points)
        self.h = self.L.or_new(nsv, wsp, ipp, ko_eps, buffer)
        if not self.h:
            raise ValueError("bad oracle world parameters")
        if self.L.or_set_form(self.h, pi_form) != 0:
            raise ValueError("bad form of the Pi_t equation")
        self.outer_bc = outer_bc
        self.nsv = nsv
        self.patches = []

    def close(self):
        if self.h:
            self.L.or_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_patch(self, d):
        """d: dict with keys of a patch description (see workloads.patch)."""
        n, npp = _i(d["n"])
        lo, lop = _d(d["lo"])
        hi, hip = _d(d["hi"])
        per, perp = _i(d.get("periodic", (0, 0, 0)))
        eu, eup = _d(d.get("euler", (0, 0, 0)))
        c0, c0p = _d(d.get("c0", (0, 0, 0)))
        vel, velp = _d(d.get("vel", (0, 0, 0)))
        pid = self.L.or_add_patch(self.h, d.get("coord", CART), int(d.get("is_global", 0)), npp, lop, hip, perp,
                                  eup, d.get("motion", STATIC), c0p, velp, float(d.get("radius", 0.0)),
                                  float(d.get("speed", 0.0)), float(d.get("phase", 0.0)),
                                  int(d.get("sv_mask", 1)))
        if pid < 0:
            raise ValueError("oracle rejected patch")
        if any(x != 0.0 for x in d.get("spin", (0.0, 0.0, 0.0))):
            sp, spp = _d(d["spin"])
            if self.L.or_set_spin(self.h, pid, spp) != 0:
                raise ValueError("oracle rejected spin")
        if pid == 0 and self.outer_bc != 0 and self.L.or_set_outer_bc(self.h, self.outer_bc) != 0:
            raise ValueError("oracle rejected the outer boundary condition")
        self.patches.append(dict(d))
        return pid

    def set_exact(self, sv, ex):
        if ex["kind"] == "plane":
            k, kp = _d(ex["kappa"])
            self.L.or_set_exact_plane(self.h, sv, ex.get("A", 1.0), ex.get("B", 0.0), kp, ex.get("psi", 0.0))
        elif ex["kind"] == "gauss":
            a, ap = _d(ex["amp"])
            xc, xcp = _d(np.asarray(ex["centers"]).reshape(-1))
            w, wp = _d(ex["widths"])
            if self.L.or_set_exact_gauss(self.h, sv, len(a), ap, xcp, wp) != 0:
                raise ValueError("too many pulses")
        else:
            raise ValueError(ex["kind"])

    def shape(self, pid):
        n = self.patches[pid]["n"]
        return (5, n[2], n[1], n[0])

    def full_shape(self, pid):
        n = self.patches[pid]["n"]
        return (5, n[2] + 2 * NG, n[1] + 2 * NG, n[0] + 2 * NG)

    def set_state(self, pid, sv, arr, t0=0.0):
        a, ap = _d(arr)
        assert a.size == int(np.prod(self.shape(pid)))
        if self.L.or_set_state(self.h, pid, sv, ap, t0) != 0:
            raise ValueError("set_state")

    def get_state(self, pid, sv=0):
        out = np.empty(self.shape(pid))
        _, op = _d(out)
        if self.L.or_get_state(self.h, pid, sv, op) != 0:
            raise ValueError("get_state")
        return out

    def get_full(self, pid, sv=0):
        out = np.empty(self.full_shape(pid))
        _, op = _d(out)
        self.L.or_get_full(self.h, pid, sv, op)
        return out

    def set_full(self, pid, sv, arr):
        a, ap = _d(arr)
        assert a.size == int(np.prod(self.full_shape(pid)))
        self.L.or_set_full(self.h, pid, sv, ap)

    def init_exact(self, t0=0.0):
        self.L.or_init_exact(self.h, t0)

    def prepare(self):
        rc = self.L.or_prepare(self.h)
        if rc:
            raise RuntimeError("oracle flags failed rc=%d" % rc)

    def flags(self):
        n = self.patches[0]["n"]
        f = np.empty((n[2], n[1], n[0]), dtype=np.uint8)
        c = np.empty((n[2], n[1], n[0]), dtype=np.int32)
        rc = self.L.or_get_flags(self.h, f.ctypes.data_as(C.POINTER(C.c_uint8)), c.ctypes.data_as(C.POINTER(C.c_int32)))
        if rc:
            raise RuntimeError("oracle flags failed rc=%d" % rc)
        return f, c

    def exchange_ghosts(self, t):
        rc = self.L.or_exchange_ghosts(self.h, t)
        if rc:
            raise RuntimeError("oracle exchange failed rc=%d" % rc)

    def step(self, dt, n=1):
        rc = self.L.or_step(self.h, dt, n)
        if rc:
            raise RuntimeError("oracle step failed rc=%d" % rc)

    @property
    def t(self):
        return self.L.or_time(self.h)

    def counters(self):
        out = (C.c_longlong * 6)()
        self.L.or_counters(self.h, out)
        return dict(skip_local=out[0], skip_eff=out[1], skip_uncover=out[2], n_uncover=out[3],
                    skip_outer=out[4], n_outer=out[5])

    def cover_full(self):
        """Covering local patch (or -1) of every cell of the global patch's padded
        array [n2+6][n1+6][n0+6]: interior cells as in flags(), physical ghost
        cells (outer ghosts that are not periodic copies) from the covered-ghost
        list of the current step."""
        n = self.patches[0]["n"]
        c = np.empty((n[2] + 2 * NG, n[1] + 2 * NG, n[0] + 2 * NG), dtype=np.int32)
        rc = self.L.or_cover_full(self.h, c.ctypes.data_as(C.POINTER(C.c_int32)))
        if rc:
            raise RuntimeError("oracle flags failed rc=%d" % rc)
        return c

    def diag(self, pid, sv=0):
        out = np.zeros(27)
        _, op = _d(out)
        self.L.or_diag(self.h, pid, sv, op)
        return dict(max=out[0:5].copy(), sumsq=out[5:10].copy(), err_max=out[10:15].copy(),
                    err_sumsq=out[15:20].copy(), int_rel_err=out[20], live=int(out[21]), volume=out[22],
                    energy=out[23], constraint=out[24:27].copy())

    # --- unit entry points -------------------------------------------------
    def metric(self, pid, sv, t, xp):
        x, xpp = _d(xp)
        g = np.zeros(16)
        c = np.zeros(4)
        sg = np.zeros(1)
        _, gp = _d(g)
        _, cp = _d(c)
        _, sgp = _d(sg)
        self.L.or_metric_at(self.h, pid, sv, t, xpp, gp, cp, sgp)
        return g.reshape(4, 4), c, sg[0]

    def jac(self, pid, t, xp):
        x, xpp = _d(xp)
        E = np.zeros(16)
        _, ep = _d(E)
        self.L.or_jac_at(self.h, pid, t, xpp, ep)
        return E.reshape(4, 4)

    def map_fwd(self, pid, t, xp):
        x, xpp = _d(xp)
        X = np.zeros(3)
        _, Xp = _d(X)
        self.L.or_map_fwd(self.h, pid, t, xpp, Xp)
        return X

    def map_inv(self, pid, t, X):
        x, Xp = _d(X)
        xp = np.zeros(3)
        _, xpp = _d(xp)
        self.L.or_map_inv(self.h, pid, t, Xp, xpp)
        return xp

    def rotation(self, pid):
        R = np.zeros(9)
        _, rp = _d(R)
        self.L.or_rotation(self.h, pid, rp)
        return R.reshape(3, 3)

    def transform(self, d, xd, r, xr, t, state):
        _, xdp = _d(xd)
        _, xrp = _d(xr)
        s, sp = _d(state)
        out = np.zeros(5)
        _, op = _d(out)
        self.L.or_transform(self.h, d, xdp, r, xrp, t, sp, op)
        return out

    def interp(self, d, sv, t, X):
        _, Xp = _d(X)
        out = np.zeros(5)
        xd = np.zeros(3)
        _, op = _d(out)
        _, xdp = _d(xd)
        ok = self.L.or_interp(self.h, d, sv, t, Xp, op, xdp)
        return ok, out, xd

    def exact_bg(self, sv, t, X):
        _, Xp = _d(X)
        out = np.zeros(5)
        _, op = _d(out)
        self.L.or_exact_bg(self.h, sv, t, Xp, op)
        return out

    def exact_patch(self, pid, sv, t, xp):
        _, xpp = _d(xp)
        out = np.zeros(5)
        _, op = _d(out)
        self.L.or_exact_patch(self.h, pid, sv, t, xpp, op)
        return out

    def rhs(self, pid, sv, t):
        out = np.empty(self.shape(pid))
        _, op = _d(out)
        self.L.or_rhs(self.h, pid, sv, t, op)
        return out

    def rhs_outer(self, sv=0):
        """Sommerfeld right-hand side at the outer ghost cells of the global
        patch (full padded array [5][n2+6][n1+6][n0+6], NaN elsewhere)."""
        out = np.full(self.full_shape(0), np.nan)
        _, op = _d(out)
        if self.L.or_rhs_outer(self.h, sv, op) != 0:
            raise ValueError("no global patch or state vector")
        return out

    def stencil(self, pid, op, d, e, i, j, k, sv=0):
        return self.L.or_stencil(self.h, pid, sv, op, d, e, i, j, k)


def set_threads(n):
    """Threads of the oracle's OpenMP loops (timing runs); returns the new maximum."""
    lib().or_set_threads(int(n))
    return lib().or_max_threads()


def lagrange(P, q):
    s = C.c_int(0)
    w = np.zeros(8)
    _, wp = _d(w)
    lib().or_lagrange(P, q, C.byref(s), wp)
    return s.value, w[:P].copy()


def world_from_config(cfg):
    """Build an oracle world from a workload config (see workloads.py)."""
    w = OracleWorld(wave_speed=cfg["wave_speed"], interp_points=cfg["interp_points"],
                    ko_eps=cfg.get("ko_eps", 0.005), buffer=cfg.get("buffer", 4), pi_form=cfg.get("pi_form", 0),
                    outer_bc=cfg.get("outer_bc", 0))
    for d in cfg["patches"]:
        w.add_patch(d)
    for sv, ex in enumerate(cfg.get("exact", [])):
        if ex is not None:
            w.set_exact(sv, ex)
    return w
