"""Thin ctypes binding of libpw (include/pw.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libpw.so; this module only
converts Python/numpy arguments to the C structures and back.  There is no
fallback: if the library is missing or fails to load, ``load()`` raises.

torch is imported before the library is loaded so that the process holds a
single HIP runtime (torch's bundled runtime has the same soname libpw links to),
which lets libpw run on torch streams and allocate through torch's caching
allocator.
"""
import ctypes as C
import os

import numpy as np

try:  # one HIP runtime per process: load torch's first
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpw.so")

PW_FP64, PW_MIXED, PW_MIXED_INC = 0, 1, 2
PW_CART, PW_SPH, PW_CYL = 0, 1, 2
PW_FORM_PAPER, PW_FORM_FIRST_ORDER = 0, 1
PW_BC_EXACT, PW_BC_SOMMERFELD = 0, 1
PW_STATIC, PW_LINEAR, PW_CIRCLE = 0, 1, 2
PW_FLAG_LIVE, PW_FLAG_EFFGHOST, PW_FLAG_DEACT = 0, 1, 2
PW_SCHED_BATCHED, PW_SCHED_PER_PATCH = 0, 1
PW_ORDER_BANDS, PW_ORDER_OCTANTS = 0, 1
PW_CHAIN_GLOBAL, PW_CHAIN_LOCAL_AFTER, PW_CHAIN_LOCAL_BEFORE = 0, 1, 2
PW_TILE_32X8, PW_TILE_16X16, PW_TILE_128X4, PW_TILE_128X8 = 0, 1, 1, 2
PW_EXACT_NONE, PW_EXACT_PLANE, PW_EXACT_GAUSS = 0, 1, 2
STATUS = {0: "PW_OK", -1: "PW_EINVAL", -2: "PW_ENOMEM", -3: "PW_EDEVICE", -4: "PW_ESTATE", -5: "PW_EOVERLAP",
          -6: "PW_EMOTION"}

EXPORTS = ["pw_create", "pw_create_patch", "pw_set_exact", "pw_init_exact", "pw_set_state", "pw_get_state",
           "pw_get_state_full", "pw_get_flags", "pw_exchange_ghosts", "pw_rk4_step", "pw_get_time",
           "pw_diagnostics", "pw_counters", "pw_live_cells", "pw_enable_timing", "pw_kernel_times",
           "pw_get_tuning", "pw_set_tuning", "pw_autotune", "pw_last_error", "pw_destroy", "pw_get_state_noalloc"]
KERNEL_CLASSES = ["pose", "ghost_s1", "ghost_s2", "ghost_s3", "ghost_s4", "stage_s1", "stage_s2", "stage_s3",
                  "stage_s4", "flags", "finalize", "gstage_s1", "gstage_s2", "gstage_s3", "gstage_s4", "g2l", "l2g"]

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_uint64, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("n_state_vectors", C.c_int32), ("wave_speed", C.c_double * 4),
                ("interp_points", C.c_int32 * 4), ("buffer_width", C.c_int32), ("ko_eps", C.c_double),
                ("schedule", C.c_int32), ("use_graph", C.c_int32), ("stream", C.c_void_p),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_user", C.c_void_p), ("pi_form", C.c_int32),
                ("outer_bc", C.c_int32)]


class PatchDesc(C.Structure):
    _fields_ = [("coord", C.c_int32), ("is_global", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("periodic", C.c_int32 * 3), ("euler_zyz", C.c_double * 3),
                ("motion", C.c_int32), ("c0", C.c_double * 3), ("vel", C.c_double * 3), ("radius", C.c_double),
                ("speed", C.c_double), ("phase", C.c_double), ("sv_mask", C.c_uint32), ("spin", C.c_double * 3)]


class ExactDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("amp", C.c_double), ("offset", C.c_double), ("kappa", C.c_double * 3),
                ("phase", C.c_double), ("n_pulses", C.c_int32), ("pulse_amp", C.c_double * 32),
                ("pulse_center", (C.c_double * 3) * 32), ("pulse_width", C.c_double * 32)]


class Diag(C.Structure):
    _fields_ = [("max_abs", C.c_double * 5), ("sum_sq", C.c_double * 5), ("err_max", C.c_double * 5),
                ("err_sum_sq", C.c_double * 5), ("int_rel_err", C.c_double), ("live_cells", C.c_double),
                ("volume", C.c_double), ("energy", C.c_double), ("constraint_max", C.c_double * 3)]


class Tuning(C.Structure):
    _fields_ = [("tile_z_global", C.c_int32), ("tile_z_local", C.c_int32), ("g2l_run", C.c_int32),
                ("l2g_run", C.c_int32), ("global_order", C.c_int32), ("chain", C.c_int32),
                ("local_tile", C.c_int32), ("global_tile", C.c_int32)]


class Counters(C.Structure):
    _fields_ = [("skip_local", C.c_int64), ("skip_eff", C.c_int64), ("skip_uncover", C.c_int64),
                ("n_uncover", C.c_int64), ("steps", C.c_int64), ("skip_outer", C.c_int64), ("n_outer", C.c_int64)]


_lib = None


def load():
    """Load libpw.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise RuntimeError("libpw.so is not built: run __graft_entry__.build() or paper_2002_00088_amd/build.py")
    L = C.CDLL(LIB)
    vp = C.c_void_p
    dp = C.POINTER(C.c_double)
    L.pw_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
    L.pw_create_patch.argtypes = [vp, C.POINTER(PatchDesc), C.POINTER(C.c_int32)]
    L.pw_set_exact.argtypes = [vp, C.c_int32, C.POINTER(ExactDesc)]
    L.pw_init_exact.argtypes = [vp, C.c_double]
    L.pw_set_state.argtypes = [vp, C.c_int32, C.c_int32, dp, C.c_int64, C.c_int32, C.c_double]
    L.pw_get_state.argtypes = [vp, C.c_int32, C.c_int32, dp, C.c_int64, C.c_int32]
    L.pw_get_state_full.argtypes = [vp, C.c_int32, C.c_int32, dp, C.c_int64]
    L.pw_get_state_noalloc.argtypes = [vp, C.c_int32, C.c_int32, dp, C.c_int64]
    L.pw_get_flags.argtypes = [vp, C.POINTER(C.c_uint8), C.POINTER(C.c_int32), C.c_int64]
    L.pw_exchange_ghosts.argtypes = [vp, C.c_double]
    L.pw_rk4_step.argtypes = [vp, C.c_double, C.c_int32]
    L.pw_get_time.argtypes = [vp, dp]
    L.pw_diagnostics.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(Diag)]
    L.pw_counters.argtypes = [vp, C.POINTER(Counters)]
    L.pw_live_cells.argtypes = [vp, C.POINTER(C.c_int64)]
    L.pw_enable_timing.argtypes = [vp, C.c_int32]
    L.pw_kernel_times.argtypes = [vp, dp, C.POINTER(C.c_int64)]
    L.pw_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.pw_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.pw_autotune.argtypes = [vp, C.c_double, C.c_int32, C.POINTER(Tuning)]
    L.pw_last_error.restype = C.c_char_p
    L.pw_last_error.argtypes = [vp]
    L.pw_destroy.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("pw_last_error", "pw_destroy"):
            getattr(L, name).restype = C.c_int32
    L.pw_destroy.restype = None
    _lib = L
    return L


class PwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


def patch_desc(d):
    pd = PatchDesc()
    pd.coord = int(d.get("coord", PW_CART))
    pd.is_global = int(d.get("is_global", 0))
    for a in range(3):
        pd.n[a] = int(d["n"][a])
        pd.lo[a] = float(d["lo"][a])
        pd.hi[a] = float(d["hi"][a])
        pd.periodic[a] = int(d.get("periodic", (0, 0, 0))[a])
        pd.euler_zyz[a] = float(d.get("euler", (0, 0, 0))[a])
        pd.c0[a] = float(d.get("c0", (0, 0, 0))[a])
        pd.vel[a] = float(d.get("vel", (0, 0, 0))[a])
        pd.spin[a] = float(d.get("spin", (0, 0, 0))[a])
    pd.motion = int(d.get("motion", PW_STATIC))
    pd.radius = float(d.get("radius", 0.0))
    pd.speed = float(d.get("speed", 0.0))
    pd.phase = float(d.get("phase", 0.0))
    pd.sv_mask = int(d.get("sv_mask", 1))
    return pd


def exact_desc(ex):
    e = ExactDesc()
    if ex is None:
        e.kind = PW_EXACT_NONE
    elif ex["kind"] == "plane":
        e.kind = PW_EXACT_PLANE
        e.amp = float(ex.get("A", 1.0))
        e.offset = float(ex.get("B", 0.0))
        e.phase = float(ex.get("psi", 0.0))
        for a in range(3):
            e.kappa[a] = float(ex["kappa"][a])
    elif ex["kind"] == "gauss":
        e.kind = PW_EXACT_GAUSS
        n = len(ex["amp"])
        e.n_pulses = n
        for g in range(n):
            e.pulse_amp[g] = float(ex["amp"][g])
            e.pulse_width[g] = float(ex["widths"][g])
            for a in range(3):
                e.pulse_center[g][a] = float(ex["centers"][g][a])
    else:
        raise ValueError(ex["kind"])
    return e


class Context:
    """One libpw context (one global patch plus local patches) on the current GPU."""

    def __init__(self, precision=PW_FP64, wave_speed=(1.0,), interp_points=None, buffer_width=4, ko_eps=0.005,
                 schedule=PW_SCHED_BATCHED, use_graph=True, stream=None, torch_alloc=False, pi_form=0, outer_bc=0):
        self.L = load()
        cfg = Config()
        cfg.precision = precision
        cfg.n_state_vectors = len(wave_speed)
        if interp_points is None:
            interp_points = [6] * len(wave_speed)
        for s, v in enumerate(wave_speed):
            cfg.wave_speed[s] = float(v)
            cfg.interp_points[s] = int(interp_points[s])
        cfg.buffer_width = buffer_width
        cfg.ko_eps = ko_eps
        cfg.schedule = schedule
        cfg.use_graph = 1 if use_graph else 0
        cfg.pi_form = pi_form
        cfg.outer_bc = outer_bc
        cfg.stream = stream
        self._keep = []
        self.n_alloc = 0  # device allocations made through the torch allocator callbacks
        if torch_alloc:
            dev = torch.cuda.current_device()

            def _alloc(nbytes, user):
                self.n_alloc += 1
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)

            def _free(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            a, f = ALLOC_FN(_alloc), FREE_FN(_free)
            self._keep += [a, f]
            cfg.dev_alloc = a
            cfg.dev_free = f
        self.h = C.c_void_p()
        rc = self.L.pw_create(C.byref(cfg), C.byref(self.h))
        if rc != 0:
            raise PwError(rc, "pw_create failed")
        self.nsv = len(wave_speed)
        self.patches = []

    def _chk(self, rc):
        if rc != 0:
            raise PwError(rc, self.L.pw_last_error(self.h).decode())

    def close(self):
        if self.h:
            self.L.pw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def create_patch(self, d):
        pd = patch_desc(d)
        pid = C.c_int32()
        self._chk(self.L.pw_create_patch(self.h, C.byref(pd), C.byref(pid)))
        self.patches.append(dict(d))
        return pid.value

    def set_exact(self, sv, ex):
        e = exact_desc(ex)
        self._chk(self.L.pw_set_exact(self.h, sv, C.byref(e)))

    def init_exact(self, t0=0.0):
        self._chk(self.L.pw_init_exact(self.h, t0))

    def shape(self, pid):
        n = self.patches[pid]["n"]
        return (5, n[2], n[1], n[0])

    def set_state(self, pid, sv, arr, t0=0.0):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        self._chk(self.L.pw_set_state(self.h, pid, sv, a.ctypes.data_as(C.POINTER(C.c_double)), a.size, 0, t0))

    def set_state_device(self, pid, sv, ptr, n, t0=0.0):
        self._chk(self.L.pw_set_state(self.h, pid, sv, C.cast(C.c_void_p(ptr), C.POINTER(C.c_double)), n, 1, t0))

    def get_state(self, pid, sv=0):
        out = np.empty(self.shape(pid))
        self._chk(self.L.pw_get_state(self.h, pid, sv, out.ctypes.data_as(C.POINTER(C.c_double)), out.size, 0))
        return out

    def get_state_noalloc(self, pid, sv=0, out=None):
        """pw_get_state_noalloc into a host array (a new one unless `out` is given)."""
        if out is None:
            out = np.empty(self.shape(pid))
        assert out.dtype == np.float64 and out.flags.c_contiguous and out.size == int(np.prod(self.shape(pid)))
        self._chk(self.L.pw_get_state_noalloc(self.h, pid, sv, out.ctypes.data_as(C.POINTER(C.c_double)),
                                              out.size))
        return out

    def get_state_full(self, pid, sv=0):
        n = self.patches[pid]["n"]
        out = np.empty((5, n[2] + 6, n[1] + 6, n[0] + 6))
        self._chk(self.L.pw_get_state_full(self.h, pid, sv, out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
        return out

    def flags(self):
        n = self.patches[0]["n"]
        f = np.empty((n[2], n[1], n[0]), dtype=np.uint8)
        c = np.empty((n[2], n[1], n[0]), dtype=np.int32)
        self._chk(self.L.pw_get_flags(self.h, f.ctypes.data_as(C.POINTER(C.c_uint8)),
                                      c.ctypes.data_as(C.POINTER(C.c_int32)), f.size))
        return f, c

    def exchange_ghosts(self, t):
        self._chk(self.L.pw_exchange_ghosts(self.h, t))

    def rk4_step(self, dt, n=1):
        self._chk(self.L.pw_rk4_step(self.h, dt, n))

    @property
    def t(self):
        v = C.c_double()
        self._chk(self.L.pw_get_time(self.h, C.byref(v)))
        return v.value

    def diagnostics(self, pid, sv=0):
        d = Diag()
        self._chk(self.L.pw_diagnostics(self.h, pid, sv, C.byref(d)))
        return dict(max=np.array(d.max_abs[:]), sumsq=np.array(d.sum_sq[:]), err_max=np.array(d.err_max[:]),
                    err_sumsq=np.array(d.err_sum_sq[:]), int_rel_err=d.int_rel_err, live=int(d.live_cells),
                    volume=d.volume, energy=d.energy, constraint=np.array(d.constraint_max[:]))

    def counters(self):
        c = Counters()
        self._chk(self.L.pw_counters(self.h, C.byref(c)))
        return dict(skip_local=c.skip_local, skip_eff=c.skip_eff, skip_uncover=c.skip_uncover,
                    n_uncover=c.n_uncover, steps=c.steps, skip_outer=c.skip_outer, n_outer=c.n_outer)

    def tuning(self):
        t = Tuning()
        self._chk(self.L.pw_get_tuning(self.h, C.byref(t)))
        return {f: getattr(t, f) for f, _ in Tuning._fields_}

    def set_tuning(self, **kw):
        t = Tuning(**{**self.tuning(), **kw})
        self._chk(self.L.pw_set_tuning(self.h, C.byref(t)))

    def autotune(self, dt, steps_per_trial=3):
        """Time candidate tunings on this context (advances the state; set the
        initial data afterwards) and keep the fastest; returns it."""
        t = Tuning()
        self._chk(self.L.pw_autotune(self.h, dt, steps_per_trial, C.byref(t)))
        return {f: getattr(t, f) for f, _ in Tuning._fields_}

    def enable_timing(self, on=True):
        self._chk(self.L.pw_enable_timing(self.h, 1 if on else 0))

    def kernel_times(self):
        n = len(KERNEL_CLASSES)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        self._chk(self.L.pw_kernel_times(self.h, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES)}

    def live_cells(self):
        v = C.c_int64()
        self._chk(self.L.pw_live_cells(self.h, C.byref(v)))
        return v.value


def context_from_config(cfg, precision=PW_FP64, schedule=PW_SCHED_BATCHED, use_graph=True, stream=None,
                        torch_alloc=False):
    ctx = Context(precision=precision, wave_speed=cfg["wave_speed"], interp_points=cfg["interp_points"],
                  buffer_width=cfg.get("buffer", 4), ko_eps=cfg.get("ko_eps", 0.005), schedule=schedule,
                  use_graph=use_graph, stream=stream, torch_alloc=torch_alloc, pi_form=cfg.get("pi_form", 0),
                  outer_bc=cfg.get("outer_bc", 0))
    for d in cfg["patches"]:
        ctx.create_patch(d)
    for sv, ex in enumerate(cfg.get("exact", [])):
        if ex is not None:
            ctx.set_exact(sv, ex)
    return ctx
