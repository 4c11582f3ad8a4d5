"""ctypes binding of libgrlbm.so (the C ABI of include/grlbm.h), same names.

Argument marshalling only: every step of the solver runs in the HIP library.  The
library is loaded on first use; if it is missing this module raises instead of
falling back to anything else.

A parameter dict (lattice units, the keys produced by `inputs`) converts to
`lbm_params` with `make_params`.  `Solver` is a small convenience wrapper that owns a
context and checks every status.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrlbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EDIVERGED, LBM_ESTATE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
                -4: "LBM_EDIVERGED", -5: "LBM_ESTATE"}
LBM_STORE_F32, LBM_STORE_F16 = 0, 1
LBM_START_FIRST_ORDER, LBM_START_EQUILIBRIUM = 0, 1


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3),
        ("collision", ctypes.c_int32), ("storage", ctypes.c_int32), ("mu_law", ctypes.c_int32),
        ("layout_pad", ctypes.c_int32), ("start", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("mu_ref", ctypes.c_double), ("kappa_ref", ctypes.c_double),
        ("T_ref", ctypes.c_double), ("T_S", ctypes.c_double),
        ("omega", ctypes.c_double * 5),
        ("sensor_gain", ctypes.c_double), ("J_min", ctypes.c_double), ("omega_min", ctypes.c_double),
        ("rho_min", ctypes.c_double), ("p_min", ctypes.c_double),
        ("rho_ref", ctypes.c_double), ("E_ref", ctypes.c_double),
    ]


class lbm_diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("Ek", ctypes.c_double), ("eps_s", ctypes.c_double), ("eps_d", ctypes.c_double),
        ("dtotal", ctypes.c_double * 5),
        ("nonfinite", ctypes.c_int64),
    ]


class lbm_launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("odd_lds", ctypes.c_int32)]

    def as_dict(self):
        return dict(block=self.block, nontemporal=self.nontemporal,
                    blocks_per_cu=self.blocks_per_cu, odd_lds=self.odd_lds)


class lbm_batch_tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("grid", ctypes.c_int32)]

    def as_dict(self):
        return dict(block=self.block, nontemporal=self.nontemporal,
                    blocks_per_cu=self.blocks_per_cu, grid=self.grid)


class lbm_batch_stats(ctypes.Structure):
    _fields_ = [("clock", ctypes.c_int64), ("arena_bytes", ctypes.c_size_t),
                ("arena_free_bytes", ctypes.c_size_t), ("arena_largest_free", ctypes.c_size_t),
                ("live_instances", ctypes.c_int32), ("active_instances", ctypes.c_int32),
                ("active_cells", ctypes.c_int64), ("tuning", lbm_batch_tuning),
                ("graph_steps", ctypes.c_int32)]


class LbmError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

# name -> (restype, argtypes)
_P = ctypes.POINTER
_vp = ctypes.c_void_p
class lbm_mms(ctypes.Structure):
    """Constants of the manufactured solution (include/grlbm_mms.h), lattice units."""
    _fields_ = [(n, ctypes.c_double) for n in
                ("rho0", "U", "P0", "a", "K", "W", "gamma", "mu", "kappa")]


SIGNATURES = {
    "lbm_state_bytes": (ctypes.c_size_t, [_P(lbm_params)]),
    "lbm_create": (ctypes.c_int, [_P(lbm_params), _vp, _P(_vp)]),
    "lbm_create_in": (ctypes.c_int, [_P(lbm_params), _vp, ctypes.c_size_t, _vp, _P(_vp)]),
    "lbm_init_fields": (ctypes.c_int, [_vp, _P(ctypes.c_double)]),
    "lbm_init_fields_device": (ctypes.c_int, [_vp, _vp]),
    "lbm_step": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int32]),
    "lbm_moments": (ctypes.c_int, [_vp, _P(ctypes.c_double)]),
    "lbm_moments_device": (ctypes.c_int, [_vp, _vp]),
    "lbm_diagnostics": (ctypes.c_int, [_vp, _P(lbm_diag), ctypes.c_int32, _P(ctypes.c_int32)]),
    "lbm_get_populations": (ctypes.c_int, [_vp, _P(ctypes.c_float), _P(ctypes.c_int64)]),
    "lbm_set_populations": (ctypes.c_int, [_vp, _P(ctypes.c_float), ctypes.c_int64]),
    "lbm_set_launch": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "lbm_get_launch": (ctypes.c_int, [_vp, _P(lbm_launch)]),
    "lbm_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, _P(lbm_launch), _P(ctypes.c_float), _P(lbm_launch),
                                    _P(ctypes.c_float), ctypes.c_int32, _P(ctypes.c_int32)]),
    "lbm_set_source": (ctypes.c_int, [_vp, _vp]),
    "lbm_mms_source": (ctypes.c_int, [_P(lbm_mms), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_double, _vp, _vp]),
    "lbm_get_step": (ctypes.c_int, [_vp, _P(ctypes.c_int64)]),
    "lbm_destroy": (ctypes.c_int, [_vp]),
    "lbm_step_noalloc": (ctypes.c_int, [_P(lbm_params), _vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                        _vp, ctypes.c_int32, _vp]),
    "lbm_bw_probe": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32, _P(ctypes.c_double)]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_batch_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        _vp, _P(_vp)]),
    "lbm_batch_add": (ctypes.c_int, [_vp, _P(lbm_params), _P(ctypes.c_double), ctypes.c_int64,
                                     _P(ctypes.c_int32)]),
    "lbm_batch_run": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "lbm_batch_query": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_int64), _P(ctypes.c_int32)]),
    "lbm_batch_moments": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_double)]),
    "lbm_batch_populations": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_float), _P(ctypes.c_int64)]),
    "lbm_batch_remove": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "lbm_batch_nonfinite": (ctypes.c_int, [_vp, _P(ctypes.c_int32), ctypes.c_int32, _P(ctypes.c_int32)]),
    "lbm_batch_info": (ctypes.c_int, [_vp, _P(lbm_batch_stats)]),
    "lbm_batch_set_tuning": (ctypes.c_int, [_vp, _P(lbm_batch_tuning)]),
    "lbm_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, _P(lbm_batch_tuning), _P(ctypes.c_float),
                                          _P(lbm_batch_tuning), _P(ctypes.c_float), ctypes.c_int32,
                                          _P(ctypes.c_int32)]),
    "lbm_batch_destroy": (ctypes.c_int, [_vp]),
}


def load(path: str = LIB_PATH):
    """Load the HIP library (raises FileNotFoundError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with paper_2609_16361_amd.build.build() "
            "(there is no fallback implementation)")
    # PyTorch ships its own HIP runtime with the same soname.  Loading torch first
    # makes libgrlbm.so bind to that runtime, so one process never holds two HIP
    # runtimes (which leaves whichever initialises second without a device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, where):
    if status != LBM_OK:
        msg = load().lbm_last_error().decode(errors="replace")
        raise LbmError(status, where, msg)


def make_params(p: dict, storage: int | None = None, layout_pad: int = 0) -> lbm_params:
    o = lbm_params()
    o.nx, o.ny, o.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    for a in range(3):
        o.bc[a] = int(p["bc"][a])
    o.collision = int(p["collision"])
    o.storage = int(p.get("storage", LBM_STORE_F32) if storage is None else storage)
    o.mu_law = int(p["mu_law"])
    o.layout_pad = int(p.get("layout_pad", layout_pad))
    o.start = int(p.get("start", LBM_START_FIRST_ORDER))
    o.gamma = float(p["gamma"])
    o.mu_ref = float(p["mu_ref"])
    o.kappa_ref = float(p["kappa_ref"])
    o.T_ref = float(p["T_ref"])
    o.T_S = float(p["T_S"])
    for k in range(5):
        o.omega[k] = float(p["omega"][k])
    o.sensor_gain = float(p["sensor_gain"])
    o.J_min = float(p["J_min"])
    o.omega_min = float(p["omega_min"])
    o.rho_min = float(p["rho_min"])
    o.p_min = float(p["p_min"])
    o.rho_ref = float(p["rho_ref"])
    o.E_ref = float(p["E_ref"])
    return o


# ---------------------------------------------------------- C names, thin wrappers
def lbm_state_bytes(params: lbm_params) -> int:
    return int(load().lbm_state_bytes(ctypes.byref(params)))


def lbm_create(params: lbm_params, stream: int | None = None) -> int:
    h = _vp()
    _check(load().lbm_create(ctypes.byref(params), stream, ctypes.byref(h)), "lbm_create")
    return h.value


def lbm_create_in(params: lbm_params, dev_ptr: int, nbytes: int, stream: int | None = None) -> int:
    h = _vp()
    _check(load().lbm_create_in(ctypes.byref(params), dev_ptr, nbytes, stream, ctypes.byref(h)),
           "lbm_create_in")
    return h.value


def lbm_init_fields(ctx: int, Q: np.ndarray) -> None:
    q = np.ascontiguousarray(Q, dtype=np.float64)
    _check(load().lbm_init_fields(ctx, q.ctypes.data_as(_P(ctypes.c_double))), "lbm_init_fields")


def lbm_init_fields_device(ctx: int, dev_ptr: int) -> None:
    _check(load().lbm_init_fields_device(ctx, dev_ptr), "lbm_init_fields_device")


def lbm_step(ctx: int, n: int, diag_every: int = 0) -> None:
    _check(load().lbm_step(ctx, int(n), int(diag_every)), "lbm_step")


def lbm_moments(ctx: int, shape) -> np.ndarray:
    out = np.empty((5,) + tuple(shape), dtype=np.float64)
    _check(load().lbm_moments(ctx, out.ctypes.data_as(_P(ctypes.c_double))), "lbm_moments")
    return out


def lbm_moments_device(ctx: int, dev_ptr: int) -> None:
    _check(load().lbm_moments_device(ctx, dev_ptr), "lbm_moments_device")


def lbm_diagnostics(ctx: int, max_records: int = 4096):
    """Returns (records as a list of dicts, status).  EDIVERGED is returned, not
    raised, so callers can inspect the records."""
    buf = (lbm_diag * max_records)()
    cnt = ctypes.c_int32(0)
    st = load().lbm_diagnostics(ctx, buf, max_records, ctypes.byref(cnt))
    if st not in (LBM_OK, LBM_EDIVERGED):
        _check(st, "lbm_diagnostics")
    recs = []
    for i in range(cnt.value):
        d = buf[i]
        recs.append(dict(step=d.step, Ek=d.Ek, eps_s=d.eps_s, eps_d=d.eps_d,
                         dtotal=list(d.dtotal), nonfinite=d.nonfinite))
    return recs, st


def lbm_get_populations(ctx: int, shape):
    f = np.empty((35,) + tuple(shape), dtype=np.float32)
    step = ctypes.c_int64(0)
    _check(load().lbm_get_populations(ctx, f.ctypes.data_as(_P(ctypes.c_float)), ctypes.byref(step)),
           "lbm_get_populations")
    return f, step.value


def lbm_set_populations(ctx: int, f: np.ndarray, step: int) -> None:
    ff = np.ascontiguousarray(f, dtype=np.float32)
    _check(load().lbm_set_populations(ctx, ff.ctypes.data_as(_P(ctypes.c_float)), int(step)),
           "lbm_set_populations")


def lbm_set_launch(ctx: int, block: int, nontemporal: bool, blocks_per_cu: int = 0,
                   odd_lds: bool = True) -> None:
    _check(load().lbm_set_launch(ctx, int(block), int(bool(nontemporal)), int(blocks_per_cu),
                                 int(bool(odd_lds))),
           "lbm_set_launch")


def lbm_get_step(ctx: int) -> int:
    s = ctypes.c_int64(0)
    _check(load().lbm_get_step(ctx, ctypes.byref(s)), "lbm_get_step")
    return s.value


def lbm_destroy(ctx: int) -> None:
    _check(load().lbm_destroy(ctx), "lbm_destroy")


def lbm_step_noalloc(params: lbm_params, F_dev: int, step: int, n: int, diag_every: int = 0,
                     rec_dev: int | None = None, rec_max: int = 0, stream: int | None = None) -> None:
    """F_dev, rec_dev: device addresses (e.g. tensor.data_ptr()); rec_dev receives
    9 floats per diagnostic step."""
    _check(load().lbm_step_noalloc(ctypes.byref(params), F_dev, int(step), int(n), int(diag_every), rec_dev,
                                   int(rec_max), stream), "lbm_step_noalloc")


def lbm_bw_probe(nbytes: int, iters: int = 10) -> float:
    g = ctypes.c_double(0.0)
    _check(load().lbm_bw_probe(int(nbytes), int(iters), ctypes.byref(g)), "lbm_bw_probe")
    return g.value


def lbm_set_source(ctx: int, S_dev: int | None) -> None:
    """S_dev: device address of S[5][nz][ny][nx] FP32 (e.g. tensor.data_ptr()), or
    None to switch the source off."""
    _check(load().lbm_set_source(ctx, S_dev), "lbm_set_source")


def lbm_mms_source(m: dict, nx: int, ny: int, nz: int, t: float, S_dev: int, stream: int | None = None) -> None:
    """Manufactured-solution source at lattice time t into S_dev (FP32 [5][nz][ny][nx])."""
    mm = lbm_mms(*[float(m[n]) for n, _ in lbm_mms._fields_])
    _check(load().lbm_mms_source(ctypes.byref(mm), int(nx), int(ny), int(nz), float(t), S_dev, stream),
           "lbm_mms_source")


def lbm_get_launch(ctx: int) -> dict:
    out = lbm_launch()
    _check(load().lbm_get_launch(ctx, ctypes.byref(out)), "lbm_get_launch")
    return out.as_dict()


def lbm_autotune(ctx: int, trial_steps: int = 20, max_tried: int = 32):
    """Returns (best launch dict, best us/step, [(launch dict, us/step), ...])."""
    best = lbm_launch()
    bus = ctypes.c_float(0)
    tried = (lbm_launch * max_tried)()
    tus = (ctypes.c_float * max_tried)()
    n = ctypes.c_int32(0)
    _check(load().lbm_autotune(ctx, int(trial_steps), ctypes.byref(best), ctypes.byref(bus), tried, tus,
                               int(max_tried), ctypes.byref(n)), "lbm_autotune")
    return best.as_dict(), bus.value, [(tried[i].as_dict(), tus[i]) for i in range(n.value)]


def lbm_last_error() -> str:
    return load().lbm_last_error().decode(errors="replace")


# ----------------------------------------------------------------- convenience
class Solver:
    """One context.  `stream` is a hipStream_t handle (e.g.
    torch.cuda.current_stream().cuda_stream) or None for a private stream."""

    def __init__(self, params: dict, stream: int | None = None, storage: int | None = None,
                 block: int | None = None, nontemporal: bool | None = None, layout_pad: int = 0,
                 blocks_per_cu: int | None = None, odd_lds: bool = True):
        self.params = dict(params)
        self.cparams = make_params(params, storage=storage, layout_pad=layout_pad)
        self.shape = (self.cparams.nz, self.cparams.ny, self.cparams.nx)
        self.ctx = lbm_create(self.cparams, stream)
        if block is not None or nontemporal is not None or blocks_per_cu is not None or not odd_lds:
            # unspecified settings keep the library's defaults for this grid
            d = lbm_get_launch(self.ctx)
            lbm_set_launch(self.ctx, d["block"] if block is None else block,
                           d["nontemporal"] if nontemporal is None else bool(nontemporal),
                           d["blocks_per_cu"] if blocks_per_cu is None else blocks_per_cu, odd_lds)

    def init(self, Q):
        lbm_init_fields(self.ctx, np.asarray(Q, dtype=np.float64).reshape((5,) + self.shape))

    def step(self, n, diag_every=0):
        lbm_step(self.ctx, n, diag_every)

    def set_source(self, S_dev):
        lbm_set_source(self.ctx, S_dev)

    def autotune(self, trial_steps=20):
        """Pick the fastest launch shape on the current state (left unchanged)."""
        return lbm_autotune(self.ctx, trial_steps)

    def launch(self):
        return lbm_get_launch(self.ctx)

    def moments(self):
        return lbm_moments(self.ctx, self.shape)

    def diagnostics(self):
        return lbm_diagnostics(self.ctx)

    def populations(self):
        return lbm_get_populations(self.ctx, self.shape)

    def set_populations(self, f, step):
        lbm_set_populations(self.ctx, f, step)

    @property
    def step_count(self):
        return lbm_get_step(self.ctx)

    def close(self):
        if self.ctx:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------- batches
def lbm_batch_create(arena_bytes: int, max_instances: int, max_tiles: int, graph_steps: int = 16,
                     stream: int | None = None) -> int:
    h = _vp()
    _check(load().lbm_batch_create(int(arena_bytes), int(max_instances), int(max_tiles),
                                   int(graph_steps), stream, ctypes.byref(h)), "lbm_batch_create")
    return h.value


def lbm_batch_add(batch: int, params: lbm_params, Q: np.ndarray, steps: int) -> int:
    q = np.ascontiguousarray(Q, dtype=np.float64)
    i = ctypes.c_int32(-1)
    _check(load().lbm_batch_add(batch, ctypes.byref(params), q.ctypes.data_as(_P(ctypes.c_double)),
                                int(steps), ctypes.byref(i)), "lbm_batch_add")
    return i.value


def lbm_batch_run(batch: int, n: int) -> None:
    _check(load().lbm_batch_run(batch, int(n)), "lbm_batch_run")


def lbm_batch_query(batch: int, inst: int):
    d = ctypes.c_int64(0)
    f = ctypes.c_int32(0)
    _check(load().lbm_batch_query(batch, int(inst), ctypes.byref(d), ctypes.byref(f)), "lbm_batch_query")
    return d.value, bool(f.value)


def lbm_batch_moments(batch: int, inst: int, shape) -> np.ndarray:
    out = np.empty((5,) + tuple(shape), dtype=np.float64)
    _check(load().lbm_batch_moments(batch, int(inst), out.ctypes.data_as(_P(ctypes.c_double))),
           "lbm_batch_moments")
    return out


def lbm_batch_populations(batch: int, inst: int, shape):
    f = np.empty((35,) + tuple(shape), dtype=np.float32)
    s = ctypes.c_int64(0)
    _check(load().lbm_batch_populations(batch, int(inst), f.ctypes.data_as(_P(ctypes.c_float)),
                                        ctypes.byref(s)), "lbm_batch_populations")
    return f, s.value


def lbm_batch_remove(batch: int, inst: int) -> None:
    _check(load().lbm_batch_remove(batch, int(inst)), "lbm_batch_remove")


def lbm_batch_nonfinite(batch: int, max_ids: int) -> list:
    ids = (ctypes.c_int32 * max(1, int(max_ids)))()
    count = ctypes.c_int32()
    _check(load().lbm_batch_nonfinite(batch, ids, int(max_ids), ctypes.byref(count)), "lbm_batch_nonfinite")
    return [int(ids[i]) for i in range(min(count.value, int(max_ids)))]


def lbm_batch_info(batch: int) -> dict:
    s = lbm_batch_stats()
    _check(load().lbm_batch_info(batch, ctypes.byref(s)), "lbm_batch_info")
    return dict(clock=s.clock, arena_bytes=s.arena_bytes, arena_free_bytes=s.arena_free_bytes,
                arena_largest_free=s.arena_largest_free, live_instances=s.live_instances,
                active_instances=s.active_instances, active_cells=s.active_cells,
                tuning=s.tuning.as_dict(), graph_steps=s.graph_steps)


def lbm_batch_set_tuning(batch: int, block: int, nontemporal: bool, blocks_per_cu: int, grid: int) -> None:
    t = lbm_batch_tuning(int(block), int(bool(nontemporal)), int(blocks_per_cu), int(grid))
    _check(load().lbm_batch_set_tuning(batch, ctypes.byref(t)), "lbm_batch_set_tuning")


def lbm_batch_autotune(batch: int, trial_steps: int = 20, max_tried: int = 64):
    """Returns (best tuning dict, best us/step, [(tuning dict, us/step), ...])."""
    best = lbm_batch_tuning()
    bus = ctypes.c_float(0)
    tried = (lbm_batch_tuning * max_tried)()
    tus = (ctypes.c_float * max_tried)()
    n = ctypes.c_int32(0)
    _check(load().lbm_batch_autotune(batch, int(trial_steps), ctypes.byref(best), ctypes.byref(bus),
                                     tried, tus, int(max_tried), ctypes.byref(n)), "lbm_batch_autotune")
    return best.as_dict(), bus.value, [(tried[i].as_dict(), tus[i]) for i in range(n.value)]


def lbm_batch_destroy(batch: int) -> None:
    _check(load().lbm_batch_destroy(batch), "lbm_batch_destroy")


class Batch:
    """Owns one lbm_batch; instances are added from parameter dicts."""

    def __init__(self, arena_bytes: int, max_instances: int = 1024, max_tiles: int = 1 << 20,
                 graph_steps: int = 16, stream: int | None = None):
        self.h = lbm_batch_create(arena_bytes, max_instances, max_tiles, graph_steps, stream)
        self.shapes = {}

    def add(self, params: dict, Q, steps: int, storage: int | None = None) -> int:
        p = make_params(params, storage=storage)
        i = lbm_batch_add(self.h, p, np.asarray(Q, dtype=np.float64), steps)
        self.shapes[i] = (p.nz, p.ny, p.nx)
        return i

    def run(self, n: int) -> None:
        lbm_batch_run(self.h, n)

    def query(self, i: int):
        return lbm_batch_query(self.h, i)

    def moments(self, i: int):
        return lbm_batch_moments(self.h, i, self.shapes[i])

    def populations(self, i: int):
        return lbm_batch_populations(self.h, i, self.shapes[i])

    def remove(self, i: int) -> None:
        lbm_batch_remove(self.h, i)
        self.shapes.pop(i, None)

    def nonfinite(self) -> list:
        """Ids of the live instances whose state is no longer finite."""
        return lbm_batch_nonfinite(self.h, max(1, len(self.shapes)))

    def info(self) -> dict:
        return lbm_batch_info(self.h)

    def autotune(self, trial_steps: int = 20):
        return lbm_batch_autotune(self.h, trial_steps)

    def set_tuning(self, block, nontemporal, blocks_per_cu, grid):
        lbm_batch_set_tuning(self.h, block, nontemporal, blocks_per_cu, grid)

    def close(self):
        if self.h:
            lbm_batch_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
