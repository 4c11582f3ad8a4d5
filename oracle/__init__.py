"""FP64 CPU oracle of the five-field gradient-reconstruction LBM (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The product path (the HIP library and its
Python binding) never imports this package; the two share no code.

The arithmetic lives in oracle.c (Algorithm 1 of the paper step by step, FP64, two
buffers, push streaming).  This module only marshals numpy arrays.

Parameters are passed as a plain dict in lattice units with the keys
  nx, ny, nz, bc (3 ints: 0 periodic, 1 zero gradient), collision (0 regularized
  with sensor, 1 BGK), mu_law (0 constant, 1 Sutherland), start (0 first-order,
  1 equilibrium; optional, default 0), gamma, mu_ref, kappa_ref,
  T_ref, T_S, omega (5 floats), sensor_gain, J_min, omega_min, rho_min, p_min.
Extra keys are ignored.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("GRLBM_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))
_lib = None


class OraParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3),
        ("collision", ctypes.c_int32), ("mu_law", ctypes.c_int32), ("start", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("mu_ref", ctypes.c_double), ("kappa_ref", ctypes.c_double),
        ("T_ref", ctypes.c_double), ("T_S", ctypes.c_double),
        ("omega", ctypes.c_double * 5),
        ("sensor_gain", ctypes.c_double), ("J_min", ctypes.c_double),
        ("omega_min", ctypes.c_double),
        ("rho_min", ctypes.c_double), ("p_min", ctypes.c_double),
    ]


_D = ctypes.c_double


class OraCellInfo(ctypes.Structure):
    _fields_ = [
        ("Q", _D * 5), ("J", (_D * 3) * 5),
        ("rho_f", _D), ("u", _D * 3), ("k2", _D), ("p", _D), ("T", _D),
        ("mu", _D), ("kappa", _D), ("nu", _D),
        ("Phi_adv", (_D * 3) * 5), ("Pi", (_D * 3) * 5), ("gradQ_tilde", (_D * 3) * 5),
        ("M", (_D * 15) * 15),
        ("gradQ", (_D * 3) * 5),
        ("grad_u", (_D * 3) * 3),
        ("grad_T", _D * 3),
        ("theta", _D), ("s", _D), ("chi", _D),
        ("omega_h", _D * 5),
        ("tau", (_D * 3) * 3), ("q", _D * 3),
        ("Phi", (_D * 3) * 5),
        ("ek", _D), ("eps_s", _D), ("eps_d", _D),
        ("nonfinite", ctypes.c_int32),
    ]


class OraMms(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("rho0", "U", "P0", "a", "K", "W", "gamma", "mu", "kappa")]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    lib.ora_collide.argtypes = [P(OraParams), dp, dp, P(OraCellInfo)]
    lib.ora_init.argtypes = [P(OraParams), dp, dp]
    lib.ora_moments.argtypes = [P(OraParams), dp, dp]
    lib.ora_step.argtypes = [P(OraParams), dp, dp, dp]
    lib.ora_run.argtypes = [P(OraParams), dp, dp, ctypes.c_int64, ctypes.c_int64, dp]
    lib.ora_run.restype = ctypes.c_int64
    lib.ora_step_src.argtypes = [P(OraParams), dp, dp, dp, dp]
    lib.ora_mms_source.argtypes = [P(OraParams), P(OraMms), ctypes.c_double, dp]
    lib.ora_run_mms.argtypes = [P(OraParams), P(OraMms), dp, dp, dp, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double]
    lib.ora_mms_size.restype = ctypes.c_int32
    lib.ora_cell_info_size.restype = ctypes.c_int32
    lib.ora_params_size.restype = ctypes.c_int32
    lib.ora_num_threads.restype = ctypes.c_int32
    lib.ora_set_num_threads.argtypes = [ctypes.c_int32]
    lib.ora_set_num_threads.restype = None
    if lib.ora_cell_info_size() != ctypes.sizeof(OraCellInfo):
        raise RuntimeError("oracle cell-info layout mismatch")
    if lib.ora_params_size() != ctypes.sizeof(OraParams):
        raise RuntimeError("oracle params layout mismatch")
    if lib.ora_mms_size() != ctypes.sizeof(OraMms):
        raise RuntimeError("oracle manufactured-solution layout mismatch")
    _lib = lib
    return lib


def make_params(p: dict) -> OraParams:
    o = OraParams()
    o.nx, o.ny, o.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    for a in range(3):
        o.bc[a] = int(p["bc"][a])
    o.collision = int(p["collision"])
    o.mu_law = int(p["mu_law"])
    o.start = int(p.get("start", 0))
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
    return o


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def cells(p: dict) -> int:
    return int(p["nx"]) * int(p["ny"]) * int(p["nz"])


def collide(p: dict, f_in):
    """One cell: f_in[35] -> (f_out[35], info dict of every intermediate)."""
    lib = _load()
    P = make_params(p)
    fi = np.ascontiguousarray(np.asarray(f_in, dtype=np.float64).reshape(35))
    fo = np.zeros(35)
    info = OraCellInfo()
    lib.ora_collide(ctypes.byref(P), _ptr(fi), _ptr(fo), ctypes.byref(info))
    out = {}
    for name, _ in OraCellInfo._fields_:
        v = getattr(info, name)
        out[name] = np.ctypeslib.as_array(v).copy() if hasattr(v, "_length_") else v
    return fo, out


def init(p: dict, Q) -> np.ndarray:
    """Q[5][nz][ny][nx] (lattice units) -> equilibrium populations f[35][N]."""
    lib = _load()
    P = make_params(p)
    N = cells(p)
    q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(5, N))
    f = np.zeros((35, N))
    lib.ora_init(ctypes.byref(P), _ptr(q), _ptr(f))
    return f


def moments(p: dict, f) -> np.ndarray:
    """f[35][N] -> Q[5][nz][ny][nx]."""
    lib = _load()
    P = make_params(p)
    N = cells(p)
    ff = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(35, N))
    Q = np.zeros((5, N))
    lib.ora_moments(ctypes.byref(P), _ptr(ff), _ptr(Q))
    return Q.reshape(5, int(p["nz"]), int(p["ny"]), int(p["nx"]))


def step(p: dict, f):
    """One step from f[35][N]; returns (f_new, diag[9]) where diag holds the sums of
    the pre-step state: E_k, eps_s, eps_d densities, five conserved totals, and the
    number of non-finite cells."""
    lib = _load()
    P = make_params(p)
    N = cells(p)
    fi = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(35, N))
    fo = np.zeros_like(fi)
    d = np.zeros(9)
    lib.ora_step(ctypes.byref(P), _ptr(fi), _ptr(fo), _ptr(d))
    return fo, d


def run(p: dict, f, nsteps: int, diag_every: int = 0):
    """nsteps steps from f[35][N] (copied); returns (f_final, diag rows [R,9])."""
    lib = _load()
    P = make_params(p)
    N = cells(p)
    a = np.array(np.asarray(f, dtype=np.float64).reshape(35, N), copy=True, order="C")
    w = np.empty_like(a)
    rows = (nsteps + diag_every - 1) // diag_every if diag_every > 0 else 0
    d = np.zeros((max(rows, 1), 9))
    r = lib.ora_run(ctypes.byref(P), _ptr(a), _ptr(w), int(nsteps), int(diag_every), _ptr(d))
    return a, d[:r]


def num_threads() -> int:
    """Threads the oracle's parallel cell loop uses (OpenMP)."""
    return int(_load().ora_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's following steps (results do not depend on it)."""
    _load().ora_set_num_threads(int(n))


def _mms(m: dict) -> OraMms:
    o = OraMms()
    for name, _ in OraMms._fields_:
        setattr(o, name, float(m[name]))
    return o


def step_source(p: dict, f, S):
    """One step from f[35][N] with the source S[5][N] (lattice units per step) added
    as w_i S_k after the collision; returns (f_new, diag[9])."""
    lib = _load()
    P = make_params(p)
    N = cells(p)
    fi = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(35, N))
    src = np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(5, N))
    fo = np.zeros_like(fi)
    d = np.zeros(9)
    lib.ora_step_src(ctypes.byref(P), _ptr(fi), _ptr(fo), _ptr(d), _ptr(src))
    return fo, d


def mms_source(p: dict, m: dict, t: float) -> np.ndarray:
    """Source of the manufactured solution (eq. 8) at every cell at lattice time t:
    S[5][nz][ny][nx].  m holds rho0, U, P0, a, K, W, gamma, mu, kappa in lattice
    units."""
    lib = _load()
    P = make_params(p)
    M = _mms(m)
    S = np.zeros((5, cells(p)))
    lib.ora_mms_source(ctypes.byref(P), ctypes.byref(M), float(t), _ptr(S))
    return S.reshape(5, int(p["nz"]), int(p["ny"]), int(p["nx"]))


def run_mms(p: dict, m: dict, f, nsteps: int, t0: float = 0.0, t_frac: float = 0.5):
    """nsteps steps from f (copied) with the manufactured source; the source of step
    s is evaluated at lattice time t0 + s + t_frac."""
    lib = _load()
    P = make_params(p)
    M = _mms(m)
    N = cells(p)
    a = np.array(np.asarray(f, dtype=np.float64).reshape(35, N), copy=True, order="C")
    w = np.empty_like(a)
    S = np.empty((5, N))
    lib.ora_run_mms(ctypes.byref(P), ctypes.byref(M), _ptr(a), _ptr(w), _ptr(S), int(nsteps), float(t0),
                    float(t_frac))
    return a
