"""ctypes wrapper of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The product package never imports it.

All arrays are numpy float64 in the layout f[i, y, x] (D1Q3: ny = 1); the
state is the post-streaming (pre-collision) state of eq. (lbgkLB).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# the same source built with OpenMP: used only to time the CPU baseline
TIMING_LIB_PATH = os.path.join(HERE, "liboracle_omp.so")

D1Q3, D2Q9 = 1, 2
QE_POLY, QE_ENTROPIC = 0, 1
DS_EXACT, DS_QUADRATIC = 0, 1
LIM_TRIM, LIM_MEDIAN = 1, 2
LIM_ENS_THRESHOLD, LIM_ENS_SMOOTH, LIM_ENS_RATIONAL, LIM_ENS_BUDGET = 4, 8, 16, 32
TRIM_HOMOTHETY, TRIM_EHRENFEST = 0, 1
MED_FLOOR, MED_GATE = 0, 1
BC_PERIODIC, BC_CAVITY, BC_TUBE, BC_CAVITY_DIFFUSIVE = 0, 1, 2, 3
MASK_TRIM, MASK_MEDIAN, MASK_NONPOS, MASK_NOTFLUID, MASK_ENSEMBLE, MASK_POSITIVITY = 1, 2, 4, 8, 16, 32
LIM_POSITIVITY = 64
COLL_LBGK, COLL_ELBM = 0, 1


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("beta", ctypes.c_double),
        ("qe", ctypes.c_int32), ("ds_form", ctypes.c_int32), ("limiter", ctypes.c_int32),
        ("trim_mode", ctypes.c_int32), ("median_mode", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("delta_trim", ctypes.c_double), ("delta_median", ctypes.c_double),
        ("rho0", ctypes.c_double), ("lid_ux", ctypes.c_double),
        ("entropy", ctypes.c_int32),
        ("ens_c", ctypes.c_double), ("ens_k", ctypes.c_double), ("delta_ens", ctypes.c_double),
        ("collision", ctypes.c_int32), ("homothety", ctypes.c_int32), ("top_k", ctypes.c_int64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
        ("sum_dS_pre", ctypes.c_double), ("sum_dS_post", ctypes.c_double), ("max_dS", ctypes.c_double),
        ("lbgk_production", ctypes.c_double), ("limiter_production", ctypes.c_double),
        ("total_entropy", ctypes.c_double),
        ("n_trimmed", ctypes.c_int64), ("n_filtered", ctypes.c_int64),
        ("n_nonpositive", ctypes.c_int64), ("n_nonfinite", ctypes.c_int64), ("n_fluid", ctypes.c_int64),
        ("n_ensemble", ctypes.c_int64), ("mean_dS", ctypes.c_double), ("ens_threshold", ctypes.c_double),
        ("n_positivity", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _stale(path, src):
    return not os.path.exists(path) or os.path.getmtime(path) < max(
        os.path.getmtime(src), os.path.getmtime(os.path.join(HERE, "oracle.h")))


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no FP contraction)."""
    src = os.path.join(HERE, "oracle.c")
    if force or _stale(LIB_PATH, src):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-o", LIB_PATH, src, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB_PATH


def build_timing(force: bool = False) -> str:
    """The same source with -fopenmp (per-node loops over rows in parallel,
    global sums still in row-major order): the CPU baseline's timing build."""
    src = os.path.join(HERE, "oracle.c")
    if force or _stale(TIMING_LIB_PATH, src):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-o", TIMING_LIB_PATH, src, "-lm"]
        subprocess.run(cmd, check=True)
    return TIMING_LIB_PATH


_lib = None
_timing_lib = None


def _declare(L):
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_threads.restype = ctypes.c_int
    L.orc_q.argtypes = [ctypes.c_int32]
    L.orc_equilibrium.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, dp]
    L.orc_delta_s.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp]
    L.orc_delta_s.restype = ctypes.c_double
    L.orc_h.argtypes = [ctypes.c_double]
    L.orc_h.restype = ctypes.c_double
    L.orc_entropy.argtypes = [ctypes.c_int32, dp]
    L.orc_entropy.restype = ctypes.c_double
    L.orc_median.argtypes = [dp, ctypes.c_int32]
    L.orc_median.restype = ctypes.c_double
    L.orc_elbm_alpha.argtypes = [ctypes.c_int32, dp, dp, ctypes.POINTER(ctypes.c_int32)]
    L.orc_elbm_alpha.restype = ctypes.c_double
    L.orc_step.argtypes = [ctypes.POINTER(Params), dp, ctypes.POINTER(Stats),
                           ctypes.POINTER(ctypes.c_uint8), dp, dp]
    L.orc_stream.argtypes = [ctypes.POINTER(Params), dp, dp]
    L.orc_init_equilibrium.argtypes = [ctypes.POINTER(Params), dp, dp, dp]
    return L


def timing_lib():
    """ctypes handle of the OpenMP timing build (CPU baseline only)."""
    global _timing_lib
    if _timing_lib is None:
        build_timing()
        _timing_lib = _declare(ctypes.CDLL(TIMING_LIB_PATH))
    return _timing_lib


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def q_of(lattice: int) -> int:
    return 3 if lattice == D1Q3 else 9


def velocities(lattice: int):
    L = lib()
    q = q_of(lattice)
    vx, vy = ctypes.c_int32(), ctypes.c_int32()
    out = []
    for i in range(q):
        L.orc_velocity(lattice, i, ctypes.byref(vx), ctypes.byref(vy))
        out.append((vx.value, vy.value))
    return np.array(out, dtype=np.int64)


def opposite(lattice: int, i: int) -> int:
    return lib().orc_opposite(lattice, i)


def equilibrium(lattice: int, qe: int, rho: float, ux: float, uy: float = 0.0) -> np.ndarray:
    out = np.zeros(q_of(lattice))
    lib().orc_equilibrium(lattice, qe, rho, ux, uy, _dp(out))
    return out


def delta_s(form: int, f: np.ndarray, fstar: np.ndarray) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    fstar = np.ascontiguousarray(fstar, dtype=np.float64)
    return lib().orc_delta_s(len(f), form, _dp(f), _dp(fstar))


def h(x: float) -> float:
    return lib().orc_h(x)


def entropy(lattice: int, f: np.ndarray) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().orc_entropy(lattice, _dp(f))


def elbm_alpha(f, fstar):
    """alpha of the ELBM step and whether the positivity rule replaced the root"""
    f = np.ascontiguousarray(f, dtype=np.float64)
    fs = np.ascontiguousarray(fstar, dtype=np.float64)
    pr = ctypes.c_int32()
    a = lib().orc_elbm_alpha(len(f), _dp(f), _dp(fs), ctypes.byref(pr))
    return a, bool(pr.value)


def median(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().orc_median(_dp(v), len(v))


def make_params(lattice=D2Q9, nx=8, ny=8, beta=0.9, qe=QE_POLY, ds_form=DS_EXACT, limiter=0,
                trim_mode=TRIM_HOMOTHETY, median_mode=MED_FLOOR, bc=BC_PERIODIC, delta_trim=1e-3,
                delta_median=1e-3, rho0=1.0, lid_ux=0.0, entropy=False, ens_c=0.0, ens_k=0.5,
                delta_ens=0.0, collision=0, homothety=0, top_k=0) -> Params:
    if lattice == D1Q3:
        ny = 1
    return Params(lattice, nx, ny, beta, qe, ds_form, limiter, trim_mode, median_mode, bc,
                  delta_trim, delta_median, rho0, lid_ux, 1 if entropy else 0, ens_c, ens_k, delta_ens,
                  collision, homothety, top_k)


def init_equilibrium(p: Params, rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    n = p.nx * p.ny
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(n)
    dim = 1 if p.lattice == D1Q3 else 2
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(dim * n)
    f = np.zeros(q_of(p.lattice) * n)
    rc = lib().orc_init_equilibrium(ctypes.byref(p), _dp(rho), _dp(u), _dp(f))
    if rc:
        raise ValueError(f"orc_init_equilibrium failed ({rc})")
    return f.reshape(q_of(p.lattice), p.ny, p.nx)


def step(p: Params, f: np.ndarray, steps: int = 1, record: bool = False, record_lim: bool = False,
         handle=None):
    """Advance f in place by `steps` steps; returns (stats of the last step,
    mask, dS) with mask/dS of the last step when `record` is set, and also
    the Delta S of the limited states when `record_lim` is set.  `handle`
    selects another build of the same source (the timing build)."""
    assert f.dtype == np.float64 and f.flags.c_contiguous
    n = p.nx * p.ny
    st = Stats()
    mask = np.zeros(n, dtype=np.uint8) if record else None
    ds = np.zeros(n) if record else None
    dsl = np.zeros(n) if record_lim else None
    L = handle if handle is not None else lib()
    for k in range(steps):
        last = k == steps - 1
        mptr = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if (record and last) else None
        dptr = _dp(ds) if (record and last) else None
        lptr = _dp(dsl) if (record_lim and last) else None
        rc = L.orc_step(ctypes.byref(p), _dp(f), ctypes.byref(st), mptr, dptr, lptr)
        if rc:
            raise ValueError(f"orc_step failed ({rc})")
    out = (st, mask.reshape(p.ny, p.nx) if record else None, ds.reshape(p.ny, p.nx) if record else None)
    if record_lim:
        out = out + (dsl.reshape(p.ny, p.nx),)
    return out


def stream(p: Params, o: np.ndarray) -> np.ndarray:
    o = np.ascontiguousarray(o, dtype=np.float64)
    f = np.zeros_like(o)
    rc = lib().orc_stream(ctypes.byref(p), _dp(o), _dp(f))
    if rc:
        raise ValueError("orc_stream failed")
    return f


def moments(lattice: int, f: np.ndarray):
    """rho and u of every node, eq. (macro_dis), summed in index order."""
    v = velocities(lattice)
    rho = np.zeros(f.shape[1:])
    jx = np.zeros(f.shape[1:])
    jy = np.zeros(f.shape[1:])
    for i in range(f.shape[0]):
        rho += f[i]
        jx += v[i, 0] * f[i]
        jy += v[i, 1] * f[i]
    return rho, jx / rho, jy / rho
