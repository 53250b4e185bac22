"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the time loop runs in liblbm.so's HIP kernels; this module only
converts numpy arrays and descriptor fields to the C structs and back.  There
is no CPU fallback: if the library is missing, loading fails with an error.

torch is imported before the library is loaded so that the process has one
HIP runtime (torch's); torch also supplies streams and, optionally, the
device workspace.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

try:  # one HIP runtime per process: let torch load it first when present
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ERANGE = 0, -1, -2, -3, -4, -5
LBM_D1Q3, LBM_D2Q9 = 1, 2
LBM_QE_POLYNOMIAL, LBM_QE_ENTROPIC = 0, 1
LBM_LIM_NONE, LBM_LIM_TRIM, LBM_LIM_MEDIAN = 0, 1, 2
LBM_LIM_ENS_THRESHOLD, LBM_LIM_ENS_SMOOTH, LBM_LIM_ENS_RATIONAL, LBM_LIM_ENS_BUDGET = 4, 8, 16, 32
LBM_LIM_POSITIVITY = 64
LBM_COLL_LBGK, LBM_COLL_ELBM = 0, 1
LBM_TRIM_HOMOTHETY, LBM_TRIM_EHRENFEST = 0, 1
LBM_MED_FLOOR_DELTA, LBM_MED_GATE_DELTA = 0, 1
LBM_DS_EXACT, LBM_DS_QUADRATIC = 0, 1
LBM_BC_PERIODIC, LBM_BC_CAVITY, LBM_BC_TUBE_ENDS, LBM_BC_CAVITY_DIFFUSIVE = 0, 1, 2, 3
LBM_F64, LBM_F32, LBM_F16_SHIFT, LBM_BF16_SHIFT = 0, 1, 2, 3
LBM_MASK_TRIM, LBM_MASK_MEDIAN, LBM_MASK_NONPOS, LBM_MASK_NOTFLUID, LBM_MASK_ENSEMBLE = 1, 2, 4, 8, 16
LBM_MASK_POSITIVITY = 32
LBM_RUN_RECORD, LBM_RUN_ENTROPY, LBM_RUN_NO_GRAPH, LBM_RUN_NO_TUNE, LBM_RUN_ADAPTIVE = 1, 2, 4, 8, 16

STORAGE_BYTES = {LBM_F64: 8, LBM_F32: 4, LBM_F16_SHIFT: 2, LBM_BF16_SHIFT: 2}

_dp = ctypes.POINTER(ctypes.c_double)


class lbm_domain_desc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("lattice", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("beta", ctypes.c_double),
        ("qe", ctypes.c_int32), ("limiter", ctypes.c_int32), ("trim_mode", ctypes.c_int32),
        ("median_mode", ctypes.c_int32), ("ds_form", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("delta_trim", ctypes.c_double), ("delta_median", ctypes.c_double),
        ("rho0", ctypes.c_double), ("lid_ux", ctypes.c_double),
        ("rho_init", _dp), ("u_init", _dp), ("f_init", _dp),
        ("probe_x", ctypes.c_int32), ("probe_y", ctypes.c_int32),
        ("ens_c", ctypes.c_double), ("ens_k", ctypes.c_double), ("delta_ens", ctypes.c_double),
        ("collision", ctypes.c_int32), ("homothety", ctypes.c_int32), ("top_k", ctypes.c_int64),
    ]


class lbm_run_desc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("storage", ctypes.c_int32), ("device", ctypes.c_int32),
        ("stats_every", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
        ("tile_h", ctypes.c_int32), ("flags", ctypes.c_uint32), ("probe_capacity", ctypes.c_int32),
        ("graph_chunk", ctypes.c_int32), ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class lbm_entropy_stats_t(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("step", ctypes.c_int64),
        ("mass", ctypes.c_double), ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
        ("sum_dS_pre", ctypes.c_double), ("sum_dS_post", ctypes.c_double), ("max_dS", ctypes.c_double),
        ("mean_dS", ctypes.c_double), ("lbgk_production", ctypes.c_double),
        ("limiter_production", ctypes.c_double), ("total_entropy", ctypes.c_double),
        ("n_trimmed", ctypes.c_int64), ("n_filtered", ctypes.c_int64), ("n_nonpositive", ctypes.c_int64),
        ("n_nonfinite", ctypes.c_int64), ("n_fluid", ctypes.c_int64),
        ("n_ensemble", ctypes.c_int64), ("ens_threshold", ctypes.c_double),
        ("n_positivity", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "struct_size"}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None

# name -> (restype, argtypes); every symbol declared in include/lbm.h
SIGNATURES = {
    "lbm_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(lbm_domain_desc), ctypes.c_int32,
                                           ctypes.POINTER(lbm_run_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_create": (ctypes.c_int, [ctypes.POINTER(lbm_domain_desc), ctypes.c_int32, ctypes.POINTER(lbm_run_desc),
                                  ctypes.POINTER(ctypes.c_void_p)]),
    "lbm_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "lbm_synchronize": (ctypes.c_int, [ctypes.c_void_p]),
    "lbm_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp, _dp]),
    "lbm_entropy_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(lbm_entropy_stats_t)]),
    "lbm_get_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "lbm_set_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "lbm_limiter_mask": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8), _dp]),
    "lbm_kernel_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "lbm_probe_trace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                       ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "lbm_tile_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "lbm_destroy": (None, [ctypes.c_void_p]),
    "lbm_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lbm_beta_from_nu": (ctypes.c_double, [ctypes.c_double]),
    "lbm_abi_version": (ctypes.c_int, []),
    "lbm_step_static": (ctypes.c_int, [ctypes.POINTER(lbm_domain_desc), ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, _dp]),
}


def lib():
    """Load liblbm.so (built by paper_0704_0043_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_0704_0043_amd/build.py (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != LBM_OK:
        msg = lib().lbm_last_error(ctx)
        raise LbmError(rc, (msg or b"").decode() or lib().lbm_strerror(rc).decode())
    return rc


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


@dataclass
class Domain:
    """Host-side description of one domain (fields of lbm_domain_desc)."""
    lattice: int = LBM_D2Q9
    nx: int = 64
    ny: int = 64
    beta: float = 0.9
    qe: int = LBM_QE_POLYNOMIAL
    limiter: int = LBM_LIM_NONE
    trim_mode: int = LBM_TRIM_HOMOTHETY
    median_mode: int = LBM_MED_FLOOR_DELTA
    ds_form: int = LBM_DS_EXACT
    bc: int = LBM_BC_PERIODIC
    delta_trim: float = 1e-3
    delta_median: float = 1e-3
    rho0: float = 1.0
    lid_ux: float = 0.0
    ens_c: float = 0.0
    ens_k: float = 0.5
    delta_ens: float = 0.0
    collision: int = LBM_COLL_LBGK
    homothety: int = 0
    top_k: int = 0
    rho_init: np.ndarray | None = None
    u_init: np.ndarray | None = None
    f_init: np.ndarray | None = None
    probe: tuple | None = None
    _keep: list = field(default_factory=list, repr=False)

    @property
    def q(self):
        return 9 if self.lattice == LBM_D2Q9 else 3

    @property
    def dim(self):
        return 2 if self.lattice == LBM_D2Q9 else 1

    def to_c(self) -> lbm_domain_desc:
        if self.lattice == LBM_D1Q3:
            self.ny = 1
        n = self.nx * self.ny
        d = lbm_domain_desc()
        d.struct_size = ctypes.sizeof(lbm_domain_desc)
        for k in ("lattice", "nx", "ny", "beta", "qe", "limiter", "trim_mode", "median_mode", "ds_form", "bc",
                  "delta_trim", "delta_median", "rho0", "lid_ux", "ens_c", "ens_k", "delta_ens", "collision",
                  "homothety", "top_k"):
            setattr(d, k, getattr(self, k))
        self._keep = []
        for name, arr, size in (("rho_init", self.rho_init, n), ("u_init", self.u_init, self.dim * n),
                                ("f_init", self.f_init, self.q * n)):
            if arr is not None:
                a = _f64(arr, size)
                self._keep.append(a)
                setattr(d, name, a.ctypes.data_as(_dp))
        px, py = self.probe if self.probe is not None else (-1, -1)
        d.probe_x, d.probe_y = px, py
        return d


@dataclass
class Run:
    """Fields of lbm_run_desc."""
    storage: int = LBM_F32
    device: int = 0
    stats_every: int = 0
    tile_x: int = 0
    tile_y: int = 0
    tile_h: int = 0
    flags: int = 0
    probe_capacity: int = 0
    graph_chunk: int = 0
    stream: int | None = None
    workspace: int | None = None
    workspace_bytes: int = 0

    def to_c(self) -> lbm_run_desc:
        r = lbm_run_desc()
        r.struct_size = ctypes.sizeof(lbm_run_desc)
        for k in ("storage", "device", "stats_every", "tile_x", "tile_y", "tile_h", "flags", "probe_capacity",
                  "graph_chunk", "workspace_bytes"):
            setattr(r, k, getattr(self, k))
        r.stream = self.stream or None
        r.workspace = self.workspace or None
        return r


def _desc_array(domains):
    arr = (lbm_domain_desc * len(domains))()
    for k, d in enumerate(domains):
        arr[k] = d.to_c()
    return arr


def lbm_workspace_bytes(domains, run: Run) -> int:
    arr = _desc_array(domains)
    out = ctypes.c_size_t()
    rc_run = run.to_c()
    _check(lib().lbm_workspace_bytes(arr, len(domains), ctypes.byref(rc_run), ctypes.byref(out)))
    return out.value


class Context:
    """Owns an lbm_ctx handle (lbm_destroy on close)."""

    def __init__(self, handle, domains, run):
        self.handle = handle
        self.domains = list(domains)
        self.run = run

    def close(self):
        if self.handle:
            lib().lbm_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lbm_create(domains, run: Run) -> Context:
    if isinstance(domains, Domain):
        domains = [domains]
    arr = _desc_array(domains)
    rdesc = run.to_c()
    h = ctypes.c_void_p()
    _check(lib().lbm_create(arr, len(domains), ctypes.byref(rdesc), ctypes.byref(h)))
    return Context(h.value, domains, run)


def lbm_step(ctx: Context, n_steps: int) -> None:
    _check(lib().lbm_step(ctx.handle, int(n_steps)), ctx.handle)


def lbm_synchronize(ctx: Context) -> None:
    _check(lib().lbm_synchronize(ctx.handle), ctx.handle)


def lbm_moments(ctx: Context, domain: int = 0):
    d = ctx.domains[domain]
    n = d.nx * d.ny
    rho = np.empty(n)
    u = np.empty(d.dim * n)
    _check(lib().lbm_moments(ctx.handle, domain, rho.ctypes.data_as(_dp), u.ctypes.data_as(_dp)), ctx.handle)
    return rho.reshape(d.ny, d.nx), u.reshape(d.dim, d.ny, d.nx)


def lbm_entropy_stats(ctx: Context, domain: int = 0, allow_unstable: bool = False) -> dict:
    s = lbm_entropy_stats_t()
    s.struct_size = ctypes.sizeof(s)
    rc = lib().lbm_entropy_stats(ctx.handle, domain, ctypes.byref(s))
    if rc == LBM_EUNSTABLE and allow_unstable:
        out = s.as_dict()
        out["unstable"] = True
        return out
    _check(rc, ctx.handle)
    return s.as_dict()


def lbm_get_populations(ctx: Context, domain: int = 0) -> np.ndarray:
    d = ctx.domains[domain]
    f = np.empty(d.q * d.nx * d.ny)
    _check(lib().lbm_get_populations(ctx.handle, domain, f.ctypes.data_as(_dp)), ctx.handle)
    return f.reshape(d.q, d.ny, d.nx)


def lbm_set_populations(ctx: Context, f, domain: int = 0) -> None:
    d = ctx.domains[domain]
    a = _f64(f, d.q * d.nx * d.ny)
    _check(lib().lbm_set_populations(ctx.handle, domain, a.ctypes.data_as(_dp)), ctx.handle)


def lbm_limiter_mask(ctx: Context, domain: int = 0):
    d = ctx.domains[domain]
    n = d.nx * d.ny
    mask = np.empty(n, dtype=np.uint8)
    ds = np.empty(n)
    _check(lib().lbm_limiter_mask(ctx.handle, domain, mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                  ds.ctypes.data_as(_dp)), ctx.handle)
    return mask.reshape(d.ny, d.nx), ds.reshape(d.ny, d.nx)


def lbm_probe_trace(ctx: Context, domain: int = 0, max_samples: int = 1 << 20) -> np.ndarray:
    buf = np.empty(2 * max_samples, dtype=np.float32)
    n = ctypes.c_int64()
    _check(lib().lbm_probe_trace(ctx.handle, domain, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                 max_samples, ctypes.byref(n)), ctx.handle)
    return buf[: 2 * n.value].reshape(-1, 2).copy()


def lbm_tile_config(ctx: Context):
    tx, ty, th = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lbm_tile_config(ctx.handle, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(th)), ctx.handle)
    return tx.value, ty.value, th.value


def lbm_kernel_times(ctx: Context, n_steps: int):
    """Advance n_steps eagerly with events around each kernel; returns the
    average (collision, median) kernel durations in milliseconds."""
    ms = (ctypes.c_double * 2)()
    _check(lib().lbm_kernel_times(ctx.handle, int(n_steps), ms), ctx.handle)
    return ms[0], ms[1]


def lbm_destroy(ctx: Context) -> None:
    ctx.close()


LBM_STATIC_SCRATCH_BYTES = 64 << 20
LBM_STATIC_NSTATS = 14
STATIC_STATS_FIELDS = ("mass", "mom_x", "mom_y", "sum_dS_pre", "sum_dS_post", "max_dS", "limiter_production",
                       "n_trimmed", "n_filtered", "n_nonpositive", "n_nonfinite", "n_fluid", "n_ensemble",
                       "n_positivity")


def lbm_step_static(domain: Domain, storage: int, f0: int, f1: int, n_steps: int, stream: int | None = None,
                    stats: int | None = None) -> None:
    """Allocation-free stepping on caller-owned device buffers (device
    pointers as ints): the state starts in f0 and ends in f0 (even n_steps)
    or f1 (odd); `stats` is a device pointer to LBM_STATIC_NSTATS doubles."""
    d = domain.to_c()
    _check(lib().lbm_step_static(ctypes.byref(d), int(storage), stream or None, ctypes.c_void_p(f0),
                                 ctypes.c_void_p(f1), int(n_steps),
                                 ctypes.cast(ctypes.c_void_p(stats), _dp) if stats else None))


def lbm_beta_from_nu(nu: float) -> float:
    return lib().lbm_beta_from_nu(nu)


def lbm_strerror(code: int) -> str:
    return lib().lbm_strerror(code).decode()


def lbm_last_error(ctx: Context | None = None) -> str:
    return (lib().lbm_last_error(ctx.handle if ctx else None) or b"").decode()


def lbm_abi_version() -> int:
    return lib().lbm_abi_version()
