"""Python binding of libspic.so (include/spic.h), argument marshalling only.

Every function keeps the C name and forwards to the library; all arithmetic
of the mover, the moment gathering and the sort runs in the HIP kernels.
Device memory and streams come from PyTorch (torch tensors on a HIP device,
``torch.cuda.Stream``).  If the library is not built, importing the functions
works but the first call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libspic.so")

SPIC_OK, SPIC_E_ARG, SPIC_E_BUDGET, SPIC_E_HIP, SPIC_E_UNSUPPORTED, SPIC_E_STATE = 0, -1, -2, -3, -4, -5
SPIC_F32, SPIC_F64, SPIC_F32C = 1, 2, 3

EXPORTED = ("spic_ctx_create", "spic_ctx_destroy", "spic_last_error", "spic_status_str", "spic_version",
            "spic_set_option", "spic_get_option", "spic_mover", "spic_moments", "spic_sort",
            "spic_batch_submit", "spic_wait", "spic_poll", "spic_mover_noalloc", "spic_field_apply",
            "spic_field_cycle")


class SpicError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (%d): %s" % (_status_name(status), status, message))
        self.status = status
        self.message = message


class spic_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("reserved", C.c_int32),
                ("Lx", C.c_double), ("Ly", C.c_double), ("Lz", C.c_double)]


class spic_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("c", C.c_double), ("niter_mover", C.c_int32), ("sort_every", C.c_int32),
                ("step", C.c_int64), ("mover_tol", C.c_double)]


class spic_fields(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("reserved", C.c_int32)] + [(k, C.c_void_p) for k in
                                                                   ("ex", "ey", "ez", "bx", "by", "bz")]


class spic_species(C.Structure):
    _fields_ = ([("dtype", C.c_int32), ("host_resident", C.c_int32), ("n", C.c_int64), ("qom", C.c_double)]
                + [(k, C.c_void_p) for k in ("x", "y", "z", "u", "v", "w", "q")] + [("id", C.c_void_p)])


class spic_moment_array(C.Structure):
    _fields_ = [("acc_dtype", C.c_int32), ("reserved", C.c_int32), ("m", C.c_void_p)]


class spic_field_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("c", C.c_double), ("theta", C.c_double), ("fourpi", C.c_double),
                ("tol", C.c_double), ("max_iter", C.c_int32), ("restart", C.c_int32)]


class spic_em_state(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ex", "ey", "ez", "bx", "by", "bz")]


class spic_field_stats(C.Structure):
    _fields_ = [("clean_iters", C.c_int32), ("solve_iters", C.c_int32), ("clean_resid", C.c_double),
                ("solve_resid", C.c_double)]


class spic_run(C.Structure):
    _fields_ = [("grid", spic_grid), ("params", spic_params), ("fields", spic_fields),
                ("species", C.POINTER(spic_species)), ("moments", C.POINTER(spic_moment_array)),
                ("nspecies", C.c_int32), ("nsteps", C.c_int32)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libspic.so is not built (%s); run `python -m paper_2008_04397_amd.build`"
                               % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.spic_ctx_create.argtypes = [C.c_int, C.c_uint64, C.POINTER(vp)]
        L.spic_ctx_destroy.argtypes = [vp]
        L.spic_last_error.argtypes = [vp]
        L.spic_last_error.restype = C.c_char_p
        L.spic_status_str.argtypes = [C.c_int]
        L.spic_status_str.restype = C.c_char_p
        L.spic_version.argtypes = []
        L.spic_set_option.argtypes = [vp, C.c_char_p, C.c_int64]
        L.spic_get_option.argtypes = [vp, C.c_char_p, C.POINTER(C.c_int64)]
        L.spic_mover.argtypes = [vp, C.POINTER(spic_grid), C.POINTER(spic_params), C.POINTER(spic_fields),
                                 C.POINTER(spic_species), C.c_int32, C.POINTER(spic_moment_array), vp]
        L.spic_mover_noalloc.argtypes = L.spic_mover.argtypes
        L.spic_moments.argtypes = [vp, C.POINTER(spic_grid), C.POINTER(spic_species), C.c_int32,
                                   C.POINTER(spic_moment_array), C.c_int32, vp]
        L.spic_sort.argtypes = [vp, C.POINTER(spic_grid), C.POINTER(spic_species), C.c_int32, vp]
        L.spic_batch_submit.argtypes = [vp, C.POINTER(spic_run), C.c_int32, C.POINTER(C.c_uint64)]
        L.spic_wait.argtypes = [vp, C.c_uint64, C.POINTER(C.c_double)]
        L.spic_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32)]
        L.spic_field_apply.argtypes = [vp, C.POINTER(spic_grid), C.POINTER(spic_field_params),
                                       C.POINTER(spic_em_state), C.POINTER(spic_moment_array),
                                       C.POINTER(C.c_double), C.c_int32, vp, vp, vp]
        L.spic_field_cycle.argtypes = [vp, C.POINTER(spic_grid), C.POINTER(spic_field_params),
                                       C.POINTER(spic_em_state), C.POINTER(spic_moment_array),
                                       C.POINTER(C.c_double), C.c_int32, C.POINTER(spic_field_stats), vp]
        for f in EXPORTED:
            if f not in ("spic_last_error", "spic_status_str"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _status_name(st: int) -> str:
    try:
        return lib().spic_status_str(st).decode()
    except Exception:
        return str(st)


# ------------------------------------------------------------------ helpers

def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _dtype_code(t) -> int:
    import torch
    dt = t.dtype
    if dt in (torch.float32, np.float32):
        return SPIC_F32
    if dt in (torch.float64, np.float64):
        return SPIC_F64
    raise ValueError("unsupported dtype %s" % dt)


def make_grid(g) -> spic_grid:
    return spic_grid(int(g.nx), int(g.ny), int(g.nz), 0, float(g.Lx), float(g.Ly), float(g.Lz))


def make_params(dt: float, c: float = 1.0, niter: int = 3, sort_every: int = 0, step: int = 0,
                tol: float = 0.0) -> spic_params:
    """tol > 0: tolerance-terminated mover iterations, niter the cap."""
    return spic_params(float(dt), float(c), int(niter), int(sort_every), int(step), float(tol))


def make_fields(f: Dict[str, "object"]) -> spic_fields:
    code = _dtype_code(f["ex"])
    return spic_fields(code, 0, *[_ptr(f[k]) for k in ("ex", "ey", "ez", "bx", "by", "bz")])


def make_species(sp: Dict[str, "object"], qom: float, host_resident: bool = False) -> spic_species:
    n = int(sp["x"].numel() if hasattr(sp["x"], "numel") else sp["x"].size)
    return spic_species(_dtype_code(sp["x"]), int(bool(host_resident)), n, float(qom),
                        *[_ptr(sp[k]) for k in ("x", "y", "z", "u", "v", "w", "q")], _ptr(sp.get("id")))


def make_moments(m) -> spic_moment_array:
    """A [10][nodes] tensor (FP64 or FP32 accumulation), or a float32
    [2][10][nodes] tensor for compensated FP32 (high and low planes)."""
    if getattr(m, "dim", lambda: 2)() == 3:
        return spic_moment_array(SPIC_F32C, 0, _ptr(m))
    return spic_moment_array(_dtype_code(m), 0, _ptr(m))


def _arr(ctype, items):
    items = list(items)
    return (ctype * max(1, len(items)))(*items)


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ context

class Context:
    """Owns a spic_ctx handle (device, HBM budget for library scratch)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = C.c_void_p()
        st = lib().spic_ctx_create(int(device), int(hbm_budget_bytes), C.byref(h))
        if st != SPIC_OK:
            raise SpicError(st, "spic_ctx_create(device=%d)" % device)
        self.handle = h
        self.device = device

    def check(self, st: int):
        if st != SPIC_OK:
            raise SpicError(st, lib().spic_last_error(self.handle).decode())
        return st

    def close(self):
        if getattr(self, "handle", None):
            lib().spic_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key: str, value: int):
        return self.check(lib().spic_set_option(self.handle, key.encode(), int(value)))

    def get_option(self, key: str) -> int:
        v = C.c_int64()
        self.check(lib().spic_get_option(self.handle, key.encode(), C.byref(v)))
        return v.value


def spic_ctx_create(device: int = 0, hbm_budget_bytes: int = 0) -> Context:
    return Context(device, hbm_budget_bytes)


def spic_ctx_destroy(ctx: Context):
    ctx.close()


def spic_version() -> int:
    return int(lib().spic_version())


def spic_status_str(st: int) -> str:
    return lib().spic_status_str(int(st)).decode()


def spic_mover(ctx: Context, grid, params: spic_params, fields, species: Sequence[dict], qoms: Sequence[float],
               moments: Optional[Sequence] = None, stream=None, raw: bool = False) -> int:
    """One fused step of every species (moments overwritten when given)."""
    g = make_grid(grid)
    f = make_fields(fields)
    sp = _arr(spic_species, [make_species(s, q) for s, q in zip(species, qoms)])
    mom = _arr(spic_moment_array, [make_moments(m) for m in moments]) if moments is not None else None
    st = lib().spic_mover(ctx.handle, C.byref(g), C.byref(params), C.byref(f), sp, len(species), mom,
                          _stream(stream))
    return st if raw else ctx.check(st)


def spic_mover_noalloc(ctx: Context, grid, params: spic_params, fields, species: Sequence[dict],
                       qoms: Sequence[float], moments: Optional[Sequence] = None, stream=None,
                       raw: bool = False) -> int:
    """spic_mover with a sort of every species before its move (sort_every
    must be 1), all scratch in the library's fixed per-GPU array."""
    g = make_grid(grid)
    f = make_fields(fields)
    sp = _arr(spic_species, [make_species(s, q) for s, q in zip(species, qoms)])
    mom = _arr(spic_moment_array, [make_moments(m) for m in moments]) if moments is not None else None
    st = lib().spic_mover_noalloc(ctx.handle, C.byref(g), C.byref(params), C.byref(f), sp, len(species), mom,
                                  _stream(stream))
    return st if raw else ctx.check(st)


def make_field_params(dt: float, c: float = 1.0, theta: float = 1.0, fourpi: float = 4.0 * np.pi,
                      tol: float = 1e-10, max_iter: int = 200, restart: int = 30) -> spic_field_params:
    return spic_field_params(float(dt), float(c), float(theta), float(fourpi), float(tol), int(max_iter),
                             int(restart))


def make_em(fields: dict) -> spic_em_state:
    """spic_em_state of six FP64 device tensors keyed ex..bz."""
    return spic_em_state(*[_ptr(fields[k]) for k in ("ex", "ey", "ez", "bx", "by", "bz")])


def spic_field_apply(ctx: Context, grid, fparams: spic_field_params, fields: dict, moments: Sequence,
                     qoms: Sequence[float], x, y, stream=None, raw: bool = False) -> int:
    """y = the field operator applied to x ([3, nodes] FP64 device tensors)."""
    g = make_grid(grid)
    em = make_em(fields)
    mom = _arr(spic_moment_array, [make_moments(m) for m in moments]) if len(moments) else None
    q = (C.c_double * max(1, len(qoms)))(*[float(v) for v in qoms])
    st = lib().spic_field_apply(ctx.handle, C.byref(g), C.byref(fparams), C.byref(em), mom, q, len(moments),
                                _ptr(x), _ptr(y), _stream(stream))
    return st if raw else ctx.check(st)


def spic_field_cycle(ctx: Context, grid, fparams: spic_field_params, fields: dict, moments: Sequence,
                     qoms: Sequence[float], stream=None, raw: bool = False):
    """One field cycle on six FP64 device tensors (updated in place); returns
    the spic_field_stats (or the status with raw=True)."""
    g = make_grid(grid)
    em = make_em(fields)
    mom = _arr(spic_moment_array, [make_moments(m) for m in moments]) if len(moments) else None
    q = (C.c_double * max(1, len(qoms)))(*[float(v) for v in qoms])
    stats = spic_field_stats()
    st = lib().spic_field_cycle(ctx.handle, C.byref(g), C.byref(fparams), C.byref(em), mom, q, len(moments),
                                C.byref(stats), _stream(stream))
    if raw:
        return st
    ctx.check(st)
    return stats


def spic_moments(ctx: Context, grid, species: Sequence[dict], moments: Sequence, accumulate: bool = False,
                 stream=None, qoms: Optional[Sequence[float]] = None, raw: bool = False) -> int:
    g = make_grid(grid)
    qoms = list(qoms) if qoms is not None else [0.0] * len(species)
    sp = _arr(spic_species, [make_species(s, q) for s, q in zip(species, qoms)])
    mom = _arr(spic_moment_array, [make_moments(m) for m in moments])
    st = lib().spic_moments(ctx.handle, C.byref(g), sp, len(species), mom, int(bool(accumulate)), _stream(stream))
    return st if raw else ctx.check(st)


def spic_sort(ctx: Context, grid, species: Sequence[dict], stream=None, raw: bool = False) -> int:
    g = make_grid(grid)
    sp = _arr(spic_species, [make_species(s, 0.0) for s in species])
    st = lib().spic_sort(ctx.handle, C.byref(g), sp, len(species), _stream(stream))
    return st if raw else ctx.check(st)


def spic_poll(ctx: Context, ticket: int) -> bool:
    done = C.c_int32()
    ctx.check(lib().spic_poll(ctx.handle, int(ticket), C.byref(done)))
    return bool(done.value)


def resolved_launch(ctx: Context, dtype: str) -> Dict[str, int]:
    """The tiled-kernel launch settings the library resolves for particles of
    the given precision ("f32"/"f64") with FP64 moments (read-only option
    keys "f32:<name>" / "f64:<name>"; no resolution logic here)."""
    keys = ("tile_variant", "tile_block", "bank_align", "sort_ordered", "sort_rows", "halo", "mover_cache",
            "mover_halo", "tile_group")
    return {k: ctx.get_option("%s:%s" % (dtype, k)) for k in keys}


# --------------------------------------------------------- tensor helpers

def to_device(arrs: Dict[str, np.ndarray], dtype, device="cuda") -> Dict[str, "object"]:
    """Copy a dict of numpy arrays to device tensors (floats cast to dtype)."""
    import torch
    out = {}
    for k, v in arrs.items():
        t = torch.from_numpy(np.ascontiguousarray(v))
        if t.is_floating_point():
            t = t.to(dtype)
        out[k] = t.to(device)
    return out


def to_host(arrs: Dict[str, "object"]) -> Dict[str, np.ndarray]:
    return {k: v.detach().cpu().numpy() for k, v in arrs.items()}


def moment_buffers(grid, nsp: int, dtype=None, device="cuda", compensated: bool = False):
    """Moment outputs: [10][nodes] of dtype, or with compensated=True the
    float32 [2][10][nodes] high and low planes of SPIC_F32C (moments =
    high + low)."""
    import torch
    nn = grid.nx * grid.ny * grid.nz
    if compensated:
        return [torch.zeros((2, 10, nn), dtype=torch.float32, device=device) for _ in range(nsp)]
    dtype = dtype or torch.float64
    return [torch.zeros((10, nn), dtype=dtype, device=device) for _ in range(nsp)]


# ----------------------------------------------------------- batch engine

class Run:
    """One multi-step run for spic_batch_submit.

    species: list of dicts of tensors (device tensors, or pinned host tensors
    for host-resident species); qoms: charge-to-mass ratio per species;
    moments: list of device tensors [10, nodes] or None.
    """

    def __init__(self, grid, params, fields, species, qoms, moments=None, nsteps=1):
        self.grid, self.params, self.fields = grid, params, fields
        self.species, self.qoms, self.moments, self.nsteps = list(species), list(qoms), moments, int(nsteps)

    def _host(self, s):
        x = s["x"]
        return (not hasattr(x, "is_cuda")) or (not x.is_cuda)

    def to_c(self):
        sps = [make_species(s, q, host_resident=self._host(s)) for s, q in zip(self.species, self.qoms)]
        sp_arr = _arr(spic_species, sps)
        mom_arr = _arr(spic_moment_array, [make_moments(m) for m in self.moments]) if self.moments is not None else None
        r = spic_run()
        r.grid = make_grid(self.grid)
        r.params = self.params
        r.fields = make_fields(self.fields)
        r.species = C.cast(sp_arr, C.POINTER(spic_species))
        r.moments = C.cast(mom_arr, C.POINTER(spic_moment_array)) if mom_arr is not None else None
        r.nspecies = len(self.species)
        r.nsteps = self.nsteps
        return r, (sp_arr, mom_arr)


def spic_batch_submit(ctx: Context, runs: Sequence[Run], raw: bool = False):
    """Submit runs; returns their tickets.  The runs' tensors are kept
    referenced by the context until their ticket has been waited on."""
    cs, keep = [], []
    for r in runs:
        c, k = r.to_c()
        cs.append(c)
        keep.append(k)
    arr = _arr(spic_run, cs)
    tickets = (C.c_uint64 * max(1, len(runs)))()
    st = lib().spic_batch_submit(ctx.handle, arr, len(runs), tickets)
    if raw and st != SPIC_OK:
        return st
    ctx.check(st)
    if not hasattr(ctx, "_inflight"):
        ctx._inflight = {}
    out = []
    for i, r in enumerate(runs):
        ctx._inflight[int(tickets[i])] = r
        out.append(int(tickets[i]))
    return out


def spic_wait(ctx: Context, ticket: int) -> float:
    """Block until the ticket's run is done; returns its device seconds and
    releases the run's tensors."""
    secs = C.c_double()
    st = lib().spic_wait(ctx.handle, int(ticket), C.byref(secs))
    getattr(ctx, "_inflight", {}).pop(int(ticket), None)
    ctx.check(st)
    return secs.value


def pinned_like(arrs: Dict[str, np.ndarray], dtype) -> Dict[str, "object"]:
    """Copy numpy arrays into pinned (page-locked) host tensors."""
    import torch
    out = {}
    for k, v in arrs.items():
        t = torch.from_numpy(np.ascontiguousarray(v))
        if t.is_floating_point():
            t = t.to(dtype)
        out[k] = t.pin_memory()
    return out
