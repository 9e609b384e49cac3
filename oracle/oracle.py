"""ctypes wrapper of the FP64 C oracle (oracle/spic_oracle.c).

Test infrastructure only.  Arrays are numpy float64; every call copies its
inputs so the caller's arrays are never modified unless the function says so.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspic_oracle.so")

_F6 = ("ex", "ey", "ez", "bx", "by", "bz")


class OGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad", C.c_int32),
                ("Lx", C.c_double), ("Ly", C.c_double), ("Lz", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        gp = C.POINTER(OGrid)
        L.oracle_weights.argtypes = [gp, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int64), dp]
        L.oracle_gather.argtypes = [gp] + [dp] * 6 + [dp] * 3 + [C.c_int64, dp]
        L.oracle_mover.argtypes = [gp, C.c_double, C.c_double, C.c_int, C.c_double] + [dp] * 6 + [dp] * 6 + [C.c_int64]
        L.oracle_mover_tol.argtypes = ([gp, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double] + [dp] * 6 +
                                       [dp] * 6 + [C.c_int64, C.POINTER(C.c_int32)])
        L.oracle_deposit.argtypes = [gp] + [dp] * 7 + [C.c_int64, dp, C.c_int]
        L.oracle_max_threads.argtypes = []
        L.oracle_set_threads.argtypes = [C.c_int]
        for f in ("oracle_weights", "oracle_gather", "oracle_mover", "oracle_mover_tol", "oracle_deposit",
                  "oracle_max_threads", "oracle_set_threads"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _grid(g) -> OGrid:
    return OGrid(int(g.nx), int(g.ny), int(g.nz), 0, float(g.Lx), float(g.Ly), float(g.Lz))


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64)).copy()


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the count in effect."""
    return int(lib().oracle_set_threads(int(n)))


def weights(g, x: float, y: float, z: float):
    """(nodes[8], W[8]) of a point (tensor-product reading of Eq. 3)."""
    node = np.zeros(8, dtype=np.int64)
    w = np.zeros(8, dtype=np.float64)
    rc = lib().oracle_weights(C.byref(_grid(g)), float(x), float(y), float(z),
                              node.ctypes.data_as(C.POINTER(C.c_int64)), _p(w))
    assert rc == 0
    return node, w


def gather(g, fields: Dict[str, np.ndarray], x, y, z) -> np.ndarray:
    """Eq. 4 at points (x, y, z): returns [6, n] = Ex, Ey, Ez, Bx, By, Bz."""
    f = [_f64(fields[k]) for k in _F6]
    x, y, z = _f64(x).ravel(), _f64(y).ravel(), _f64(z).ravel()
    n = x.size
    out = np.zeros((6, n), dtype=np.float64)
    rc = lib().oracle_gather(C.byref(_grid(g)), *[_p(a) for a in f], _p(x), _p(y), _p(z), n, _p(out))
    assert rc == 0
    return out


def mover(g, dt: float, c: float, niter: int, qom: float, fields: Dict[str, np.ndarray],
          sp: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    """One implicit step of one species; returns a new state dict."""
    f = [_f64(fields[k]) for k in _F6]
    st = {k: _f64(sp[k]) for k in ("x", "y", "z", "u", "v", "w")}
    n = st["x"].size
    rc = lib().oracle_mover(C.byref(_grid(g)), float(dt), float(c), int(niter), float(qom),
                            *[_p(a) for a in f], *[_p(st[k]) for k in ("x", "y", "z", "u", "v", "w")], n)
    assert rc == 0
    out = dict(sp)
    out.update(st)
    return out


def mover_tol(g, dt: float, c: float, niter: int, tol: float, qom: float, fields: Dict[str, np.ndarray],
              sp: Dict[str, np.ndarray]):
    """One implicit step with the tolerance-terminated iteration (Sec. II:
    the count may be set by a prescribed error tolerance): each particle
    stops after pass k >= 2 once max_d |vbar^k - vbar^(k-1)| < tol, at most
    niter passes; tol = 0 is the fixed count.  Returns (new state, passes
    per particle)."""
    f = [_f64(fields[k]) for k in _F6]
    st = {k: _f64(sp[k]) for k in ("x", "y", "z", "u", "v", "w")}
    n = st["x"].size
    it = np.zeros(n, dtype=np.int32)
    rc = lib().oracle_mover_tol(C.byref(_grid(g)), float(dt), float(c), int(niter), float(tol), float(qom),
                                *[_p(a) for a in f], *[_p(st[k]) for k in ("x", "y", "z", "u", "v", "w")], n,
                                it.ctypes.data_as(C.POINTER(C.c_int32)))
    assert rc == 0
    out = dict(sp)
    out.update(st)
    return out, it


def deposit(g, sp: Dict[str, np.ndarray], mom: Optional[np.ndarray] = None) -> np.ndarray:
    """The ten moments [10, nodes] of one species (accumulated into mom if given)."""
    a = {k: _f64(sp[k]) for k in ("x", "y", "z", "u", "v", "w", "q")}
    n = a["x"].size
    nn = g.nx * g.ny * g.nz
    acc = 1
    if mom is None:
        mom = np.zeros((10, nn), dtype=np.float64)
        acc = 0
    assert mom.dtype == np.float64 and mom.shape == (10, nn) and mom.flags.c_contiguous
    rc = lib().oracle_deposit(C.byref(_grid(g)), *[_p(a[k]) for k in ("x", "y", "z", "u", "v", "w", "q")],
                              n, _p(mom), acc)
    assert rc == 0
    return mom


def step(g, dt: float, c: float, niter: int, qom: float, fields, sp, tol: float = 0.0):
    """Fused step of one species: (new state, moments of the new state);
    tol > 0 takes the tolerance-terminated iteration with niter as the cap."""
    new = mover(g, dt, c, niter, qom, fields, sp) if tol == 0.0 else mover_tol(g, dt, c, niter, tol, qom, fields,
                                                                                  sp)[0]
    return new, deposit(g, new)


def run(h, fields, species: Sequence[Dict[str, np.ndarray]], nsteps: int,
        qoms: Optional[Sequence[float]] = None):
    """nsteps fused steps of every species with fixed fields.

    Returns (final states, moments of the last step [nsp, 10, nodes]).
    """
    qoms = list(qoms if qoms is not None else h.qoms)
    g = h.grid
    states = [dict(s) for s in species]
    moms = None
    for _ in range(nsteps):
        moms = []
        for s, st in enumerate(states):
            states[s], m = step(g, h.dt, h.c, h.niter, qoms[s], fields, st)
            moms.append(m)
    return states, (np.stack(moms) if moms else None)
