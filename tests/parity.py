"""Comparison helpers shared by the GPU parity tests.

Tolerances (stated once, used everywhere):
  FP64 path vs the FP64 oracle, per step and at the end:
    positions  max |dx_d| (minimal image)      <= 1e-12 * L_d
    velocities max |dv|                        <= 1e-12 * max_p |v|
    moments    rel-L2 per (species, component) <= 1e-12
  FP32 particles, one step from the identical (FP32-rounded) state:
    positions  <= 1e-5 * L_d   (an FP32 wrap alone costs ~ulp(L_d))
    velocities <= 1e-5 * max(max_p |v|, vth)
  FP32 particles with FP64 accumulation, moments vs the oracle's FP64
  deposit of the same FP32 particle state: rel-L2 <= 1e-6.
"""
from __future__ import annotations

import numpy as np

POS64, VEL64, MOM64 = 1e-12, 1e-12, 1e-12
POS32, VEL32, MOM32 = 1e-5, 1e-5, 1e-6


def by_id(st):
    if "id" not in st:
        return st
    order = np.argsort(st["id"], kind="stable")
    return {k: np.asarray(v)[order] for k, v in st.items()}


def pos_err(a, b, L):
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    d = d - L * np.round(d / L)
    return float(np.abs(d).max()) if d.size else 0.0


def vmax(st):
    if np.asarray(st["u"]).size == 0:
        return 0.0
    return float(np.sqrt(np.asarray(st["u"], np.float64) ** 2 + np.asarray(st["v"], np.float64) ** 2
                         + np.asarray(st["w"], np.float64) ** 2).max())


def state_errors(gpu, ora, grid):
    """(max position error / L per axis, max velocity error) after id alignment."""
    gpu, ora = by_id(gpu), by_id(ora)
    if "id" in gpu and "id" in ora:
        assert np.array_equal(gpu["id"], ora["id"]), "particle ids differ"
    pe = max(pos_err(gpu[k], ora[k], L) / L for k, L in zip(("x", "y", "z"), grid.L))
    ve = max(float(np.abs(np.asarray(gpu[k], np.float64) - ora[k]).max()) if ora[k].size else 0.0
             for k in ("u", "v", "w"))
    return pe, ve


def assert_state(gpu, ora, grid, pos_tol, vel_tol, vscale=None):
    pe, ve = state_errors(gpu, ora, grid)
    vs = vscale if vscale is not None else max(vmax(ora), 1e-300)
    assert pe <= pos_tol, "position error %.3e > %.1e (relative to L)" % (pe, pos_tol)
    assert ve <= vel_tol * vs, "velocity error %.3e > %.1e * %.3e" % (ve, vel_tol, vs)
    return pe, ve / vs


def rel_l2(a, b):
    """Per-component rel-L2 of a vs reference b, both [10, nodes]."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    out = []
    for k in range(b.shape[0]):
        nb = np.linalg.norm(b[k])
        na = np.linalg.norm(a[k] - b[k])
        out.append(na / nb if nb > 0 else (0.0 if na == 0 else np.inf))
    return np.array(out)


def assert_moments(a, b, tol):
    r = rel_l2(a, b)
    assert np.all(r <= tol), "moment rel-L2 %s > %.1e" % (np.array2string(r, precision=2), tol)
    return float(r.max())
