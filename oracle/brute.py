"""Brute-force numpy reference for tiny inputs (a handful of particles).

Test infrastructure only.  It shares no cell-index logic with the C oracle:
  * the weight of node g for particle p is Eq. 3 written out over *every*
    node of the grid, with the minimal-image distance of the periodic box and
    the tensor-product reading W = prod_d max(0, 1 - |x_g,d - x_p,d| / dx_d);
  * the gather (Eq. 4) and the moments (the moment equation of Sec. II) are
    sums over all nodes with those weights;
  * the mean velocity is obtained from the implicit equation of motion it
    solves, vbar = v^n + (q dt/2m) E + (q dt/2mc) vbar x B, by a dense 3x3
    linear solve (numpy.linalg.solve) instead of the closed form of Eq. 2.
"""
from __future__ import annotations

from typing import Dict

import numpy as np


def node_coords(g):
    dx, dy, dz = g.Lx / g.nx, g.Ly / g.ny, g.Lz / g.nz
    i, j, k = np.meshgrid(np.arange(g.nx), np.arange(g.ny), np.arange(g.nz), indexing="ij")
    return (i * dx).ravel(), (j * dy).ravel(), (k * dz).ravel()


def _min_image(d, L):
    return d - L * np.round(d / L)


def weights_all(g, x, y, z) -> np.ndarray:
    """W(x_g - x_p) for every node g (flat node order), Eq. 3."""
    gx, gy, gz = node_coords(g)
    dx, dy, dz = g.Lx / g.nx, g.Ly / g.ny, g.Lz / g.nz
    wx = np.maximum(0.0, 1.0 - np.abs(_min_image(gx - x, g.Lx)) / dx)
    wy = np.maximum(0.0, 1.0 - np.abs(_min_image(gy - y, g.Ly)) / dy)
    wz = np.maximum(0.0, 1.0 - np.abs(_min_image(gz - z, g.Lz)) / dz)
    return wx * wy * wz


def gather(g, fields: Dict[str, np.ndarray], x, y, z) -> np.ndarray:
    W = weights_all(g, x, y, z)
    return np.array([np.sum(fields[k] * W) for k in ("ex", "ey", "ez", "bx", "by", "bz")])


def _cross_matrix(b):
    """M with M @ v == v x b."""
    bx, by, bz = b
    return np.array([[0.0, bz, -by], [-bz, 0.0, bx], [by, -bx, 0.0]])


def move1(g, dt, c, niter, qom, fields, x, v):
    """One implicit step of one particle; x, v are length-3 arrays."""
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    L = np.array([g.Lx, g.Ly, g.Lz])
    xb = x.copy()
    vbar = v.copy()
    for _ in range(niter):
        F = gather(g, fields, *xb)
        E, B = F[:3], F[3:]
        rhs = v + qom * dt / 2.0 * E
        A = np.eye(3) - _cross_matrix(qom * dt / (2.0 * c) * B)
        vbar = np.linalg.solve(A, rhs)
        xb = x + vbar * dt / 2.0
    v_new = 2.0 * vbar - v
    x_new = np.mod(x + vbar * dt, L)
    x_new = np.where(x_new >= L, 0.0, x_new)
    return x_new, v_new


def mover(g, dt, c, niter, qom, fields, sp):
    out = {k: np.array(sp[k], dtype=np.float64, copy=True) for k in ("x", "y", "z", "u", "v", "w")}
    for p in range(out["x"].size):
        xn, vn = move1(g, dt, c, niter, qom, fields,
                       [out["x"][p], out["y"][p], out["z"][p]], [out["u"][p], out["v"][p], out["w"][p]])
        out["x"][p], out["y"][p], out["z"][p] = xn
        out["u"][p], out["v"][p], out["w"][p] = vn
    res = dict(sp)
    res.update(out)
    return res


def deposit(g, sp) -> np.ndarray:
    nn = g.nx * g.ny * g.nz
    mom = np.zeros((10, nn))
    for p in range(np.asarray(sp["x"]).size):
        W = weights_all(g, sp["x"][p], sp["y"][p], sp["z"][p])
        u, v, w, q = sp["u"][p], sp["v"][p], sp["w"][p], sp["q"][p]
        vals = (1.0, u, v, w, u * u, u * v, u * w, v * v, v * w, w * w)
        for k in range(10):
            mom[k] += q * vals[k] * W
    return mom
