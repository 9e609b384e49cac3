"""Seeded synthetic inputs for the implicit mover and moment gathering.

This module only *draws inputs*: node-centred E/B arrays of a Harris current
sheet and the particle species (SoA positions, velocities, charges, ids) that
both the GPU path and the CPU oracle consume.  It holds none of the method's
arithmetic (no weights, no gather, no rotation, no deposit), so sharing it
between the two sides does not couple them.

Workloads follow the paper's reconnection setup (Sec. IV: a Harris-type
current sheet, four species, ion/electron charge-to-mass ratio 64,
omega_pi*dt = 0.25, three predictor-corrector iterations), with the box
sizes and particle counts of the benchmark configurations below.

Layout conventions (shared by every consumer):
  * node arrays have nx*ny*nz entries, node (i, j, k) at flat index
    (i*ny + j)*nz + k, position (i*dx, j*dy, k*dz); the box is periodic so
    node n_d is node 0;
  * species order: 0 sheet electrons, 1 sheet ions, 2 background electrons,
    3 background ions;
  * particles are generated cell by cell in flat cell order, so a fresh
    species is already sorted by cell.

Random streams are keyed by (seed, purpose, species, x-slab) so any x-slab of
any species can be regenerated alone (used to stream very large runs and to
draw subsamples) and the concatenation over slabs equals the whole species.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Iterator, List, Optional, Sequence, Tuple

import numpy as np

BOX_L = (20.0, 10.0, 2.5)

SHEET_E, SHEET_I, BG_E, BG_I = 0, 1, 2, 3
SPECIES_NAMES = ("sheet_e", "sheet_i", "bg_e", "bg_i")


@dataclasses.dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    Lx: float = BOX_L[0]
    Ly: float = BOX_L[1]
    Lz: float = BOX_L[2]

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def cells(self) -> int:
        return self.nodes

    @property
    def d(self) -> Tuple[float, float, float]:
        return (self.Lx / self.nx, self.Ly / self.ny, self.Lz / self.nz)

    @property
    def L(self) -> Tuple[float, float, float]:
        return (self.Lx, self.Ly, self.Lz)


@dataclasses.dataclass(frozen=True)
class Harris:
    """Physical parameters of one Harris-sheet box."""
    grid: Grid
    ppc: int
    dt: float = 0.25
    niter: int = 3
    c: float = 1.0
    B0: float = 0.0195
    delta: float = 0.5
    pert: float = 0.01          # perturbation amplitude relative to B0
    qom_e: float = -64.0
    qom_i: float = 1.0
    vth_e: float = 0.045
    vth_i: float = 0.0126
    n_bg: float = 0.1
    drift_z: float = 0.0        # sheet drift along z (0 unless a test asks)
    seed: int = 2008_04397

    @property
    def qoms(self) -> Tuple[float, float, float, float]:
        return (self.qom_e, self.qom_i, self.qom_e, self.qom_i)

    @property
    def vths(self) -> Tuple[float, float, float, float]:
        return (self.vth_e, self.vth_i, self.vth_e, self.vth_i)

    @property
    def n_per_species(self) -> int:
        return self.grid.cells * self.ppc

    @property
    def n_total(self) -> int:
        return 4 * self.n_per_species


# ---------------------------------------------------------------------------
# The benchmark workloads (all boxes use L = (20, 10, 2.5)).
# ---------------------------------------------------------------------------

def harris_32x16x4() -> Harris:
    """32x16x4 cells, 27 ppc x 4 species (221,184 particles), 10 steps, FP64."""
    return Harris(Grid(32, 16, 4), ppc=27)


def harris_128x64x32() -> Harris:
    """128x64x32 cells, 64 ppc x 4 species (67,108,864 particles), 20 steps."""
    return Harris(Grid(128, 64, 32), ppc=64)


def harris_512x256x32() -> Harris:
    """512x256x32 cells, 125 ppc x 4 species (~2.1e9 particles), 5 steps."""
    return Harris(Grid(512, 256, 32), ppc=125)


STEPS = {"harris_32x16x4": 10, "harris_128x64x32": 20, "harris_512x256x32": 5}


# ---------------------------------------------------------------------------
# Random streams
# ---------------------------------------------------------------------------

_P_FIELDS, _P_VEL, _P_POS = 1000, 2000, 3000


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng([int(k) & 0xFFFFFFFF for k in key])


# ---------------------------------------------------------------------------
# Fields
# ---------------------------------------------------------------------------

def make_fields(h: Harris, dtype=np.float64) -> Dict[str, np.ndarray]:
    """Node E, B of a Harris sheet plus a seeded uniform perturbation.

    B_x(y) = B0 tanh((y - Ly/2)/delta), B_y = B_z = 0, E = 0, and every one of
    the six components gets pert*B0*U(-1, 1) per node so the E path and all B
    components are exercised.  Generated in FP64, then cast.
    """
    g = h.grid
    dx, dy, dz = g.d
    y = np.arange(g.ny, dtype=np.float64) * dy
    bx_y = h.B0 * np.tanh((y - 0.5 * g.Ly) / h.delta)
    out = {}
    rng = _rng(h.seed, _P_FIELDS)
    shape = (g.nx, g.ny, g.nz)
    for name in ("ex", "ey", "ez", "bx", "by", "bz"):
        base = np.zeros(shape, dtype=np.float64)
        if name == "bx":
            base += bx_y[None, :, None]
        noise = rng.uniform(-1.0, 1.0, size=shape) * (h.pert * h.B0)
        out[name] = np.ascontiguousarray((base + noise).reshape(-1).astype(dtype))
    return out


def uniform_fields(g: Grid, E=(0.0, 0.0, 0.0), B=(0.0, 0.0, 0.0), dtype=np.float64):
    n = g.nodes
    vals = dict(zip(("ex", "ey", "ez", "bx", "by", "bz"), tuple(E) + tuple(B)))
    return {k: np.full(n, v, dtype=dtype) for k, v in vals.items()}


# ---------------------------------------------------------------------------
# Particles
# ---------------------------------------------------------------------------

def _lattice_side(ppc: int) -> int:
    m = int(round(ppc ** (1.0 / 3.0)))
    return m if m ** 3 == ppc else 0


def _density(h: Harris, s: int, y: np.ndarray) -> np.ndarray:
    if s in (SHEET_E, SHEET_I):
        return 1.0 / np.cosh((y - 0.5 * h.grid.Ly) / h.delta) ** 2
    return np.full_like(y, h.n_bg)


def species_slab(h: Harris, s: int, i0: int, i1: int, dtype=np.float64,
                 with_id: bool = True) -> Dict[str, np.ndarray]:
    """Particles of species ``s`` living in x-slabs [i0, i1), cell-major order.

    Positions sit on a cube-root lattice (a + 1/2)/m inside each cell when ppc
    is a perfect cube, else they are seeded-uniform inside the cell.  Density
    is carried by the charge q = sign(qom) * n(y) * dx*dy*dz / ppc.  Velocities
    are Maxwellian with sigma = vth of the species (+ drift_z for the sheet).
    """
    g = h.grid
    dx, dy, dz = g.d
    ppc = h.ppc
    m = _lattice_side(ppc)
    ny, nz = g.ny, g.nz
    per_slab = ny * nz * ppc
    cols = []
    for i in range(i0, i1):
        jj, kk = np.meshgrid(np.arange(ny), np.arange(nz), indexing="ij")
        if m:
            a = (np.arange(m) + 0.5) / m
            fa, fb, fc = np.meshgrid(a, a, a, indexing="ij")
            fx = np.broadcast_to(fa.reshape(1, 1, -1), (ny, nz, ppc))
            fy = np.broadcast_to(fb.reshape(1, 1, -1), (ny, nz, ppc))
            fz = np.broadcast_to(fc.reshape(1, 1, -1), (ny, nz, ppc))
        else:
            rp = _rng(h.seed, _P_POS, s, i)
            fx = rp.random((ny, nz, ppc))
            fy = rp.random((ny, nz, ppc))
            fz = rp.random((ny, nz, ppc))
        x = ((i + fx) * dx).reshape(-1)
        y = ((jj[:, :, None] + fy) * dy).reshape(-1)
        z = ((kk[:, :, None] + fz) * dz).reshape(-1)
        rv = _rng(h.seed, _P_VEL, s, i)
        vth = h.vths[s]
        u = rv.normal(0.0, vth, per_slab)
        v = rv.normal(0.0, vth, per_slab)
        w = rv.normal(0.0, vth, per_slab)
        if s in (SHEET_E, SHEET_I) and h.drift_z != 0.0:
            w = w + (h.drift_z if s == SHEET_I else -h.drift_z)
        qom = h.qoms[s]
        q = math.copysign(1.0, qom) * _density(h, s, y) * (dx * dy * dz / ppc)
        cols.append((x, y, z, u, v, w, q))
    names = ("x", "y", "z", "u", "v", "w", "q")
    out = {k: np.ascontiguousarray(np.concatenate([c[n] for c in cols]).astype(dtype))
           for n, k in enumerate(names)}
    if with_id:
        out["id"] = np.arange(i0 * per_slab, i1 * per_slab, dtype=np.int64)
    return out


def make_species(h: Harris, s: int, dtype=np.float64, with_id: bool = True):
    return species_slab(h, s, 0, h.grid.nx, dtype=dtype, with_id=with_id)


def make_all_species(h: Harris, dtype=np.float64, with_id: bool = True) -> List[Dict[str, np.ndarray]]:
    return [make_species(h, s, dtype, with_id) for s in range(4)]


def round_state(sp: Dict[str, np.ndarray], dtype) -> Dict[str, np.ndarray]:
    """Round a species to ``dtype`` (the id array is kept as is)."""
    return {k: (v if k == "id" else np.ascontiguousarray(v.astype(dtype))) for k, v in sp.items()}


def upcast(sp: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    return {k: (v if k == "id" else np.ascontiguousarray(v.astype(np.float64))) for k, v in sp.items()}


# ---------------------------------------------------------------------------
# Subsamples and small generic inputs
# ---------------------------------------------------------------------------

def _mix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (a published integer hash), vectorised."""
    x = x.astype(np.uint64)
    with np.errstate(over="ignore"):
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        x = x ^ (x >> np.uint64(31))
    return x


def subsample_mask(ids: np.ndarray, k: int = 64, seed: int = 7) -> np.ndarray:
    """Seeded 1/k subsample by a hash of the particle id.

    A plain stride would select the same lattice site in every cell; hashing
    the id spreads the sample over sites, cells and velocities.
    """
    with np.errstate(over="ignore"):
        h = _mix64(ids.astype(np.uint64) + np.uint64(seed) * np.uint64(0x9E3779B97F4A7C15))
    return (h % np.uint64(k)) == 0


def random_particles(g: Grid, n: int, vth: float, seed: int, q_scale: float = 1.0,
                     dtype=np.float64) -> Dict[str, np.ndarray]:
    """n particles uniform in the box, Maxwellian velocities, random charges."""
    r = _rng(seed, 77)
    out = {
        "x": r.uniform(0.0, g.Lx, n), "y": r.uniform(0.0, g.Ly, n), "z": r.uniform(0.0, g.Lz, n),
        "u": r.normal(0.0, vth, n), "v": r.normal(0.0, vth, n), "w": r.normal(0.0, vth, n),
        "q": r.uniform(0.5, 1.5, n) * q_scale,
    }
    out = {k: np.ascontiguousarray(v.astype(dtype)) for k, v in out.items()}
    out["id"] = np.arange(n, dtype=np.int64)
    return out


# ---------------------------------------------------------------------------
# Batched ensemble and serving request streams
# ---------------------------------------------------------------------------

def ensemble_boxes(n_boxes: int = 64, seed: int = 4, scale: float = 1.0) -> List[Harris]:
    """Independent periodic Harris boxes of uneven size.

    Per box: nx in {16, 32, 64, 128}, ny = nx/2, nz in {4, 8}, ppc in
    {8, 27, 64}, B0 ~ U[0.01, 0.03], mass ratio in {25, 64, 100} (qom_e =
    -mass ratio, qom_i = 1).  ``scale`` < 1 shrinks nx (tests).
    """
    r = _rng(seed, 4000)
    boxes = []
    for b in range(n_boxes):
        nx = int(r.choice([16, 32, 64, 128]))
        nz = int(r.choice([4, 8]))
        ppc = int(r.choice([8, 27, 64]))
        B0 = float(r.uniform(0.01, 0.03))
        mr = float(r.choice([25, 64, 100]))
        if scale != 1.0:
            nx = max(4, int(nx * scale))
        g = Grid(nx, max(2, nx // 2), nz)
        boxes.append(Harris(g, ppc=ppc, B0=B0, qom_e=-mr, seed=seed * 1000 + b))
    return boxes


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival: float       # seconds after stream start
    box: Harris
    steps: int


def serving_stream(n_req: int = 1000, rate: float = 20.0, seed: int = 5,
                   max_nx: int = 256, min_nx: int = 16,
                   steps_range: Tuple[int, int] = (10, 200)) -> List[Request]:
    """Poisson arrivals (mean ``rate``/s) of Harris-box runs of mixed size.

    nx in powers of two from min_nx to max_nx, ny = nx/2, nz in {4, 8},
    ppc uniform integer in 8..64, steps uniform in steps_range.
    """
    r = _rng(seed, 5000)
    t = 0.0
    reqs = []
    sizes = [n for n in (16, 32, 64, 128, 256) if min_nx <= n <= max_nx]
    for k in range(n_req):
        t += float(r.exponential(1.0 / rate))
        nx = int(r.choice(sizes))
        nz = int(r.choice([4, 8]))
        ppc = int(r.integers(8, 65))
        steps = int(r.integers(steps_range[0], steps_range[1] + 1))
        g = Grid(nx, max(2, nx // 2), nz)
        reqs.append(Request(k, t, Harris(g, ppc=ppc, seed=seed * 100000 + k), steps))
    return reqs


# ---------------------------------------------------------------------------
# Device-side generator for workloads that are never compared with the
# oracle (serving streams, the 2.1e9-particle streamed box): the same recipe
# as species_slab (lattice positions, Maxwellian velocities, density in q),
# drawn with torch's seeded generator on the GPU, so inputs of millions of
# particles are produced in milliseconds.  Values differ from species_slab's.
# ---------------------------------------------------------------------------

def species_tensors(h: Harris, s: int, i0: int = 0, i1: Optional[int] = None, device="cuda", dtype=None,
                    seed_offset: int = 0, with_id: bool = False):
    import torch
    dtype = dtype or torch.float32
    g = h.grid
    i1 = g.nx if i1 is None else i1
    dx, dy, dz = g.d
    ppc = h.ppc
    m = _lattice_side(ppc)
    gen = torch.Generator(device=device)
    gen.manual_seed((h.seed * 1_000_003 + s * 10_007 + i0 * 101 + seed_offset) & 0x7FFFFFFFFFFFFFFF)
    nxs = i1 - i0
    ncell = nxs * g.ny * g.nz
    n = ncell * ppc
    cell = torch.arange(ncell, device=device, dtype=torch.int64).repeat_interleave(ppc)
    k = cell % g.nz
    j = (cell // g.nz) % g.ny
    i = cell // (g.nz * g.ny) + i0
    if m:
        a = torch.arange(ppc, device=device, dtype=torch.int64).repeat(ncell)
        fa = ((a // (m * m)) + 0.5) / m
        fb = (((a // m) % m) + 0.5) / m
        fc = ((a % m) + 0.5) / m
    else:
        fa = torch.rand(n, generator=gen, device=device, dtype=torch.float64)
        fb = torch.rand(n, generator=gen, device=device, dtype=torch.float64)
        fc = torch.rand(n, generator=gen, device=device, dtype=torch.float64)
    x = (i.double() + fa) * dx
    y = (j.double() + fb) * dy
    z = (k.double() + fc) * dz
    vth = h.vths[s]
    u = torch.randn(n, generator=gen, device=device, dtype=torch.float32) * vth
    v = torch.randn(n, generator=gen, device=device, dtype=torch.float32) * vth
    w = torch.randn(n, generator=gen, device=device, dtype=torch.float32) * vth
    if s in (SHEET_E, SHEET_I) and h.drift_z != 0.0:
        w = w + (h.drift_z if s == SHEET_I else -h.drift_z)
    if s in (SHEET_E, SHEET_I):
        dens = 1.0 / torch.cosh((y - 0.5 * g.Ly) / h.delta) ** 2
    else:
        dens = torch.full_like(y, h.n_bg)
    q = math.copysign(1.0, h.qoms[s]) * dens * (dx * dy * dz / ppc)
    out = {"x": x.to(dtype), "y": y.to(dtype), "z": z.to(dtype), "u": u.to(dtype), "v": v.to(dtype),
           "w": w.to(dtype), "q": q.to(dtype)}
    if with_id:  # the particle's index in the whole box (cell-major, then lattice site)
        out["id"] = (i0 * g.ny * g.nz) * ppc + torch.arange(n, device=device, dtype=torch.int64)
    return out


def fields_tensors(h: Harris, device="cuda", dtype=None):
    """make_fields (numpy, seeded) moved to the device: fields are small."""
    import torch
    dtype = dtype or torch.float32
    return {k: torch.from_numpy(v).to(device=device, dtype=dtype) for k, v in make_fields(h).items()}
