"""FP64 reference of the implicit field solve that closes the cycle (Sec. II,
step 3: a linear system from the implicit-in-time discretisation of
Maxwell's equations, solved with GMRes, and a Poisson equation solved with
CG each cycle so that the continuity equation holds -- "divergence
cleaning"; Sec. VI names the solver's residual as the next GPU port).

Test infrastructure only: this module is plain numpy / scipy.sparse, it
shares no code with the HIP path, and it uses direct solves (a sparse LU
for the field system, FFT for the periodic Poisson equation) where the GPU
path iterates.

The paper does not print the discretisation, so this reading is used (the
library follows it too):

* grid: the periodic node grid of the particle step (n_d distinct nodes per
  axis, spacing L_d / n_d, flat node index (i * ny + j) * nz + k); vector
  fields are [3, nodes] arrays;
* D_d: the central difference (f(+e_d) - f(-e_d)) / (2 dx_d); curl, div
  and grad are built from the D_d, and the Poisson operator is
  div(grad) -- so a gradient correction changes the discrete divergence by
  exactly the Poisson right-hand side;
* susceptibility of species s at a node: mu_s = (fourpi / 2) theta dt^2 qom_s
  rho_s R(b_s), b_s = qom_s dt B / (2 c), where R(b) is the rotation of the
  mover's Eq. 2 -- R(b) v solves vhat = v + vhat x b;
* implicit current: Jhat = sum_s R(b_s) (J_s - (dt / 2) div P_s), with
  (div P)_a = sum_b D_b P_ab;
* field equation for E^theta (the theta-implicit Ampere law with Faraday's
  law substituted):
      (I + mu) E^theta + (c theta dt)^2 curl curl E^theta
          = E^n + theta dt (c curl B^n - fourpi Jhat);
* update: E^{n+1} = (E^theta - (1 - theta) E^n) / theta,
  B^{n+1} = B^n - c dt curl E^theta;
* divergence cleaning, before the solve: E^n <- E^n - grad phi with
  div grad phi = div E^n - fourpi rho_bar, rho_bar = sum_s rho_s without
  its components along the null space of div grad (the modes constant or
  alternating along each axis; alternating only where n_d is even).
"""
from __future__ import annotations

from typing import Dict, Sequence, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

FIELD_KEYS = ("ex", "ey", "ez", "bx", "by", "bz")


def spacing(g) -> Tuple[float, float, float]:
    return g.Lx / g.nx, g.Ly / g.ny, g.Lz / g.nz


def _shift_index(g, axis: int, s: int) -> np.ndarray:
    """Flat index of the node s steps along `axis` from every node (periodic)."""
    i, j, k = np.meshgrid(np.arange(g.nx), np.arange(g.ny), np.arange(g.nz), indexing="ij")
    ijk = [i, j, k]
    n = (g.nx, g.ny, g.nz)
    ijk[axis] = (ijk[axis] + s) % n[axis]
    return ((ijk[0] * g.ny + ijk[1]) * g.nz + ijk[2]).ravel()


def diff_matrix(g, axis: int) -> sp.csr_matrix:
    """D_axis as a sparse [nodes, nodes] matrix."""
    N = g.nx * g.ny * g.nz
    h = spacing(g)[axis]
    rows = np.arange(N)
    plus, minus = _shift_index(g, axis, 1), _shift_index(g, axis, -1)
    data = np.r_[np.full(N, 1.0 / (2 * h)), np.full(N, -1.0 / (2 * h))]
    # a 2-node axis maps +1 and -1 to the same node: the entries add to 0
    return sp.csr_matrix((data, (np.r_[rows, rows], np.r_[plus, minus])), shape=(N, N))


def operators(g):
    """(Dx, Dy, Dz, curl [3N, 3N], div [N, 3N], grad [3N, N], lap [N, N])."""
    Dx, Dy, Dz = (diff_matrix(g, a) for a in range(3))
    Z = sp.csr_matrix(Dx.shape)
    curl = sp.bmat([[Z, -Dz, Dy], [Dz, Z, -Dx], [-Dy, Dx, Z]]).tocsr()
    div = sp.hstack([Dx, Dy, Dz]).tocsr()
    grad = sp.vstack([Dx, Dy, Dz]).tocsr()
    lap = (div @ grad).tocsr()
    return Dx, Dy, Dz, curl, div, grad, lap


def rotation(b: np.ndarray) -> np.ndarray:
    """R(b) for b [..., 3]: the matrix taking v to the solution vhat of
    vhat = v + vhat x b (the rotation of the mover's Eq. 2), [..., 3, 3]."""
    b = np.asarray(b, np.float64)
    bx, by, bz = b[..., 0], b[..., 1], b[..., 2]
    b2 = bx * bx + by * by + bz * bz
    # vhat = (v + v x b + (v . b) b) / (1 + |b|^2); (v x b)_a = sum_c X_ac v_c
    X = np.zeros(b.shape[:-1] + (3, 3))
    X[..., 0, 1], X[..., 0, 2] = bz, -by
    X[..., 1, 0], X[..., 1, 2] = -bz, bx
    X[..., 2, 0], X[..., 2, 1] = by, -bx
    R = np.eye(3) + X + b[..., :, None] * b[..., None, :]
    return R / (1.0 + b2)[..., None, None]


def _bfield(fields) -> np.ndarray:
    return np.stack([np.asarray(fields[k], np.float64) for k in ("bx", "by", "bz")], axis=-1)  # [N, 3]


def susceptibility(g, fields, moments: Sequence[np.ndarray], qoms: Sequence[float], dt: float, c: float,
                   theta: float, fourpi: float) -> np.ndarray:
    """mu at every node, [N, 3, 3]."""
    B = _bfield(fields)
    mu = np.zeros(B.shape[:1] + (3, 3))
    for m, q in zip(moments, qoms):
        R = rotation(q * dt / (2.0 * c) * B)
        mu += (0.5 * fourpi * theta * dt * dt * q * np.asarray(m[0], np.float64))[:, None, None] * R
    return mu


def implicit_current(g, fields, moments, qoms, dt, c) -> np.ndarray:
    """Jhat, [3, N]."""
    Dx, Dy, Dz, *_ = operators(g)
    D = (Dx, Dy, Dz)
    B = _bfield(fields)
    J = np.zeros((3, B.shape[0]))
    pidx = {(0, 0): 4, (0, 1): 5, (0, 2): 6, (1, 1): 7, (1, 2): 8, (2, 2): 9}
    for m, q in zip(moments, qoms):
        m = np.asarray(m, np.float64)
        divP = np.zeros((3, B.shape[0]))
        for a in range(3):
            for b in range(3):
                divP[a] += D[b] @ m[pidx[(min(a, b), max(a, b))]]
        R = rotation(q * dt / (2.0 * c) * B)  # [N, 3, 3]
        src = m[1:4] - 0.5 * dt * divP  # [3, N]
        J += np.einsum("nab,bn->an", R, src)
    return J


def field_matrix(g, mu: np.ndarray, dt: float, c: float, theta: float) -> sp.csr_matrix:
    """(I + mu) + (c theta dt)^2 curl curl, acting on [3N] = (Ex..., Ey..., Ez...)."""
    N = mu.shape[0]
    _, _, _, curl, *_ = operators(g)
    rows, cols, vals = [], [], []
    idx = np.arange(N)
    for a in range(3):
        for b in range(3):
            rows.append(a * N + idx)
            cols.append(b * N + idx)
            vals.append(mu[:, a, b] + (1.0 if a == b else 0.0))
    M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * N, 3 * N))
    return (M + (c * theta * dt) ** 2 * (curl @ curl)).tocsr()


def apply_field(g, mu, dt, c, theta, x: np.ndarray) -> np.ndarray:
    """The field operator on x [3, N] (the residual's matrix-vector product)."""
    A = field_matrix(g, mu, dt, c, theta)
    return (A @ np.asarray(x, np.float64).ravel()).reshape(3, -1)


def null_modes(g) -> np.ndarray:
    """Orthonormal basis of the null space of div grad, [m, N]: products of a
    constant or (even n_d only) alternating pattern along each axis."""
    pats = []
    for n in (g.nx, g.ny, g.nz):
        p = [np.ones(n)]
        if n % 2 == 0:
            p.append((-1.0) ** np.arange(n))
        pats.append(p)
    out = []
    for a in pats[0]:
        for b in pats[1]:
            for cc in pats[2]:
                v = (a[:, None, None] * b[None, :, None] * cc[None, None, :]).ravel()
                out.append(v / np.linalg.norm(v))
    return np.array(out)


def project_range(g, r: np.ndarray) -> np.ndarray:
    """r without its components along the null modes of div grad."""
    Q = null_modes(g)
    return r - Q.T @ (Q @ r)


def poisson_fft(g, r: np.ndarray) -> np.ndarray:
    """phi with div grad phi = r (r in the range), phi orthogonal to the null
    space: div grad is diagonal in the discrete Fourier basis with symbol
    -sum_d (sin(2 pi k_d / n_d) / dx_d)^2."""
    hx, hy, hz = spacing(g)
    R = np.fft.fftn(np.asarray(r, np.float64).reshape(g.nx, g.ny, g.nz))
    kx = np.sin(2 * np.pi * np.arange(g.nx) / g.nx) / hx
    ky = np.sin(2 * np.pi * np.arange(g.ny) / g.ny) / hy
    kz = np.sin(2 * np.pi * np.arange(g.nz) / g.nz) / hz
    sym = -(kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2)
    zero = np.abs(sym) < 1e-12 * np.abs(sym).max() if np.abs(sym).max() > 0 else np.ones_like(sym, bool)
    phi_hat = np.where(zero, 0.0, R / np.where(zero, 1.0, sym))
    return np.real(np.fft.ifftn(phi_hat)).ravel()


def clean(g, fields, moments, fourpi: float) -> Tuple[np.ndarray, np.ndarray]:
    """Divergence cleaning of E: (E_clean [3, N], phi)."""
    _, _, _, _, div, grad, _ = operators(g)
    E = np.stack([np.asarray(fields[k], np.float64) for k in ("ex", "ey", "ez")])
    rho = np.zeros(g.nx * g.ny * g.nz)  # no species: vacuum
    for m in moments:
        rho = rho + np.asarray(m[0], np.float64)
    r = div @ E.ravel() - fourpi * project_range(g, rho)
    phi = poisson_fft(g, project_range(g, r))
    return E - (grad @ phi).reshape(3, -1), phi


def field_cycle(g, fields: Dict[str, np.ndarray], moments: Sequence[np.ndarray], qoms: Sequence[float],
                dt: float, c: float, theta: float, fourpi: float) -> Dict[str, np.ndarray]:
    """One field cycle: clean E^n, solve the field equation for E^theta by a
    sparse LU, update E and B.  Returns the new six field arrays."""
    _, _, _, curl, *_ = operators(g)
    En, _ = clean(g, fields, moments, fourpi)
    Bn = np.stack([np.asarray(fields[k], np.float64) for k in ("bx", "by", "bz")])
    mu = susceptibility(g, fields, moments, qoms, dt, c, theta, fourpi)
    Jh = implicit_current(g, fields, moments, qoms, dt, c)
    rhs = En + theta * dt * (c * (curl @ Bn.ravel()).reshape(3, -1) - fourpi * Jh)
    A = field_matrix(g, mu, dt, c, theta)
    Eth = spla.spsolve(A.tocsc(), rhs.ravel()).reshape(3, -1)
    E1 = (Eth - (1.0 - theta) * En) / theta
    B1 = Bn - c * dt * (curl @ Eth.ravel()).reshape(3, -1)
    return {"ex": E1[0], "ey": E1[1], "ez": E1[2], "bx": B1[0], "by": B1[1], "bz": B1[2]}


def rhs_vector(g, fields, moments, qoms, dt, c, theta, fourpi, E=None) -> np.ndarray:
    """The right-hand side of the field equation, [3, N] (with E^n = E if
    given, else the fields' E)."""
    _, _, _, curl, *_ = operators(g)
    if E is None:
        E = np.stack([np.asarray(fields[k], np.float64) for k in ("ex", "ey", "ez")])
    Bn = np.stack([np.asarray(fields[k], np.float64) for k in ("bx", "by", "bz")])
    Jh = implicit_current(g, fields, moments, qoms, dt, c)
    return E + theta * dt * (c * (curl @ Bn.ravel()).reshape(3, -1) - fourpi * Jh)
