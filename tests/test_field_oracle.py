"""Pins of the field-solve oracle (oracle/field.py) against closed forms,
exact discrete identities and an independent Fourier solve -- nothing here
re-derives a value the oracle computes the same way.

F1  a central difference of a discrete Fourier mode is the mode times
    its symbol sin(2 pi m / n) / dx;
F2  div curl = 0 and curl grad = 0 exactly;
F3  curl is symmetric, curl curl positive semidefinite, and
    curl curl = grad div - (vector) div grad;
F4  R(b) inverts v -> v - v x b, R(0) = I;
F5  with B = 0 the susceptibility is (fourpi / 2) theta dt^2 sum qom rho I;
F6  a transverse wave is an eigenvector of the field operator with
    eigenvalue 1 + mu + (c theta dt)^2 s^2;
F7  the cycle's E^theta solves the field equation (residual), and with a
    uniform scalar susceptibility it equals a per-mode 3x3 Fourier solve;
F8  the implicit current: with B = 0 it is J - (dt/2) div P, checked on a
    cosine pressure profile;
F9  divergence cleaning: div E_clean = fourpi rho (range part), the
    correction is curl free, the null modes are in the kernel of div grad;
F10 theta = 1: E^{n+1} = E^theta and B^{n+1} = B^n - c dt curl E^{n+1}.
"""
import numpy as np
import pytest

from oracle import field as F
from paper_2008_04397_amd import workloads as W


def _grid(nx=6, ny=4, nz=5, L=(3.0, 2.0, 2.5)):
    return W.Grid(nx, ny, nz, *L)


def _fields(g, rng, scale=1.0):
    N = g.nx * g.ny * g.nz
    return {k: scale * rng.standard_normal(N) for k in F.FIELD_KEYS}


def _moments(g, rng, nsp=2):
    N = g.nx * g.ny * g.nz
    out = []
    for s in range(nsp):
        m = rng.standard_normal((10, N)) * 0.1
        m[0] = (1.0 if s else -1.0) * (1.0 + 0.2 * rng.random(N))
        out.append(m)
    return out


def _node_ijk(g):
    i, j, k = np.meshgrid(np.arange(g.nx), np.arange(g.ny), np.arange(g.nz), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def test_f1_difference_of_a_fourier_mode():
    g = _grid(8, 6, 5)
    h = F.spacing(g)
    idx = _node_ijk(g)
    n = (g.nx, g.ny, g.nz)
    for axis in range(3):
        D = F.diff_matrix(g, axis)
        for m in range(n[axis]):
            ph = 2 * np.pi * m * idx[axis] / n[axis]
            got = D @ np.cos(ph)
            want = -np.sin(2 * np.pi * m / n[axis]) / h[axis] * np.sin(ph)
            assert np.allclose(got, want, atol=1e-12 / h[axis])


def test_f2_div_curl_and_curl_grad_vanish():
    g = _grid()
    rng = np.random.default_rng(1)
    _, _, _, curl, div, grad, _ = F.operators(g)
    E = rng.standard_normal(3 * g.nx * g.ny * g.nz)
    phi = rng.standard_normal(g.nx * g.ny * g.nz)
    assert np.abs(div @ (curl @ E)).max() < 1e-12 * np.abs(curl @ E).max()
    assert np.abs(curl @ (grad @ phi)).max() < 1e-12 * np.abs(grad @ phi).max()


def test_f3_curl_curl_is_symmetric_semidefinite_and_the_vector_identity():
    g = _grid(4, 4, 3)
    rng = np.random.default_rng(2)
    Dx, Dy, Dz, curl, div, grad, lap = F.operators(g)
    C = curl.toarray()
    assert np.array_equal(C, C.T)
    w = np.linalg.eigvalsh(C @ C)
    assert w.min() > -1e-10 * w.max()
    E = rng.standard_normal(3 * g.nx * g.ny * g.nz)
    N = g.nx * g.ny * g.nz
    vec_lap = np.concatenate([lap @ E[a * N:(a + 1) * N] for a in range(3)])
    assert np.allclose(curl @ (curl @ E), grad @ (div @ E) - vec_lap, atol=1e-11 * np.abs(vec_lap).max())


def test_f4_rotation_inverts_the_implicit_cross_product():
    rng = np.random.default_rng(3)
    b = rng.standard_normal((50, 3))
    v = rng.standard_normal((50, 3))
    R = F.rotation(b)
    lhs = np.einsum("nab,nb->na", R, v - np.cross(v, b))
    assert np.allclose(lhs, v, atol=1e-13)
    assert np.array_equal(F.rotation(np.zeros(3)), np.eye(3))


def test_f5_susceptibility_without_magnetic_field():
    g = _grid()
    rng = np.random.default_rng(4)
    f = _fields(g, rng)
    for k in ("bx", "by", "bz"):
        f[k][:] = 0.0
    mom = _moments(g, rng)
    qoms, dt, c, theta, fourpi = (-64.0, 1.0), 0.25, 1.0, 0.8, 4 * np.pi
    mu = F.susceptibility(g, f, mom, qoms, dt, c, theta, fourpi)
    scal = 0.5 * fourpi * theta * dt * dt * (qoms[0] * mom[0][0] + qoms[1] * mom[1][0])
    assert np.allclose(mu, scal[:, None, None] * np.eye(3), rtol=1e-14, atol=0)


def test_f6_transverse_wave_is_an_eigenvector():
    g = _grid(8, 4, 4)
    dt, c, theta = 0.3, 1.0, 1.0
    N = g.nx * g.ny * g.nz
    mu0 = 0.7
    mu = np.broadcast_to(mu0 * np.eye(3), (N, 3, 3)).copy()
    i, _, _ = _node_ijk(g)
    for m in range(1, g.nx):
        e = np.zeros((3, N))
        e[1] = np.cos(2 * np.pi * m * i / g.nx)  # E_y(x): transverse
        s = np.sin(2 * np.pi * m / g.nx) / F.spacing(g)[0]
        lam = 1.0 + mu0 + (c * theta * dt) ** 2 * s * s
        assert np.allclose(F.apply_field(g, mu, dt, c, theta, e), lam * e, atol=1e-12 * lam)


def _fourier_solve(g, rhs, mu0, a):
    """(1 + mu0) E + a curl curl E = rhs mode by mode: curl -> i s x, so
    curl curl -> |s|^2 I - s s^T with s_d = sin(2 pi k_d / n_d) / dx_d."""
    hx, hy, hz = F.spacing(g)
    R = np.fft.fftn(rhs.reshape(3, g.nx, g.ny, g.nz), axes=(1, 2, 3))
    sx = np.sin(2 * np.pi * np.arange(g.nx) / g.nx) / hx
    sy = np.sin(2 * np.pi * np.arange(g.ny) / g.ny) / hy
    sz = np.sin(2 * np.pi * np.arange(g.nz) / g.nz) / hz
    out = np.zeros_like(R)
    for i in range(g.nx):
        for j in range(g.ny):
            for k in range(g.nz):
                s = np.array([sx[i], sy[j], sz[k]])
                M = (1.0 + mu0) * np.eye(3) + a * (s @ s * np.eye(3) - np.outer(s, s))
                out[:, i, j, k] = np.linalg.solve(M, R[:, i, j, k])
    return np.real(np.fft.ifftn(out, axes=(1, 2, 3))).reshape(3, -1)


def test_f7_field_equation_solution():
    g = _grid(6, 4, 5)
    rng = np.random.default_rng(5)
    f = _fields(g, rng, 0.1)
    mom = _moments(g, rng)
    qoms, dt, c, theta, fourpi = (-25.0, 1.0), 0.25, 1.0, 0.75, 4 * np.pi
    new = F.field_cycle(g, f, mom, qoms, dt, c, theta, fourpi)
    En, _ = F.clean(g, f, mom, fourpi)
    Eth = theta * np.stack([new[k] for k in ("ex", "ey", "ez")]) + (1 - theta) * En
    mu = F.susceptibility(g, f, mom, qoms, dt, c, theta, fourpi)
    rhs = F.rhs_vector(g, f, mom, qoms, dt, c, theta, fourpi, E=En)
    res = F.apply_field(g, mu, dt, c, theta, Eth) - rhs
    assert np.linalg.norm(res) < 1e-12 * np.linalg.norm(rhs)
    # uniform scalar susceptibility: against an independent Fourier solve
    N = g.nx * g.ny * g.nz
    for k in ("bx", "by", "bz"):
        f[k][:] = 0.0
    mom_u = [np.zeros((10, N)), np.zeros((10, N))]
    mom_u[0][0], mom_u[1][0] = -0.9, 0.9
    mu_u = F.susceptibility(g, f, mom_u, qoms, dt, c, theta, fourpi)
    mu0 = mu_u[0, 0, 0]
    assert np.allclose(mu_u, mu0 * np.eye(3))
    b = rng.standard_normal((3, N))
    A = F.field_matrix(g, mu_u, dt, c, theta)
    x_lu = F.spla.spsolve(A.tocsc(), b.ravel()).reshape(3, -1)
    x_ft = _fourier_solve(g, b, mu0, (c * theta * dt) ** 2)
    assert np.allclose(x_lu, x_ft, atol=1e-12 * np.abs(x_ft).max())


def test_f8_implicit_current_without_magnetic_field():
    g = _grid(8, 4, 4)
    rng = np.random.default_rng(6)
    N = g.nx * g.ny * g.nz
    f = _fields(g, rng)
    for k in ("bx", "by", "bz"):
        f[k][:] = 0.0
    i, _, _ = _node_ijk(g)
    m = np.zeros((10, N))
    m[1:4] = rng.standard_normal((3, N))
    m[4] = np.cos(2 * np.pi * i / g.nx)  # P_xx(x)
    dt, c = 0.4, 1.0
    J = F.implicit_current(g, f, [m], [1.0], dt, c)
    h = F.spacing(g)[0]
    dPxx = -np.sin(2 * np.pi / g.nx) / h * np.sin(2 * np.pi * i / g.nx)
    assert np.allclose(J[0], m[1] - 0.5 * dt * dPxx, atol=1e-13)
    assert np.allclose(J[1:], m[2:4], atol=1e-13)


def test_f9_divergence_cleaning():
    rng = np.random.default_rng(7)
    for dims in ((6, 4, 5), (5, 3, 7), (8, 8, 2)):
        g = _grid(*dims)
        _, _, _, curl, div, grad, lap = F.operators(g)
        f = _fields(g, rng)
        mom = _moments(g, rng)
        fourpi = 4 * np.pi
        Ec, phi = F.clean(g, f, mom, fourpi)
        rho = mom[0][0] + mom[1][0]
        target = fourpi * F.project_range(g, rho)
        assert np.allclose(div @ Ec.ravel(), target, atol=1e-11 * np.abs(target).max())
        E = np.stack([f[k] for k in ("ex", "ey", "ez")])
        assert np.abs(curl @ (Ec - E).ravel()).max() < 1e-11 * np.abs(Ec - E).max()
        Q = F.null_modes(g)
        assert np.allclose(Q @ Q.T, np.eye(Q.shape[0]), atol=1e-13)
        assert np.abs(lap @ Q.T).max() < 1e-12
        assert Q.shape[0] == np.prod([2 if n % 2 == 0 else 1 for n in dims])


def test_f10_theta_one_update():
    g = _grid(4, 4, 3)
    rng = np.random.default_rng(8)
    f = _fields(g, rng, 0.1)
    mom = _moments(g, rng)
    qoms, dt, c, fourpi = (-4.0, 1.0), 0.2, 1.5, 4 * np.pi
    new = F.field_cycle(g, f, mom, qoms, dt, c, 1.0, fourpi)
    _, _, _, curl, *_ = F.operators(g)
    E1 = np.stack([new[k] for k in ("ex", "ey", "ez")])
    B0 = np.stack([f[k] for k in ("bx", "by", "bz")])
    B1 = np.stack([new[k] for k in ("bx", "by", "bz")])
    assert np.allclose(B1, B0 - c * dt * (curl @ E1.ravel()).reshape(3, -1), atol=1e-13)


def test_f11_vacuum_cycle():
    """No species: no susceptibility or current; cleaning removes div E."""
    g = _grid(6, 4, 5)
    rng = np.random.default_rng(9)
    f = _fields(g, rng, 0.1)
    new = F.field_cycle(g, f, [], [], 0.25, 1.0, 0.5, 4 * np.pi)
    _, _, _, curl, div, grad, lap = F.operators(g)
    Ec, _ = F.clean(g, f, [], 4 * np.pi)
    assert np.abs(div @ Ec.ravel()).max() < 1e-12 * np.abs(Ec).max() / min(F.spacing(g))
    assert all(np.all(np.isfinite(v)) for v in new.values())


def test_f12_right_hand_side_closed_forms():
    """Vacuum with B_z(x) = cos(2 pi m x / Lx): the right-hand side is
    E + theta dt c curl B with (curl B)_y = -D_x B_z from the symbol; a
    uniform current with B = 0 enters as -theta dt fourpi J."""
    g = _grid(8, 4, 4)
    N = g.nx * g.ny * g.nz
    i, _, _ = _node_ijk(g)
    rng = np.random.default_rng(10)
    f = _fields(g, rng, 0.1)
    for k in ("bx", "by", "bz"):
        f[k][:] = 0.0
    m = 3
    f["bz"][:] = np.cos(2 * np.pi * m * i / g.nx)
    dt, c, theta, fourpi = 0.3, 1.5, 0.7, 4 * np.pi
    E = np.stack([f[k] for k in ("ex", "ey", "ez")])
    rhs = F.rhs_vector(g, f, [], [], dt, c, theta, fourpi)
    s = np.sin(2 * np.pi * m / g.nx) / F.spacing(g)[0]
    want = E.copy()
    want[1] += theta * dt * c * s * np.sin(2 * np.pi * m * i / g.nx)
    assert np.allclose(rhs, want, atol=1e-13)
    f["bz"][:] = 0.0
    mom = np.zeros((10, N))
    mom[1:4] = np.array([0.2, -0.1, 0.05])[:, None]
    rhs = F.rhs_vector(g, f, [mom], [1.0], dt, c, theta, fourpi)
    assert np.allclose(rhs, E - theta * dt * fourpi * mom[1:4], atol=1e-13)


# plausible mistakes planted in the oracle (each must fail a pin above)
def _mut_curl_sign(mp):
    real = F.operators

    def ops(g):
        Dx, Dy, Dz, curl, div, grad, lap = real(g)
        Z = F.sp.csr_matrix(Dx.shape)
        bad = F.sp.bmat([[Z, Dz, Dy], [Dz, Z, -Dx], [-Dy, Dx, Z]]).tocsr()
        return Dx, Dy, Dz, bad, div, grad, lap
    mp.setattr(F, "operators", ops)


def _mut_mu_factor(mp):
    real = F.susceptibility
    mp.setattr(F, "susceptibility", lambda *a: 2.0 * real(*a))


def _mut_rotation_sense(mp):
    real = F.rotation
    mp.setattr(F, "rotation", lambda b: np.swapaxes(real(b), -1, -2))


def _mut_pressure_half(mp):
    real = F.implicit_current

    def jh(g, fields, moments, qoms, dt, c):
        return real(g, fields, moments, qoms, 2.0 * dt, c) - 0.0 * dt
    mp.setattr(F, "implicit_current", jh)


def _mut_clean_sign(mp):
    real = F.clean

    def cl(g, fields, moments, fourpi):
        Ec, phi = real(g, fields, moments, fourpi)
        E = np.stack([np.asarray(fields[k], np.float64) for k in ("ex", "ey", "ez")])
        return 2 * E - Ec, phi
    mp.setattr(F, "clean", cl)


def _mut_rhs_current_sign(mp):
    real = F.rhs_vector

    def rv(g, fields, moments, qoms, dt, c, theta, fourpi, E=None):
        return real(g, fields, moments, qoms, dt, c, theta, -fourpi, E=E)
    mp.setattr(F, "rhs_vector", rv)


PINS = [test_f1_difference_of_a_fourier_mode, test_f2_div_curl_and_curl_grad_vanish,
        test_f3_curl_curl_is_symmetric_semidefinite_and_the_vector_identity,
        test_f4_rotation_inverts_the_implicit_cross_product, test_f5_susceptibility_without_magnetic_field,
        test_f6_transverse_wave_is_an_eigenvector, test_f7_field_equation_solution,
        test_f8_implicit_current_without_magnetic_field, test_f9_divergence_cleaning, test_f10_theta_one_update,
        test_f11_vacuum_cycle, test_f12_right_hand_side_closed_forms]


@pytest.mark.parametrize("mutate", [_mut_curl_sign, _mut_mu_factor, _mut_rotation_sense, _mut_pressure_half,
                                    _mut_clean_sign, _mut_rhs_current_sign])
def test_planted_mistakes_fail_a_pin(mutate, monkeypatch):
    with monkeypatch.context() as mp:
        mutate(mp)
        failed = 0
        for pin in PINS:
            try:
                pin()
            except AssertionError:
                failed += 1
    assert failed >= 1, mutate.__name__
