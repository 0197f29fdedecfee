"""Pins for the oracle's validation pieces (CPU only): the elastic sphere's edge springs (Sec. 6.2.3),
target points (Sec. 6.2.2), the pressure (eq. pressure_poisson_k), the channel-flow series (Sec.
6.2.2) and the circle's pressure jump (Sec. 6.1), each against an independent fact of the paper or
of the mathematics."""

import numpy as np
import pytest

import workloads as wl
from oracle import fluid, forces, validation
from oracle.modes import spectral_shape, wavevector


def _mesh():
    X0, tris = wl.icosphere(2, 0.3, (0.5, 0.5, 0.5))
    return X0, tris


def test_spring_energy_equals_the_triangle_energy_and_the_area_at_rest():
    X0, tris = _mesh()
    sigma = 1.7
    edges, K = forces.spring_stiffness(X0, tris, sigma)
    # the paper: at the reference state the elastic energy equals the surface energy with gamma = sigma
    assert forces.spring_energy(X0, edges, K) == pytest.approx(sigma * forces.surface_area(X0, tris), rel=1e-12)
    Y = X0 + 0.02 * np.random.default_rng(1).standard_normal(X0.shape)
    assert forces.spring_energy(Y, edges, K) == pytest.approx(forces.elastic_energy(Y, X0, tris, sigma), rel=1e-12)


def test_spring_stiffness_is_half_the_cotangent_sum():
    X0, tris = wl.latlong_sphere(5, 7, radius=0.3)  # irregular triangles
    edges, K = forces.spring_stiffness(X0, tris, 2.0)
    cot = {}
    for t in tris:
        for r in range(3):
            A, B, C = int(t[r]), int(t[(r + 1) % 3]), int(t[(r + 2) % 3])
            u, v = X0[A] - X0[C], X0[B] - X0[C]
            ang = np.arccos(np.dot(u, v) / np.linalg.norm(u) / np.linalg.norm(v))
            key = (min(A, B), max(A, B))
            cot[key] = cot.get(key, 0.0) + 1.0 / np.tan(ang)
    ref = np.array([0.5 * 2.0 * cot[(int(i), int(j))] for i, j in edges])
    assert np.allclose(K, ref, rtol=1e-10, atol=1e-12)


def test_spring_force_is_minus_the_energy_gradient():
    X0, tris = _mesh()
    edges, K = forces.spring_stiffness(X0, tris, 1.0)
    rng = np.random.default_rng(2)
    Y = X0 + 0.03 * rng.standard_normal(X0.shape)
    F = forces.spring_force(Y, edges, K)
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * np.abs(F).max()
    h = 1e-6
    for j, a in [(0, 0), (7, 1), (100, 2), (161, 0)]:
        Yp, Ym = Y.copy(), Y.copy()
        Yp[j, a] += h
        Ym[j, a] -= h
        g = (forces.spring_energy(Yp, edges, K) - forces.spring_energy(Ym, edges, K)) / (2 * h)
        assert abs(-g - F[j, a]) < 1e-7 * np.abs(F).max()


def test_target_force_is_minus_the_spring_energy_gradient():
    rng = np.random.default_rng(3)
    X, T = rng.standard_normal((9, 2)), rng.standard_normal((9, 2))
    F = forces.target_force(X, T, 40.0)
    h = 1e-6
    for j, a in [(0, 0), (4, 1), (8, 0)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[j, a] += h
        Xm[j, a] -= h
        E = lambda Z: 20.0 * np.sum((T - Z) ** 2)
        assert abs(-(E(Xp) - E(Xm)) / (2 * h) - F[j, a]) < 1e-6


@pytest.mark.parametrize("Ns", [(8, 6), (6, 5, 4)])
def test_pressure_makes_the_momentum_balance_divergence_free(Ns):
    """f - rho s - grad p is divergence free mode by mode (that is what defines p); with u = 0 the
    pressure is the Stokes pressure of the same force."""
    rng = np.random.default_rng(4)
    d = len(Ns)
    shp = (d,) + spectral_shape(Ns)
    f = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    u = fluid.project(rng.standard_normal(shp) + 1j * rng.standard_normal(shp), Ns, 1.3)
    p = fluid.pressure(f, u, Ns, 1.3, 0.8)
    k = wavevector(Ns, 1.3)
    g = f - 0.8 * fluid.nonlinear(u, Ns, 1.3) - np.stack([1j * k[a] * p for a in range(d)])
    div = sum(k[a] * g[a] for a in range(d))
    nz = sum(k[a] ** 2 for a in range(d)) > 0
    assert np.abs(div[nz]).max() < 1e-12 * np.abs(f).max()
    assert np.allclose(fluid.pressure(f, None, Ns, 1.3, 0.8), fluid.stokes_pressure(f, Ns, 1.3), atol=1e-14)


def test_channel_series_tends_to_the_steady_profile_and_flux():
    D, f0, mu, rho = 0.5, 100.0, 0.1, 1.0
    y = np.linspace(0.0, D, 41)
    u = validation.poiseuille_velocity(y, 1e3, D, f0, mu, rho, terms=4000)
    assert np.allclose(u, f0 / (2 * mu) * y * (D - y), atol=1e-6 * f0 * D * D / mu)
    assert validation.poiseuille_flux(1e3, D, f0, mu, rho) == pytest.approx(
        validation.poiseuille_steady_flux(D, f0, mu), rel=1e-9)
    assert validation.effective_width(validation.poiseuille_steady_flux(D, f0, mu), f0, mu) == pytest.approx(D)


def test_channel_series_solves_the_heat_equation_and_integrates_to_the_flux():
    D, f0, mu, rho = 0.5, 100.0, 0.1, 1.0
    t, h, dt = 0.05, 1e-3, 1e-5
    y = np.linspace(0.1, 0.4, 7)
    U = lambda yy, tt: validation.poiseuille_velocity(yy, tt, D, f0, mu, rho, terms=4000)
    ut = (U(y, t + dt) - U(y, t - dt)) / (2 * dt)
    uyy = (U(y + h, t) - 2 * U(y, t) + U(y - h, t)) / (h * h)
    assert np.allclose(ut, mu / rho * uyy + f0 / rho, rtol=0, atol=2e-3 * f0 / rho)
    yq = (np.arange(4000) + 0.5) * D / 4000  # midpoint rule
    flux = np.sum(U(yq, t)) * D / 4000
    assert flux == pytest.approx(validation.poiseuille_flux(t, D, f0, mu, rho), rel=1e-6)


def test_circle_pressure_has_zero_mean_and_the_laplace_jump():
    F, r, L = 1.0, 0.125, 1.0
    p1, p2 = validation.circle_pressure_jump(F, r, L)
    assert p1 * (L * L - np.pi * r * r) + p2 * np.pi * r * r == pytest.approx(0.0, abs=1e-15)
    assert p1 - p2 == pytest.approx(F / r)


def test_steady_wall_system_satisfies_no_slip_and_force_balance():
    # a symmetric matrix with a null direction, as the wall's Stokes matrix has: the solve must still
    # meet every equation it states
    rng = np.random.default_rng(7)
    Nb = 6
    B = rng.standard_normal((2 * Nb, 2 * Nb - 1))
    A = B @ B.T
    S, ubar = validation.steady_wall_system(A, Nb, 3.0, 1.0)
    assert np.abs(A @ S.ravel() + np.tile(ubar, Nb)).max() < 1e-11
    assert S.sum(axis=0) == pytest.approx([-3.0, 0.0], abs=1e-12)


def test_steady_channel_converges_first_order_and_three_halves_against_the_effective_width():
    """Sec. 6.2.2, steady channel with D = L: the relative velocity error is first order against the
    channel width D and faster (3/2 order reported) against the effective width D_e; the effective
    boundary width tends to about 0.4 h."""
    f0, mu, L = 100.0, 0.1, 1.0
    res = []
    for N in (8, 16, 32):
        S, ubar, uhat, ux = validation.steady_channel(N, f0, mu, L)
        assert S.sum(axis=0) == pytest.approx([-f0, 0.0], abs=1e-9 * f0)
        # the grid mean of a trigonometric polynomial is its k = 0 mode: the mean flow
        assert ux.mean() == pytest.approx(ubar[0], rel=1e-12)
        # mirror symmetry about the wall: u(y) = u(L - y)
        assert np.abs(ux[1:] - ux[:0:-1]).max() < 1e-9 * np.abs(ux).max()
        res.append(validation.steady_channel_errors(ux, ubar[0], N, f0, mu, L) + (N,))
    for (e0, d0, _, _), (e1, d1, _, _) in zip(res, res[1:]):
        assert 0.8 < np.log2(e0 / e1) < 1.3
        assert np.log2(d0 / d1) > 1.4
    De, N = res[-1][2], res[-1][3]
    assert 0.35 < (L - De) * N / L < 0.5
