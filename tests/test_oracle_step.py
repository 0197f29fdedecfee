"""Pins for the oracle's force laws and its Alg. 1 stepper (CPU only).

Forces: zero net force and F = -grad E by central differences (Secs. 6.2.1, 6.2.3).
Stepper: the discrete momentum identity (Sec. 5.3), translation invariance
under an arbitrary shift (Sec. 5.2), second-order temporal self-convergence
(Sec. 6.2.1), and volume conservation of the divergence-free flow (Sec. 5.1).
Mesh: the lat-long sphere is closed (Euler characteristic 2) and
counter-clockwise seen from outside (positive enclosed volume).
"""

import numpy as np
import pytest

from oracle import diagnostics, forces, step
from oracle.modes import wavevector, spectral_shape
from tests.helpers import rel_l2
from workloads import ellipse_2d, latlong_sphere, stokes2d_case


def _fd_grad(E, X, h=1e-6, idx=None):
    g = np.zeros_like(X)
    it = idx if idx is not None else [(i, a) for i in range(X.shape[0]) for a in range(X.shape[1])]
    for (i, a) in it:
        Xp = X.copy(); Xp[i, a] += h
        Xm = X.copy(); Xm[i, a] -= h
        g[i, a] = (E(Xp) - E(Xm)) / (2 * h)
    return g


def test_tension2d_force_is_energy_gradient():
    rng = np.random.default_rng(1)
    X = ellipse_2d(24, (0.4, 0.6)) + 0.01 * rng.standard_normal((24, 2))
    K = 1.3
    F = forces.tension_force_2d(X, K)
    w = 2 * np.pi / 24
    g = _fd_grad(lambda Y: forces.tension_energy_2d(Y, K), X)
    assert rel_l2(w * F, -g) < 1e-7
    assert np.max(np.abs(F.sum(axis=0))) < 1e-10 * np.max(np.abs(F))


def test_surface_tension_force_is_area_gradient():
    X, tris = latlong_sphere(6, 8, radius=0.3, center=(0.5, 0.5, 0.5), scale=(1.1, 1.0, 0.9))
    rng = np.random.default_rng(2)
    X = X + 0.01 * rng.standard_normal(X.shape)
    gamma = 0.7
    F = forces.surface_tension_force_3d(X, tris, gamma)
    g = _fd_grad(lambda Y: forces.surface_tension_energy_3d(Y, tris, gamma), X)
    assert rel_l2(F, -g) < 1e-7
    assert np.max(np.abs(F.sum(axis=0))) < 1e-12 * np.max(np.abs(F))


def test_latlong_mesh_closed_and_outward():
    for (R, P) in [(4, 5), (10, 12), (200, 200)]:
        X, tris = latlong_sphere(R, P, radius=0.25, center=(0.5, 0.5, 0.5))
        V, T = X.shape[0], tris.shape[0]
        edges = set()
        for t in tris:
            for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
                edges.add((min(a, b), max(a, b)))
        assert V - len(edges) + T == 2
        # every directed edge appears once and its reverse once: consistently oriented closed surface
        directed = {}
        for t in tris:
            for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
                directed[(a, b)] = directed.get((a, b), 0) + 1
        assert all(v == 1 for v in directed.values())
        assert all((b, a) in directed for (a, b) in directed)
        assert diagnostics.enclosed_volume(X, tris) > 0
    assert T == 79996 and V == 40000
    vol = diagnostics.enclosed_volume(X, tris)
    assert abs(vol - 4 / 3 * np.pi * 0.25 ** 3) < 1e-3 * vol


def _ns2d_setup(N=12, M=24):
    Ns = (N, N)
    X = ellipse_2d(M, (0.45, 0.55), 0.25, 0.2)
    shp = spectral_shape(Ns)
    uh = np.zeros((2,) + shp, dtype=complex)
    uh[1][0, 1] = 1.0 / 2j  # u0 = (0, sin 2 pi x), Sec. 6.2.1
    uh[1][0, -1] = -1.0 / 2j
    force = step.ForceLaw("tension2d", 1.0)
    U = step.interp_velocity(X, uh, Ns, 1.0)
    return Ns, X, U, uh, force


def test_momentum_identity():
    """rho L^d (uhat_0^{m+1} - uhat_0^m) / dt = sum_j w_j F_j^{m+1/2} (Sec. 5.3)."""
    Ns, X, U, uh, force = _ns2d_setup()
    X = X + np.array([0.03, 0.0])  # break the symmetry so that the net force is nonzero per component
    L, rho, mu, dt = 1.0, 1.3, 0.02, 2e-3
    Xn, Un, un, mid = step.ns_step(X, U, uh, force, Ns, L, rho, mu, dt, return_mid=True)
    lhs = rho * L ** 2 * (un[:, 0, 0] - uh[:, 0, 0]) / dt
    rhs = diagnostics.net_force(mid["F"], mid["w"])
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * max(1.0, np.max(np.abs(mid["F"])))
    # with a force law of zero net force the mean flow stays constant
    assert np.max(np.abs(un[:, 0, 0] - uh[:, 0, 0])) < 1e-13


def test_translation_invariance_ns():
    """Shifting every point by r shifts the whole trajectory: X_r(T) - r = X(T), uhat_r = uhat e^{-ik.r}."""
    Ns, X, U, uh, force = _ns2d_setup()
    L, rho, mu, dt = 1.0, 1.0, 0.01, 2e-3
    r = np.array([0.31415926535, 0.27182818284])
    k = wavevector(Ns, L)
    ph = np.exp(-1j * (k[0] * r[0] + k[1] * r[1]))
    Xa, Ua, ua = X.copy(), U.copy(), uh.copy()
    Xb, Ub, ub = X + r, U.copy(), uh * ph
    for _ in range(4):
        Xa, Ua, ua = step.ns_step(Xa, Ua, ua, force, Ns, L, rho, mu, dt)
        Xb, Ub, ub = step.ns_step(Xb, Ub, ub, force, Ns, L, rho, mu, dt)
    assert np.max(np.abs(Xb - r - Xa)) < 1e-13
    assert rel_l2(ub, ua * ph) < 1e-12
    assert rel_l2(Ub, Ua) < 1e-12


def test_translation_invariance_stokes():
    case = stokes2d_case()
    Ns, L, mu, dt = case["N"], case["L"], case["mu"], case["dt"]
    force = step.ForceLaw("tension2d", case["K"])
    X = case["X"]
    r = np.array([0.1234567, -0.7654321])
    U, _ = step.stokes_velocity(X, force, Ns, L, mu)
    Ur, _ = step.stokes_velocity(X + r, force, Ns, L, mu)
    assert rel_l2(Ur, U) < 1e-12
    Xa, Ua = X, U
    Xb, Ub = X + r, Ur
    for _ in range(3):
        Xa, Ua, _ = step.stokes_step(Xa, Ua, force, Ns, L, mu, dt)
        Xb, Ub, _ = step.stokes_step(Xb, Ub, force, Ns, L, mu, dt)
    assert np.max(np.abs(Xb - r - Xa)) < 1e-13


def test_temporal_second_order():
    """Self-convergence of the midpoint/Crank-Nicolson stepper is second order (Sec. 6.2.1)."""
    Ns, X0, U0, uh0, force = _ns2d_setup(N=8, M=16)
    L, rho, mu = 1.0, 1.0, 0.05
    T = 0.04

    def run(nsteps):
        X, U, uh = X0.copy(), U0.copy(), uh0.copy()
        dt = T / nsteps
        for _ in range(nsteps):
            X, U, uh = step.ns_step(X, U, uh, force, Ns, L, rho, mu, dt)
        return X

    x1, x2, x3 = run(4), run(8), run(16)
    e1 = np.max(np.abs(x1 - x3))
    e2 = np.max(np.abs(x2 - x3))
    ratio = e1 / e2
    assert 4.0 < ratio < 6.5, ratio  # (1 - 1/16)/(1/4 - 1/16) = 5 for an exact second-order method


def test_divergence_free_and_area_conserved_continuous_limit():
    """k.uhat = 0 after each step (Sec. 5.1); enclosed area changes only at the time-step error level."""
    Ns, X, U, uh, force = _ns2d_setup(N=16, M=40)
    L, rho, mu, dt = 1.0, 1.0, 0.01, 1e-3
    A0 = diagnostics.enclosed_area(X)
    for _ in range(5):
        X, U, uh = step.ns_step(X, U, uh, force, Ns, L, rho, mu, dt)
    assert diagnostics.divergence_residual(uh, Ns, L) < 1e-13
    assert abs(diagnostics.enclosed_area(X) - A0) < 1e-7 * A0


def test_batched_stokes2d_workload_is_seeded():
    import workloads
    a = workloads.batched_stokes2d(count=64, seed=4)
    b = workloads.batched_stokes2d(count=64, seed=4)
    assert len(a) == 64
    for x, y in zip(a, b):
        assert x["N"] == y["N"] and np.array_equal(x["X"], y["X"])
        assert x["N"][0] in (64, 128, 256, 512)
        assert 256 <= x["X"].shape[0] <= 8192
