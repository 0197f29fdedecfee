"""Pins for the oracle's transform gradients (CPU only): central finite differences of the
direct sums themselves (App. A eqs. type1 and type2), on tiny inputs, for strengths, spectra and
positions, and the adjoint identities they rest on."""

import numpy as np
import pytest

from oracle import nudft
from oracle.modes import spectral_shape


def _loss1(X, c, w, Ns, L, scale):
    return float(np.real(np.vdot(w, nudft.type1(X, c, Ns, L, scale))))  # Re sum conj(w) f


def _loss2(X, f, w, Ns, L):
    return float(np.real(np.vdot(w, nudft.type2(X, f, Ns, L))))


@pytest.mark.parametrize("Ns", [(6, 5), (5, 4, 6)])
def test_type1_grad_matches_finite_differences(Ns):
    rng = np.random.default_rng(51)
    d, M, L, scale = len(Ns), 7, 1.3, 0.7
    X = rng.uniform(-1, 2, (M, d))
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    w = rng.standard_normal(spectral_shape(Ns)) + 1j * rng.standard_normal(spectral_shape(Ns))
    gc, gX = nudft.type1_grad(X, c, w, Ns, L, scale)  # dL/df-bar convention: the gradient of f is w
    h = 1e-6
    for j in range(M):
        for part, unit in ((0, 1.0), (1, 1j)):
            cp, cm = c.copy(), c.copy()
            cp[j] += h * unit
            cm[j] -= h * unit
            fd = (_loss1(X, cp, w, Ns, L, scale) - _loss1(X, cm, w, Ns, L, scale)) / (2 * h)
            ref = gc[j].real if part == 0 else gc[j].imag
            assert abs(fd - ref) < 1e-7 * max(1.0, abs(ref))
        for a in range(d):
            Xp, Xm = X.copy(), X.copy()
            Xp[j, a] += h
            Xm[j, a] -= h
            fd = (_loss1(Xp, c, w, Ns, L, scale) - _loss1(Xm, c, w, Ns, L, scale)) / (2 * h)
            assert abs(fd - gX[j, a]) < 1e-6 * max(1.0, abs(gX[j, a]))


@pytest.mark.parametrize("Ns", [(6, 5), (5, 4, 6)])
def test_type2_grad_matches_finite_differences(Ns):
    rng = np.random.default_rng(52)
    d, M, L = len(Ns), 6, 0.9
    X = rng.uniform(-1, 2, (M, d))
    shp = spectral_shape(Ns)
    f = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    w = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    gf, gX = nudft.type2_grad(X, f, w, Ns, L)
    h = 1e-6
    flat = f.ravel()
    for q in rng.choice(flat.size, 8, replace=False):
        for part, unit in ((0, 1.0), (1, 1j)):
            fp, fm = flat.copy(), flat.copy()
            fp[q] += h * unit
            fm[q] -= h * unit
            fd = (_loss2(X, fp.reshape(shp), w, Ns, L) - _loss2(X, fm.reshape(shp), w, Ns, L)) / (2 * h)
            ref = gf.ravel()[q].real if part == 0 else gf.ravel()[q].imag
            assert abs(fd - ref) < 1e-7 * max(1.0, abs(ref))
    for j in range(M):
        for a in range(d):
            Xp, Xm = X.copy(), X.copy()
            Xp[j, a] += h
            Xm[j, a] -= h
            fd = (_loss2(Xp, f, w, Ns, L) - _loss2(Xm, f, w, Ns, L)) / (2 * h)
            assert abs(fd - gX[j, a]) < 1e-6 * max(1.0, abs(gX[j, a]))


def test_position_gradients_of_a_shift_sum_to_a_translation_derivative():
    """Translating all points by r multiplies type-1 by exp(-i k.r), so sum_j grad_X[j] equals the
    derivative of the loss along a uniform shift: Re sum_k conj(w) (-i k) f(k)."""
    rng = np.random.default_rng(53)
    Ns, L = (6, 7), 1.0
    X = rng.random((9, 2))
    c = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    w = rng.standard_normal(spectral_shape(Ns)) + 1j * rng.standard_normal(spectral_shape(Ns))
    f = nudft.type1(X, c, Ns, L)
    _, gX = nudft.type1_grad(X, c, w, Ns, L)
    for a in range(2):
        shift = float(np.real(np.vdot(w, -nudft._ik_weighted(f, Ns, L, a))))
        assert abs(gX[:, a].sum() - shift) < 1e-10 * max(1.0, abs(shift))


@pytest.mark.parametrize("Ns", [(8, 6), (6, 5, 4)])
def test_stokes_map_grad_matches_finite_differences(Ns):
    from oracle import step
    rng = np.random.default_rng(54)
    d, M, L, mu = len(Ns), 5, 1.0, 0.7
    X = rng.random((M, d))
    S = rng.standard_normal((M, d))
    W = rng.standard_normal((M, d))
    loss = lambda X_, S_: float(np.sum(W * step.stokes_map(X_, S_, Ns, L, mu)[0]))
    gS, gX = step.stokes_map_grad(X, S, W, Ns, L, mu)
    h = 1e-6
    for j in range(M):
        for a in range(d):
            Sp, Sm = S.copy(), S.copy()
            Sp[j, a] += h
            Sm[j, a] -= h
            fd = (loss(X, Sp) - loss(X, Sm)) / (2 * h)
            assert abs(fd - gS[j, a]) < 1e-7 * max(1.0, abs(gS[j, a]))
            Xp, Xm = X.copy(), X.copy()
            Xp[j, a] += h
            Xm[j, a] -= h
            fd = (loss(Xp, S) - loss(Xm, S)) / (2 * h)
            assert abs(fd - gX[j, a]) < 1e-6 * max(1.0, abs(gX[j, a]))


def _wobbly_sphere(seed):
    import workloads as wl
    X, tris = wl.latlong_sphere(4, 6, radius=0.2, center=(0.5, 0.5, 0.5))
    return X + 0.01 * np.random.default_rng(seed).standard_normal(X.shape), tris


def test_surface_force_jvp_matches_finite_differences_and_is_symmetric():
    from oracle import forces
    X, tris = _wobbly_sphere(61)
    rng = np.random.default_rng(62)
    V, W = rng.standard_normal(X.shape), rng.standard_normal(X.shape)
    J = forces.surface_tension_force_3d_jvp(X, tris, 1.3, V)
    h = 1e-6
    fd = (forces.surface_tension_force_3d(X + h * V, tris, 1.3) -
          forces.surface_tension_force_3d(X - h * V, tris, 1.3)) / (2 * h)
    assert np.abs(J - fd).max() < 1e-7 * np.abs(fd).max()
    # F = -gamma grad(area): the Jacobian is a Hessian, <W, J V> = <V, J W>
    JW = forces.surface_tension_force_3d_jvp(X, tris, 1.3, W)
    assert abs(np.sum(W * J) - np.sum(V * JW)) < 1e-12 * abs(np.sum(W * J))
    # a rigid translation does not change the force
    T = np.tile(rng.standard_normal(3), (X.shape[0], 1))
    assert np.abs(forces.surface_tension_force_3d_jvp(X, tris, 1.3, T)).max() < 1e-12 * np.abs(J).max()


def test_tension_force_jvp_is_the_force_of_the_direction():
    from oracle import forces
    rng = np.random.default_rng(63)
    X, V = rng.standard_normal((11, 2)), rng.standard_normal((11, 2))
    h = 1e-3  # the force is linear: the central difference is exact up to rounding
    fd = (forces.tension_force_2d(X + h * V, 0.7) - forces.tension_force_2d(X - h * V, 0.7)) / (2 * h)
    assert np.allclose(forces.tension_force_2d_jvp(V, 0.7), fd, rtol=1e-9, atol=1e-9)


def _trajectory_fd_check(X, force_kind, K, tris, Ns, mu, dt, steps, target, comps):
    from oracle import step
    loss, gX, gK = step.stokes_trajectory_grad(X, step.ForceLaw(force_kind, K, tris), Ns, 1.0, mu, dt, steps,
                                               target)

    def L(X0, k):
        XT = step.stokes_trajectory(X0, step.ForceLaw(force_kind, k, tris), Ns, 1.0, mu, dt, steps)
        return step.trajectory_loss(XT, target)

    assert loss == pytest.approx(L(X, K), rel=1e-14)
    h = 1e-5
    fdK = (L(X, K + h) - L(X, K - h)) / (2 * h)
    assert abs(gK - fdK) < 1e-7 * max(abs(fdK), 1e-3)
    scale = np.abs(gX).max()
    for j, a in comps:
        Xp, Xm = X.copy(), X.copy()
        Xp[j, a] += h
        Xm[j, a] -= h
        fd = (L(Xp, K) - L(Xm, K)) / (2 * h)
        assert abs(gX[j, a] - fd) < 1e-7 * scale, (j, a, gX[j, a], fd)


def test_stokes_trajectory_grad_matches_finite_differences_3d_surface_tension():
    X, tris = _wobbly_sphere(64)
    target = 0.5 + (X - 0.5) * np.array([1.2, 1.0, 0.8])
    comps = [(0, 0), (3, 1), (10, 2), (17, 0), (X.shape[0] - 1, 1)]
    _trajectory_fd_check(X, "surface3d", 1.0, tris, (8, 8, 8), 1.0, 2e-2, 3, target, comps)


def test_stokes_trajectory_grad_matches_finite_differences_2d_tension():
    import workloads as wl
    X = wl.ellipse_2d(24, center=(0.43, 0.57), a=0.3, b=0.2)
    target = wl.ellipse_2d(24, center=(0.5, 0.5), a=0.25, b=0.25)
    _trajectory_fd_check(X, "tension2d", 0.8, None, (12, 12), 1.0, 1e-2, 4, target, [(0, 0), (5, 1), (23, 0)])
