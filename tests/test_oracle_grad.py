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
