"""Pins for the oracle's Fourier-space fluid operators (CPU only).

Projection: k.Q = 0, idempotence, gradients removed (Secs. 2, 5.1).
Stokes solve: the Fourier Stokes equations with the paper's pressure (eq.
stokeslet) hold mode by mode; the normal-force circle gives u = 0 (Sec. 6.1,
printed in the paper); the Stokes energy identity (Sec. 5.4 with eq. stokeslet).
Nonlinear term: brute-force truncated convolution (Sec. 3.1), independence of
the padded length, zero mean (Sec. 5.3), skew identity (Sec. 5.4) and
translation covariance (Sec. 5.2).
Viscous factor: a sine shear flow decays by (1-a)/(1+a) per step (Alg. 1).
"""

import json
import os

import numpy as np
import pytest

from oracle import fluid, nudft, step
from oracle.modes import wavevector, ksquared, nyquist_mask, spectral_shape
from tests.helpers import rel_l2, random_real_field_hat
from workloads import circle_2d

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _div_free(Ns, d, seed, L=1.0):
    uh = random_real_field_hat(Ns, d, seed)
    uh = fluid.project(uh, Ns, L)
    return fluid.zero_nyquist(uh, Ns)


@pytest.mark.parametrize("Ns", [(8, 8), (6, 5, 4)])
def test_projection(Ns):
    d = len(Ns)
    L = 1.4
    rng = np.random.default_rng(1)
    shp = (d,) + spectral_shape(Ns)
    P = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    Q = fluid.project(P, Ns, L)
    k = wavevector(Ns, L)
    kdq = sum(k[a] * Q[a] for a in range(d))
    assert np.max(np.abs(kdq)) < 1e-12 * np.max(np.abs(P))
    assert rel_l2(fluid.project(Q, Ns, L), Q) < 1e-14
    phi = rng.standard_normal(spectral_shape(Ns)) + 0j
    grad = np.stack([1j * k[a] * phi for a in range(d)])
    assert np.max(np.abs(fluid.project(grad, Ns, L))) < 1e-12 * np.max(np.abs(grad))
    zero = (slice(None),) + (0,) * d
    assert np.allclose(Q[zero], P[zero])


@pytest.mark.parametrize("Ns", [(8, 8), (6, 5, 4)])
def test_stokeslet_solves_fourier_stokes(Ns):
    """-i k phat - mu |k|^2 uhat + fhat = 0 and k.uhat = 0 for k != 0 (eqs. stokes, stokeslet)."""
    d = len(Ns)
    L, mu = 1.2, 0.7
    rng = np.random.default_rng(2)
    shp = (d,) + spectral_shape(Ns)
    f = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    u = fluid.stokeslet(f, Ns, L, mu)
    p = fluid.stokes_pressure(f, Ns, L)
    k = wavevector(Ns, L)
    k2 = ksquared(Ns, L)
    nz = k2 > 0
    for a in range(d):
        res = -1j * k[a] * p - mu * k2 * u[a] + f[a]
        assert np.max(np.abs(res[nz])) < 1e-12 * np.max(np.abs(f))
    assert np.max(np.abs(sum(k[a] * u[a] for a in range(d)))) < 1e-12


def test_normal_force_circle_gives_zero_velocity():
    """Printed in the paper: the normal-force circle has u = 0 to machine error below the transition."""
    g = json.load(open(os.path.join(GOLDEN, "circle_normal_force.json")))
    L, mu, M = g["L"], g["mu"], g["N_b"]
    X = circle_2d(M, center=tuple(g["center"]), r=g["radius"])
    th = 2 * np.pi * np.arange(M) / M
    F = g["force_magnitude"] * np.stack([np.cos(th), np.sin(th)], axis=1)
    for N in g["N_below_transition"]:
        Ns = (N, N)
        fh = step.spread_force(X, F, 2 * np.pi / M, Ns, L)
        uh = fluid.stokeslet(fh, Ns, L, mu)
        uh[:, nyquist_mask(Ns)] = 0.0
        U = step.interp_velocity(X, uh, Ns, L)
        assert np.max(np.abs(U)) < g["machine_error_bound"], N
    # and the tangential force is not trivial (sanity of the same pipeline)
    Ft = np.stack([-np.sin(th), np.cos(th)], axis=1)
    uh = fluid.stokeslet(step.spread_force(X, Ft, 2 * np.pi / M, (32, 32), L), (32, 32), L, mu)
    assert np.max(np.abs(step.interp_velocity(X, uh, (32, 32), L))) > 1e-3


def test_stokes_energy_identity():
    """sum_j w_j F_j . U_j = mu L^d sum_k |k|^2 |uhat|^2 (Sec. 5.4 with the Stokeslet)."""
    L, mu = 1.0, 0.8
    rng = np.random.default_rng(3)
    M = 30
    X = rng.random((M, 3))
    F = rng.standard_normal((M, 3))
    F -= F.mean(axis=0)
    Ns = (8, 8, 8)
    fh = step.spread_force(X, F, 1.0, Ns, L)
    uh = fluid.stokeslet(fh, Ns, L, mu)
    uh[:, nyquist_mask(Ns)] = 0.0
    U = step.interp_velocity(X, uh, Ns, L)
    lhs = float(np.sum(F * U))
    rhs = mu * L ** 3 * float(np.sum(ksquared(Ns, L) * np.sum(np.abs(uh) ** 2, axis=0)))
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


@pytest.mark.parametrize("Ns", [(6, 6), (8, 6), (4, 4, 4), (5, 5)])
def test_nonlinear_matches_truncated_convolution(Ns):
    d = len(Ns)
    L = 1.1
    rng = np.random.default_rng(4)
    shp = (d,) + spectral_shape(Ns)
    uh = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)  # general complex input
    s_fft = fluid.nonlinear(uh, Ns, L)
    s_conv = fluid.nonlinear_convolution(uh, Ns, L)
    assert rel_l2(s_fft, s_conv) < 1e-13


def test_nonlinear_padding_independent():
    """Any padded length above 3N/2 gives the same shat (Sec. 3.1); 3N/2 itself suffices once -N/2 is zeroed."""
    Ns = (8, 8, 8)
    uh = _div_free(Ns, 3, 5)
    a = fluid.nonlinear(uh, Ns, 1.0)
    b = fluid.nonlinear(uh, Ns, 1.0, npad=(13, 14, 15))
    assert rel_l2(a, b) < 1e-13
    # 3N/2 = 12 with the Nyquist modes zeroed: products reach |m| <= N-2, aliases land beyond N/2
    c = fluid._truncate(
        np.fft.fftn(sum(np.fft.ifftn(fluid._embed(uh[1], Ns, (12, 12, 12))) * 12 ** 3 *
                        np.fft.ifftn(fluid._embed(1j * wavevector(Ns, 1.0)[1] * uh[0], Ns, (12, 12, 12))) * 12 ** 3
                        for _ in [0])) / 12 ** 3, Ns, (12, 12, 12))
    ref = fluid._truncate(
        np.fft.fftn(np.fft.ifftn(fluid._embed(uh[1], Ns, (16, 16, 16))) * 16 ** 3 *
                    np.fft.ifftn(fluid._embed(1j * wavevector(Ns, 1.0)[1] * uh[0], Ns, (16, 16, 16))) * 16 ** 3)
        / 16 ** 3, Ns, (16, 16, 16))
    assert rel_l2(c, ref) < 1e-13
    with pytest.raises(ValueError):
        fluid.nonlinear(uh, Ns, 1.0, npad=(12, 12, 12))


@pytest.mark.parametrize("Ns", [(12, 12), (8, 8, 8)])
def test_nonlinear_conservation_identities(Ns):
    """shat(0) = 0 (Sec. 5.3) and sum_k shat . conj(uhat) = 0 (Sec. 5.4) for divergence-free real u."""
    d = len(Ns)
    uh = _div_free(Ns, d, 6)
    s = fluid.nonlinear(uh, Ns, 1.0)
    zero = (slice(None),) + (0,) * d
    scale = np.max(np.abs(s))
    assert np.max(np.abs(s[zero])) < 1e-13 * scale
    assert abs(np.sum(s * np.conj(uh))) < 1e-13 * scale * np.sum(np.abs(uh))


def test_nonlinear_translation_covariance():
    """shat(uhat e^{-ik.r}) = shat(uhat) e^{-ik.r} (Sec. 5.2)."""
    Ns = (8, 10)
    L = 1.0
    uh = _div_free(Ns, 2, 7)
    r = np.array([0.31415926, 0.27182818])
    k = wavevector(Ns, L)
    ph = np.exp(-1j * (k[0] * r[0] + k[1] * r[1]))
    assert rel_l2(fluid.nonlinear(uh * ph, Ns, L), fluid.nonlinear(uh, Ns, L) * ph) < 1e-13


def test_sine_shear_decays_by_crank_nicolson_factor():
    """u0 = (0, sin 2 pi x / L) has shat = 0, so with f = 0 each step multiplies uhat by (1-a)/(1+a)."""
    Ns = (16, 16)
    L, rho, mu, dt = 1.0, 1.0, 0.01, 1e-3
    shp = spectral_shape(Ns)
    uh = np.zeros((2,) + shp, dtype=complex)
    # sin(2 pi x) = (e^{i k x} - e^{-i k x}) / 2i  at m_x = +-1
    uh[1][0, 1] = 1.0 / 2j
    uh[1][0, -1] = -1.0 / 2j
    assert np.max(np.abs(fluid.nonlinear(uh, Ns, L))) < 1e-14
    a = mu * dt * (2 * np.pi / L) ** 2 / (2 * rho)
    f0 = np.zeros_like(uh)
    u = uh
    for n in range(1, 4):
        _, u = fluid.ns_update(f0, u, Ns, L, rho, mu, dt)
        assert rel_l2(u, uh * ((1 - a) / (1 + a)) ** n) < 1e-14
