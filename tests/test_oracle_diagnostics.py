"""Pins of the oracle's diagnostics (CPU only): each one against a value fixed independently of it.

* kinetic energy (Sec. 5.4): (rho/2) times the integral of |u|^2 -- a closed form for a single cosine
  mode, and the grid quadrature h^d sum |u|^2 of a random real field (exact for a trigonometric
  polynomial sampled on its own grid);
* dissipation (Sec. 5.4): mu times the integral of |grad u|^2, with the gradient written out
  analytically for a sum of explicit sine/cosine modes;
* power (Sec. 5.4, eq. pote_energ_derivative): the boundary sum sum_j w_j F_j . U_j equals
  L^d sum_k fhat . conj(uhat) when fhat is the spread of the forces and U the interpolation of uhat;
* divergence residual (Sec. 5.1): 1 for a pure gradient field, 0 for a divergence-free one, and a
  closed-form ratio for one solenoidal mode plus one gradient mode;
* enclosed area and volume (Sec. 6.2): the exact area of a regular polygon inscribed in an ellipse,
  and the exact volumes of a triangulated box and tetrahedron.

Each pin is followed by a check that a plausible slip in the oracle (a dropped L^d, a halved sum,
a flipped sign, a missing weight) would fail it; the slip is planted in a copy of the oracle
function on the CPU, never in the product path.
"""

import numpy as np
import pytest

from oracle import diagnostics, nudft
from oracle.modes import spectral_shape

L_BOX = 1.7  # L != 1 so that a dropped L^d shows
RHO = 1.3
MU = 0.37


def _grid(Ns, L):
    """Grid coordinates x_a[j] = j L / N_a as a list of arrays broadcastable to spectral_shape(Ns)."""
    d = len(Ns)
    out = []
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = int(Ns[a])
        out.append((np.arange(Ns[a]) * (L / Ns[a])).reshape(shape))
    return out


def _coeffs(u, Ns):
    """Fourier coefficients (K_N, FFT order) of grid samples u of a trigonometric polynomial:
    u(x_j) = sum_k uhat(k) exp(i k.x_j).  The DFT is the plain library routine."""
    d = len(Ns)
    return np.fft.fftn(u, axes=tuple(range(1, d + 1))) / float(np.prod(Ns))


def _random_trig_field(Ns, L, seed, nterms=6):
    """A real vector field made of a few explicit modes A cos(k.x + phi) per component, |m_a| < N_a/2,
    with its samples on the N grid and its exact gradient there: returns (u, du) with
    u[c] (spectral_shape) and du[c][b] = d u_c / d x_b."""
    rng = np.random.default_rng(seed)
    d = len(Ns)
    x = _grid(Ns, L)
    shp = spectral_shape(Ns)
    u = np.zeros((d,) + shp)
    du = np.zeros((d, d) + shp)
    for c in range(d):
        for _ in range(nterms):
            m = [int(rng.integers(-(Ns[a] // 2) + 1, Ns[a] // 2)) for a in range(d)]
            A = rng.standard_normal()
            phi = rng.uniform(0, 2 * np.pi)
            k = [2 * np.pi * m[a] / L for a in range(d)]
            arg = sum(k[a] * x[a] for a in range(d)) + phi
            u[c] += A * np.cos(arg)
            for b in range(d):
                du[c, b] += -A * k[b] * np.sin(arg)
    return u, du


# ---- kinetic energy -----------------------------------------------------------------------------

def _kinetic_pins(fn):
    """True when fn(uhat, L, rho) meets both kinetic-energy pins."""
    ok = True
    # closed form: u = (A cos(k.x + phi), 0, 0), integral of u^2 over the box = A^2 L^d / 2
    for Ns in [(8, 6), (6, 8, 5)]:
        d = len(Ns)
        x = _grid(Ns, L_BOX)
        A, phi, m = 0.8, 0.3, [1, 2, 1][:d]
        arg = sum(2 * np.pi * m[a] / L_BOX * x[a] for a in range(d)) + phi
        u = np.zeros((d,) + spectral_shape(Ns))
        u[0] = A * np.cos(arg)
        want = 0.5 * RHO * A * A * L_BOX ** d / 2
        ok &= abs(fn(_coeffs(u, Ns), L_BOX, RHO) - want) < 1e-12 * want
    # quadrature: (rho/2) h^d sum_grid |u|^2 for a random real field sampled on its grid (Parseval)
    for Ns in [(8, 8), (6, 4, 5)]:
        d = len(Ns)
        rng = np.random.default_rng(11)
        u = rng.standard_normal((d,) + spectral_shape(Ns))
        hd = float(np.prod([L_BOX / n for n in Ns]))
        want = 0.5 * RHO * hd * float(np.sum(u * u))
        ok &= abs(fn(_coeffs(u, Ns), L_BOX, RHO) - want) < 1e-12 * want
    return bool(ok)


def test_kinetic_energy_pins():
    assert _kinetic_pins(diagnostics.kinetic_energy)


def test_kinetic_energy_pins_catch_slips():
    ke = diagnostics.kinetic_energy
    assert not _kinetic_pins(lambda u, L, rho: ke(u, 1.0, rho))           # dropped L^d
    assert not _kinetic_pins(lambda u, L, rho: 2.0 * ke(u, L, rho))        # half/full-spectrum factor
    assert not _kinetic_pins(lambda u, L, rho: ke(u, L, rho) / rho)        # dropped rho


# ---- dissipation --------------------------------------------------------------------------------

def _dissipation_pins(fn):
    ok = True
    for Ns, seed in [((8, 10), 3), ((6, 8, 6), 4)]:
        d = len(Ns)
        u, du = _random_trig_field(Ns, L_BOX, seed)
        hd = float(np.prod([L_BOX / n for n in Ns]))
        # mu times the integral of |grad u|^2, by the grid quadrature of the exact gradient
        want = MU * hd * float(np.sum(du * du))
        ok &= abs(fn(_coeffs(u, Ns), Ns, L_BOX, MU) - want) < 1e-11 * want
    # closed form: u = (0, A sin(2 pi m x / L)) -> integral |grad u|^2 = A^2 (2 pi m / L)^2 L^d / 2
    Ns = (8, 8)
    x = _grid(Ns, L_BOX)
    A, m = 1.1, 3
    u = np.zeros((2,) + spectral_shape(Ns))
    u[1] = A * np.sin(2 * np.pi * m * x[0] / L_BOX)
    want = MU * A * A * (2 * np.pi * m / L_BOX) ** 2 * L_BOX ** 2 / 2
    ok &= abs(fn(_coeffs(u, Ns), Ns, L_BOX, MU) - want) < 1e-12 * want
    return bool(ok)


def test_dissipation_pins():
    assert _dissipation_pins(diagnostics.dissipation)


def test_dissipation_pins_catch_slips():
    ds = diagnostics.dissipation
    assert not _dissipation_pins(lambda u, Ns, L, mu: ds(u, Ns, 1.0, mu))  # L dropped everywhere
    assert not _dissipation_pins(lambda u, Ns, L, mu: ds(u, Ns, L, mu) / L ** len(Ns))  # the L^d of the final law
    assert not _dissipation_pins(lambda u, Ns, L, mu: 0.5 * ds(u, Ns, L, mu))


# ---- power --------------------------------------------------------------------------------------

def _power_case(Ns, M, seed):
    rng = np.random.default_rng(seed)
    d = len(Ns)
    X = rng.uniform(-0.5, 2.0, (M, d)) * L_BOX
    F = rng.standard_normal((M, d))
    w = rng.uniform(0.2, 1.5, M)
    # a real field: odd N per axis, so K_N is symmetric and U is real
    u = rng.standard_normal((d,) + spectral_shape(Ns))
    uhat = _coeffs(u, Ns)
    U = np.stack([nudft.type2(X, uhat[a], Ns, L_BOX) for a in range(d)], axis=1)
    assert np.max(np.abs(U.imag)) < 1e-11 * np.max(np.abs(U))
    U = U.real
    fhat = np.stack([nudft.type1(X, w * F[:, a], Ns, L_BOX, scale=L_BOX ** -d) for a in range(d)])
    return F, w, U, fhat, uhat


def _power_pins(fn):
    ok = True
    for Ns, M, seed in [((7, 9), 40, 5), ((5, 7, 5), 30, 6)]:
        d = len(Ns)
        F, w, U, fhat, uhat = _power_case(Ns, M, seed)
        want = L_BOX ** d * float(np.real(np.sum(fhat * np.conj(uhat))))
        got = fn(F, w, U)
        ok &= abs(got - want) < 1e-10 * np.sqrt(np.sum((w[:, None] * F) ** 2) * np.sum(U * U))
        # a single point: w F . U by hand
        ok &= abs(fn(F[:1], w[:1], U[:1]) - w[0] * float(F[0] @ U[0])) < 1e-14 * (1 + abs(w[0] * F[0] @ U[0]))
    return bool(ok)


def test_power_pins():
    assert _power_pins(diagnostics.power)


def test_power_pins_catch_slips():
    pw = diagnostics.power
    assert not _power_pins(lambda F, w, U: pw(F, 1.0, U))     # weight dropped
    assert not _power_pins(lambda F, w, U: -pw(F, w, U))      # sign
    assert not _power_pins(lambda F, w, U: pw(F, w * w, U))   # weight applied twice


# ---- divergence residual ------------------------------------------------------------------------

def _divergence_pins(fn):
    ok = True
    Ns = (8, 6, 7)
    d = 3
    shp = spectral_shape(Ns)
    rng = np.random.default_rng(9)
    # a pure gradient field uhat = i k phi: |k.uhat| = |k| |uhat| mode by mode, the ratio is 1
    phi = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    m = [np.fft.fftfreq(n, 1.0 / n) for n in Ns]
    kz, ky, kx = np.meshgrid(*[2 * np.pi * mm / L_BOX for mm in reversed(m)], indexing="ij")
    grad = np.stack([1j * kx * phi, 1j * ky * phi, 1j * kz * phi])
    ok &= abs(fn(grad, Ns, L_BOX) - 1.0) < 1e-13
    # one solenoidal mode (amplitude a, k1 . a = 0) and one gradient mode (i k2 phi2):
    # ratio = |k2|^2 |phi2| / max(|k1| |a|, |k2|^2 |phi2|)
    for amp in (0.05, 3.0):
        uh = np.zeros((d,) + shp, dtype=complex)
        m1, m2 = (1, 2, 0), (0, -1, 3)  # (m_x, m_y, m_z)
        k1 = np.array(m1) * 2 * np.pi / L_BOX
        k2 = np.array(m2) * 2 * np.pi / L_BOX
        a = np.cross(k1, [0.3, -0.7, 1.1]) * (1 + 0.5j)
        idx1 = (m1[2] % Ns[2], m1[1] % Ns[1], m1[0] % Ns[0])
        idx2 = (m2[2] % Ns[2], m2[1] % Ns[1], m2[0] % Ns[0])
        for c in range(d):
            uh[(c,) + idx1] = a[c]
            uh[(c,) + idx2] = 1j * k2[c] * amp
        num = float(k2 @ k2) * amp
        den = max(np.linalg.norm(k1) * np.linalg.norm(a), num)
        ok &= abs(fn(uh, Ns, L_BOX) - num / den) < 1e-13
        ok &= num / den < 1.0 if amp == 0.05 else abs(num / den - 1.0) < 1e-15
    # a divergence-free field alone, and the zero field
    uh0 = np.zeros((d,) + shp, dtype=complex)
    uh0[(slice(None),) + idx1] = a
    ok &= fn(uh0, Ns, L_BOX) < 1e-15
    ok &= fn(np.zeros((d,) + shp, dtype=complex), Ns, L_BOX) == 0.0
    return bool(ok)


def test_divergence_residual_pins():
    assert _divergence_pins(diagnostics.divergence_residual)


def test_divergence_residual_pins_catch_slips():
    dv = diagnostics.divergence_residual
    assert not _divergence_pins(lambda u, Ns, L: 0.0)                       # a residual that reports nothing
    assert not _divergence_pins(lambda u, Ns, L: dv(u[[1, 0, 2]], Ns, L))   # components swapped
    assert not _divergence_pins(lambda u, Ns, L: dv(np.conj(u), Ns, L) * 0.5)


# ---- enclosed area and volume -------------------------------------------------------------------

def _area_pins(fn):
    ok = True
    for M, a, b, c in [(7, 0.3, 0.2, (0.4, 0.7)), (128, 0.3, 0.2, (5.3, -2.1)), (1000, 1.0, 0.5, (0.0, 0.0))]:
        th = 2 * np.pi * np.arange(M) / M
        X = np.stack([c[0] + a * np.cos(th), c[1] + b * np.sin(th)], axis=1)
        want = 0.5 * M * a * b * np.sin(2 * np.pi / M)  # M triangles of area (1/2) a b sin(2 pi / M)
        ok &= abs(fn(X) - want) < 1e-13 * (1 + abs(want)) * (1 + np.max(np.abs(X)))
        ok &= abs(fn(X[::-1]) + want) < 1e-13 * (1 + abs(want)) * (1 + np.max(np.abs(X)))  # clockwise: negative
    sq = np.array([[0.0, 0.0], [2.0, 0.0], [2.0, 3.0], [0.0, 3.0]])
    ok &= abs(fn(sq) - 6.0) < 1e-15
    return bool(ok)


def test_enclosed_area_pins():
    assert _area_pins(diagnostics.enclosed_area)


def test_enclosed_area_pins_catch_slips():
    ar = diagnostics.enclosed_area
    assert not _area_pins(lambda X: -ar(X))
    assert not _area_pins(lambda X: 2.0 * ar(X))
    assert not _area_pins(lambda X: abs(ar(X)))


def _box_mesh(lo, hi):
    """The 12 triangles of an axis-aligned box, counter-clockwise seen from outside."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    V = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]])
    T = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7], [0, 1, 5], [0, 5, 4],
                  [1, 2, 6], [1, 6, 5], [2, 3, 7], [2, 7, 6], [3, 0, 4], [3, 4, 7]])
    return V, T


def test_enclosed_volume_exact():
    V, T = _box_mesh((0.3, -1.0, 2.0), (1.3, 1.5, 2.5))
    assert abs(diagnostics.enclosed_volume(V, T) - 1.0 * 2.5 * 0.5) < 1e-14
    assert abs(diagnostics.enclosed_volume(V, T[:, ::-1]) + 1.25) < 1e-14  # reversed orientation
    tet = np.array([[0.1, 0.2, 0.3], [1.1, 0.2, 0.3], [0.1, 1.2, 0.3], [0.1, 0.2, 1.3]])
    tris = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]])
    assert abs(diagnostics.enclosed_volume(tet, tris) - 1.0 / 6.0) < 1e-15
