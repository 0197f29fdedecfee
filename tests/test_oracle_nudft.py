"""Pins for the oracle's direct nonuniform Fourier sums (CPU only).

Each test checks the oracle against something other than itself: the DFT on
grid points (App. A, remark after eq. type1), a brute-force loop that forms
each phase in one piece, adjointness, and the closed-form Dirichlet kernel
and its discrete moment identities (Sec. 4, eqs. FSIB_kern_odd and
sum_square_FSIB and the zeroth-moment identity before it).
"""

import itertools

import numpy as np
import pytest

from oracle import nudft
from oracle.modes import mode_numbers, spectral_shape
from tests.helpers import rel_l2


def _grid_points(Ns, L):
    d = len(Ns)
    axes = [np.arange(int(n)) * (L / int(n)) for n in Ns]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")  # numpy axis b <-> physical axis d-1-b
    return np.stack([mesh[d - 1 - a].ravel() for a in range(d)], axis=1)


def test_mode_numbers_match_eq_kNh():
    assert list(mode_numbers(4)) == [0, 1, -2, -1]
    assert list(mode_numbers(5)) == [0, 1, 2, -2, -1]
    for n in range(1, 12):
        m = mode_numbers(n)
        assert sorted(m) == list(range(-(n // 2), n - n // 2))


@pytest.mark.parametrize("Ns", [(8,), (7,), (8, 6), (5, 9), (4, 6, 5), (6, 6, 6)])
def test_type1_on_grid_is_dft(Ns):
    """Points on the uniform grid x = jL/N reduce type-1 to the DFT (App. A)."""
    L = 1.7
    rng = np.random.default_rng(11)
    shp = spectral_shape(Ns)
    cgrid = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    X = _grid_points(Ns, L)
    f = nudft.type1(X, cgrid.ravel(), Ns, L)
    ref = np.fft.fftn(cgrid)
    assert rel_l2(f, ref) < 1e-13


@pytest.mark.parametrize("Ns", [(8,), (8, 6), (4, 6, 5)])
def test_type2_on_grid_is_inverse_dft(Ns):
    L = 0.9
    rng = np.random.default_rng(12)
    shp = spectral_shape(Ns)
    fh = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    X = _grid_points(Ns, L)
    c = nudft.type2(X, fh, Ns, L)
    ref = np.fft.ifftn(fh) * float(np.prod(shp))
    assert rel_l2(c, ref.ravel()) < 1e-13


@pytest.mark.parametrize("Ns", [(6,), (5, 4), (4, 3, 5)])
def test_type1_type2_match_bruteforce(Ns):
    d = len(Ns)
    rng = np.random.default_rng(13)
    M = 9
    L = 2.0
    X = rng.uniform(-3.0, 5.0, (M, d))  # unfolded coordinates: periodicity is part of the sum
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    f = nudft.type1(X, c, Ns, L, scale=0.3)
    assert rel_l2(f, nudft.type1_bruteforce(X, c, Ns, L, scale=0.3)) < 1e-13
    shp = spectral_shape(Ns)
    fh = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    assert rel_l2(nudft.type2(X, fh, Ns, L), nudft.type2_bruteforce(X, fh, Ns, L)) < 1e-13


def test_multi_transform_and_blocking():
    """T > 1 transforms and several point blocks give the same as one at a time."""
    rng = np.random.default_rng(14)
    Ns = (6, 5, 4)
    M = 50
    X = rng.random((M, 3))
    c = rng.standard_normal((2, M)) + 1j * rng.standard_normal((2, M))
    old = nudft._BLOCK_ELEMS
    try:
        nudft._BLOCK_ELEMS = 7 * 30  # blocks of 7 points
        f = nudft.type1(X, c, Ns)
        g = nudft.type2(X, f, Ns)
    finally:
        nudft._BLOCK_ELEMS = old
    for t in range(2):
        assert rel_l2(f[t], nudft.type1_bruteforce(X, c[t], Ns)) < 1e-13
        assert rel_l2(g[t], nudft.type2_bruteforce(X, f[t], Ns)) < 1e-13


@pytest.mark.parametrize("Ns", [(16, 12), (6, 7, 8)])
def test_adjointness(Ns):
    """<type2(v), c> = <v, type1(c)>: spreading and interpolation are adjoint (Sec. 5.4)."""
    d = len(Ns)
    rng = np.random.default_rng(15)
    M = 40
    X = rng.random((M, d))
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    v = rng.standard_normal(spectral_shape(Ns)) + 1j * rng.standard_normal(spectral_shape(Ns))
    lhs = np.vdot(nudft.type2(X, v, Ns), c)
    rhs = np.vdot(v, nudft.type1(X, c, Ns))
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def _dirichlet(x, n_odd, L):
    """sin(n pi x / L) / sin(pi x / L) (eq. FSIB_kern_odd without the 1/L)."""
    s = np.sin(np.pi * x / L)
    return np.where(np.abs(s) < 1e-300, float(n_odd), np.sin(n_odd * np.pi * x / L) / np.where(s == 0, 1, s))


@pytest.mark.parametrize("N", [9, 10, 16])
def test_spread_interp_is_dirichlet_kernel(N):
    """spread then interp of one unit source is L^-d prod_a delta_{L,N'}(x_a - y_a) L (Sec. 4).

    For even N the -N/2 modes are dropped (the symmetric N-1 mode set), for
    odd N all modes are kept; N' is the size of the symmetric set.
    """
    L = 1.3
    d = 2
    Ns = (N, N)
    rng = np.random.default_rng(16)
    y = rng.random((1, d)) * L
    x = rng.random((20, d)) * L
    f = nudft.type1(y, np.ones(1), Ns, L, scale=L ** (-d))
    n_sym = N if N % 2 else N - 1
    if N % 2 == 0:
        for a in range(d):
            m = mode_numbers(N)
            sl = [slice(None)] * d
            sl[d - 1 - a] = np.nonzero(m == -N // 2)[0]
            f[tuple(sl)] = 0.0
    U = nudft.type2(x, f, Ns, L)
    ref = L ** (-d) * np.prod([_dirichlet(x[:, a] - y[0, a], n_sym, L) for a in range(d)], axis=0)
    assert np.max(np.abs(U - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("N", [7, 11])
def test_sinc_kernel_moments_via_oracle(N):
    """Zeroth moment sum_j delta_{L,N}(x - jh) h = 1 and sum of squares = 1/h (Sec. 4), odd N, any x."""
    L = 1.0
    h = L / N
    rng = np.random.default_rng(17)
    xs = rng.random(5)
    grid = (np.arange(N) * h)[:, None]
    for x in xs:
        # delta_{L,N}(x - y_j) = interp at x of spread (scale 1/L) of a unit source at y_j
        vals = np.array([nudft.type2(np.array([[x]]), nudft.type1(grid[j:j + 1], np.ones(1), (N,), L, 1.0 / L),
                                     (N,), L)[0] for j in range(N)])
        assert abs(np.sum(vals) * h - 1.0) < 1e-12
        assert abs(np.sum(np.abs(vals) ** 2) * h - 1.0 / h) < 1e-10 / h


def test_unfolded_coordinates_are_periodic():
    rng = np.random.default_rng(18)
    Ns = (5, 6, 4)
    X = rng.random((7, 3))
    c = rng.standard_normal(7) + 0j
    shift = np.array([3.0, -2.0, 11.0])
    assert rel_l2(nudft.type1(X + shift, c, Ns), nudft.type1(X, c, Ns)) < 1e-13


def test_empty_point_set():
    f = nudft.type1(np.zeros((0, 2)), np.zeros(0, complex), (4, 4))
    assert f.shape == (4, 4) and not np.any(f)
    assert nudft.type2(np.zeros((0, 2)), f, (4, 4)).shape == (0,)


def test_type1_at_modes_matches_bruteforce_and_full():
    rng = np.random.default_rng(19)
    Ns = (5, 4, 6)
    X = rng.uniform(-1, 2, (11, 3))
    c = rng.standard_normal(11) + 1j * rng.standard_normal(11)
    full = nudft.type1(X, c, Ns, 1.3, scale=0.5)
    brute = nudft.type1_bruteforce(X, c, Ns, 1.3, scale=0.5)
    ms = [mode_numbers(n) for n in Ns]
    picks = [(0, 0, 0), (1, 2, 3), (4, 3, 5), (2, 0, 1)]  # FFT-order indices (ix, iy, iz)
    modes = np.array([[ms[0][i], ms[1][j], ms[2][k]] for (i, j, k) in picks])
    got = nudft.type1_at_modes(X, c, modes, 1.3, scale=0.5)
    for q, (i, j, k) in enumerate(picks):
        assert abs(got[q] - brute[k, j, i]) < 1e-13 * np.max(np.abs(brute))
        assert abs(got[q] - full[k, j, i]) < 1e-13 * np.max(np.abs(full))
