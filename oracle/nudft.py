"""Direct nonuniform Fourier sums (type-1 and type-2) -- oracle side.

Test infrastructure only (see the package docstring).

type1:  fhat(k) = scale * sum_j c_j exp(-i k.x_j),  k in K_N      (App. A, eq. type1)
type2:  c_j     = sum_{k in K_N} fhat(k) exp(+i k.x_j)             (App. A, eq. type2)

With scale = L^-d and c_j = w_j F_j, type1 is the FSIB force spreading
(Sec. 3.1, eq. force_spreading_quad); type2 of the velocity coefficients is the
velocity interpolation (eq. velo_intp_fini).

The sums are evaluated exactly (to rounding): per-axis phase tables
E_a[j, m] = exp(-+ i 2 pi m x_{j,a} / L) built by direct cos/sin in FP64, and
the tensor-product sum contracted with a complex matrix product over blocks of
points.  No grid, no kernel, no FFT.  ``*_bruteforce`` are pure loops for tiny
inputs that form every phase exp(-i k.x_j) in one piece.
"""

import numpy as np

from .modes import mode_numbers, spectral_shape

_BLOCK_ELEMS = 1 << 24  # complex entries per block of the tensor-product table


def _phase_table(x, N, L, sign):
    """E[j, i] = exp(sign * i * 2*pi*m_i*x_j/L) for the FFT-ordered modes m_i of K_N."""
    m = mode_numbers(N).astype(np.float64)
    xf = np.mod(np.asarray(x, dtype=np.float64), L) / L  # periodicity; exact in exact arithmetic
    ang = (2.0 * np.pi) * np.outer(xf, m)
    return np.cos(ang) + (1j * sign) * np.sin(ang)


def _as_trans(c, M):
    c = np.asarray(c, dtype=np.complex128)
    single = c.ndim == 1
    c = c.reshape(1, M) if single else c.reshape(c.shape[0], M)
    return c, single


def type1(X, c, Ns, L=1.0, scale=1.0):
    """Type-1 sum fhat(k) = scale * sum_j c_j exp(-i k.x_j) over k in K_N.

    X: (M, d) real positions (any real values; the sum is L-periodic in x).
    c: (M,) or (T, M) complex strengths.
    Ns: per-axis mode counts (N_x, N_y[, N_z]).
    Returns (spectral_shape) or (T, spectral_shape) complex128, FFT order, x fastest.
    """
    X = np.asarray(X, dtype=np.float64)
    M, d = X.shape
    assert d == len(Ns)
    c, single = _as_trans(c, M)
    T = c.shape[0]
    shp = spectral_shape(Ns)
    out = np.zeros((T,) + shp, dtype=np.complex128)
    if M > 0:
        if d == 1:
            E0 = _phase_table(X[:, 0], Ns[0], L, -1.0)
            out[:] = c @ E0
        elif d == 2:
            E0 = _phase_table(X[:, 0], Ns[0], L, -1.0)
            E1 = _phase_table(X[:, 1], Ns[1], L, -1.0)
            for t in range(T):
                out[t] = E1.T @ (c[t][:, None] * E0)
        elif d == 3:
            n0, n1, n2 = (int(n) for n in Ns)
            blk = max(1, _BLOCK_ELEMS // max(1, n1 * n2))
            flat = out.reshape(T, n2 * n1, n0)
            for j0 in range(0, M, blk):
                j1 = min(M, j0 + blk)
                E0 = _phase_table(X[j0:j1, 0], n0, L, -1.0)
                E1 = _phase_table(X[j0:j1, 1], n1, L, -1.0)
                E2 = _phase_table(X[j0:j1, 2], n2, L, -1.0)
                A = (E2[:, :, None] * E1[:, None, :]).reshape(j1 - j0, n2 * n1)
                for t in range(T):
                    flat[t] += A.T @ (c[t, j0:j1][:, None] * E0)
        else:
            raise ValueError("dimension must be 1, 2 or 3")
    out *= scale
    return out[0] if single else out


def type2(X, fhat, Ns, L=1.0):
    """Type-2 sum c_j = sum_{k in K_N} fhat(k) exp(+i k.x_j).

    fhat: (spectral_shape) or (T, spectral_shape) complex, FFT order.
    Returns (M,) or (T, M) complex128.
    """
    X = np.asarray(X, dtype=np.float64)
    M, d = X.shape
    assert d == len(Ns)
    shp = spectral_shape(Ns)
    f = np.asarray(fhat, dtype=np.complex128)
    single = f.shape == shp
    f = f.reshape((-1,) + shp)
    T = f.shape[0]
    out = np.zeros((T, M), dtype=np.complex128)
    if M == 0:
        return out[0] if single else out
    if d == 1:
        F0 = _phase_table(X[:, 0], Ns[0], L, +1.0)
        out[:] = f @ F0.T
    elif d == 2:
        F0 = _phase_table(X[:, 0], Ns[0], L, +1.0)
        F1 = _phase_table(X[:, 1], Ns[1], L, +1.0)
        for t in range(T):
            G = f[t] @ F0.T  # (N_y, M): sum over m_x
            out[t] = np.sum(F1 * G.T, axis=1)
    elif d == 3:
        n0, n1, n2 = (int(n) for n in Ns)
        blk = max(1, _BLOCK_ELEMS // max(1, n1 * n2))
        for j0 in range(0, M, blk):
            j1 = min(M, j0 + blk)
            F0 = _phase_table(X[j0:j1, 0], n0, L, +1.0)
            F1 = _phase_table(X[j0:j1, 1], n1, L, +1.0)
            F2 = _phase_table(X[j0:j1, 2], n2, L, +1.0)
            A = (F2[:, :, None] * F1[:, None, :]).reshape(j1 - j0, n2 * n1)
            for t in range(T):
                G = f[t].reshape(n2 * n1, n0) @ F0.T  # (N_z*N_y, block): sum over m_x
                out[t, j0:j1] = np.sum(A * G.T, axis=1)
    else:
        raise ValueError("dimension must be 1, 2 or 3")
    return out[0] if single else out


def type1_at_modes(X, c, modes, L=1.0, scale=1.0):
    """Type-1 sum at selected integer mode vectors: out[q] = scale * sum_j c_j exp(-i 2 pi m_q.x_j / L).

    modes: (K, d) integers in physical-axis order.  Direct sum, one phase per (point, mode); for
    checking sampled outputs of a transform too large to evaluate in full.
    """
    X = np.asarray(X, dtype=np.float64)
    m = np.asarray(modes, dtype=np.float64)
    xf = np.mod(X, L) / L
    out = np.zeros(m.shape[0], dtype=np.complex128)
    c = np.asarray(c, dtype=np.complex128)
    blk = max(1, _BLOCK_ELEMS // max(1, m.shape[0]))
    for j0 in range(0, X.shape[0], blk):
        ang = (2.0 * np.pi) * (xf[j0:j0 + blk] @ m.T)
        out += c[j0:j0 + blk] @ (np.cos(ang) - 1j * np.sin(ang))
    return scale * out


def _all_wavevectors(Ns, L):
    """(n_modes, d) array of k = 2*pi*m/L for every mode of K_N, in C order of spectral_shape."""
    d = len(Ns)
    grids = np.meshgrid(*[mode_numbers(Ns[d - 1 - a]) for a in range(d)], indexing="ij")
    # grids[b] varies along numpy axis b, which is physical axis d-1-b
    m = np.stack([grids[d - 1 - a].ravel() for a in range(d)], axis=1).astype(np.float64)
    return (2.0 * np.pi / L) * m


def type1_bruteforce(X, c, Ns, L=1.0, scale=1.0):
    """Loop over points and modes; each phase exp(-i k.x_j) formed in one piece (tiny inputs only)."""
    X = np.asarray(X, dtype=np.float64)
    c = np.asarray(c, dtype=np.complex128)
    K = _all_wavevectors(Ns, L)
    out = np.zeros(K.shape[0], dtype=np.complex128)
    for j in range(X.shape[0]):
        for q in range(K.shape[0]):
            out[q] += c[j] * np.exp(-1j * float(np.dot(K[q], X[j])))
    return scale * out.reshape(spectral_shape(Ns))


def type2_bruteforce(X, fhat, Ns, L=1.0):
    """Loop over points and modes (tiny inputs only)."""
    X = np.asarray(X, dtype=np.float64)
    f = np.asarray(fhat, dtype=np.complex128).ravel()
    K = _all_wavevectors(Ns, L)
    out = np.zeros(X.shape[0], dtype=np.complex128)
    for j in range(X.shape[0]):
        acc = 0j
        for q in range(K.shape[0]):
            acc += f[q] * np.exp(1j * float(np.dot(K[q], X[j])))
        out[j] = acc
    return out


# ---- gradients of the sums (for the adjoint of the transforms) ----
#
# Convention: for a real loss L and complex arrays, the gradient is dL/dRe + i dL/dIm (the
# conjugate-Wirtinger convention of torch.autograd); positions are real.  For a linear map the
# gradient of the input is the adjoint applied to the gradient of the output.


def _ik_weighted(f, Ns, L, axis):
    """i k_axis f(k) on the FFT-ordered spectrum (physical axis `axis`)."""
    shp = spectral_shape(Ns)
    d = len(Ns)
    k = (2.0 * np.pi / L) * mode_numbers(Ns[axis]).astype(np.float64)
    bshape = [1] * d
    bshape[d - 1 - axis] = Ns[axis]
    f = np.asarray(f, dtype=np.complex128)
    return f * (1j * k.reshape(bshape)) if f.shape == shp else f * (1j * k.reshape([1] + bshape))


def type1_grad(X, c, g, Ns, L=1.0, scale=1.0):
    """Gradients of type1 given the output gradient g (same shape as the output).

    grad_c_j = scale * sum_k g(k) exp(+i k.x_j)                        (the adjoint: a type-2 sum)
    grad_X[j, a] = Re( scale * c_j * conj( sum_k i k_a g(k) exp(+i k.x_j) ) )
    (the phase derivative d/dx_a exp(-i k.x) = -i k_a exp(-i k.x)).
    """
    X = np.asarray(X, dtype=np.float64)
    M, d = X.shape
    c, single = _as_trans(c, M)
    g = np.asarray(g, dtype=np.complex128).reshape((c.shape[0],) + spectral_shape(Ns))
    gc = scale * type2(X, g, Ns, L)
    gX = np.zeros((M, d))
    for a in range(d):
        h = type2(X, _ik_weighted(g, Ns, L, a), Ns, L)
        gX[:, a] = np.sum(np.real(scale * c * np.conj(h)), axis=0)
    return (gc[0] if single else gc), gX


def type2_grad(X, fhat, g, Ns, L=1.0):
    """Gradients of type2 given the output gradient g ((M,) or (T, M)).

    grad_fhat(k) = sum_j g_j exp(-i k.x_j)                             (the adjoint: a type-1 sum)
    grad_X[j, a] = Re( conj(g_j) * sum_k i k_a fhat(k) exp(+i k.x_j) )
    """
    X = np.asarray(X, dtype=np.float64)
    M, d = X.shape
    g, single = _as_trans(g, M)
    f = np.asarray(fhat, dtype=np.complex128).reshape((g.shape[0],) + spectral_shape(Ns))
    gf = type1(X, g, Ns, L)
    gX = np.zeros((M, d))
    for a in range(d):
        dv = type2(X, _ik_weighted(f, Ns, L, a), Ns, L)
        gX[:, a] = np.sum(np.real(np.conj(g) * dv), axis=0)
    return (gf[0] if single else gf), gX
