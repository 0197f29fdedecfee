"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module holds geometry and random draws only -- none of the method's
arithmetic.  Both the HIP path and the CPU oracle receive the arrays it
returns.  All draws use numpy's PCG64 ``default_rng(seed)`` in a fixed order.

Workloads (L = 1 throughout):

* ``ellipse_2d``      closed curve X_j = c + (a cos th_j, b sin th_j), th_j = 2 pi j / M.
* ``latlong_sphere``  triangulated sphere (rings x longitudes, polar fans),
                      counter-clockwise seen from outside.
* ``icosphere``       icosahedral sphere refined by 4-splits (10 4^level + 2 vertices).
* ``stokes2d_case``   2D Stokes ellipse, N = 32^2, M = 128, centre drawn from seed 1.
* ``ns3d_case``       3D Navier-Stokes ellipsoid, N = 128^3, lat-long 200 x 200 = 40,000 points.
* ``diff_stokes3d_case`` differentiable 3D Stokes, N = 64^3, lat-long 100 x 100 = 10,000 points,
                      20 steps, target ellipsoid with semi-axes drawn from seed 5.
* ``nufft_points``    half uniform in the unit torus, half on a sphere of radius 0.2
                      (the NUFFT micro-benchmark point law), complex N(0,1) strengths.
"""

import numpy as np


def ellipse_2d(M, center=(0.5, 0.5), a=0.3, b=0.2, rotation=0.0):
    th = 2.0 * np.pi * np.arange(M) / M
    x = a * np.cos(th)
    y = b * np.sin(th)
    cr, sr = np.cos(rotation), np.sin(rotation)
    X = np.stack([center[0] + cr * x - sr * y, center[1] + sr * x + cr * y], axis=1)
    return X.astype(np.float64)


def circle_2d(M, center=(0.5, 0.5), r=0.125):
    return ellipse_2d(M, center, r, r)


def latlong_sphere(n_rings, n_lon, radius=1.0, center=(0.0, 0.0, 0.0), scale=(1.0, 1.0, 1.0)):
    """Lat-long triangulated sphere.

    Rings at polar angle th_i = pi (i + 1/2) / n_rings, longitudes ph_j = 2 pi j / n_lon;
    vertex index i * n_lon + j.  Each quad between rings i, i+1 splits along the
    (i,j)-(i+1,j+1) diagonal; each polar ring is closed by a fan from its vertex 0.
    Triangles are counter-clockwise seen from outside.  Returns (X (M,3) float64, tris (T,3) int32).
    """
    R, P = int(n_rings), int(n_lon)
    th = np.pi * (np.arange(R) + 0.5) / R
    ph = 2.0 * np.pi * np.arange(P) / P
    st, ct = np.sin(th)[:, None], np.cos(th)[:, None]
    Xu = np.stack([(st * np.cos(ph)[None, :]).ravel(),
                   (st * np.sin(ph)[None, :]).ravel(),
                   np.broadcast_to(ct, (R, P)).ravel()], axis=1)
    X = np.asarray(center, dtype=np.float64)[None, :] + radius * Xu * np.asarray(scale, dtype=np.float64)[None, :]

    def v(i, j):
        return i * P + (j % P)

    tris = []
    for i in range(R - 1):
        for j in range(P):
            tris.append((v(i, j), v(i + 1, j), v(i + 1, j + 1)))
            tris.append((v(i, j), v(i + 1, j + 1), v(i, j + 1)))
    for j in range(1, P - 1):
        tris.append((v(0, 0), v(0, j), v(0, j + 1)))
    for j in range(1, P - 1):
        tris.append((v(R - 1, 0), v(R - 1, j + 1), v(R - 1, j)))
    return X, np.asarray(tris, dtype=np.int32)


def vertex_triangle_csr(tris, M):
    """Vertex -> incident-triangle lists in CSR form (ptr (M+1,), idx (3T,)), int32, sorted by triangle."""
    tris = np.asarray(tris, dtype=np.int64)
    verts = tris.ravel()
    tid = np.repeat(np.arange(tris.shape[0]), 3)
    order = np.lexsort((tid, verts))
    counts = np.bincount(verts, minlength=M)
    ptr = np.zeros(M + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(counts)
    return ptr.astype(np.int32), tid[order].astype(np.int32)


def icosphere(level, radius=1.0, center=(0.0, 0.0, 0.0)):
    """Icosahedral sphere (Sec. 6.2.3): the regular icosahedron refined `level` times, each triangle
    split into four through its edge midpoints, which are pushed out to the sphere.  10 4^level + 2
    vertices, triangles counter-clockwise seen from outside.  Returns (X (M,3) float64, tris int32)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(int(level)):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                mid[key] = len(V) - 1
            return mid[key]

        G = []
        for a, b, c in F:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            G += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = G
    X = np.asarray(center, dtype=np.float64)[None, :] + radius * np.array(V)
    return X, np.asarray(F, dtype=np.int32)


def vertex_neighbor_csr(tris, M):
    """Vertex -> linked-vertex lists (the mesh edges, both directions) in CSR form, int32, sorted."""
    tris = np.asarray(tris, dtype=np.int64)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.unique(np.concatenate([e, e[:, ::-1]]), axis=0)  # sorted by (i, j)
    counts = np.bincount(e[:, 0], minlength=M)
    ptr = np.zeros(M + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(counts)
    return ptr.astype(np.int32), e[:, 1].astype(np.int32)


def stokes2d_case(seed=1, M=128, N=32):
    """2D Stokes ellipse: semi-axes 0.3/0.2 about a seeded random centre; K = 1, mu = 1, dt = 1e-3."""
    rng = np.random.default_rng(seed)
    c = rng.random(2)
    return dict(X=ellipse_2d(M, center=c), N=(N, N), L=1.0, K=1.0, mu=1.0, rho=1.0, dt=1e-3,
                force="tension2d")


def batched_stokes2d(count=64, seed=4, sizes=(64, 128, 256, 512), m_range=(256, 8192)):
    """Independent 2D Stokes instances: N_i from `sizes`, M_i log-uniform in m_range, ellipses of
    semi-major axis 0.3 and aspect ratio U[1, 3] with a random centre and rotation; K = 1, mu = 1,
    dt = 1e-3.  Draw order per instance: N, M, aspect, centre (2), rotation."""
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        m = int(np.floor(np.exp(rng.uniform(np.log(m_range[0]), np.log(m_range[1])))))
        aspect = rng.uniform(1.0, 3.0)
        c = rng.random(2)
        rot = rng.uniform(0.0, np.pi)
        X = ellipse_2d(m, center=c, a=0.3, b=0.3 / aspect, rotation=rot)
        cases.append(dict(X=X, N=(n, n), L=1.0, K=1.0, mu=1.0, dt=1e-3, force="tension2d"))
    return cases


def ns3d_case(n_rings=200, n_lon=200, N=128):
    """3D Navier-Stokes: sphere of radius 0.25 stretched by (1.2, 1, 0.8) about (1/2,1/2,1/2);
    surface tension K = 1, rho = 1, mu = 0.01, dt = 5e-4, uhat^0 = 0."""
    X, tris = latlong_sphere(n_rings, n_lon, radius=0.25, center=(0.5, 0.5, 0.5), scale=(1.2, 1.0, 0.8))
    return dict(X=X, tris=tris, N=(N, N, N), L=1.0, K=1.0, mu=0.01, rho=1.0, dt=5e-4,
                force="surface3d")


def diff_stokes3d_case(seed=5, n_rings=100, n_lon=100, N=64, steps=20):
    """Differentiable 3D Stokes: lat-long sphere of radius 0.25 about (1/2,1/2,1/2), surface tension
    K = 1, mu = 1, dt = 1e-3, `steps` steps; target = the same vertices on an ellipsoid with semi-axes
    drawn U[0.2, 0.3] (three draws), i.e. c + axes * (X0 - c) / 0.25."""
    rng = np.random.default_rng(seed)
    axes = rng.uniform(0.2, 0.3, 3)
    c = np.array([0.5, 0.5, 0.5])
    X, tris = latlong_sphere(n_rings, n_lon, radius=0.25, center=tuple(c))
    target = c[None, :] + axes[None, :] * (X - c[None, :]) / 0.25
    return dict(X=X, tris=tris, target=target, axes=axes, N=(N, N, N), L=1.0, K=1.0, mu=1.0, dt=1e-3,
                steps=steps, force="surface3d")


def nufft_points(M, seed=3, dim=3, cluster_radius=0.2):
    """Half uniform in [0,1)^dim, half on a sphere of radius 0.2 about the centre; shuffled.

    Returns (X (M,dim) float64, c (M,) complex128 with N(0,1) real and imaginary parts).
    """
    rng = np.random.default_rng(seed)
    h = M // 2
    X = np.empty((M, dim))
    X[:h] = rng.random((h, dim))
    g = rng.standard_normal((M - h, dim))
    X[h:] = 0.5 + cluster_radius * g / np.linalg.norm(g, axis=1)[:, None]
    X = X[rng.permutation(M)]
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    return X, c


def random_modes(shape, seed, ntrans=None):
    """Complex N(0,1) Fourier coefficients of the given spectral shape."""
    rng = np.random.default_rng(seed)
    full = shape if ntrans is None else (ntrans,) + tuple(shape)
    return rng.standard_normal(full) + 1j * rng.standard_normal(full)


def random_points(M, dim, seed, lo=0.0, hi=1.0):
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.random((M, dim))
