"""Type-2 interpolation of point sets mixing a tight cluster (one or two crowded tiles, so
consecutive sorted points share most of their cells) with sparse uniform points partly outside
[0, 1), against the oracle's direct sums: complex transforms (ntrans = 2) and the real velocity
channels of the fluid path."""

import numpy as np
import pytest

from oracle import nudft
from oracle.modes import spectral_shape
from oracle.step import interp_velocity
from tests.gpu_helpers import announce, dev, host, half, rel_l2, cdtype, rdtype

pytestmark = pytest.mark.gpu

BAR = {"f64": 1e-10, "f32": 1e-5}
TOL = {"f64": 1e-11, "f32": 1e-5}


@pytest.fixture(scope="module")
def fsib():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


def _points(M, dim, seed):
    rng = np.random.default_rng(seed)
    h = M // 2
    X = np.empty((M, dim))
    X[:h] = 0.31 + 0.02 * rng.random((h, dim))  # a cluster inside a tile or two
    X[h:] = rng.uniform(-0.3, 1.3, (M - h, dim))  # sparse, partly outside [0, 1)
    return X[rng.permutation(M)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dim,Ns,M", [(2, (40, 36), 901), (3, (20, 18, 22), 1203)])
def test_type2_cluster_and_sparse(fsib, prec, dim, Ns, M):
    announce(f"interp cluster+sparse type2 {prec} dim={dim} N={Ns}")
    X = _points(M, dim, 81 + dim)
    f = np.stack([np.random.default_rng(90 + t).standard_normal(spectral_shape(Ns)) +
                  1j * np.random.default_rng(95 + t).standard_normal(spectral_shape(Ns)) for t in range(2)])
    plan = fsib.Plan(dim, Ns, prec=prec, tol=TOL[prec], ntrans=2, max_points=M)
    out = host(plan.interp(dev(X), dev(f, cdtype(prec))))
    ref = np.stack([nudft.type2(X, f[t], Ns, 1.0) for t in range(2)])
    err = rel_l2(out, ref)
    print(f"type2 cluster+sparse {prec} dim={dim}: {err:.2e}")
    assert err < BAR[prec]
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dim,Ns,M", [(2, (32, 32), 700), (3, (16, 20, 16), 1100)])
def test_velocity_interp_cluster_and_sparse(fsib, prec, dim, Ns, M):
    announce(f"interp cluster+sparse velocity {prec} dim={dim} N={Ns}")
    X = _points(M, dim, 83 + dim)
    rng = np.random.default_rng(97)
    uhat = np.fft.fftn(rng.standard_normal((dim,) + tuple(reversed(Ns))), axes=tuple(range(1, dim + 1)))
    uhat /= np.prod(Ns)
    # a real field's spectrum with the -N/2 modes zeroed (the fluid path's velocity)
    for a in range(dim):
        n = Ns[a]
        if n % 2 == 0:
            sl = [slice(None)] * (dim + 1)
            sl[dim - a] = n // 2
            uhat[tuple(sl)] = 0.0
    plan = fsib.Plan(dim, Ns, prec=prec, tol=TOL[prec], max_points=M, fluid=True)
    out = host(plan.velocity_interp(dev(X), dev(half(uhat, Ns[0]), cdtype(prec))))
    ref = interp_velocity(X, uhat, Ns, 1.0)
    err = rel_l2(out, ref)
    print(f"velocity cluster+sparse {prec} dim={dim}: {err:.2e}")
    assert err < BAR[prec]
    plan.close()
