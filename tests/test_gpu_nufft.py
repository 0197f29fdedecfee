"""GPU parity of the nonuniform transforms (App. A) against the oracle's direct sums.

Bar: relative l2 error over all outputs <= 1e-10 with the GPU in FP64 (plan tol 1e-11) and
<= 1e-5 with the GPU in FP32 (plan tol 1e-5).  Sizes span several tiles and a ragged number of
points; edge cases cover empty and single-point inputs, points on period boundaries and far
outside the box, all points in one tile, odd N and several transforms per call.
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import nudft
from oracle.modes import spectral_shape
from tests.gpu_helpers import announce, dev, host, rel_l2, cdtype

pytestmark = pytest.mark.gpu

BAR = {"f64": 1e-10, "f32": 1e-5}
TOL = {"f64": 1e-11, "f32": 1e-5}


@pytest.fixture(scope="module")
def fsib():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


CASES = [
    # (dim, Ns, M, seed)
    (2, (32, 32), 1000, 1),
    (2, (17, 24), 777, 2),
    (3, (16, 16, 16), 2000, 3),
    (3, (24, 13, 18), 1501, 4),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dim,Ns,M,seed", CASES)
def test_type1_matches_direct_sum(fsib, prec, dim, Ns, M, seed):
    announce(f"type1 prec={prec} dim={dim} N={Ns} M={M}")
    X, c = workloads.nufft_points(M, seed=seed, dim=dim)
    X = X * 1.3 - 0.2  # L = 1.3, points partly outside [0, L)
    L = 1.3
    ref = nudft.type1(X, c, Ns, L, scale=0.7)
    plan = fsib.Plan(dim, Ns, L=L, prec=prec, tol=TOL[prec], max_points=M)
    out = plan.spread(dev(X), dev(c, cdtype(prec)), scale=0.7)
    err = rel_l2(host(out), ref)
    print(f"type1 {prec} dim={dim} N={Ns} rel_l2={err:.3e} w={plan.info()['w']}")
    assert err < BAR[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dim,Ns,M,seed", CASES)
def test_type2_matches_direct_sum(fsib, prec, dim, Ns, M, seed):
    announce(f"type2 prec={prec} dim={dim} N={Ns} M={M}")
    X, _ = workloads.nufft_points(M, seed=seed, dim=dim)
    f = workloads.random_modes(spectral_shape(Ns), seed + 100)
    ref = nudft.type2(X, f, Ns, 1.0)
    plan = fsib.Plan(dim, Ns, L=1.0, prec=prec, tol=TOL[prec], max_points=M)
    out = plan.interp(dev(X), dev(f, cdtype(prec)))
    err = rel_l2(host(out), ref)
    print(f"type2 {prec} dim={dim} N={Ns} rel_l2={err:.3e}")
    assert err < BAR[prec]


def test_multiple_transforms(fsib):
    announce("ntrans=3 type1/type2 3D f64")
    Ns = (12, 10, 14)
    X, _ = workloads.nufft_points(500, seed=5, dim=3)
    rng = np.random.default_rng(6)
    c = rng.standard_normal((3, 500)) + 1j * rng.standard_normal((3, 500))
    plan = fsib.Plan(3, Ns, prec="f64", tol=1e-11, ntrans=3, max_points=500)
    out = host(plan.spread(dev(X), dev(c)))
    assert rel_l2(out, nudft.type1(X, c, Ns)) < 1e-10
    f = workloads.random_modes(spectral_shape(Ns), 7, ntrans=3)
    back = host(plan.interp(dev(X), dev(f)))
    assert rel_l2(back, nudft.type2(X, f, Ns)) < 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjointness(fsib, prec):
    """<interp(v), c> = <v, spread(c)> to rounding of the plan precision (the kernels are adjoint)."""
    announce(f"adjointness {prec}")
    Ns = (20, 16, 12)
    X, c = workloads.nufft_points(3000, seed=8, dim=3)
    v = workloads.random_modes(spectral_shape(Ns), 9)
    plan = fsib.Plan(3, Ns, prec=prec, tol=1e-6 if prec == "f32" else 1e-9, max_points=3000)
    s = host(plan.spread(dev(X), dev(c, cdtype(prec)))).astype(np.complex128)
    g = host(plan.interp(dev(X), dev(v, cdtype(prec)))).astype(np.complex128)
    lhs, rhs = np.vdot(g, c), np.vdot(v, s)
    bound = 1e-5 if prec == "f32" else 1e-13
    assert abs(lhs - rhs) < bound * np.linalg.norm(g) * np.linalg.norm(c)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_edge_points(fsib, prec):
    """Points at 0, L - ulp, L, -L, 1e6 L, negative, a single point, and an empty set."""
    announce(f"edge points {prec}")
    L = 1.0
    Ns = (16, 16, 16)
    pts = np.array([[0.0, 0.0, 0.0], [np.nextafter(L, 0), 0.5, 0.25], [L, L, L], [-L, 0.3, -0.7],
                    [1e6 * L + 0.125, -3e5 * L, 0.5], [-1e-17, 0.999999999999, 2.5]])
    rng = np.random.default_rng(10)
    c = rng.standard_normal(len(pts)) + 1j * rng.standard_normal(len(pts))
    plan = fsib.Plan(3, Ns, prec=prec, tol=TOL[prec], max_points=64)
    out = host(plan.spread(dev(pts), dev(c, cdtype(prec))))
    assert rel_l2(out, nudft.type1(pts, c, Ns)) < BAR[prec] * 10
    one = host(plan.spread(dev(pts[3:4]), dev(c[3:4], cdtype(prec))))
    assert rel_l2(one, nudft.type1(pts[3:4], c[3:4], Ns)) < BAR[prec] * 10
    empty = host(plan.spread(dev(np.zeros((0, 3))), dev(np.zeros(0, complex), cdtype(prec))))
    assert np.all(empty == 0)
    e2 = host(plan.interp(dev(np.zeros((0, 3))), dev(np.ones(spectral_shape(Ns), complex), cdtype(prec))))
    assert e2.shape == (0,)
    plan.check()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_all_points_in_one_tile(fsib, prec):
    """Maximum contention: every point inside one fine-grid tile."""
    announce(f"one tile {prec}")
    Ns = (32, 32, 32)
    rng = np.random.default_rng(11)
    X = 0.40 + 0.01 * rng.random((4000, 3))
    c = rng.standard_normal(4000) + 1j * rng.standard_normal(4000)
    plan = fsib.Plan(3, Ns, prec=prec, tol=TOL[prec], max_points=4000)
    out = host(plan.spread(dev(X), dev(c, cdtype(prec))))
    assert rel_l2(out, nudft.type1(X, c, Ns)) < BAR[prec]


def test_nonfinite_positions_flagged(fsib):
    announce("non-finite positions")
    Ns = (8, 8)
    X = np.array([[0.1, 0.2], [np.nan, 0.5], [0.3, np.inf]])
    plan = fsib.Plan(2, Ns, prec="f64", tol=1e-8, max_points=8)
    plan.spread(dev(X), dev(np.ones(3, complex)))
    with pytest.raises(fsib.FSIBError) as ei:
        plan.check()
    assert ei.value.status == 6
    plan.check()  # flag cleared


def test_too_many_points_rejected(fsib):
    plan = fsib.Plan(2, (8, 8), prec="f64", tol=1e-8, max_points=4)
    with pytest.raises(fsib.FSIBError) as ei:
        plan.spread(dev(np.zeros((5, 2))), dev(np.ones(5, complex)))
    assert ei.value.status == 1
