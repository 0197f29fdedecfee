"""fsib_spread_noalloc (type-1 through the library's static per-GPU scratch, App. A eq. type1) against
fsib_spread on the same plan and inputs: two calls in a row, the second with fewer points, each
compared with the plan's own fsib_spread (bitwise on a deterministic plan; to rounding on the default
plan) and with the oracle's direct sums; point counts beyond max_points within the scratch; and the
clear refusal of a transform too large for the scratch."""

import ctypes

import numpy as np
import pytest
import torch

import workloads
from oracle import nudft
from tests.gpu_helpers import announce, cdtype, dev, host, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


@pytest.mark.parametrize("prec,deterministic", [("f64", True), ("f32", True), ("f64", False)])
def test_noalloc_matches_spread(F, prec, deterministic):
    announce(f"fsib_spread_noalloc vs fsib_spread {prec} deterministic={deterministic}")
    Ns = (20, 16, 24)
    tol = 1e-10 if prec == "f64" else 1e-5
    plan = F.Plan(3, Ns, prec=prec, tol=tol, max_points=6000, deterministic=deterministic)
    for M, seed in ((6000, 71), (1733, 72)):  # the second call smaller than the first
        X, c = workloads.nufft_points(M, seed=seed, dim=3)
        X[:10] += 3.0  # positions outside [0, 1) fold
        Xd, cd = dev(X), dev(c, cdtype(prec))
        ref = host(plan.spread(Xd, cd))
        out = torch.full(tuple(reversed(Ns)), float("nan"), dtype=cdtype(prec), device="cuda")
        got = host(plan.spread_noalloc(Xd, cd, out))
        if deterministic:
            assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
        else:
            assert rel_l2(got, ref) < (1e-14 if prec == "f64" else 1e-6)
        assert rel_l2(got, nudft.type1(X, c, Ns)) < (1e-9 if prec == "f64" else 1e-5)
    plan.close()


def test_noalloc_beyond_max_points_and_2d(F):
    announce("fsib_spread_noalloc beyond max_points, 2D, ntrans 2")
    Ns = (40, 36)
    plan = F.Plan(2, Ns, prec="f64", tol=1e-9, ntrans=2, max_points=16, deterministic=True)
    X, c1 = workloads.nufft_points(5000, seed=73, dim=2)
    c = np.stack([c1, np.conj(c1) * 0.5j])
    out = torch.zeros((2,) + tuple(reversed(Ns)), dtype=torch.complex128, device="cuda")
    got = host(plan.spread_noalloc(dev(X), dev(c), out, scale=0.25))
    assert rel_l2(got, nudft.type1(X, c, Ns, scale=0.25)) < 1e-8
    with pytest.raises(F.FSIBError):  # the plan's own entry point keeps its max_points
        plan.spread(dev(X), dev(c))
    plan.close()


def test_noalloc_refuses_oversize(F):
    announce("fsib_spread_noalloc refuses a transform beyond the scratch")
    from paper_2302_08694_amd import _binding as B
    lib = B.load_library()
    plan = F.Plan(3, (128, 128, 128), prec="f64", tol=1e-6, max_points=8, upsampfac=2.0)  # 256^3 grid: 268 MB
    X = torch.rand((8, 3), dtype=torch.float64, device="cuda")
    c = torch.ones(8, dtype=torch.complex128, device="cuda")
    out = torch.zeros((128, 128, 128), dtype=torch.complex128, device="cuda")
    st = lib.fsib_spread_noalloc(plan._h, 8, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), 1.0, None)
    assert st == 1
    assert b"bytes of scratch" in lib.fsib_last_error()
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0  # nothing was enqueued
    fl = F.Plan(3, (16, 16, 16), prec="f64", tol=1e-6, max_points=8, fluid=True)
    st = lib.fsib_spread_noalloc(fl._h, 8, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), 1.0, None)
    assert st == 7
    plan.close()
    fl.close()
