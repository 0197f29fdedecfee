"""Spreading variants of 2D plans (tuning knob spread_threads: 64, 128 or 256 threads per 16 x 16 tile,
i.e. 4, 2 or 1 cells per lane) and their autotuning.

Each cell of a tile is summed by one lane in the order of the sorted points whatever the variant, so
on a deterministic plan (fixed order inside every bin) the three variants give bitwise equal type-1
sums (App. A, eqs. type1_conv and type1_deco), for complex strengths and for the real force spreading
of a fluid plan; the results also match the oracle's direct sums to the plan's tolerance.  Heavy tiles
(crowded points split over several workgroups) are included.  The knob is refused outside its values
and on 3D plans, and the autotuner leaves one of the variants set.
"""

import numpy as np
import pytest

import workloads
from oracle import nudft
from tests.gpu_helpers import announce, cdtype, dev, host, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


def _points(M, seed):
    rng = np.random.default_rng(seed)
    # half uniform, half crowded near one point (heavy tiles that split)
    X = np.concatenate([rng.random((M // 2, 2)), 0.3 + 0.01 * rng.random((M - M // 2, 2))])
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    return X, c


@pytest.mark.parametrize("prec,tol,bar", [("f64", 1e-10, 1e-9), ("f32", 1e-5, 1e-4)])
def test_variants_bitwise_equal(F, prec, tol, bar):
    announce(f"2D spreading variants {prec}")
    Ns = (48, 40)
    X, c = _points(6000, 71)
    plan = F.Plan(2, Ns, prec=prec, tol=tol, max_points=X.shape[0], deterministic=True)
    Xd, cd = dev(X), dev(c, cdtype(prec))
    base = plan.tuning()
    outs = {}
    for nt in (64, 128, 256):
        plan.tuning(**{**base, "spread_threads": nt})
        outs[nt] = host(plan.spread(Xd, cd))
    for nt in (128, 256):
        assert np.array_equal(outs[nt].view(np.uint8), outs[64].view(np.uint8)), nt
    ref = nudft.type1(X, c, Ns)
    err = rel_l2(outs[64], ref)
    print(f"2D spread variants {prec}: bitwise equal, rel_l2 vs oracle {err:.2e}")
    assert err < bar
    plan.close()


def test_variants_fluid_force_spread(F):
    announce("2D spreading variants, real force spreading of a fluid plan")
    case = workloads.stokes2d_case(M=400, N=48)
    X = dev(case["X"])
    S = dev(np.random.default_rng(72).standard_normal((400, 2)))
    plan = F.Plan(2, case["N"], prec="f64", tol=1e-10, max_points=400, fluid=True, deterministic=True)
    base = plan.tuning()
    outs = []
    for nt in (64, 128, 256):
        plan.tuning(**{**base, "spread_threads": nt})
        outs.append(host(plan.force_spread(X, S, scale=1.0)))
    for o in outs[1:]:
        assert np.array_equal(o.view(np.uint8), outs[0].view(np.uint8))
    plan.close()


def test_variant_knob_checks_and_autotune(F):
    from paper_2302_08694_amd.tune import autotune
    announce("spread_threads knob checks and autotune")
    p2 = F.Plan(2, (32, 32), prec="f32", tol=1e-5, max_points=2000)
    p3 = F.Plan(3, (16, 16, 16), prec="f32", tol=1e-5, max_points=2000)
    with pytest.raises(F.FSIBError):
        p2.tuning(spread_threads=32)
    with pytest.raises(F.FSIBError):
        p3.tuning(spread_threads=128)
    p3.tuning(spread_threads=256)
    X, c = _points(2000, 73)
    Xd, cd = dev(X), dev(c, cdtype("f32"))
    res = autotune(p2, lambda: p2.spread(Xd, cd), reps=1)
    assert res["best"]["spread_threads"] in (0, 64, 128, 256)
    assert res["best"] == p2.tuning()
    tried = {t[0]["spread_threads"] for t in res["trials"]}
    assert {64, 128, 256} <= tried
    print(f"autotune chose {res['best']}")
    p2.close()
    p3.close()
