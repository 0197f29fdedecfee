"""Batched independent 2D Stokes simulations captured in one HIP graph.

Every replay of the captured graph is checked against the same batch stepped eagerly (with eager
work and synchronisations between the replays), and the final states against the CPU oracle's
Stokes steps (eq. stokeslet with the midpoint update of eqs. spatial_1 and spatial_4).
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import step
from tests.gpu_helpers import announce, host, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


def _oracle(cases, steps):
    out = []
    for c in cases:
        law = step.ForceLaw("tension2d", c["K"])
        X = c["X"].copy()
        U, _ = step.stokes_velocity(X, law, c["N"], 1.0, c["mu"])
        for _ in range(steps):
            X, U, _ = step.stokes_step(X, U, law, c["N"], 1.0, c["mu"], c["dt"])
        out.append((X, U))
    return out


@pytest.mark.parametrize("prec,tol,bar", [("f64", 1e-11, 1e-10), ("f32", 1e-5, 3e-5)])
def test_batched_stokes_graph_replays(F, prec, tol, bar):
    from paper_2302_08694_amd.batch import StokesBatch
    announce(f"batched 2D Stokes graph {prec}")
    cases = workloads.batched_stokes2d(count=4, seed=4, sizes=(16, 24, 32), m_range=(48, 160))
    eager = StokesBatch(cases, prec=prec, tol=tol)
    snaps = []
    for _ in range(2):
        eager.step(2)
        torch.cuda.synchronize()
        snaps.append([(host(it["X"]), host(it["U"])) for it in eager.items])
    gb = StokesBatch(cases, prec=prec, tol=tol)
    gb.capture(2)
    for r in range(2):
        gb.replay()
        torch.cuda.synchronize()
        # the same kernels as the eager steps; the order of points inside a bin comes from atomics,
        # so sums may differ in the last bits (FP32: ~1e-7 relative)
        rep = 1e-12 if prec == "f64" else 1e-6
        for it, (Xe, Ue) in zip(gb.items, snaps[r]):
            X0 = it["X0"].cpu().numpy()
            assert rel_l2(host(it["X"]) - X0, Xe - X0) < rep
            assert rel_l2(host(it["U"]), Ue) < rep
        # eager work of the program between replays
        junk = torch.randn(1 << 16, device="cuda")
        float(junk.abs().sum().item())
        torch.cuda.synchronize()
    refs = _oracle(cases, 4)
    for it, c, (Xo, Uo) in zip(gb.items, cases, refs):
        ex = rel_l2(host(it["X"]) - c["X"], Xo - c["X"])
        eu = rel_l2(host(it["U"]), Uo)
        print(f"batch {prec} N={c['N']} M={it['M']}: dX {ex:.2e} U {eu:.2e}")
        assert max(ex, eu) < bar
    eager.close()
    gb.close()
