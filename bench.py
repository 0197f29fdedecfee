"""FSIB hot-path benchmark on one MI355X.

Workload: 3D Navier-Stokes FSIB, N = 128^3 Fourier modes, M = 40,000 surface points (lat-long
200 x 200 sphere of radius 0.25 stretched to an ellipsoid 0.3/0.25/0.2), surface tension K = 1,
rho = 1, mu = 0.01, dt = 5e-4, uhat^0 = 0.  One step = one Alg. 1 step (fsib_step): force,
type-1 spread, two dealiased Fourier updates, two type-2 interpolations, the position updates.
Inputs are synthetic and resident on the device before timing starts.

    python bench.py [--gpus 1] [--steps 100] [--warmup 5] [--no-cpu-baseline]

Prints one JSON line: FSIB steps/s in FP64 at NUFFT tolerance 1e-5 (value), with the FP32 form,
the NUFFT spread+interp points/s at 128^3, the NUFFT micro-benchmark (256^3, 2e6 points), the
batched 2D Stokes form (64 uneven instances, HIP graph), the differentiable 3D Stokes form (64^3,
10,000 points, 20 checkpointed steps), the roofline of the dominant kernel and the CPU oracle
timed on the host.
"""

import argparse
import json
import os
import sys
import time

import numpy as np


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--upsampfac", type=float, default=0.0,
                    help="fine-grid oversampling of the FP64 and FP32 step plans (0: the plan's automatic choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=128, help="modes per axis")
    ap.add_argument("--rings", type=int, default=200)
    ap.add_argument("--fp64-only", action="store_true", help="skip the FP32 form and the NUFFT timings")
    ap.add_argument("--no-nufft-micro", action="store_true", help="skip the NUFFT micro-benchmark legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 2D Stokes leg")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiable 3D Stokes leg")
    ap.add_argument("--no-lowmem", action="store_true", help="skip the low-memory (oversampling 1.25) leg")
    ap.add_argument("--nufft-only", action="store_true", help="run only the NUFFT micro-benchmark legs")
    ap.add_argument("--nufft-case", default=None,
                    help="with --nufft-only: one case N:M:prec:tol (e.g. 256:2000000:f32:1e-5) instead of all")
    ap.add_argument("--nufft-reps", type=int, default=10, help="timed transforms per direction and NUFFT case")
    ap.add_argument("--serial", action="store_true",
                    help="run the point side of each half step on the caller's stream (plan tuning overlap = 0) "
                         "instead of concurrently on the plan's second stream")
    ap.add_argument("--batch-lanes", type=int, default=0,
                    help="run only a few steps of the 64-instance 2D Stokes batch (FP32, tol 1e-5) with this many "
                         "lanes of library groups (1: one launch per stage over all plans), e.g. for a kernel trace")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 512 MiB device copy (reference for hardware byte counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def setup(F, torch, prec, tol, N, rings, upsampfac=0.0, overlap=True, deterministic=False):
    import workloads
    case = workloads.ns3d_case(n_rings=rings, n_lon=rings, N=N)
    X0, tris = case["X"], case["tris"]
    M = X0.shape[0]
    ptr, idx = workloads.vertex_triangle_csr(tris, M)
    dev = "cuda:0"
    plan = F.Plan(3, case["N"], L=case["L"], prec=prec, tol=tol, max_points=M, fluid=True, navier_stokes=True,
                  upsampfac=upsampfac, deterministic=deterministic)
    if not overlap:
        plan.tuning(overlap=0)
    force = F.Force("surface3d", case["K"], torch.as_tensor(tris).to(dev), torch.as_tensor(ptr).to(dev),
                    torch.as_tensor(idx).to(dev))
    params = F.FluidParams("navier_stokes", rho=case["rho"], mu=case["mu"], dt=case["dt"])
    X = torch.as_tensor(X0).to(dev).contiguous()
    U = torch.zeros((M, 3), dtype=plan.rdtype, device=dev)
    uh = torch.zeros((3,) + plan.half_shape, dtype=plan.cdtype, device=dev)
    return dict(plan=plan, force=force, params=params, X=X, U=U, uh=uh, M=M, X0=X0, tris=tris, case=case)


ROUND = 10  # steps per round from the initial state (the specified dt is above the explicit
            # surface-tension stability limit at h = 1/128: the uninterrupted run turns non-finite
            # near step 60, so timing restarts from the initial state every ROUND steps)


def reset(s):
    s["X"].copy_(s["Xinit"])
    s["U"].zero_()
    s["uh"].zero_()


def time_steps(torch, s, steps, warmup, prof_class=None):
    plan, force, params = s["plan"], s["force"], s["params"]
    if "Xinit" not in s:  # the initial state (every call starts from it)
        s["Xinit"] = s["X"].clone()
    reset(s)
    if warmup > 0:
        plan.steps(params, force, s["X"], s["U"], s["uh"], warmup)
    reset(s)
    if prof_class:
        plan.profile(prof_class, max_launches=64 * steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # rounds of ROUND steps from the initial state, each one fsib_steps call (the interpolation of
    # U^{m+1} overlaps the next step's products)
    for k in range(0, steps, ROUND):
        if k > 0:
            reset(s)  # inside the timed region
        plan.steps(params, force, s["X"], s["U"], s["uh"], min(ROUND, steps - k))
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    prof = None
    if prof_class:
        prof = plan.profile_read()
        plan.profile(None)
    # state after ROUND steps from the initial state, for the FP32-vs-FP64 comparison
    reset(s)
    plan.steps(params, force, s["X"], s["U"], s["uh"], ROUND)
    torch.cuda.synchronize()
    return (el, prof) if prof_class else el


def time_reps(torch, s, reps=30):
    """Median over `reps` repetitions of one round (ROUND steps from the initial state, one fsib_steps
    call), each timed with a HIP event pair on the stream the steps are issued on; the state reset
    between repetitions lies outside the events."""
    plan, force, params = s["plan"], s["force"], s["params"]
    if "Xinit" not in s:  # the initial state (every repetition starts from it)
        s["Xinit"] = s["X"].clone()
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    reset(s)
    plan.steps(params, force, s["X"], s["U"], s["uh"], ROUND)  # warm-up
    for e0, e1 in ev:
        reset(s)
        e0.record(st)
        plan.steps(params, force, s["X"], s["U"], s["uh"], ROUND)
        e1.record(st)
    torch.cuda.synchronize()
    ms = sorted(e0.elapsed_time(e1) / ROUND for e0, e1 in ev)
    return {"reps": reps, "steps_per_rep": ROUND, "median_ms_per_step": ms[len(ms) // 2],
            "min_ms_per_step": ms[0], "max_ms_per_step": ms[-1], "median_steps_per_s": 1e3 / ms[len(ms) // 2],
            "method": "HIP events on the issuing stream around each repetition of one fsib_steps call of "
                      f"{ROUND} steps from the initial state, after one warm-up repetition"}


def stokes2d_small(F, torch, reps=30):
    """The 2D Stokes ellipse (N = 32^2, M = 128, tension K = 1, mu = 1, dt = 1e-3, FP64 at tol 1e-12):
    10 steps from U^0, eager (one fsib_steps call) and replayed from a HIP graph; median over `reps`
    repetitions timed with HIP events.  Returns the timings and the final positions."""
    import workloads
    c = workloads.stokes2d_case()
    X0 = c["X"]
    M = X0.shape[0]
    dev = "cuda:0"
    plan = F.Plan(2, c["N"], L=c["L"], prec="f64", tol=1e-12, max_points=M, fluid=True)
    force = F.Force("tension2d", c["K"])
    params = F.FluidParams("stokes", mu=c["mu"], dt=c["dt"])
    Xi = torch.as_tensor(X0).to(dev)
    X = Xi.clone()
    U = torch.zeros((M, 2), dtype=torch.float64, device=dev)
    uh = torch.zeros((2,) + plan.half_shape, dtype=torch.complex128, device=dev)

    def run():
        X.copy_(Xi)
        plan.velocity(params, force, X, uh, out=U)
        plan.steps(params, force, X, U, uh, 10)

    st = torch.cuda.current_stream()
    run()
    torch.cuda.synchronize()
    Xf = X.cpu().numpy()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(st)
        run()
        e1.record(st)
    torch.cuda.synchronize()
    eager = sorted(e0.elapsed_time(e1) / 10 for e0, e1 in ev)
    side = torch.cuda.Stream()
    side.wait_stream(st)
    with torch.cuda.stream(side):
        run()
    st.wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    g.replay()
    torch.cuda.synchronize()
    gdiff = float(np.max(np.abs(X.cpu().numpy() - Xf)))
    for e0, e1 in ev:
        e0.record(st)
        g.replay()
        e1.record(st)
    torch.cuda.synchronize()
    graph = sorted(e0.elapsed_time(e1) / 10 for e0, e1 in ev)
    del g
    plan.close()
    med = lambda v: v[len(v) // 2]
    res = {"workload": "2D Stokes FSIB, N=32^2, M=128 ellipse 0.3/0.2 at a seeded centre, tension K=1, mu=1, "
                       "dt=1e-3, 10 steps, FP64 tol 1e-12",
           "eager_steps_per_s": 1e3 / med(eager), "eager_median_ms_per_step": med(eager),
           "graph_steps_per_s": 1e3 / med(graph), "graph_median_ms_per_step": med(graph),
           "graph_max_abs_diff_X_vs_eager": gdiff, "reps": reps,
           "method": "median over repetitions of U^0 (fsib_velocity) + 10 steps (fsib_steps), HIP events"}
    return res, Xf


def time_steps_graph(torch, s, steps):
    """The same rounds (state reset + one fsib_steps call of ROUND steps) captured once in a HIP graph
    and replayed; returns (seconds per step, max |X_graph - X_eager| after one round)."""
    plan, force, params = s["plan"], s["force"], s["params"]
    reset(s)
    plan.steps(params, force, s["X"], s["U"], s["uh"], ROUND)
    torch.cuda.synchronize()
    X_eager = s["X"].clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        reset(s)
        plan.steps(params, force, s["X"], s["U"], s["uh"], ROUND)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        reset(s)
        plan.steps(params, force, s["X"], s["U"], s["uh"], ROUND)
    g.replay()
    torch.cuda.synchronize()
    diff = float((s["X"] - X_eager).abs().max().item())
    rounds = max(1, steps // ROUND)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(rounds):
        g.replay()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / (rounds * ROUND)
    del g
    torch.cuda.synchronize()
    return el, diff


def time_nufft(torch, s, reps=20):
    """Force spreading and velocity interpolation at the surface points (sort + spread + FFT + deconvolution)."""
    plan = s["plan"]
    X = s["X"]
    M = s["M"]
    S = torch.randn((M, 3), dtype=plan.rdtype, device=X.device)
    fh = plan.force_spread(X, S, 1.0)
    fh[..., -1] = 0
    U = plan.velocity_interp(X, fh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.force_spread(X, S, 1.0, out=fh)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        plan.velocity_interp(X, fh, out=U)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ts, ti = (t1 - t0) / reps, (t2 - t1) / reps
    return dict(spread_pts_per_s=M / ts, interp_pts_per_s=M / ti, spread_interp_pts_per_s=M / (ts + ti),
                spread_ms=ts * 1e3, interp_ms=ti * 1e3)


def touched_cells(torch, X, nf, w):
    """Fine-grid cells inside at least one point's w^3 kernel support (counted on the device)."""
    dev = X.device
    occ = torch.zeros(nf ** 3, dtype=torch.bool, device=dev)
    xf = torch.remainder(X, 1.0) * nf
    i0 = torch.ceil(xf - w / 2.0).to(torch.int64)  # first cell of the support along each axis
    off = torch.arange(w, device=dev)
    ix = torch.remainder(i0[:, 0:1] + off, nf)  # (M, w)
    for dz in range(w):
        iz = torch.remainder(i0[:, 2] + dz, nf)
        for dy in range(w):
            iy = torch.remainder(i0[:, 1] + dy, nf)
            occ[((iz * nf + iy) * nf)[:, None] + ix] = True
    n = int(occ.sum().item())
    del occ
    return n


def time_nufft_micro(F, torch, N, M, prec, tol, reps=10):
    """Type-1 and type-2 of M complex strengths at N^3 modes with the NUFFT micro-benchmark's point law.

    Returns points/s of the full transforms (sort + spread + FFT + deconvolution and the reverse)
    and, from HIP events around the spreading and interpolation kernels alone, their time and
    fraction of HBM bandwidth: spreading writes the fine grid once and reads each point's record
    (24 B of coordinates + its strength); interpolation reads each touched fine cell once and each
    point's record, and writes one value per point.
    """
    import workloads
    dev = "cuda:0"
    X0, c0 = workloads.nufft_points(M, seed=3, dim=3)
    plan = F.Plan(3, (N, N, N), prec=prec, tol=tol, max_points=M)
    info = plan.info()
    nf, w = info["n_fine"][0], info["w"]
    X = torch.as_tensor(X0).to(dev)
    c = torch.as_tensor(c0).to(dev).to(plan.cdtype)
    fh = torch.as_tensor(workloads.random_modes((N, N, N), 38)).to(dev).to(plan.cdtype)
    out1 = plan.spread(X, c)
    out2 = plan.interp(X, fh)
    torch.cuda.synchronize()
    res = {"N": N, "M": M, "prec": prec, "tol": tol, "w": w, "n_fine": nf}
    for kind, call, cls in (("type1", lambda: plan.spread(X, c, out=out1), "spread"),
                            ("type2", lambda: plan.interp(X, fh, out=out2), "interp")):
        call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        plan.profile(cls, max_launches=4 * reps)
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        ms, n, _ = plan.profile_read()
        plan.profile(None)
        res[f"{kind}_pts_per_s"] = M / t
        res[f"{kind}_ms"] = t * 1e3
        res[f"{cls}_kernel_us"] = ms * 1e3 / max(n, 1)
    sc = 4 if prec == "f32" else 8
    touched = touched_cells(torch, X, nf, w)
    b_spread = M * (24 + 2 * sc) + nf ** 3 * 2 * sc
    b_interp = M * (24 + 2 * sc) + touched * 2 * sc
    res["spread_kernel_frac_hbm"] = b_spread / (res["spread_kernel_us"] * 1e-6) / (HBM_PEAK_GBS * 1e9)
    res["interp_kernel_frac_hbm"] = b_interp / (res["interp_kernel_us"] * 1e-6) / (HBM_PEAK_GBS * 1e9)
    res["touched_cell_fraction"] = touched / nf ** 3
    res["spread_interp_pts_per_s"] = M / ((res["type1_ms"] + res["type2_ms"]) * 1e-3)
    plan.close()
    del X, c, fh, out1, out2
    torch.cuda.empty_cache()
    return res


def batched_stokes(F, torch, steps=50, graph_steps=10):
    """64 independent 2D Stokes instances (uneven N and M), FP32 batched under a HIP graph, against
    the same batch launched eagerly and the plain FP64 path; instance-steps per second.  The stream
    count of each batch is picked by the batch's autotuner from timed probes."""
    import workloads
    from paper_2302_08694_amd.batch import StokesBatch
    cases = workloads.batched_stokes2d(count=64, seed=4)
    res = {"instances": len(cases), "steps": steps, "points": int(sum(c["X"].shape[0] for c in cases)),
           "n_modes": sorted(set(int(c["N"][0]) for c in cases))}
    finals = {}
    for prec, tol in (("f32", 1e-5), ("f64", 1e-5)):
        b = StokesBatch(cases, prec=prec, tol=tol)
        tune = b.autotune()
        res[f"{prec}_streams"] = len(b.streams)
        res[f"{prec}_autotune_ms_per_batch_step"] = {str(k): v * 1e3 for k, v in tune.items()}
        b.step(1)
        b.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        te = time.perf_counter() - t0
        res[f"{prec}_eager_instance_steps_per_s"] = len(cases) * steps / te
        if prec == "f32":
            b.reset()
            b.capture(graph_steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps // graph_steps):
                b.replay()
            torch.cuda.synchronize()
            tg = time.perf_counter() - t0
            res["f32_graph_instance_steps_per_s"] = len(cases) * steps / tg
        finals[prec] = [(it["X"].cpu().numpy(), it["X0"].cpu().numpy()) for it in b.items]
        b.close()
    num = sum(float(np.sum((x32 - x64) ** 2)) for (x32, _), (x64, _) in zip(finals["f32"], finals["f64"]))
    den = sum(float(np.sum((x64 - x0) ** 2)) for (x64, x0) in finals["f64"])
    res["f32_rel_err_displacement_vs_f64"] = (num / max(den, 1e-300)) ** 0.5
    # the same cases on multi-instance plans, one per group of equal N, stepped through library Groups
    # (fsib_group_steps): the groups are split into lanes, each lane one Group on its own stream whose
    # every stage is one launch over the lane's plans of all its N.  The autotuner picks each plan's
    # knobs and the lane count (1: one launch per stage for the whole batch; the number of groups:
    # every group on its own stream) from timed batch steps.
    from paper_2302_08694_amd.batch import StokesGroupBatch
    for prec, tol in (("f32", 1e-5), ("f64", 1e-5)):
        b = StokesGroupBatch(cases, prec=prec, tol=tol)
        res["grouped_plans"] = len(b.groups)
        tuned = b.autotune()
        lanes = tuned.pop("lanes")
        res[f"{prec}_grouped_tuning"] = {str(k): v for k, v in tuned.items()}
        res[f"{prec}_lanes_ms_per_batch_step"] = {str(k): v * 1e3 for k, v in lanes.items()}
        res[f"{prec}_lanes_chosen"] = b.lanes
        b.step(1)
        rates = []  # median of three timed runs from the initial state
        for _ in range(3):
            b.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.step(steps)
            torch.cuda.synchronize()
            rates.append(len(cases) * steps / (time.perf_counter() - t0))
        res[f"{prec}_grouped_eager_instance_steps_per_s"] = sorted(rates)[1]
        Xg = [x.cpu().numpy() for x in b.positions()]
        b.reset()
        b.capture(graph_steps)
        rates = []
        for _ in range(3):
            b.reset()  # the captured steps read and write the same state tensors
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps // graph_steps):
                b.replay()
            torch.cuda.synchronize()
            rates.append(len(cases) * steps / (time.perf_counter() - t0))
        res[f"{prec}_grouped_graph_instance_steps_per_s"] = sorted(rates)[1]
        num = sum(float(np.sum((xg - x64) ** 2)) for xg, (x64, _) in zip(Xg, finals["f64"]))
        res[f"{prec}_grouped_rel_err_displacement_vs_f64"] = (num / max(den, 1e-300)) ** 0.5
        b.close()
    return res


def differentiable_stokes(F, torch, reps=5):
    """Loss and gradients (initial positions, stiffness) of 20 checkpointed Stokes steps at 64^3 modes
    with 10,000 surface-tension points: FP32 and FP64 forward + adjoint, wall time per gradient
    evaluation next to the forward alone, and the FP32 gradients' error against the FP64 ones."""
    import workloads
    from paper_2302_08694_amd.autograd import ForceLaw, stokes_trajectory
    c = workloads.diff_stokes3d_case()
    X0, tris, M = c["X"], c["tris"], c["X"].shape[0]
    ptr, idx = workloads.vertex_triangle_csr(tris, M)
    d = lambda a: torch.as_tensor(a).to("cuda:0")
    law = ForceLaw("surface3d", d(tris), d(ptr), d(idx))
    tgt = d(c["target"])
    res = {"n_modes": c["N"][0], "points": M, "steps": c["steps"], "dt": c["dt"], "checkpointed": True}
    grads = {}
    for prec, tol in (("f32", 1e-6), ("f64", 1e-10)):
        plan = F.Plan(3, c["N"], prec=prec, tol=tol, max_points=M, fluid=True)

        def evaluate(grad):
            X = d(X0).requires_grad_(grad)
            K = torch.tensor(c["K"], dtype=torch.float64, device="cuda:0", requires_grad=grad)
            XT = stokes_trajectory(plan, X, K, law, c["mu"], c["dt"], c["steps"], checkpoint=True)
            loss = torch.sum((XT - tgt) ** 2)
            if grad:
                loss.backward()
                return loss, X.grad, K.grad
            return loss, None, None

        for grad in (False, True):
            for _ in range(2):  # warm-up (allocator growth, first autograd graph)
                evaluate(grad)
            torch.cuda.synchronize()
            # median of separately synchronised evaluations: the 20-step trajectory issues ~20 small
            # host-side operations per step, so single evaluations carry host jitter
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                out = evaluate(grad)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            res[f"{prec}_tol"] = tol
            res[f"{prec}_{'forward_backward' if grad else 'forward'}_ms"] = float(np.median(ts)) * 1e3
        grads[prec] = (float(out[0].detach()), out[1].cpu().numpy(), float(out[2]))
        plan.close()
    (l32, g32, k32), (l64, g64, k64) = grads["f32"], grads["f64"]
    res["loss_f64"] = l64
    res["f32_rel_err_loss"] = abs(l32 - l64) / abs(l64)
    res["f32_rel_err_grad_X0"] = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    res["f32_rel_err_grad_K"] = abs(k32 - k64) / abs(k64)
    return res


# (N, M, prec, tol): the micro-benchmark's point law (half uniform, half on a sphere of radius 0.2)
# at 256^3 with 2e6 points, and scaled to 128^3 with 2.5e5 points (same points per fine cell)
NUFFT_MICRO = [(128, 250_000, "f32", 1e-5), (128, 250_000, "f64", 1e-5),
               (256, 2_000_000, "f32", 1e-5), (256, 2_000_000, "f64", 1e-5), (256, 2_000_000, "f64", 1e-10)]


def nufft_micro(F, torch, cases=None, reps=10):
    res = []
    for N, M, prec, tol in (cases or NUFFT_MICRO):
        log(f"nufft micro N={N} M={M} {prec} tol {tol:g}")
        r = time_nufft_micro(F, torch, N, M, prec, tol, reps)
        log(f"  type1 {r['type1_ms']:.3f} ms type2 {r['type2_ms']:.3f} ms spread kernel {r['spread_kernel_us']:.1f} us "
            f"({r['spread_kernel_frac_hbm']:.2f} HBM) interp kernel {r['interp_kernel_us']:.1f} us "
            f"({r['interp_kernel_frac_hbm']:.2f} HBM)")
        res.append(r)
    return res


def cpu_stokes2d(X_gpu):
    """The oracle's 10-step trajectory of the 2D Stokes ellipse, on all host cores and on one thread, and
    the GPU's final positions against it."""
    import workloads
    from oracle import step
    try:
        from threadpoolctl import threadpool_limits
    except Exception:
        threadpool_limits = None
    c = workloads.stokes2d_case()
    force = step.ForceLaw("tension2d", c["K"])

    def traj():
        X = c["X"].copy()
        U, _ = step.stokes_velocity(X, force, c["N"], c["L"], c["mu"])
        for _ in range(10):
            X, U, _ = step.stokes_step(X, U, force, c["N"], c["L"], c["mu"], c["dt"])
        return X

    t0 = time.perf_counter()
    Xo = traj()
    t_all = (time.perf_counter() - t0) / 10
    t_one = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            traj()
            t_one = (time.perf_counter() - t0) / 10
    disp = Xo - c["X"]
    res = {"seconds_per_step_all_cores": t_all, "steps_per_s_all_cores": 1.0 / t_all,
           "seconds_per_step_1_thread": t_one, "steps_per_s_1_thread": None if t_one is None else 1.0 / t_one,
           "sample": "the whole 10-step trajectory (direct sums)"}
    if X_gpu is not None:
        res["gpu_rel_err_displacement_vs_oracle"] = float(np.linalg.norm(X_gpu - Xo) / np.linalg.norm(disp))
    return res


def cpu_nufft_micro(nmodes=256, ntargets=4096, N=256, M=2_000_000):
    """Direct type-1 sums at `nmodes` random modes and type-2 sums at `ntargets` random points of the
    NUFFT micro-benchmark (256^3 modes, 2e6 points), timed on the host and extrapolated to the full
    transforms (linear in modes and in targets).  The type-1 subset is 256 modes: the oracle forms one
    phase per (point, mode) with single-threaded cos/sin, about 16 s for 5e8 phases on the machine's host."""
    import workloads
    from oracle import nudft
    from oracle.modes import mode_numbers
    X, c = workloads.nufft_points(M, seed=3, dim=3)
    rng = np.random.default_rng(7)
    m = np.stack([mode_numbers(N)[rng.integers(0, N, nmodes)] for _ in range(3)], axis=1)
    t0 = time.perf_counter()
    nudft.type1_at_modes(X, c, m)
    t1 = time.perf_counter() - t0
    f = workloads.random_modes((N, N, N), 38)
    sel = rng.choice(M, ntargets, replace=False)
    t0 = time.perf_counter()
    nudft.type2(X[sel], f, (N, N, N))
    t2 = time.perf_counter() - t0
    del f
    full1 = t1 * N ** 3 / nmodes
    full2 = t2 * M / ntargets
    return {"type1_subset_s": t1, "type1_subset": f"{nmodes} random modes x {M} points",
            "type2_subset_s": t2, "type2_subset": f"{ntargets} random points x {N}^3 modes",
            "type1_full_extrapolated_s": full1, "type2_full_extrapolated_s": full2,
            "type1_pts_per_s": M / full1, "type2_pts_per_s": M / full2}


def cpu_baseline(N, rings, sample_points=16384):
    """The FP64 oracle on a bounded sample of one step, extrapolated to steps/s.

    Sample: the oracle's force spreading and one velocity interpolation of `sample_points` of the
    M surface points at the full N^3 mode set (direct sums, cost linear in the points), and one
    dealiased nonlinear term at the full size.  A step is one spreading, two interpolations and
    two nonlinear terms.
    """
    import workloads
    from oracle import fluid, step
    from oracle.modes import spectral_shape
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        blas_threads = os.cpu_count()
    case = workloads.ns3d_case(n_rings=rings, n_lon=rings, N=N)
    X = case["X"]
    M = X.shape[0]
    Ns = case["N"]
    rng = np.random.default_rng(0)
    sel = rng.choice(M, size=min(sample_points, M), replace=False)
    Xs = X[sel]
    Fs = rng.standard_normal((len(sel), 3))
    t0 = time.perf_counter()
    fh = step.spread_force(Xs, Fs, 1.0, Ns, 1.0)
    t1 = time.perf_counter()
    step.interp_velocity(Xs, fh, Ns, 1.0)
    t2 = time.perf_counter()
    uh = fluid.zero_nyquist(fluid.project(fh, Ns, 1.0), Ns)
    t3 = time.perf_counter()
    fluid.nonlinear(uh, Ns, 1.0)
    t4 = time.perf_counter()
    scale = M / len(sel)
    t_step = (t1 - t0) * scale + 2 * (t2 - t1) * scale + 2 * (t4 - t3)
    return {"value": 1.0 / t_step, "unit": "steps/s", "cores": int(blas_threads), "kind": "oracle",
            "sample": (f"oracle force spreading + velocity interpolation of {len(sel)} of {M} points at N={N}^3 "
                       f"(direct sums, {t1 - t0:.2f}s + {t2 - t1:.2f}s, scaled by M/{len(sel)}) and one dealiased "
                       f"nonlinear term at N={N}^3 ({t4 - t3:.2f}s); step = 1 spread + 2 interp + 2 nonlinear; "
                       f"extrapolated {t_step:.1f} s/step"),
            "seconds_per_step": t_step}


ROOFLINE_CLASS = "fft_strided"
ROOFLINE_KERNEL = "fsib::k_fft_c2c<double, false, 192, 8>"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc runs (FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0, factors from a plain 512 MiB copy); None once the kernel changes after the counters
TRAFFIC_BYTES_PER_LAUNCH = 165.4e6
TRAFFIC_SOURCE = "profiles/fft_strided_ns128_f64_hbm_counters.md"


def roofline(ms, n, nbytes):
    """Achieved algorithmic bandwidth of the dominant kernel from the event timings."""
    if n == 0 or ms <= 0:
        return None
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"kernel": ROOFLINE_KERNEL, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": TRAFFIC_BYTES_PER_LAUNCH,
            "traffic_unit": "bytes per launch", "traffic_source": TRAFFIC_SOURCE, "launches": n,
            "avg_launch_us": ms * 1e3 / n, "algorithmic_bytes_per_launch": nbytes / n,
            "method": "HIP events around each launch on its stream over a second timed pass of the same steps "
                      "(the first, uninstrumented pass gives value); bytes = every input and output element of the "
                      "pass once; unless --serial, the passes share the GPU with the point side of the step "
                      "running concurrently on a second stream"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    import paper_2302_08694_amd as F
    if F.device_count() < 1:
        raise SystemExit("no HIP device visible")
    if a.nufft_only:
        cases = None
        if a.nufft_case:
            n_, m_, p_, t_ = a.nufft_case.split(":")
            cases = [(int(n_), int(m_), p_, float(t_))]
        print(json.dumps({"metric": "NUFFT micro-benchmark only (profiling run)",
                          "nufft_micro": nufft_micro(F, torch, cases, a.nufft_reps)}), flush=True)
        return
    if a.batch_lanes > 0:
        import workloads
        from paper_2302_08694_amd.batch import StokesGroupBatch
        cases = workloads.batched_stokes2d(count=64, seed=4)
        b = StokesGroupBatch(cases, prec="f32", tol=1e-5, lanes=a.batch_lanes)
        b.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(5)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 5 * 1e3
        print(json.dumps({"metric": "batched 2D Stokes steps only (profiling run)", "lanes": b.lanes,
                          "plans": len(b.groups), "ms_per_batch_step": ms}), flush=True)
        b.close()
        return
    log("setup FP64")
    s64 = setup(F, torch, "f64", a.tol, a.n, a.rings, upsampfac=a.upsampfac, overlap=not a.serial)
    info64 = s64["plan"].info()
    log(f"plan f64: {info64}")
    # value: the steps timed without instrumentation; then the same steps again with the dominant
    # kernel (the strided FFT passes along y and z) bracketed by HIP events on its launch stream
    t64 = time_steps(torch, s64, a.steps, a.warmup)
    reps64 = time_reps(torch, s64)
    log(f"f64 median of {reps64['reps']} repetitions: {reps64['median_ms_per_step']:.3f} ms/step")
    t64p, (prof_ms, prof_n, prof_bytes) = time_steps(torch, s64, a.steps, 0, ROOFLINE_CLASS)
    log(f"f64 {t64 * 1e3:.3f} ms/step ({t64p * 1e3:.3f} with events); {ROOFLINE_CLASS}: {prof_n} launches, "
        f"{prof_ms:.3f} ms")
    X64 = s64["X"].cpu().numpy()
    tg64, gdiff64 = time_steps_graph(torch, s64, a.steps)
    log(f"f64 under a HIP graph {tg64 * 1e3:.3f} ms/step (max |X - X_eager| {gdiff64:.2e})")
    graph64 = {"steps_per_s": 1.0 / tg64, "ms_per_step": tg64 * 1e3, "max_abs_diff_X_vs_eager": gdiff64,
               "method": f"one round (state reset + {ROUND} steps) captured once, replayed {max(1, a.steps // ROUND)} times"}
    ws64 = s64["plan"].info()["workspace_bytes"]
    U64max = float(s64["U"].abs().max().item())
    nu64 = None if a.fp64_only else time_nufft(torch, s64)
    s64["plan"].close()
    del s64
    if a.calibrate_copy:
        src = torch.ones(512 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.fp64_only:
        out = {"metric": "FSIB steps/sec, FP64 only (profiling run)", "value": 1.0 / t64, "unit": "steps/s",
               "ms_per_step": t64 * 1e3, "f64_hip_graph": graph64, "roofline": roofline(prof_ms, prof_n, prof_bytes)}
        print(json.dumps(out), flush=True)
        return
    log("setup FP32")
    s32 = setup(F, torch, "f32", a.tol, a.n, a.rings, upsampfac=a.upsampfac, overlap=not a.serial)
    t32 = time_steps(torch, s32, a.steps, a.warmup)
    reps32 = time_reps(torch, s32)
    log(f"f32 {t32 * 1e3:.3f} ms/step (median of repetitions {reps32['median_ms_per_step']:.3f})")
    X32 = s32["X"].cpu().numpy()
    ws32 = s32["plan"].info()["workspace_bytes"]
    U32max = float(s32["U"].abs().max().item())
    nu32 = time_nufft(torch, s32)
    s32["plan"].close()
    del s32
    d64 = X64 - s64_X0(a)
    err32 = float(np.linalg.norm(X32 - X64) / max(np.linalg.norm(d64), 1e-300))
    out = {
        "metric": "FSIB steps/sec (3D Navier-Stokes, 128^3 modes, M=40,000) with NUFFT spread+interp pts/sec, "
                  "FP64 and FP32 at tol 1e-5",
        "value": 1.0 / t64,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": t64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D Navier-Stokes FSIB, N={a.n}^3, M={a.rings * a.rings} lat-long ellipsoid "
                               f"(0.3/0.25/0.2), surface tension K=1, rho=1, mu=0.01, dt=5e-4, NUFFT tol {a.tol:g}",
                   "n_modes": a.n, "points": a.rings * a.rings, "tol": a.tol,
                   "fine_grid_f64": info64["n_fine"][0], "kernel_width_f64": info64["w"],
                   "point_side": "caller's stream (serial)" if a.serial else
                                 "second stream, concurrent with the dealiased products",
                   "timing": f"rounds of {ROUND} steps from the initial state (one fsib_steps call each), "
                             "state reset inside the timed region (dt = 5e-4 exceeds the explicit surface-tension stability limit at this "
                             "resolution; the uninterrupted trajectory becomes non-finite near step 60)"},
        "state_after_timed_steps": {"f64_max_abs_U": U64max, "f32_max_abs_U": U32max,
                                    "f64_finite": bool(np.all(np.isfinite(X64))),
                                    "f32_finite": bool(np.all(np.isfinite(X32)))},
        "median_of_repetitions": reps64,
        "fp32": {"steps_per_s": 1.0 / t32, "ms_per_step": t32 * 1e3, "median_of_repetitions": reps32,
                 "rel_err_displacement_vs_fp64": err32, "steps_compared": ROUND},
        "f64_hip_graph": graph64,
        "nufft_at_128": {"f64": nu64, "f32": nu32},
        "roofline": roofline(prof_ms, prof_n, prof_bytes),
        "ms_per_step_with_events": t64p * 1e3,
    }
    log("deterministic FP64 plan")
    sd = setup(F, torch, "f64", a.tol, a.n, a.rings, upsampfac=a.upsampfac, overlap=not a.serial, deterministic=True)
    repsd = time_reps(torch, sd)
    Xd1 = sd["X"].cpu().numpy()
    reset(sd)
    sd["plan"].steps(sd["params"], sd["force"], sd["X"], sd["U"], sd["uh"], ROUND)
    torch.cuda.synchronize()
    Xd2 = sd["X"].cpu().numpy()
    sd["plan"].close()
    del sd
    out["f64_deterministic"] = {"median_ms_per_step": repsd["median_ms_per_step"],
                                "median_steps_per_s": repsd["median_steps_per_s"],
                                "cost_vs_default": repsd["median_ms_per_step"] / reps64["median_ms_per_step"] - 1.0,
                                "bitwise_equal_repeat": bool(np.array_equal(Xd1.view(np.uint8), Xd2.view(np.uint8))),
                                "method": "plan with deterministic = 1 (bins ordered by original point index), "
                                          "median of 30 repetitions of 10 steps; two rounds from the initial state compared bitwise"}
    log(f"  {out['f64_deterministic']}")
    log("2D Stokes, N=32^2, M=128, 10 steps")
    out["stokes2d_small"], Xc1 = stokes2d_small(F, torch)
    log(f"  {out['stokes2d_small']}")
    if not a.no_nufft_micro:
        out["nufft_micro"] = nufft_micro(F, torch)
    if not a.no_batch:
        log("batched 2D Stokes (64 instances)")
        out["batched_2d_stokes"] = batched_stokes(F, torch)
        log(f"  {out['batched_2d_stokes']}")
    if not a.no_lowmem:
        log("smaller fine grids (oversampling 1.25 and 1.5)")
        lm = {}
        for prec, tol, up in (("f32", 1e-3, 1.25), ("f64", 1e-5, 1.25), ("f32", 1e-4, 1.5)):
            s = setup(F, torch, prec, tol, a.n, a.rings, upsampfac=up)
            t = time_steps(torch, s, a.steps, a.warmup)
            info = s["plan"].info()
            Xl = s["X"].cpu().numpy()
            lm[f"{prec}_sigma{up:g}"] = {"tol": tol, "w": info["w"], "n_fine": info["n_fine"][0], "steps_per_s": 1.0 / t,
                        "ms_per_step": t * 1e3, "workspace_bytes": info["workspace_bytes"],
                        "rel_err_displacement_vs_fp64": float(np.linalg.norm(Xl - X64) /
                                                              max(np.linalg.norm(d64), 1e-300))}
            s["plan"].close()
            del s
        lm["default_workspace_bytes"] = {"f64": ws64, "f32": ws32}
        out["lowmem"] = lm
        log(f"  {lm}")
    if not a.no_diff:
        log("differentiable 3D Stokes (64^3, 10,000 points, 20 checkpointed steps)")
        out["differentiable_stokes"] = differentiable_stokes(F, torch)
        log(f"  {out['differentiable_stokes']}")
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(a.n, a.rings)
        log("cpu oracle: 2D Stokes trajectory")
        out["cpu_baseline"]["stokes2d_small"] = cpu_stokes2d(Xc1)
        log(f"  {out['cpu_baseline']['stokes2d_small']}")
        if not a.no_nufft_micro:
            log("cpu oracle: NUFFT micro-benchmark subsets")
            out["cpu_baseline"]["nufft_micro"] = cpu_nufft_micro()
            log(f"  {out['cpu_baseline']['nufft_micro']}")
    print(json.dumps(out), flush=True)


def s64_X0(a):
    import workloads
    return workloads.ns3d_case(n_rings=a.rings, n_lon=a.rings, N=a.n)["X"]


if __name__ == "__main__":
    main()
