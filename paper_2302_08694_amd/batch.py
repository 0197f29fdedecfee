"""Many independent 2D Stokes FSIB simulations advanced together.

Each instance has its own plan (its own N, M and workspace); a step of the batch is one fsib_step
per instance.  Instances are spread over `streams` HIP streams forked from the current one (and
joined back after each batch step), so the small kernels of different instances run concurrently
on the chip's XCDs.  `capture(steps)` records `steps` batch steps into one HIP graph
(torch.cuda.CUDAGraph on ROCm; the stream fork/join becomes parallel branches of the graph), so a
replay launches every kernel of every instance with no host work in between.  The library calls
allocate nothing and synchronise nothing while stepping, so they are capturable as they are.
Streams keep the default priority.
"""

import torch

from ._binding import FluidParams, Force, Plan


class StokesBatch:
    def __init__(self, cases, prec="f32", tol=1e-5, device="cuda", streams=8):
        self.prec = prec
        self.streams = [torch.cuda.Stream() for _ in range(max(1, streams))]
        self.items = []
        for c in cases:
            X0 = torch.as_tensor(c["X"], dtype=torch.float64, device=device).contiguous()
            M = X0.shape[0]
            plan = Plan(2, c["N"], L=c.get("L", 1.0), prec=prec, tol=tol, max_points=M, fluid=True)
            params = FluidParams("stokes", mu=c["mu"], dt=c["dt"])
            force = Force("tension2d", c["K"])
            uh = torch.zeros((2,) + plan.half_shape, dtype=plan.cdtype, device=device)
            U = plan.velocity(params, force, X0, uh)  # U^0 = U(X^0)
            self.items.append(dict(plan=plan, params=params, force=force, X=X0.clone(), U=U, uh=uh,
                                   X0=X0, U0=U.clone(), uh0=uh.clone(), M=M))
        self.graph = None
        self.graph_steps = 0

    def reset(self):
        for it in self.items:
            it["X"].copy_(it["X0"])
            it["U"].copy_(it["U0"])
            it["uh"].copy_(it["uh0"])

    def step(self, n=1):
        main = torch.cuda.current_stream()
        for _ in range(n):
            for s in self.streams:
                s.wait_stream(main)
            for i, it in enumerate(self.items):
                with torch.cuda.stream(self.streams[i % len(self.streams)]):
                    it["plan"].step(it["params"], it["force"], it["X"], it["U"], it["uh"])
            for s in self.streams:
                main.wait_stream(s)

    def autotune(self, candidates=(1, 4, 8, 16), steps=2):
        """Pick the stream count by timing `steps` eager batch steps per candidate (the state is
        restored afterwards); returns {candidate: seconds per batch step}."""
        import time
        saved = [(it["X"].clone(), it["U"].clone(), it["uh"].clone()) for it in self.items]
        times = {}
        for c in candidates:
            self.streams = [torch.cuda.Stream() for _ in range(c)]
            self.step(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            self.step(steps)
            torch.cuda.synchronize()
            times[c] = (time.perf_counter() - t0) / steps
        best = min(times, key=times.get)
        self.streams = [torch.cuda.Stream() for _ in range(best)]
        for it, (X, U, uh) in zip(self.items, saved):
            it["X"].copy_(X)
            it["U"].copy_(U)
            it["uh"].copy_(uh)
        torch.cuda.synchronize()
        return times

    def capture(self, steps):
        """Record `steps` batch steps into a graph; the state is left as it was."""
        saved = [(it["X"].clone(), it["U"].clone(), it["uh"].clone()) for it in self.items]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # warm-up outside the capture
            self.step(1)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(steps)
        for it, (X, U, uh) in zip(self.items, saved):
            it["X"].copy_(X)
            it["U"].copy_(U)
            it["uh"].copy_(uh)
        torch.cuda.synchronize()
        self.graph, self.graph_steps = g, steps
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def close(self):
        self.graph = None
        for it in self.items:
            it["plan"].close()
        self.items = []


class StokesGroupBatch:
    """The same simulations with one multi-instance plan per group of cases that share N, L, mu, dt
    and K (ninst > 1): each stage of a step is one launch over all instances of a group.  The groups'
    plans are split into `lanes` library Groups (fsib_group_steps), each stepped on its own stream:
    inside a lane every stage is one launch over all of the lane's plans, whatever their N; lanes run
    concurrently.  lanes=1 gives one launch per stage for the whole batch; lanes equal to the number of
    groups gives every group its own stream.  Plans are assigned to lanes largest first, each to the
    lane with the least work so far (work ~ instances x fine-grid cells + points).  fused=False is
    lanes = number of groups.  `autotune()` picks the plans' knobs and the lane count from timed steps.
    Same interface as StokesBatch; `positions()` returns each case's X in the order of `cases`."""

    def __init__(self, cases, prec="f32", tol=1e-5, device="cuda", fused=True, lanes=None):
        self.prec = prec
        keys = {}
        for i, c in enumerate(cases):
            key = (tuple(c["N"]), c.get("L", 1.0), c["mu"], c["dt"], c["K"])
            keys.setdefault(key, []).append(i)
        self.groups = []
        for (N, L, mu, dt, K), idx in keys.items():
            Xs = [torch.as_tensor(cases[i]["X"], dtype=torch.float64) for i in idx]
            counts = [x.shape[0] for x in Xs]
            X0 = torch.cat(Xs).to(device).contiguous()
            plan = Plan(2, N, L=L, prec=prec, tol=tol, max_points=X0.shape[0], fluid=True, ninst=len(idx))
            plan.set_instances(counts)
            params = FluidParams("stokes", mu=mu, dt=dt)
            force = Force("tension2d", K)
            uh = torch.zeros(plan.field_shape, dtype=plan.cdtype, device=device)
            U = plan.velocity(params, force, X0, uh)
            fine = plan.info()["n_fine"]
            work = len(idx) * fine[0] * fine[1] + X0.shape[0]
            self.groups.append(dict(plan=plan, params=params, force=force, X=X0.clone(), U=U, uh=uh, X0=X0,
                                    U0=U.clone(), uh0=uh.clone(), idx=idx, counts=counts, work=work))
        self.lane_groups = []
        self.streams = []
        self.set_lanes(lanes if lanes is not None else (1 if fused else len(self.groups)))
        self.graph = None
        self.graph_steps = 0

    def set_lanes(self, lanes):
        """Split the plans into `lanes` library Groups (largest work first, each to the least loaded
        lane), each stepped on its own stream."""
        from ._binding import Group
        for grp, _ in self.lane_groups:
            grp.close()
        # a library group holds at most 8 plans
        lanes = max(1, -(-len(self.groups) // 8), min(int(lanes), len(self.groups)))
        load = [0] * lanes
        members = [[] for _ in range(lanes)]
        for g in sorted(self.groups, key=lambda g: -g["work"]):
            open_lanes = [i for i in range(lanes) if len(members[i]) < 8]
            k = min(open_lanes, key=lambda i: load[i])
            members[k].append(g)
            load[k] += g["work"]
        self.lane_groups = [(Group([g["plan"] for g in m]), m) for m in members if m]
        self.streams = [torch.cuda.Stream() for _ in self.lane_groups]
        self.lanes = len(self.lane_groups)

    def reset(self):
        for g in self.groups:
            g["X"].copy_(g["X0"])
            g["U"].copy_(g["U0"])
            g["uh"].copy_(g["uh0"])

    def step(self, n=1):
        def run(grp, gs):
            grp.steps([g["params"] for g in gs], [g["force"] for g in gs], [g["X"] for g in gs],
                      [g["U"] for g in gs], [g["uh"] for g in gs], n)
        if len(self.lane_groups) == 1:
            run(*self.lane_groups[0])
            return
        main = torch.cuda.current_stream()
        for s in self.streams:
            s.wait_stream(main)
        for (grp, gs), s in zip(self.lane_groups, self.streams):
            with torch.cuda.stream(s):
                run(grp, gs)
        for s in self.streams:
            main.wait_stream(s)

    def _save(self):
        return [(g["X"].clone(), g["U"].clone(), g["uh"].clone()) for g in self.groups]

    def _restore(self, saved):
        for g, (X, U, uh) in zip(self.groups, saved):
            g["X"].copy_(X)
            g["U"].copy_(U)
            g["uh"].copy_(uh)
        torch.cuda.synchronize()

    def autotune(self, reps=3, lanes=None):
        """Tune each plan's knobs (paper_2302_08694_amd.tune) on timed steps of that plan alone, give
        the plans that share a lane the spreading variant of the lane's largest plan (a launch over
        plans needs one workgroup size), then pick the lane count (candidates `lanes`, default 1, 2
        and the number of groups) from timed batch steps.  The state is restored afterwards.  Returns
        {N: chosen knobs, "lanes": {candidate: seconds per batch step}}."""
        import time
        from .tune import autotune
        saved = self._save()
        chosen = {}
        for g in self.groups:
            run = lambda g=g: g["plan"].step(g["params"], g["force"], g["X"], g["U"], g["uh"])
            chosen[g["plan"].n_modes[0]] = autotune(g["plan"], run, reps=reps)["best"]
        self._restore(saved)
        least = -(-len(self.groups) // 8)  # lanes needed for groups of at most 8 plans
        cands = lanes if lanes is not None else sorted({least, min(max(2, least), len(self.groups)), len(self.groups)})
        times = {}
        for c in cands:
            self._lanes_with_shared_variant(c)
            self.step(1)
            torch.cuda.synchronize()
            nrep = max(5, reps)
            t0 = time.perf_counter()
            for _ in range(nrep):
                self.step(1)
            torch.cuda.synchronize()
            times[c] = (time.perf_counter() - t0) / nrep
            self._restore(saved)
        best = min(times, key=times.get)
        self._lanes_with_shared_variant(best)
        for g in self.groups:
            chosen[g["plan"].n_modes[0]] = g["plan"].tuning()
        chosen["lanes"] = times
        return chosen

    def _lanes_with_shared_variant(self, lanes):
        self.set_lanes(lanes)
        for _, gs in self.lane_groups:
            top = max(gs, key=lambda g: g["work"])
            v = top["plan"].tuning()["spread_threads"]
            for g in gs:
                g["plan"].tuning(**{**g["plan"].tuning(), "spread_threads": v})

    def positions(self):
        out = [None] * sum(len(g["idx"]) for g in self.groups)
        for g in self.groups:
            for i, X in zip(g["idx"], torch.split(g["X"], g["counts"])):
                out[i] = X
        return out

    def capture(self, steps):
        saved = self._save()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.step(1)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            self.step(steps)
        self._restore(saved)
        self.graph, self.graph_steps = gr, steps
        return gr

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def close(self):
        self.graph = None
        for grp, _ in self.lane_groups:
            grp.close()
        self.lane_groups = []
        for g in self.groups:
            g["plan"].close()
        self.groups = []
