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
    and K (ninst > 1): each stage of a step is one launch over all instances of a group, so a batch
    step costs a few launches per group instead of per instance.  With fused=True (the default) the
    groups' plans form one library Group (fsib_group_steps) and each stage is one launch over all
    groups, of every N; with fused=False the groups run on their own streams.  Same interface as
    StokesBatch; `positions()` returns each case's X in the order of `cases`."""

    def __init__(self, cases, prec="f32", tol=1e-5, device="cuda", fused=True):
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
            self.groups.append(dict(plan=plan, params=params, force=force, X=X0.clone(), U=U, uh=uh, X0=X0,
                                    U0=U.clone(), uh0=uh.clone(), idx=idx, counts=counts))
        self.streams = [torch.cuda.Stream() for _ in self.groups]
        self.fused = None
        if fused:
            from ._binding import Group
            self.fused = Group([g["plan"] for g in self.groups])
        self.graph = None
        self.graph_steps = 0

    def reset(self):
        for g in self.groups:
            g["X"].copy_(g["X0"])
            g["U"].copy_(g["U0"])
            g["uh"].copy_(g["uh0"])

    def step(self, n=1):
        if self.fused is not None:
            gs = self.groups
            self.fused.steps([g["params"] for g in gs], [g["force"] for g in gs], [g["X"] for g in gs],
                             [g["U"] for g in gs], [g["uh"] for g in gs], n)
            return
        main = torch.cuda.current_stream()
        for _ in range(n):
            for s in self.streams:
                s.wait_stream(main)
            for g, s in zip(self.groups, self.streams):
                with torch.cuda.stream(s):
                    g["plan"].step(g["params"], g["force"], g["X"], g["U"], g["uh"])
            for s in self.streams:
                main.wait_stream(s)

    def autotune(self, reps=3):
        """Tune each group's plan knobs (paper_2302_08694_amd.tune) on timed steps of that group;
        the state is restored afterwards.  Returns {N: chosen knobs}."""
        from .tune import autotune
        chosen = {}
        for g in self.groups:
            saved = (g["X"].clone(), g["U"].clone(), g["uh"].clone())
            run = lambda g=g: g["plan"].step(g["params"], g["force"], g["X"], g["U"], g["uh"])
            chosen[g["plan"].n_modes[0]] = autotune(g["plan"], run, reps=reps)["best"]
            g["X"].copy_(saved[0])
            g["U"].copy_(saved[1])
            g["uh"].copy_(saved[2])
        torch.cuda.synchronize()
        return chosen

    def positions(self):
        out = [None] * sum(len(g["idx"]) for g in self.groups)
        for g in self.groups:
            for i, X in zip(g["idx"], torch.split(g["X"], g["counts"])):
                out[i] = X
        return out

    def capture(self, steps):
        saved = [(g["X"].clone(), g["U"].clone(), g["uh"].clone()) for g in self.groups]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.step(1)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            self.step(steps)
        for g, (X, U, uh) in zip(self.groups, saved):
            g["X"].copy_(X)
            g["U"].copy_(U)
            g["uh"].copy_(uh)
        torch.cuda.synchronize()
        self.graph, self.graph_steps = gr, steps
        return gr

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def close(self):
        self.graph = None
        if self.fused is not None:
            self.fused.close()
            self.fused = None
        for g in self.groups:
            g["plan"].close()
        self.groups = []
