"""Timed search over a plan's launch-shape knobs (fsib_plan_tuning).

    autotune(plan, run, reps=3) -> {"best": {...}, "trials": [(knobs, seconds), ...]}

`run()` performs one representative unit of work on the plan (a time step, a pair of transforms);
it is called once per trial to warm up and then `reps` times under the clock.  The search is one
pass of coordinate descent: the spreading variant of 2D plans (threads, i.e. cells per lane, of a
16 x 16 tile), the XCD run length of spreading, then that of interpolation, the heavy-tile split,
the points per interpolation wavefront and, on Navier-Stokes plans with 192-point dealiasing lines,
the FFT stages of the fused products pass, each over a short candidate list, keeping the best value
of each before moving on.  The knobs change only the launch shape (and, for the split, the order in
which partial tiles are summed), so results agree to rounding whatever is chosen.
"""

import time

import torch

CANDIDATES = {
    "spread_threads": (64, 128, 256),  # spreading variant: threads (cells per lane) of a 2D tile
    "xcd_chunk_spread": (0, 4, 16, 64),
    "xcd_chunk_interp": (0, 16, 64, 256),
    "split": (256, 512, 1024, 2048),
    "interp_points": (4, 8),
    "nl_stages": (0, 2, 3),  # fused products x pass: per half step (0), 16 x 12 in registers, 8 x 8 x 3 via LDS
}


def _time(run, reps):
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def autotune(plan, run, reps=3, candidates=None):
    cands = dict(CANDIDATES if candidates is None else candidates)
    if plan.dim == 3:
        cands.pop("spread_threads", None)  # one spreading variant for 3D tiles
    if plan.info()["n_dealias"][0] != 192:
        cands.pop("nl_stages", None)  # one products kernel for other dealiasing lengths
    best = plan.tuning()
    trials = []
    best_t = _time(run, reps)
    trials.append((dict(best), best_t))
    for knob, values in cands.items():
        for v in values:
            if v == best[knob] or (knob == "split" and v < plan.tuning()["split"] and v < best["split"]):
                continue
            try:
                trial = plan.tuning(**{**best, knob: v})
            except Exception:  # a value the plan cannot take (e.g. a split below its creation value)
                continue
            t = _time(run, reps)
            trials.append((dict(trial), t))
            if t < best_t:
                best_t, best = t, dict(trial)
        plan.tuning(**best)
    return {"best": best, "seconds": best_t, "trials": trials}
