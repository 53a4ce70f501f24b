"""Autotuner of the frame's launch shapes.

For each persistent kernel of the update (probe-ray traversal, shadow-ray
traversal, hit shading, matrix-core blend) it times a set of grid sizes
(multiples of the compute-unit count, plus 0 = one workgroup per work unit),
for the shadow rays how their tasks are spread over lanes (batches of 64, or
per-wave ranges with lane refill at an idle-lane threshold), for frames that
answer a query batch the batch's share in the shadow launch, and for the
blend its tile shape (1, 2 or 4 workgroups per block of 8 probes), on the
live workload with the library's own kernel timing, and keeps the fastest.
The choice is returned as a dict, can be saved as JSON and applied to
another context with ``apply``.  Tuning runs real frames: call it during
warm-up.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional

# the kernels a stage runs on: the shadow rays by refill mode, and the
# traversals with a share of a query batch when the frames are
# irf_update_probes_query frames
TRACE = ("trace", "trace_query")
SHADOW = ("shadow", "shadow_refill", "shadow_query")
# knobs in the order they are tuned (one at a time, the others held); the
# blend's grid is tuned again after its tile shape, since the best grid
# depends on the shape.  query_shadow (the query batch's share in the shadow
# launch) is timed over both traversals and tuned only on frames that answer
# queries.  shadow_refill is timed over both traversals too: with lane
# refill the shadow launch takes no share of a query batch, so the whole
# batch moves into the trace launch.
KNOBS = (("trace_blocks", TRACE), ("shadow_refill", TRACE + SHADOW), ("query_shadow", TRACE + SHADOW),
         ("shadow_blocks", SHADOW), ("shade_blocks", ("shade",)), ("blend_blocks", ("blend_mma",)),
         ("blend_rsplit", ("blend_mma",)), ("blend_blocks", ("blend_mma",)))


def candidates(cu: int, knob: str = "trace_blocks") -> list:
    """Values tried for one knob: grid sizes (0 = one workgroup per work
    unit, else multiples of the compute-unit count), or for the shadow rays'
    lane refill the idle-lane threshold (0 = batches of 64)."""
    if knob == "shadow_refill":
        return [0, 4, 8, 16, 32]
    if knob == "blend_rsplit":
        return [4, 2, 1]
    if knob == "query_shadow":
        return [0, 250, 500, 750]
    return [0] + [cu * k for k in (1, 2, 4, 8, 16)]


def autotune(ctx, rotations: Iterable, frames_per_candidate: int = 3, cu: Optional[int] = None,
             step=None) -> Dict[str, int]:
    """Tunes ctx in place.  `rotations` supplies the frames' rotations (used
    in turn, from the start again when they run out); `step(R)` runs one
    frame (default: ctx.update_probes; a step that calls
    ctx.update_probes_query also tunes the query batch's split)."""
    import itertools
    torch = ctx.torch
    if cu is None:
        cu = torch.cuda.get_device_properties(ctx.device).multi_processor_count
    step = step or ctx.update_probes
    rot = itertools.cycle(list(rotations))
    chosen = {}
    report = {}
    for knob, kernels in KNOBS:
        times = {}
        for c in candidates(cu, knob):
            ctx.set_tuning(**{knob: c})
            step(next(rot))                       # settle
            torch.cuda.synchronize()
            ctx.profile(True)
            ctx.profile_read(reset=True)
            for _ in range(frames_per_candidate):
                step(next(rot))
            torch.cuda.synchronize()
            prof = ctx.profile_read(reset=True)
            ctx.profile(False)
            ran = [prof[k] for k in kernels if k in prof]
            if not ran or (knob == "query_shadow" and "trace_query" not in prof):
                break
            times[c] = sum(ms for _, ms in ran) / max(n for n, _ in ran)
        if times:
            best = min(times, key=times.get)
            ctx.set_tuning(**{knob: best})
            chosen[knob] = best
            report[knob if knob not in report else knob + "_again"] = {str(k): round(1e3 * v, 2)
                                                                      for k, v in times.items()}
    ctx.tuning_report = report
    return chosen


def save(tuning: Dict[str, int], path: str, workload: str, report: Optional[dict] = None) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"workload": workload, "tuning": tuning, "candidate_us": report or {}}, f, indent=1)


def load(path: str) -> Dict[str, int]:
    with open(path) as f:
        return {k: int(v) for k, v in json.load(f)["tuning"].items()}


def apply(ctx, tuning: Dict[str, int]) -> None:
    ctx.set_tuning(**tuning)
