"""GPU side of the parity protocol (tests/parity.py): run workloads through
the HIP library and through the FP64 oracle on the same seeded inputs and
compare every ray, texel and query.

Every frame goes through the substitution step (the oracle adopts the
library's decision on the rays it flags and where the two differ), so no
probe, texel or ray is left out of the value comparison.  Each comparison
prints its plain-1e-5 pass rate and the counts of elements that needed the
oracle's float32 sensitivity allowance; those counts are held to budgets
(WIDENED_MAX, BEYOND_MAX of the elements compared).
"""
import numpy as np

from tests import parity as P

U32 = P.U32
# budgets, as fractions of the elements of one comparison: elements beyond
# 1e-5 s within their kappa allowance (capped at 1e-3 s), and elements whose
# allowance exceeds 1e-3 s (the float32 evaluation of the oracle's own steps
# stays below 0.5 % and 0.6 % on these workloads)
WIDENED_MAX = 0.02
BEYOND_MAX = 0.01


def gpu_records(ctx):
    """All volumes' ray records of the last frame, in the oracle's order
    (per volume, per active probe in index order, per ray)."""
    recs = [ctx.ray_records(v) for v in range(len(ctx.volumes))]
    return np.concatenate(recs) if recs else np.zeros(0)


def gpu_atlases(gv):
    return (gv.irradiance[..., :3].float().cpu().numpy().astype(np.float64),
            gv.distance.float().cpu().numpy().astype(np.float64))


def copy_states(ctx, ov, torch, max_diff_frac=0.01):
    """After classification: the GPU's states must match the oracle's except
    on probes with an ambiguous ray; those take the oracle's state so both
    sides continue from identical states.  Returns the differing count."""
    total = 0
    for gv, o in zip(ctx.volumes, ov):
        gs = gv.states.cpu().numpy()
        diff = np.nonzero(gs != o.states)[0]
        assert len(diff) <= max(2, max_diff_frac * len(gs)), len(diff)
        if len(diff):
            gs[diff] = o.states[diff]
            gv.states.copy_(torch.from_numpy(gs))
        total += len(diff)
    return total


def frame(torch, ctx, osc, ov, lights, R, tag, launch=None):
    """One GPU frame (ctx.update_probes(R), or launch()) and the oracle's
    frame with substitution.  Returns (verdicts, report, oracle records,
    GPU records)."""
    if launch is None:
        ctx.update_probes(R)
    else:
        launch()
    torch.cuda.synchronize()
    per_vol = [ctx.ray_records(v) for v in range(len(ctx.volumes))]
    rec_g = np.concatenate(per_vol) if per_vol else np.zeros(0)
    rec_o, rep = P.oracle_frame(osc, lights, ov, R, rec_g["tri"], rec_g["vis"])
    print(f"[parity] {tag}: {rep.line()}", flush=True)
    assert rep.unflagged_flips == 0, rep.line()
    o_mag = P.origin_magnitude(ov, [len(r) for r in per_vol])
    vs, t_bad = P.ray_checks(tag, rec_g["rgb"], rec_g["d"], rec_g["t"], rec_o, o_mag)
    assert t_bad == 0, f"{tag}: {t_bad} hit distances beyond the float32 direction error"
    for v, (gv, o) in enumerate(zip(ctx.volumes, ov)):
        assert np.array_equal(gv.states.cpu().numpy(), o.states), f"{tag}: states of volume {v}"
        gi, gd = gpu_atlases(gv)
        vs += P.texel_checks(f"{tag} volume {v}", gi, gd, o)
    return vs, rep, rec_o, rec_g


def queries(torch, ctx, ov, q, tag, stage=True):
    """End to end (each side's own atlases) and, with stage=True, the GPU
    query on the oracle's atlases rounded to float32 (this overwrites the
    GPU atlases)."""
    import oracle
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    pos, nrm, view = t(q.pos), t(q.nrm), t(q.view)
    eg = ctx.query_irradiance(pos, nrm, view).cpu().numpy()
    eo, ko = oracle.query(ov, q.pos, q.nrm, q.view)
    out = [P.compare(f"{tag} query end-to-end", eg, eo, ko)]
    if stage:
        ovr = oracle.copy_volumes(ov)
        for gv, o in zip(ctx.volumes, ovr):
            o.irr[:] = o.irr.astype(np.float32)
            o.dist[:] = o.dist.astype(np.float32)
            o.irr_kappa[:] = 0.0
            o.dist_kappa[:] = 0.0
            gv.irradiance[..., :3].copy_(torch.from_numpy(o.irr.astype(np.float32)))
            gv.distance.copy_(torch.from_numpy(o.dist.astype(np.float32)))
        es = ctx.query_irradiance(pos, nrm, view).cpu().numpy()
        eo32, ko32 = oracle.query(ovr, q.pos, q.nrm, q.view)
        out.append(P.compare(f"{tag} query stage", es, eo32, ko32))
    return out


def check(verdicts, widened_max=WIDENED_MAX, beyond_max=BEYOND_MAX):
    """Prints every verdict; asserts none fails and the counts stay within
    their budgets."""
    for v in verdicts:
        print("[parity]", v.line(), flush=True)
    bad = [(v.name, v.fail, round(v.worst_allowed, 3), v.where[:3]) for v in verdicts if not v.ok]
    assert not bad, bad
    over = [(v.name, v.widened, v.beyond_cap, v.n) for v in verdicts
            if v.widened > widened_max * v.n or v.beyond_cap > beyond_max * v.n]
    assert not over, over


def flips(rec_g, rec_o):
    """Rays whose hit or shadow bits differ, and how many of them the oracle
    did not flag (must be none)."""
    import oracle
    f = (rec_g["tri"] != rec_o["tri"]) | (rec_g["vis"] != rec_o["vis"])
    return f, {"rays": len(f), "flips": int(f.sum()),
               "unflagged_flips": int((f & ((rec_o["flags"] & oracle.F_AMBIGUOUS) == 0)).sum())}
