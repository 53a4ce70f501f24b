"""Shared helpers of the GPU parity tests: run a workload through the HIP
library and through the oracle on the same seeded inputs, and compare.

Tolerances.  Floating-point results are compared per element as
|gpu - oracle| <= 1e-5 * max(|oracle|, tau) + 8 u kappa, with tau = 1e-3 x
the largest |oracle| value of that channel, u = 2^-24 and kappa the
oracle's own estimate of the float32 sensitivity of that value (large only
where the Chebyshev visibility weight is ill-conditioned).  Rays whose
nearest hit or shadow decision differs between the float32 tracer and the
oracle are accepted only where the oracle flagged them as ambiguous; such
rays, the probes they feed and (next frame) the rays whose hit-shading query
used those probes are 'tainted' and checked by validity instead of value.
"""
import numpy as np

U32 = 2.0 ** -24


def tau(o, axis=0):
    return 1e-3 * np.max(np.abs(o), axis=axis, keepdims=True) + 1e-30


def within(g, o, kappa=None, rel=1e-5, tau_v=None):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    t = tau(o.reshape(-1, o.shape[-1]) if o.ndim > 1 else o.reshape(-1, 1)) if tau_v is None else tau_v
    tol = rel * np.maximum(np.abs(o), t.reshape((1,) * (o.ndim - 1) + (-1,)) if o.ndim > 1 else t.ravel()[0])
    if kappa is not None:
        tol = tol + 8 * U32 * np.asarray(kappa)
    return np.abs(g - o) <= tol, tol


def run_classify(ctx, w, o_scene, o_vols):
    import oracle
    ctx.classify(w.classify_rotations)
    nb, nf, tf = oracle.classify(o_scene, o_vols, w.classify_rotations)
    return nb, nf, tf


def gpu_states(ctx):
    return [v.states.cpu().numpy() for v in ctx.volumes]


def sync_states_check(ctx, o_vols):
    g = gpu_states(ctx)
    return [np.array_equal(a, v.states) for a, v in zip(g, o_vols)]


def compare_records(g, o, taint_probes_prev=None, probe_base=0):
    """Per-ray comparison of one volume.  Returns (tainted_ray_mask, report)."""
    assert len(g) == len(o), (len(g), len(o))
    flip_tri = g["tri"] != o["tri"]
    flip_vis = g["vis"] != o["vis"]
    flagged = o["flags"] != 0
    bad_flip = (flip_tri | flip_vis) & ~flagged
    tainted = flip_tri | flip_vis
    if taint_probes_prev is not None and taint_probes_prev.size:
        cage = o["cage"]
        used_tainted = np.isin(cage, taint_probes_prev) & (cage >= 0)
        tainted = tainted | used_tainted.any(axis=1)
    report = {"rays": len(g), "flagged": int(flagged.sum()), "flips": int((flip_tri | flip_vis).sum()),
              "unflagged_flips": int(bad_flip.sum()), "tainted": int(tainted.sum())}
    return tainted, bad_flip, report


def texel_check(gv, ov, probes, rec_o=None, slot_of=None, rel=1e-5):
    """Compare the atlases of `probes` (oracle float64 vs GPU): per texel
    |g - o| <= rel * max(|o|, tau) + 8 u kappa, kappa = the oracle's float32
    sensitivity of that texel (its rays' radiance, its blend weights and
    rounding, carried through the hysteresis)."""
    gi = gv.irradiance[..., :3].float().cpu().numpy().astype(np.float64)
    gd = gv.distance.float().cpu().numpy().astype(np.float64)
    oi, od = ov.irr, ov.dist
    ti = tau(oi.reshape(-1, 3))
    td = tau(od.reshape(-1, 2))
    worst = 0.0
    bad = []
    for q in probes:
        tol_i = rel * np.maximum(np.abs(oi[q]), ti.reshape(1, 1, 3)) + 8 * U32 * ov.irr_kappa[q]
        tol_d = rel * np.maximum(np.abs(od[q]), td.reshape(1, 1, 2)) + 8 * U32 * ov.dist_kappa[q]
        ei = np.abs(gi[q] - oi[q]) / tol_i
        ed = np.abs(gd[q] - od[q]) / tol_d
        m = max(ei.max(), ed.max())
        worst = max(worst, m)
        if m > 1:
            bad.append((q, float(ei.max()), float(ed.max())))
    return worst, bad


def slots_of(rec_g, n_rays):
    probes = rec_g["probe"]
    probe_list = probes[::n_rays]
    return {int(q): np.arange(i * n_rays, (i + 1) * n_rays) for i, q in enumerate(probe_list)}
