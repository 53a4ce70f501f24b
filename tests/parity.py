"""The parity protocol: compare a float32 implementation of the probe
update and query (the HIP library, or the oracle's own float32 build) with
the FP64 oracle on the same seeded inputs.

Per update frame (Section "Probe Update", Eq. U):

1. The oracle runs the frame.  Every ray whose nearest hit or shadow
   decisions differ between the candidate and the oracle must carry an
   oracle flag (grazing hit, tie, near miss, edge-on, ambiguous shadow ray).
2. Substitution: the oracle runs the frame again from the same start with
   the candidate's decisions on exactly those rays (its own exact distance
   to the candidate's triangle), so every ray, texel and probe is then
   compared by value and the next frame starts from comparable atlases.
3. Every float result is compared per element against the scale
   s = max(|o|, tau), tau = 1e-3 x the largest |o| of its channel.  The
   rule is the plain |g - o| <= 1e-5 s.  Only where the oracle's float32
   sensitivity kappa of the element says float32 cannot reach that
   (8 u kappa > 1e-5 s) is an element allowed more, and then at most
   min(1e-5 s + 8 u kappa, 1e-3 s); such elements are counted ("widened").
   An element whose allowance exceeds that cap (8 u kappa > 1e-3 s, e.g. a
   hit whose previous-frame query rests on a Chebyshev variance that nearly
   cancels) cannot be held to 1e-3 by any float32 evaluation -- the oracle's
   own steps run in float32 miss it there too -- and is allowed
   1e-5 s + 8 u kappa and counted ("beyond 1e-3").

   kappa is the oracle's estimate of the float32 sensitivity of the element
   (units of u = 2^-24); it is checked as an error bound by running the
   oracle's own steps in float32 through this same protocol
   (tests/test_oracle_kappa_f32.py).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import oracle

U32 = 2.0 ** -24
REL = 1e-5
CAP = 1e-3


def channel_tau(o: np.ndarray) -> np.ndarray:
    """Per channel (last axis): 1e-3 x the largest |value|."""
    o2 = np.abs(np.asarray(o, np.float64)).reshape(-1, o.shape[-1])
    return 1e-3 * (o2.max(axis=0) if o2.size else np.zeros(o.shape[-1])) + 1e-300


@dataclass
class Verdict:
    name: str
    n: int = 0
    plain_pass: int = 0
    widened: int = 0             # beyond 1e-5 s, within the kappa allowance capped at 1e-3 s
    beyond_cap: int = 0          # beyond 1e-5 s, kappa allowance above 1e-3 s
    fail: int = 0
    worst_plain: float = 0.0     # max err / (1e-5 s)
    worst_allowed: float = 0.0   # max err / allowed
    max_rel: float = 0.0         # max err / s
    where: list = field(default_factory=list)

    @property
    def ok(self) -> bool:
        return self.fail == 0

    def line(self) -> str:
        rate = self.plain_pass / max(self.n, 1)
        return (f"{self.name}: n={self.n} plain-1e-5 pass {rate:.6f} (max rel {self.max_rel:.2e}, "
                f"worst/1e-5 {self.worst_plain:.2f}) widened {self.widened} beyond-1e-3 {self.beyond_cap} "
                f"worst/allowed {self.worst_allowed:.3f} fail {self.fail}")


def compare(name: str, g, o, kappa=None, tau=None) -> Verdict:
    """Element-wise comparison of candidate g with oracle o (channels on the
    last axis) under the rule above."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    assert g.shape == o.shape, (name, g.shape, o.shape)
    v = Verdict(name, n=int(o.size))
    if o.size == 0:
        return v
    t = channel_tau(o) if tau is None else np.asarray(tau, np.float64)
    s = np.maximum(np.abs(o), t)
    err = np.abs(g - o)
    err = np.where(np.isnan(err), np.inf, err)
    plain = REL * s
    widen = 8 * U32 * (np.zeros_like(o) if kappa is None else np.asarray(kappa, np.float64))
    undet = widen > CAP * s
    allowed = np.where(undet, plain + widen, np.minimum(plain + widen, CAP * s))
    allowed = np.maximum(allowed, plain)
    ok_plain = err <= plain
    bad = err > allowed
    v.plain_pass = int(ok_plain.sum())
    v.widened = int((~ok_plain & ~bad & ~undet).sum())
    v.beyond_cap = int((~ok_plain & ~bad & undet).sum())
    v.fail = int(bad.sum())
    v.worst_plain = float((err / plain).max())
    v.worst_allowed = float((err / allowed).max())
    v.max_rel = float((err / s).max())
    v.where = [tuple(int(i) for i in b) for b in np.argwhere(bad)[:8]]
    return v


def restore(vols, saved) -> None:
    """Copy the state of `saved` (oracle.copy_volumes) back into `vols` in place."""
    for v, p in zip(vols, saved):
        v.irr[:] = p.irr
        v.dist[:] = p.dist
        v.irr_kappa[:] = p.irr_kappa
        v.dist_kappa[:] = p.dist_kappa
        v.states[:] = p.states
        v.offsets[:] = p.offsets
        v.origin[:] = p.origin
        v.phase[:] = p.phase
        v.camera[:] = p.camera


@dataclass
class FrameReport:
    rays: int
    flagged: int
    flips: int
    unflagged_flips: int
    substituted: int

    def line(self) -> str:
        return (f"rays {self.rays} flagged {self.flagged} flips {self.flips} (unflagged {self.unflagged_flips}) "
                f"substituted {self.substituted}")


def oracle_frame(scene, lights, vols, R, cand_tri, cand_vis):
    """Steps 1-2 of the protocol for one frame of all volumes: runs the
    oracle frame in place on `vols`; where the candidate's hits or shadow
    bits differ (each such ray must be flagged) runs it again from the same
    start with the candidate's decisions on those rays.  Returns the oracle's
    records and a FrameReport."""
    saved = oracle.copy_volumes(vols)
    rec = oracle.update_frame(scene, lights, vols, R)
    cand_tri = np.asarray(cand_tri, np.int32)
    cand_vis = np.asarray(cand_vis, np.uint32)
    assert len(rec) == len(cand_tri) == len(cand_vis), (len(rec), len(cand_tri))
    flip = (rec["tri"] != cand_tri) | (rec["vis"] != cand_vis)
    flagged = (rec["flags"] & oracle.F_AMBIGUOUS) != 0
    rep = FrameReport(rays=len(rec), flagged=int(flagged.sum()), flips=int(flip.sum()),
                      unflagged_flips=int((flip & ~flagged).sum()), substituted=0)
    if flip.any():
        restore(vols, saved)
        mask = np.where(flip, 3, 0).astype(np.uint8)
        rec = oracle.update_frame(scene, lights, vols, R, force=(mask, cand_tri, cand_vis))
        assert not np.any(rec["flags"] & oracle.F_FORCE_INVALID), "a substituted triangle is not on its ray"
        assert np.array_equal(rec["tri"], cand_tri) and np.array_equal(rec["vis"], cand_vis)
        rep.substituted = int(flip.sum())
    return rec, rep


def origin_magnitude(vols, counts):
    """Per ray: a bound on the largest |coordinate| of its probe's position
    (per volume, from its window, grid and offsets); counts = rays recorded
    per volume, in order."""
    out = []
    for v, n in zip(vols, counts):
        d = v.desc
        o = np.asarray(v.origin, np.float64)
        far = o + (np.asarray(d.counts) - 1) * np.asarray(d.spacing, np.float64)
        m = float(np.maximum(np.abs(o), np.abs(far)).max() + np.abs(v.offsets).max(initial=0.0))
        out.append(np.full(int(n), m))
    return np.concatenate(out) if out else np.zeros(0)


def active_counts(vols):
    """Rays recorded per volume by the last frame (active probes x rays)."""
    act = (oracle.NEWLY_AWAKE, oracle.NEWLY_VIGILANT, oracle.AWAKE, oracle.VIGILANT)
    return [int(np.isin(v.states, act).sum()) * v.desc.rays_per_probe for v in vols]


def ray_checks(tag, g_rgb, g_d, g_t, rec, o_mag=None):
    """Per-ray radiance, recorded distance and hit distance (identical hits
    after substitution).  o_mag: per ray, the magnitude of its origin's
    coordinates (None: 0)."""
    out = [compare(f"{tag} ray radiance", g_rgb, rec["rgb"], rec["kappa"]),
           compare(f"{tag} ray distance", np.asarray(g_d)[:, None], rec["d"][:, None], rec["d_kappa"][:, None])]
    hit = rec["tri"] >= 0
    om = np.zeros(len(rec)) if o_mag is None else np.asarray(o_mag, np.float64)
    # float32 ray direction and origin: t moves by ~u (t + 4 |o|) / |cos incidence|
    t = rec["t"][hit]
    t_tol = 2e-6 * t + 8 * U32 * (t + 4 * om[hit]) / np.maximum(rec["cosi"][hit], 1e-6)
    t_bad = int((np.abs(np.asarray(g_t)[hit] - t) > t_tol).sum())
    return out, t_bad


def texel_checks(tag, g_irr, g_dist, vol):
    """Every texel (borders included) of every probe of one volume."""
    return [compare(f"{tag} irradiance texels", g_irr, vol.irr, vol.irr_kappa),
            compare(f"{tag} distance texels", g_dist, vol.dist, vol.dist_kappa)]
