"""Ragged shapes against the FP64 oracle: two volumes whose ray counts (96
and 32) are not multiples of the 64-lane wave, odd probe counts, and four
lights (the room's sun plus three point lights) -- so trace waves straddle
probe and volume boundaries, each wave's shadow slice mixes lights and
probes, and the per-batch slice map, the shadow origins carried by the tasks
and the light-side point-light segments are all exercised; the state step
runs with the room's dynamic box.  Two update frames (ray records, texels,
states) and the query on both volumes."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests.gpu_helpers import compare_records, slots_of, texel_check, within

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _workload():
    w = S.config0()
    w.volumes = [
        S.VolumeDesc(origin=(1.3, 1.1, 1.2), spacing=(2.7, 2.9, 2.6), counts=(3, 2, 3), rays_per_probe=96),
        S.VolumeDesc(origin=(0.7, 0.6, 0.9), spacing=(1.55, 1.7, 1.45), counts=(5, 3, 5), rays_per_probe=32),
    ]
    L = w.lights
    w.lights = S.Lights(L.dir_to_light, L.dir_irradiance,
                        np.array([[4.1, 6.3, 3.7], [1.6, 2.2, 6.4], [6.6, 4.4, 1.9]], np.float32),
                        np.array([[8.0, 6.0, 4.0], [3.0, 5.0, 9.0], [6.0, 6.0, 6.0]], np.float32),
                        np.array([0.1, 0.2, 0.3], np.float32))
    return w


def test_ragged_volumes_and_mixed_lights(torch):
    import oracle
    from paper_2009_10796_amd import irf
    w = _workload()
    ctx = irf.build_workload(w)
    osc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    ctx.classify(w.classify_rotations)
    oracle.classify(osc, ov, w.classify_rotations)
    for v, (gv, o) in enumerate(zip(ctx.volumes, ov)):
        gs = gv.states.cpu().numpy()
        diff = np.nonzero(gs != o.states)[0]
        print(f"[ragged] volume {v} states {np.bincount(o.states, minlength=6)} differ={len(diff)}", flush=True)
        assert len(diff) <= max(2, 0.01 * len(gs))
        if len(diff):
            gs[diff] = o.states[diff]
            gv.states.copy_(torch.from_numpy(gs))
    bases = np.cumsum([0] + [d.n_probes for d in w.volumes])
    taints = [np.zeros(0, np.int64) for _ in ov]
    shadow_rays = 0
    for f in (1, 2):
        R = w.frame_rotation(f)
        ctx.update_probes(R)
        rec_o_all = oracle.update_frame(osc, w.lights, ov, R)
        torch.cuda.synchronize()
        shadow_rays += ctx.frame_stats()["shadow_rays"]
        off = 0
        new_taint = []
        # the first volume ends mid-wave (17 active probes x 96 rays), the frame
        # in a partial wave
        assert len(ctx.ray_records(0)) % 64 != 0 and len(rec_o_all) % 64 != 0
        for v, gv in enumerate(ctx.volumes):
            rec_g = ctx.ray_records(v)
            rec_o = rec_o_all[off: off + len(rec_g)]
            off += len(rec_g)
            assert len(rec_g) % w.volumes[v].rays_per_probe == 0
            assert np.array_equal(gv.states.cpu().numpy(), ov[v].states)
            tainted, _, rep = compare_records(rec_g, rec_o, np.concatenate(taints))
            print(f"[ragged] frame {f} volume {v}: {rep}", flush=True)
            assert rep["unflagged_flips"] == 0
            assert rep["tainted"] <= 0.01 * rep["rays"] + 2
            ok, _ = within(rec_g["rgb"][~tainted], rec_o["rgb"][~tainted], kappa=rec_o["kappa"][~tainted])
            assert ok.all(), np.argwhere(~ok)[:5]
            tp = np.unique(rec_g["probe"][tainted])
            cp = [q for q in range(gv.n_probes) if q not in set(tp.tolist())]
            worst, bad = texel_check(gv, ov[v], cp, rec_o, slots_of(rec_g, w.volumes[v].rays_per_probe))
            print(f"[ragged] frame {f} volume {v}: texel worst err/tol {worst:.3f}", flush=True)
            assert not bad, bad[:5]
            new_taint.append(tp.astype(np.int64) + bases[v])
        assert off == len(rec_o_all)
        taints = new_taint
    assert shadow_rays > 0
    # query stage on the oracle's atlases (rounded to float32)
    q = S.surface_points(w.scene, 6000, 0)
    for gv, o in zip(ctx.volumes, ov):
        gv.irradiance[..., :3].copy_(torch.from_numpy(o.irr.astype(np.float32)))
        gv.distance.copy_(torch.from_numpy(o.dist.astype(np.float32)))
        o.irr[:] = o.irr.astype(np.float32)
        o.dist[:] = o.dist.astype(np.float32)
    e = ctx.query_irradiance(torch.from_numpy(q.pos).cuda(), torch.from_numpy(q.nrm).cuda(),
                             torch.from_numpy(q.view).cuda()).cpu().numpy()
    eo, ko = oracle.query(ov, q.pos, q.nrm, q.view)
    ok, _ = within(e, eo, kappa=ko)
    print(f"[ragged] query stage: fail={int((~ok).any(1).sum())} of {len(e)}", flush=True)
    assert ok.all(), np.argwhere(~ok)[:5]
    ctx.close()
