"""GPU tracking window and camera-aware volume blending (Sections "Tracking
Windows" and "Multiple Probe Volumes") against the FP64 oracle.

Workload: the city with a 9x5x9 tracking window of 1 m probes (64 rays)
inside a static 4 m volume covering the city; the camera moves 0.4 m in x
and 0.25 m in z per frame, so the window leapfrogs several times.  Per
frame: window shift, origin, phase and the classification of entering
planes; ray records and texels of both volumes; queries at surface points
around the camera, blended with the camera-centred weight.  Every frame
starts from identical inputs: the oracle's atlases, rounded to float32, are
given to both sides (oracle -> GPU input), so each frame is checked alone
and rays the float32 tracer decides otherwise do not spread."""
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
    w = S.config1(gbuffer=False)
    w.volumes = [
        S.VolumeDesc(origin=(2.0, 0.5, 3.0), spacing=(1.0, 1.0, 1.0), counts=(9, 5, 9), rays_per_probe=64,
                     tracking=True),
        S.VolumeDesc(origin=(-2.0, -2.0, -2.0), spacing=(4.0, 4.0, 4.0), counts=(6, 4, 6), rays_per_probe=64),
    ]
    return w


def test_tracking_window_parity(torch):
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
        assert len(diff) <= max(2, 0.01 * len(gs))
        gs[diff] = o.states[diff]
        gv.states.copy_(torch.from_numpy(gs))
    cam0 = np.array([6.0, 2.5, 7.0], np.float32)      # the window centre
    rots = S.rotations(w.config, 5, start_frame=1000)
    shifts = 0
    q = S.surface_points(w.scene, 60000, 4)
    for f in range(1, 9):
        for gv, o in zip(ctx.volumes, ov):
            o.irr[:] = o.irr.astype(np.float32)
            o.dist[:] = o.dist.astype(np.float32)
            o.irr_kappa[:] = 0.0
            o.dist_kappa[:] = 0.0
            gv.irradiance[..., :3].copy_(torch.from_numpy(o.irr.astype(np.float32)))
            gv.distance.copy_(torch.from_numpy(o.dist.astype(np.float32)))
        cam = (cam0 + np.float32([0.4 * f, 0.0, 0.25 * f])).astype(np.float32)
        sg = ctx.track_volume(0, cam, rots)
        so = oracle.track_volume(osc, ov[0], cam, rots)
        assert np.array_equal(sg, so), (f, sg, so)
        og, pg, cg = ctx.volume_window(0)
        assert np.array_equal(og, ov[0].origin) and np.array_equal(pg, ov[0].phase)
        assert np.array_equal(cg, ov[0].camera)
        shifts += int(np.abs(sg).sum())
        gs = ctx.volumes[0].states.cpu().numpy()
        diff = np.nonzero(gs != ov[0].states)[0]
        assert len(diff) <= max(2, 0.01 * len(gs)), (f, len(diff))
        if len(diff):
            gs[diff] = ov[0].states[diff]
            ctx.volumes[0].states.copy_(torch.from_numpy(gs))
        R = w.frame_rotation(f)
        ctx.update_probes(R)
        rec_all = oracle.update_frame(osc, w.lights, ov, R)
        torch.cuda.synchronize()
        off = 0
        for v, gv in enumerate(ctx.volumes):
            rec_g = ctx.ray_records(v)
            rec_o = rec_all[off: off + len(rec_g)]
            off += len(rec_g)
            assert np.array_equal(gv.states.cpu().numpy(), ov[v].states)
            tainted, _, rep = compare_records(rec_g, rec_o)
            assert rep["unflagged_flips"] == 0
            ok, _ = within(rec_g["rgb"][~tainted], rec_o["rgb"][~tainted], kappa=rec_o["kappa"][~tainted])
            assert ok.all(), (f, v, np.argwhere(~ok)[:5])
            tp = np.unique(rec_g["probe"][tainted])
            clean = [p for p in range(gv.n_probes) if p not in set(tp.tolist())]
            worst, bad = texel_check(gv, ov[v], clean, rec_o, slots_of(rec_g, w.volumes[v].rays_per_probe))
            print(f"[tracking] frame {f} shift {sg.tolist()} volume {v}: {rep} texel worst {worst:.3f}, "
                  f"probes checked {len(clean)} of {gv.n_probes}", flush=True)
            assert not bad, (f, v, bad[:5])
            assert rep["tainted"] <= 0.01 * rep["rays"] + 2
        assert off == len(rec_all)
        if f % 3 == 0 or f == 8:
            # queries near the camera: the camera-centred blend of the window
            near = np.all(np.abs(q.pos - cam) < [5.0, 5.0, 5.0], axis=1)
            pos, nrm, view = q.pos[near], q.nrm[near], q.view[near]
            eg = ctx.query_irradiance(*(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (pos, nrm, view)))
            eo, ko = oracle.query(ov, pos, nrm, view)
            ok, _ = within(eg.cpu().numpy(), eo, kappa=32 * ko)
            print(f"[tracking] frame {f} queries {len(pos)} fail={int((~ok).any(1).sum())}", flush=True)
            assert (~ok).any(1).mean() <= 1e-3
    assert shifts >= 3
    ctx.close()


def test_tracking_requires_a_tracking_volume(torch):
    from paper_2009_10796_amd import irf
    w = S.config0()
    ctx = irf.build_workload(w)
    with pytest.raises(irf.IrfError) as e:
        ctx.track_volume(0, [4.0, 4.0, 4.0], S.rotations(0, 1))
    assert e.value.status == irf.E_STATE
    ctx.close()
