"""GPU tracking window and camera-aware volume blending (Sections "Tracking
Windows" and "Multiple Probe Volumes") against the FP64 oracle.

Workload: the city with a 9x5x9 tracking window of 1 m probes (64 rays)
inside a static 4 m volume covering the city; the camera moves 0.4 m in x
and 0.25 m in z per frame, so the window leapfrogs several times.  Per
frame: window shift, origin, phase and the classification of entering
planes; ray records and texels of both volumes; queries at surface points
around the camera, blended with the camera-centred weight.  Both sides run
the eight frames on their own atlases (the parity protocol substitutes the
GPU's decision on the rays the oracle flags and the two decide otherwise)."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests import gpu_helpers as G

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
    G.copy_states(ctx, ov, torch)
    cam0 = np.array([6.0, 2.5, 7.0], np.float32)      # the window centre
    rots = S.rotations(w.config, 5, start_frame=1000)
    shifts = 0
    q = S.surface_points(w.scene, 60000, 4)
    verdicts = []
    for f in range(1, 9):
        cam = (cam0 + np.float32([0.4 * f, 0.0, 0.25 * f])).astype(np.float32)
        sg = ctx.track_volume(0, cam, rots)
        so = oracle.track_volume(osc, ov[0], cam, rots)
        assert np.array_equal(sg, so), (f, sg, so)
        og, pg, cg = ctx.volume_window(0)
        assert np.array_equal(og, ov[0].origin) and np.array_equal(pg, ov[0].phase)
        assert np.array_equal(cg, ov[0].camera)
        shifts += int(np.abs(sg).sum())
        G.copy_states(ctx, ov, torch)
        vs, rep, _, _ = G.frame(torch, ctx, osc, ov, w.lights, w.frame_rotation(f), f"tracking frame {f} shift {sg.tolist()}")
        verdicts += vs
        if f % 3 == 0 or f == 8:
            # queries near the camera: the camera-centred blend of the window
            near = np.all(np.abs(q.pos - cam) < [5.0, 5.0, 5.0], axis=1)
            qn = S.Queries(q.pos[near], q.nrm[near], q.view[near])
            verdicts += G.queries(torch, ctx, ov, qn, f"tracking frame {f}", stage=False)
    G.check(verdicts)
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
