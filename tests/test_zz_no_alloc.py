"""The allocation-free update frame (irf_update_probes_noalloc) against the
ordinary one (irf_update_probes): two calls in a row on one GPU -- the city
(2,048 probes x 256 rays, most of the static scratch), then the room (64
probes x 64 rays, a smaller layout over the previous call's contents) --
each compared bit for bit (atlases and states) with a separate context that
runs irf_update_probes on the same inputs; over-size frames and
differentiable contexts are refused before any launch."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _state(ctx):
    return [(v.irradiance.cpu().numpy().copy(), v.distance.cpu().numpy().copy(), v.states.cpu().numpy().copy())
            for v in ctx.volumes]


def _pair(torch, w, frames, tag):
    from paper_2009_10796_amd import irf
    a = irf.build_workload(w)     # irf_update_probes
    b = irf.build_workload(w)     # irf_update_probes_noalloc
    a.classify(w.classify_rotations)
    b.classify(w.classify_rotations)
    for gb, ga in zip(b.volumes, a.volumes):
        gb.states.copy_(ga.states)
    for f in frames:
        R = w.frame_rotation(f)
        a.update_probes(R)
        b.update_probes_noalloc(R)
        torch.cuda.synchronize()
        for v, (x, y) in enumerate(zip(_state(a), _state(b))):
            for name, p, q in zip(("irradiance", "distance", "states"), x, y):
                assert np.array_equal(p, q), f"{tag} frame {f} volume {v}: {name} differs"
        print(f"[no-alloc] {tag} frame {f}: atlases and states bit for bit", flush=True)
    with pytest.raises(irf.IrfError) as e:
        b.ray_records(0)
    assert e.value.status == irf.E_STATE
    a.close()
    b.close()


def test_noalloc_frames_match_the_allocating_frames(torch):
    print("[no-alloc] city 2048 probes x 256 rays", flush=True)
    _pair(torch, S.config1(gbuffer=False), (1, 2), "city")
    print("[no-alloc] room 64 probes x 64 rays (smaller, after the city)", flush=True)
    _pair(torch, S.config0(), (1, 2, 3), "room")


def test_noalloc_refuses_oversize_and_differentiable(torch):
    from paper_2009_10796_amd import irf
    w = S.config0()
    w.volumes = [S.VolumeDesc(origin=(0.5, 0.5, 0.5), spacing=(0.25, 0.25, 0.25), counts=(32, 32, 32),
                              rays_per_probe=256)]
    ctx = irf.build_workload(w)
    with pytest.raises(irf.IrfError) as e:
        ctx.update_probes_noalloc(w.frame_rotation(1))
    assert e.value.status == irf.E_UNSUPPORTED and "scratch" in str(e.value)
    ctx.close()
    ctx = irf.build_workload(S.config0())
    ctx.set_differentiable(True)
    with pytest.raises(irf.IrfError) as e:
        ctx.update_probes_noalloc(S.config0().frame_rotation(1))
    assert e.value.status == irf.E_UNSUPPORTED
    ctx.close()
