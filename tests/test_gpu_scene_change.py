"""Replacing the scene of a live context (a later irf_set_scene call).

Frame 1 runs on the room; then the scene is replaced by the same room
without its dynamic box (other triangles, another tree, no dynamic object)
and frame 2 runs on it, shading its hits with the frame-1 atlases.  The
oracle does the same (frame 1 on the first scene, frame 2 on the second):
states, ray records (hits in the new tree), radiance and texels, then the
query."""
import dataclasses

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


def _without_dynamic(scene):
    keep = scene.tri_object == 0
    return dataclasses.replace(scene, indices=scene.indices[keep].copy(), tri_material=scene.tri_material[keep].copy(),
                               tri_object=scene.tri_object[keep].copy())


def test_scene_replaced_between_frames(torch):
    import oracle
    from paper_2009_10796_amd import irf
    w = S.config0()
    scene_b = _without_dynamic(w.scene)
    assert 0 < len(scene_b.indices) < len(w.scene.indices) and not scene_b.tri_object.any()
    ctx = irf.build_workload(w)
    gv = ctx.volumes[0]
    osc_a, osc_b = oracle.Scene(w.scene), oracle.Scene(scene_b)
    o = oracle.Volume(w.volumes[0])
    ctx.classify(w.classify_rotations)
    oracle.classify(osc_a, [o], w.classify_rotations)
    assert G.copy_states(ctx, [o], torch) <= 1
    verdicts = []
    for f, (osc, scene) in ((1, (osc_a, None)), (2, (osc_b, scene_b))):
        if scene is not None:
            ctx.set_scene(scene)
        vs, rep, _, _ = G.frame(torch, ctx, osc, [o], w.lights, w.frame_rotation(f), f"scene change frame {f}")
        verdicts += vs
        print(f"[scene change] frame {f}: states {np.bincount(o.states, minlength=6)}", flush=True)
    verdicts += G.queries(torch, ctx, [o], w.queries, "scene change")
    G.check(verdicts)
    ctx.close()
