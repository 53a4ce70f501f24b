"""Cascaded volumes on the GPU against the FP64 oracle.

A scaled-down version of the terrain workload: fBm heightfield plus
extruded buildings, four concentric cascades (spacings 1, 2, 4, 8 m) whose
states the classification leaves uneven, a directional sun that moves 1
degree per frame, sky radiance.  Checked per volume: probe states, per-ray
hits and radiance, texels of frames 1-3; then queries at surface points,
which blend the cascades (Section "Multiple Probe Volumes").

The same checks on four cascades of 16x8x16 probes (8,192 probes, 32 rays):
above 4,096 probes the frame start compacts the active probes in two
passes (per-workgroup counts, then a scatter) instead of one workgroup.
Its third frame holds hits 0.016 m above the densest cascade's bottom probe
layer, where that cascade's blend weight is a small difference of float32
coordinates (~27 m) and so carries ~1e-4 relative error: the oracle's
float32 sensitivity takes the rounding of the hit point's coordinates into
account.
"""
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


def small_terrain(cascade_counts=(8, 4, 8), rays=64):
    return S.config3(grid_vertices=97, size=48.0, n_buildings=12, cascade_counts=cascade_counts,
                     spacings=(1.0, 2.0, 4.0, 8.0), rays=rays, center_height=3.0)


def test_cascades_parity(torch):
    _cascades_parity(torch, small_terrain())


def test_two_pass_compaction_parity(torch):
    w = small_terrain(cascade_counts=(16, 8, 16), rays=32)
    total = sum(d.n_probes for d in w.volumes)
    print(f"[cascade] {total} probes in {len(w.volumes)} volumes", flush=True)
    assert total > 4096
    _cascades_parity(torch, w)


def _cascades_parity(torch, w, frames=(1, 2, 3)):
    import oracle
    from paper_2009_10796_amd import irf
    ctx = irf.build_workload(w)
    osc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    ctx.classify(w.classify_rotations)
    oracle.classify(osc, ov, w.classify_rotations)
    for v, o in enumerate(ov):
        print(f"[cascade] volume {v} states {np.bincount(o.states, minlength=6)}", flush=True)
    print(f"[cascade] classification differs on {G.copy_states(ctx, ov, torch)} probes", flush=True)
    verdicts = []
    for f in frames:
        L = S.sun_for_frame(f)
        ctx.set_lights(L)
        vs, _, _, _ = G.frame(torch, ctx, osc, ov, L, w.frame_rotation(f), f"cascade frame {f}")
        verdicts += vs
    # queries at surface points: cascade blend, end to end and on the oracle's atlases
    verdicts += G.queries(torch, ctx, ov, S.surface_points(w.scene, 20000, 3), "cascade")
    G.check(verdicts)
    ctx.close()
