"""Blend variants on the GPU against the FP64 oracle.

* f32_valu: the vector-ALU blend (one workgroup per probe) must meet the same
  parity bar as the float32 matrix-core blend used by default.
* bf16 / f16 inputs on the matrix cores with float32 accumulation and float32
  normalisation, atlases stored in float32 or float16: the relative error
  against the oracle (floor tau = 1e-3 of the channel's largest value) is
  measured per atlas channel -- irradiance R, G, B, mean distance mu and
  mean squared distance mu2 -- after the second frame, as max and p99, and
  held to its a-priori bound: the input rounding u_in (2^-8 for bf16, 2^-11
  for f16) of the weights and of the ray values moves a normalised weighted
  mean by at most u_in of the largest value plus u_in of the value spread
  (<= 4 u_in relative at the floor), float16 storage adds its rounding
  (2^-11, twice: the frame-1 and the frame-2 texel).  The mode claimed to
  meet the precision gate of 1e-3 relative irradiance error (f16 inputs,
  float32 atlases) is asserted at 1e-3; bf16 inputs do not meet it (their
  8-bit significand on the weights and values alone allows ~4e-3).
"""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests import gpu_helpers as G
from tests import parity as P

pytestmark = pytest.mark.gpu

CHANNELS = ("E.R", "E.G", "E.B", "mu", "mu2")


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(torch, w, frames=(1, 2)):
    """Frames through the parity protocol (substitution on flagged rays);
    returns the context, the oracle volumes and the last frame's verdicts."""
    import oracle
    from paper_2009_10796_amd import irf
    ctx = irf.build_workload(w)
    osc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    ctx.classify(w.classify_rotations)
    oracle.classify(osc, ov, w.classify_rotations)
    G.copy_states(ctx, ov, torch)
    verdicts = []
    for f in frames:
        vs, _, _, _ = G.frame(torch, ctx, osc, ov, w.lights, w.frame_rotation(f), f"blend {w.volumes[0].blend} frame {f}")
        verdicts += vs
    return ctx, ov, verdicts


def channel_errors(ctx, ov):
    """Per channel (E.R, E.G, E.B, mu, mu2): (max, p99) of |g - o| / max(|o|, tau)."""
    gi, gd = G.gpu_atlases(ctx.volumes[0])
    out = {}
    for names, g, o in ((CHANNELS[:3], gi, ov[0].irr), (CHANNELS[3:], gd, ov[0].dist)):
        rel = np.abs(g - o) / np.maximum(np.abs(o), P.channel_tau(o))
        for c, name in enumerate(names):
            r = rel[..., c].ravel()
            out[name] = (float(r.max()), float(np.quantile(r, 0.99)))
    return out


@pytest.mark.parametrize("mode", ["f32_valu", "f32"])
def test_f32_blend_parity_room(torch, mode):
    """Both float32 blends meet the parity bar of the main test."""
    w = S.config0()
    for d in w.volumes:
        d.blend = mode
    ctx, ov, verdicts = _run(torch, w)
    G.check(verdicts)
    print(f"[blend] {mode} room: per-channel (max, p99) {channel_errors(ctx, ov)}", flush=True)
    ctx.close()


@pytest.mark.parametrize("mode,atlas16", [("bf16", False), ("f16", False), ("bf16", True), ("f16", True),
                                          ("f32", True)])
def test_low_precision_blend_error_city(torch, mode, atlas16):
    w = S.config1(gbuffer=False)
    for d in w.volumes:
        d.blend = mode
        d.atlas_f16 = atlas16
    ctx, ov, _ = _run(torch, w)
    e = channel_errors(ctx, ov)
    print(f"[blend] city mode={mode} atlas_f16={atlas16}: per-channel (max, p99) relative error "
          + ", ".join(f"{k} ({a:.2e}, {b:.2e})" for k, (a, b) in e.items()), flush=True)
    u_in = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11, "f32": 2.0 ** -23}[mode]
    u_st = 2 * 2.0 ** -11 if atlas16 else 0.0
    bound_max = 4 * u_in + u_st + 1e-5
    bound_p99 = 2 * u_in + u_st + 1e-5
    for k, (mx, p99) in e.items():
        assert mx <= bound_max and p99 <= bound_p99, (k, mx, p99, bound_max, bound_p99)
    if mode == "f16" and not atlas16:
        assert max(e[c][0] for c in CHANNELS[:3]) <= 1e-3, e    # the precision gate
    ctx.close()


@pytest.mark.parametrize("mode", ["f32", "bf16", "f16"])
def test_blend_tile_shapes_are_bit_exact(torch, mode):
    """The blend's tile shape (1, 2 or 4 workgroups per block of 8 probes)
    changes which workgroup multiplies a row tile, not the order of its
    products: atlases and states after two city frames are the same bits."""
    from paper_2009_10796_amd import irf
    w = S.config1(gbuffer=False)
    for d in w.volumes:
        d.blend = mode
    out = {}
    for rsplit in (4, 2, 1):
        ctx = irf.build_workload(w)
        ctx.set_tuning(blend_rsplit=rsplit)
        ctx.classify(w.classify_rotations)
        for f in (1, 2):
            ctx.update_probes(w.frame_rotation(f))
        torch.cuda.synchronize()
        out[rsplit] = [(v.irradiance.cpu().numpy().copy(), v.distance.cpu().numpy().copy(),
                        v.states.cpu().numpy().copy()) for v in ctx.volumes]
        ctx.close()
    for rsplit in (2, 1):
        for a, b in zip(out[4], out[rsplit]):
            for x, y in zip(a, b):
                assert np.array_equal(x, y), (mode, rsplit)
