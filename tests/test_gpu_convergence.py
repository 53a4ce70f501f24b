"""GPU parity of the convergence refinements (Sections "Perception-based
exponential encoding" and "Fast Convergence Heuristics") against the FP64
oracle: irradiance texels stored to the power 1/5 and blended in that
encoding, per-texel hysteresis thresholds, the query's gamma-2 cage blend.

Workloads: the room with a lighting change (the emissive quad drops to 5 %
and comes back, so texels cross both thresholds), through the matrix-core
and the vector-ALU blends; the full city (frames 1-2 and the G-buffer
query); and closed forms on the GPU alone (uniform sky, furnace)."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu
GAMMA = 5.0


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _encoded(w, blend="f32", thresholds=True):
    for d in w.volumes:
        d.irradiance_gamma = GAMMA
        d.texel_thresholds = thresholds
        d.blend = blend
    return w


def _run_frames(torch, ctx, w, osc, ov, schedule, name):
    """schedule: list of (frame, emission float32 [M,3] or None)."""
    hit_threshold = 0
    verdicts = []
    for f, em in schedule:
        if em is not None:
            ctx.set_emission(torch.from_numpy(em).cuda())
            osc.set_emission(em.astype(np.float64))
        old = ov[0].irr.copy()
        vs, rep, _, _ = G.frame(torch, ctx, osc, ov, w.lights, w.frame_rotation(f), f"convergence {name} frame {f}")
        verdicts += vs
        # with hysteresis 0.97 a texel moves by 3 % of its change, at most
        # 0.0075 below the 0.25 threshold; a lowered hysteresis moves it by
        # at least 18 % of a change above 0.25 (0.045): count those (frames
        # after the converge frame)
        moved = np.abs(ov[0].irr - old).max(-1)[:, 1:7, 1:7]
        lowered = int((moved > 0.02).sum()) if f > 1 else 0
        hit_threshold += lowered if f > 2 else 0
        print(f"[convergence] {name} frame {f}: texels with lowered hysteresis: {lowered}", flush=True)
    G.check(verdicts)
    return hit_threshold


def _query_parity(torch, ctx, w, ov, name):
    G.check(G.queries(torch, ctx, ov, w.queries, f"convergence {name}"))


def _setup(torch, w):
    import oracle
    from paper_2009_10796_amd import irf
    ctx = irf.build_workload(w)
    osc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    ctx.classify(w.classify_rotations)
    oracle.classify(osc, ov, w.classify_rotations)
    G.copy_states(ctx, ov, torch)
    return ctx, osc, ov


@pytest.mark.parametrize("blend", ["f32", "f32_valu"])
def test_encoded_room_with_lighting_change(torch, blend):
    w = _encoded(S.config0(), blend=blend)
    ctx, osc, ov = _setup(torch, w)
    em = w.scene.emission.astype(np.float32)
    dim = (em * np.float32(0.05)).astype(np.float32)
    schedule = [(1, None), (2, None), (3, dim), (4, dim), (5, em), (6, em)]
    crossed = _run_frames(torch, ctx, w, osc, ov, schedule, f"room/{blend}")
    assert crossed > 100        # the lighting change exercised the thresholds
    _query_parity(torch, ctx, w, ov, f"room/{blend}")
    ctx.close()


def test_encoded_city(torch):
    w = _encoded(S.config1())
    ctx, osc, ov = _setup(torch, w)
    _run_frames(torch, ctx, w, osc, ov, [(1, None), (2, None)], "city")
    _query_parity(torch, ctx, w, ov, "city")
    ctx.close()


def test_encoded_closed_forms_on_gpu(torch):
    """No oracle: uniform sky gives texels L^(1/5) and queries L; the furnace
    follows x_k = a x + (1 - a)(Le + rho x^5)^(1/5) in stored units."""
    from paper_2009_10796_amd import irf
    L = np.float32([0.4, 0.9, 1.3])
    d = S.VolumeDesc(origin=(0, 0, 0), spacing=(1, 1, 1), counts=(3, 2, 2), rays_per_probe=64, irradiance_gamma=GAMMA)
    ctx = irf.build_workload(S.Workload("sky", 0, S.empty_scene(), S.no_lights(sky=tuple(L)), [d]))
    ctx.update_probes(S.rotations(0, 1)[0])
    irr = ctx.volumes[0].irradiance[..., :3].cpu().numpy()
    assert np.allclose(irr, L.astype(np.float64) ** (1 / GAMMA), rtol=4e-6)
    st = S.Stream(961, 1)
    X = (st.uniform(300, 0.0, 1.0).reshape(-1, 3) * [2.0, 1.0, 1.0]).astype(np.float32)
    n = st.unit_vectors(100).astype(np.float32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    E = ctx.query_irradiance(t(X), t(n), t(n)).cpu().numpy()
    assert np.allclose(E, L, rtol=2e-5)
    ctx.close()

    Le = np.array([1.0, 2.0, 0.5])
    rho, a = 0.6, 0.75
    d = S.VolumeDesc(origin=(-1, -1, -1), spacing=(1, 1, 1), counts=(3, 3, 3), rays_per_probe=64,
                     hysteresis_irr=a, hysteresis_dist=a, max_distance=20.0, irradiance_gamma=GAMMA)
    ctx = irf.build_workload(S.Workload("furnace", 0, S.sphere_scene(4.0, 2, emission=Le.tolist(), albedo=rho),
                                        S.no_lights(), [d]))
    x = np.zeros(3)
    for f in range(6):
        ctx.update_probes(S.rotations(0, 1, start_frame=20 + f)[0])
        x = Le ** (1 / GAMMA) if f == 0 else a * x + (1 - a) * (Le + rho * x ** GAMMA) ** (1 / GAMMA)
        irr = ctx.volumes[0].irradiance[..., :3].cpu().numpy()
        assert np.allclose(irr, x, rtol=1e-5), (f, np.abs(irr - x).max())
    ctx.close()


def test_adjoint_refuses_encoded_volumes(torch):
    from paper_2009_10796_amd import irf
    w = _encoded(S.config0())
    ctx = irf.build_workload(w)
    v = ctx.volumes[0]
    gi = [torch.zeros(v.irradiance.shape, device="cuda")]
    gd = [torch.zeros(v.distance.shape, device="cuda")]
    p = torch.zeros((4, 3), device="cuda")
    with pytest.raises(irf.IrfError) as e:
        ctx.query_backward(p, p, p, p, gi, gd)
    assert e.value.status == irf.E_UNSUPPORTED
    ctx.close()
