"""The frame that also answers a query batch (irf_update_probes_query).

Its queries must equal, bit for bit, irf_query_irradiance called just
before irf_update_probes on the same stream (the atlases and states the
previous frame left), and its frame the plain frame: checked on the city
(a 480x270 G-buffer; the queries split between the probe-ray trace and
the shadow-ray launches in several proportions, on persistent and full
grids, and all in the trace launch when the shadow rays use lane refill),
on the room, on four cascades (also past 4,096 probes), on the city with a
dynamic building, whose state step can put probes to sleep before the
queries would see them (there the queries run first, as their own launch),
over frames that move the building, after autotuning, and as a captured
graph (irf_graph_capture_query) replayed against the eager frames."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests.test_gpu_cascades import small_terrain
from tests.test_gpu_dynamic_states import city_with_dynamic_building

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _tensors(torch, q):
    return [torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda() for a in (q.pos, q.nrm, q.view)]


def _same_atlases(A, B):
    return all(np.array_equal(va.irradiance.cpu().numpy(), vb.irradiance.cpu().numpy())
               and np.array_equal(va.distance.cpu().numpy(), vb.distance.cpu().numpy())
               and np.array_equal(va.states.cpu().numpy(), vb.states.cpu().numpy())
               for va, vb in zip(A.volumes, B.volumes))


def _run(torch, w, frames, tunings=(None,), scene_at=None):
    """Context A: query, then the frame; context B: the fused call.  Returns
    per frame whether queries and atlases agree bit for bit."""
    from paper_2009_10796_amd import irf
    pos, nrm, view = _tensors(torch, w.queries)
    A, B = irf.build_workload(w), irf.build_workload(w)
    for c in (A, B):
        c.classify(w.classify_rotations)
        c.update_probes(w.frame_rotation(1))
    ea, eb = torch.empty_like(pos), torch.empty_like(pos)
    out = []
    for i, f in enumerate(frames):
        if scene_at and f in scene_at:
            for c in (A, B):
                c.set_scene(scene_at[f])
        t = tunings[i % len(tunings)]
        if t:
            B.set_tuning(**t)
        A.query_irradiance(pos, nrm, view, ea)
        A.update_probes(w.frame_rotation(f))
        eb.fill_(float("nan"))
        B.update_probes_query(w.frame_rotation(f), pos, nrm, view, eb)
        torch.cuda.synchronize()
        q_same = torch.equal(ea, eb)
        a_same = _same_atlases(A, B)
        print(f"[fused] {w.name} frame {f} tuning {t}: queries equal {q_same}, frame equal {a_same}", flush=True)
        out.append((q_same, a_same))
    # n = 0: a plain frame
    A.update_probes(w.frame_rotation(99))
    B.update_probes_query(w.frame_rotation(99), pos[:0], nrm[:0], view[:0])
    torch.cuda.synchronize()
    out.append((True, _same_atlases(A, B)))
    A.close()
    B.close()
    return out


def test_fused_queries_match_query_then_frame_on_the_city(torch):
    w = S.config1(width=480, height=270)
    res = _run(torch, w, (2, 3, 4, 5, 6, 7),
               tunings=(None, {"trace_blocks": 37, "query_shadow": 0}, {"trace_blocks": 0, "query_shadow": 1000},
                        {"query_shadow": 333, "shadow_blocks": 5}, {"query_shadow": 500, "shadow_refill": 8},
                        {"query_shadow": 500, "shadow_blocks": 0, "shadow_refill": 0}))
    assert all(q and a for q, a in res), res


def test_fused_queries_match_query_then_frame_on_the_room(torch):
    res = _run(torch, S.config0(), (2, 3))
    assert all(q and a for q, a in res), res


@pytest.mark.parametrize("counts,rays", [((8, 4, 8), 64), ((16, 8, 16), 32)], ids=["1024 probes", "8192 probes"])
def test_fused_queries_match_on_cascades(torch, counts, rays):
    # four cascades (the query blends them); 8,192 probes: the frame start's
    # two-pass compaction; lane refill and batched shadow rays
    w = small_terrain(cascade_counts=counts, rays=rays)
    w.queries = S.surface_points(w.scene, 20000, 3)
    res = _run(torch, w, (2, 3, 4), tunings=({"shadow_refill": 8, "shadow_blocks": 64},
                                             {"shadow_refill": 0, "query_shadow": 500},
                                             {"shadow_refill": 0, "query_shadow": 900, "trace_blocks": 11}))
    assert all(q and a for q, a in res), res


def test_dynamic_scene_queries_run_before_the_state_step(torch):
    w, scene_a = city_with_dynamic_building()
    _, scene_b = city_with_dynamic_building((4.0, 0.0, 0.0))
    w.scene = scene_a
    w.volumes = [S.VolumeDesc(origin=(3.5, 5.5, 4.5), spacing=(1.0, 1.0, 1.0), counts=(10, 4, 6), rays_per_probe=64)]
    w.queries = S.config1(width=320, height=180).queries
    res = _run(torch, w, (2, 3, 4), scene_at={3: scene_b})
    assert all(q and a for q, a in res), res


def test_autotuner_on_fused_frames_keeps_results(torch):
    from paper_2009_10796_amd import irf, autotune
    w = S.config1(width=320, height=180)
    pos, nrm, view = _tensors(torch, w.queries)
    A, B = irf.build_workload(w), irf.build_workload(w)
    for c in (A, B):
        c.classify(w.classify_rotations)
    eb = torch.empty_like(pos)
    chosen = autotune.autotune(B, [w.frame_rotation(50 + i) for i in range(6)], frames_per_candidate=2,
                               step=lambda R: B.update_probes_query(R, pos, nrm, view, eb))
    print(f"[fused] autotuned {chosen}", flush=True)
    assert "query_shadow" in chosen and chosen["query_shadow"] in (0, 250, 500, 750)
    # the tuned context from the same state as the default one: same results
    for c in (A, B):
        for v in c.volumes:
            v.irradiance.zero_()
            v.distance.zero_()
    for va, vb in zip(A.volumes, B.volumes):
        va.states.copy_(vb.states)
    for c in (A, B):
        c.update_probes(w.frame_rotation(1))
    ea = torch.empty_like(pos)
    for f in (2, 3):
        A.query_irradiance(pos, nrm, view, ea)
        A.update_probes(w.frame_rotation(f))
        B.update_probes_query(w.frame_rotation(f), pos, nrm, view, eb)
        torch.cuda.synchronize()
        assert torch.equal(ea, eb) and _same_atlases(A, B), f
    A.close()
    B.close()


@pytest.mark.parametrize("dynamic", [False, True], ids=["static city", "dynamic building"])
def test_graph_replayed_fused_frames_match_eager(torch, dynamic):
    """irf_graph_capture_query: replays (with eager work and synchronizations
    between them) give the queries and atlases of the eager fused frames, bit
    for bit; with a dynamic building the captured frame runs the queries
    first, as its own node."""
    from paper_2009_10796_amd import irf
    if dynamic:
        w, scene = city_with_dynamic_building()
        w.scene = scene
        w.volumes = [S.VolumeDesc(origin=(3.5, 5.5, 4.5), spacing=(1.0, 1.0, 1.0), counts=(10, 4, 6),
                                  rays_per_probe=64)]
        w.queries = S.config1(width=320, height=180).queries
    else:
        w = S.config1(width=320, height=180)
    pos, nrm, view = _tensors(torch, w.queries)
    A, B = irf.build_workload(w), irf.build_workload(w)
    for c in (A, B):
        c.classify(w.classify_rotations)
        c.update_probes(w.frame_rotation(1))
    torch.cuda.synchronize()
    ea, eb = torch.empty_like(pos), torch.empty_like(pos)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = B.capture_frame_query(pos, nrm, view, eb, s)
    for f in (2, 3, 4, 5):
        A.update_probes_query(w.frame_rotation(f), pos, nrm, view, ea)
        eb.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.launch(w.frame_rotation(f))
        torch.cuda.synchronize()
        # eager work on the graph's context between replays
        extra = B.query_irradiance(pos, nrm, view)
        torch.cuda.synchronize()
        q_same, a_same = torch.equal(ea, eb), _same_atlases(A, B)
        print(f"[fused graph] dynamic={dynamic} frame {f}: queries equal {q_same}, frame equal {a_same}", flush=True)
        assert q_same and a_same, f
        assert torch.isfinite(extra).all()
    g.close()
    A.close()
    B.close()
