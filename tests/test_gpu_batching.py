"""Batched frame: persistent launches over all cascades, the frame captured as
a HIP graph, and the autotuner.  Every variant must give the same atlases,
bit for bit, as the plain eager frame (the frame's kernels are
deterministic: no atomics, fixed reduction orders).  Graph replays are also
checked on 8,192 probes, where the frame start compacts in two passes."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests.test_gpu_cascades import small_terrain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _snapshot(ctx):
    return [(v.irradiance.cpu().numpy().copy(), v.distance.cpu().numpy().copy(), v.states.cpu().numpy().copy())
            for v in ctx.volumes]


def _same(a, b):
    return all(np.array_equal(x, y) for va, vb in zip(a, b) for x, y in zip(va, vb))


def test_persistent_grids_match_default(torch):
    from paper_2009_10796_amd import irf
    w = small_terrain()
    A = irf.build_workload(w)
    B = irf.build_workload(w)
    # tiny persistent grids: every workgroup loops over many work items
    B.set_tuning(trace_blocks=7, shadow_blocks=5, shade_blocks=3, blend_blocks=2)
    # shadow rays by lane refill: per-wave task ranges, refilled at 1, 13 or
    # 64 idle lanes, on grids from one wave's worth to many; the blend's tile
    # shapes (1 or 2 workgroups per block of 8 probes, on tiny and default grids)
    Cs = []
    for refill, grid, rsplit, bgrid in ((1, 3, 1, 0), (13, 64, 2, 5), (64, 0, 1, 3)):
        c = irf.build_workload(w)
        c.set_tuning(shadow_refill=refill, shadow_blocks=grid, blend_rsplit=rsplit, blend_blocks=bgrid)
        Cs.append(c)
    for c in (A, B, *Cs):
        c.classify(w.classify_rotations)
    for f in (1, 2, 3):
        L = S.sun_for_frame(f)
        R = w.frame_rotation(f)
        for c in (A, B, *Cs):
            c.set_lights(L)
            c.update_probes(R)
        torch.cuda.synchronize()
        a = _snapshot(A)
        assert _same(a, _snapshot(B)), f
        for c in Cs:
            assert _same(a, _snapshot(c)), (f, c.get_tuning())
    for c in (A, B, *Cs):
        c.close()


@pytest.mark.parametrize("size", ["1024 probes", "8192 probes"])
def test_graph_replays_match_eager(torch, size):
    from paper_2009_10796_amd import irf
    # above 4,096 probes the captured frame holds the two-pass compaction
    w = small_terrain() if size == "1024 probes" else small_terrain(cascade_counts=(16, 8, 16), rays=32)
    A = irf.build_workload(w)
    B = irf.build_workload(w)
    for c in (A, B):
        c.classify(w.classify_rotations)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        g = B.capture_frame(s)
    q = S.surface_points(w.scene, 4096, 3)
    pos, nrm = torch.from_numpy(q.pos).cuda(), torch.from_numpy(q.nrm).cuda()
    for f in range(1, 7):
        L = S.sun_for_frame(f)
        R = w.frame_rotation(f)
        A.set_lights(L)
        B.set_lights(L)
        A.update_probes(R)
        with torch.cuda.stream(s):
            g.launch(R)
        s.synchronize()
        torch.cuda.synchronize()
        assert _same(_snapshot(A), _snapshot(B)), f
        # eager work between replays, on the same context
        ea = A.query_irradiance(pos, nrm, nrm).cpu().numpy()
        eb = B.query_irradiance(pos, nrm, nrm).cpu().numpy()
        assert np.array_equal(ea, eb)
    # a change the graph baked in is refused
    B.set_tuning(trace_blocks=11)
    with pytest.raises(irf.IrfError) as e:
        with torch.cuda.stream(s):
            g.launch(w.frame_rotation(9))
    assert e.value.status == irf.E_STATE
    g.close()
    A.close()
    B.close()


def test_autotuner_keeps_results(torch):
    from paper_2009_10796_amd import autotune, irf
    w = small_terrain()
    A = irf.build_workload(w)
    B = irf.build_workload(w)
    for c in (A, B):
        c.classify(w.classify_rotations)
        c.set_lights(S.sun_for_frame(0))
    chosen = autotune.autotune(B, S.rotations(3, 200, start_frame=100), frames_per_candidate=1)
    assert set(chosen) == {"trace_blocks", "shadow_refill", "shadow_blocks", "shade_blocks", "blend_rsplit",
                           "blend_blocks"}
    # after tuning, the same frames from the same state agree with the default launch shapes
    for c in (A, B):
        for v in c.volumes:
            v.irradiance.zero_()
            v.distance.zero_()
    B_states = [v.states.clone() for v in B.volumes]
    for va, s_ in zip(A.volumes, B_states):
        va.states.copy_(s_)
    for f in (1, 2):
        R = w.frame_rotation(f)
        A.update_probes(R)
        B.update_probes(R)
    torch.cuda.synchronize()
    assert _same(_snapshot(A), _snapshot(B))
    A.close()
    B.close()


def test_pipelined_frames_match_serial(torch):
    """The query of frame f on a second stream beside frame f+1's tracing,
    the atlas writes of f+1 ordered after that query by an event: every
    query and the final atlases equal the one-stream run bit for bit."""
    from paper_2009_10796_amd import irf
    w = small_terrain()
    A = irf.build_workload(w)
    B = irf.build_workload(w)
    for c in (A, B):
        c.classify(w.classify_rotations)
    q = S.surface_points(w.scene, 8192, 5)
    pos, nrm = torch.from_numpy(q.pos).cuda(), torch.from_numpy(q.nrm).cuda()
    frames = range(1, 9)
    serial = []
    for f in frames:
        A.set_lights(S.sun_for_frame(f))
        A.update_probes(w.frame_rotation(f))
        serial.append(A.query_irradiance(pos, nrm, nrm))
    torch.cuda.synchronize()
    Q = torch.cuda.Stream()
    piped, prev = [], None
    for f in frames:
        B.set_lights(S.sun_for_frame(f))
        B.update_probes(w.frame_rotation(f), after=prev)
        done = torch.cuda.Event()
        done.record()
        Q.wait_event(done)
        with torch.cuda.stream(Q):
            piped.append(B.query_irradiance(pos, nrm, nrm))
            prev = torch.cuda.Event()
            prev.record(Q)
    torch.cuda.current_stream().wait_event(prev)
    torch.cuda.synchronize()
    for f, (a, b) in enumerate(zip(serial, piped)):
        assert torch.equal(a, b), f
    assert _same(_snapshot(A), _snapshot(B))
    A.close()
    B.close()


def test_pipelined_frames_with_dynamic_objects(torch):
    """As above on the city with one dynamic building, moved 4 m before
    frame 3, so the state step wakes and puts probes to sleep.  The state step
    rewrites states the queries read, so with dynamic objects the whole frame
    is ordered after the previous query's event.  Every query, the states and
    the atlases equal the one-stream run bit for bit."""
    from paper_2009_10796_amd import irf
    from tests.test_gpu_dynamic_states import city_with_dynamic_building
    w, scene_a = city_with_dynamic_building()
    _, scene_b = city_with_dynamic_building((4.0, 0.0, 0.0))
    w.scene = scene_a
    w.volumes = [S.VolumeDesc(origin=(3.5, 5.5, 4.5), spacing=(1.0, 1.0, 1.0), counts=(10, 4, 6), rays_per_probe=64)]
    A = irf.build_workload(w)
    B = irf.build_workload(w)
    for c in (A, B):
        c.classify(w.classify_rotations)
    q = S.surface_points(scene_a, 8192, 5)
    pos, nrm = torch.from_numpy(q.pos).cuda(), torch.from_numpy(q.nrm).cuda()
    view = nrm
    frames = (1, 2, 3, 4)
    serial, serial_states = [], []
    for f in frames:
        if f == 3:
            A.set_scene(scene_b)
        A.update_probes(w.frame_rotation(f))
        serial.append(A.query_irradiance(pos, nrm, view))
        serial_states.append(A.volumes[0].states.clone())
    torch.cuda.synchronize()
    Q = torch.cuda.Stream()
    piped, piped_states, prev = [], [], None
    for f in frames:
        if f == 3:
            B.set_scene(scene_b)
        B.update_probes(w.frame_rotation(f), after=prev)
        done = torch.cuda.Event()
        done.record()
        Q.wait_event(done)
        with torch.cuda.stream(Q):
            piped.append(B.query_irradiance(pos, nrm, view))
            piped_states.append(B.volumes[0].states.clone())
            prev = torch.cuda.Event()
            prev.record(Q)
    torch.cuda.current_stream().wait_event(prev)
    torch.cuda.synchronize()
    changed = sum(int((a != b).sum()) for a, b in zip(serial_states[1:], serial_states[:-1]))
    print(f"[pipelined dynamic] state changes over the frames {changed}", flush=True)
    assert changed > 0
    for f, (a, b) in enumerate(zip(serial, piped)):
        assert torch.equal(a, b), f
    for f, (a, b) in enumerate(zip(serial_states, piped_states)):
        assert torch.equal(a, b), f
    assert _same(_snapshot(A), _snapshot(B))
    A.close()
    B.close()
