"""GPU adjoint (reverse of query -> blend -> hit shading, ray hits held fixed)
against the oracle's adjoint, which is pinned by central differences in FP64.

Workload: the reduced differentiable frame of tests/adjoint_case (city with
64 emissive quads, a 6x4x6 volume of 64-ray probes, frame 1 converged, then
one frame from A0 to A1 queried at surface points).  The GPU starts from the
oracle's A0 and probe states, rounded to float32 (oracle -> GPU input only).

Tolerance.  Each gradient element is a sum of terms (an upstream gradient
times the normalised blend and query weights and their Chebyshev
derivatives; the query terms are evaluated in FP64 from the float32 inputs
and stored in float32), accumulated in a fixed order (point or ray order per
texel), so that a second run gives the same bits.  The
oracle reports per element the sum of the terms' magnitudes (a) and how far
the terms move when the float32 inputs of each query (sampled moments, r,
irradiance, hit point) move by their float32 error bounds (s).  Elements are
compared as |g - o| <= 1e-5 a + s (+ 1e-7 of the array's largest |o|).  s is
large exactly where the Chebyshev factor is ill-conditioned (variance near
zero with r close to mu), as for the forward parity.
"""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests.adjoint_case import OracleFrame, workload
from tests.gpu_helpers import flips

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def frame():
    fr = OracleFrame(workload())
    for v in fr.A0:
        v.irr[:] = v.irr.astype(np.float32)
        v.dist[:] = v.dist.astype(np.float32)
    fr.target = fr.forward(S.target_emission(fr.w).astype(np.float64), fr.A0)[0]
    return fr


def _gpu_context(torch, fr):
    from paper_2009_10796_amd import irf
    ctx = irf.build_workload(fr.w)
    for gv, o in zip(ctx.volumes, fr.A0):
        gv.states.copy_(torch.from_numpy(o.states.copy()))
    return ctx


def _load_a0(torch, ctx, fr):
    for gv, o in zip(ctx.volumes, fr.A0):
        gv.irradiance.zero_()
        gv.irradiance[..., :3].copy_(torch.from_numpy(o.irr.astype(np.float32)))
        gv.distance.copy_(torch.from_numpy(o.dist.astype(np.float32)))
        gv.states.copy_(torch.from_numpy(o.states.copy()))


def _close(g, o, a=None, sens=None, name=""):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    scale = max(np.abs(o).max(), 1e-30)
    tol = 1e-7 * scale + (1e-5 * a if a is not None else 1e-4 * scale) + (sens if sens is not None else 0.0)
    err = np.abs(g - o)
    ratio = err / tol
    agg = float(np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-30))
    print(f"[adjoint] {name}: max|o|={scale:.3e} worst err/tol={ratio.max():.3f} rel L2={agg:.2e} "
          f"elements with s > 1e-3 max|o|: {int((sens > 1e-3 * scale).sum()) if sens is not None else 0}", flush=True)
    return bool(np.all(err <= tol))


def _zeros(vols):
    return [np.zeros_like(v.irr) for v in vols], [np.zeros_like(v.dist) for v in vols]


def _gpu_zeros(torch, ctx):
    dev = ctx.device
    return ([torch.zeros(v.irradiance.shape, dtype=torch.float32, device=dev) for v in ctx.volumes],
            [torch.zeros(v.distance.shape, dtype=torch.float32, device=dev) for v in ctx.volumes])


def test_query_backward_matches_oracle(torch, frame):
    import oracle
    fr = frame
    ctx = _gpu_context(torch, fr)
    # atlases: the oracle's A1, float32 (query stage alone)
    E, A1, _ = fr.forward(fr.emission, fr.A0)
    for o in A1:
        o.irr[:] = o.irr.astype(np.float32)
        o.dist[:] = o.dist.astype(np.float32)
        o.irr_kappa[:] = 0.0
        o.dist_kappa[:] = 0.0
    for gv, o in zip(ctx.volumes, A1):
        gv.irradiance.zero_()
        gv.irradiance[..., :3].copy_(torch.from_numpy(o.irr.astype(np.float32)))
        gv.distance.copy_(torch.from_numpy(o.dist.astype(np.float32)))
        gv.states.copy_(torch.from_numpy(o.states.copy()))
    q = fr.w.queries
    gout = S.Stream(951, 2).uniform(3 * len(q.pos), -1.0, 1.0).reshape(-1, 3).astype(np.float32)
    gi, gd = _zeros(A1)
    ai, ad = _zeros(A1)
    si, sd = _zeros(A1)
    oracle.query_backward(A1, q.pos, q.nrm, q.view, gout, gi, gd, ai, ad, si, sd)
    dev = ctx.device
    Gi, Gd = _gpu_zeros(torch, ctx)
    pos, nrm, view = (torch.from_numpy(a).to(dev) for a in (q.pos, q.nrm, q.view))
    ctx.query_backward(pos, nrm, view, torch.from_numpy(gout).to(dev), Gi, Gd)
    torch.cuda.synchronize()
    gi_g = Gi[0].cpu().numpy()
    assert np.all(gi_g[..., 3] == 0)
    assert np.abs(gi[0]).max() > 0 and np.abs(gd[0]).max() > 0
    assert _close(gi_g[..., :3], gi[0], ai[0], si[0], name="query dE/dirr")
    assert _close(Gd[0].cpu().numpy(), gd[0], ad[0], sd[0], name="query dE/ddist")
    # linear in the upstream gradient
    Gi2, Gd2 = _gpu_zeros(torch, ctx)
    ctx.query_backward(pos, nrm, view, torch.from_numpy(2 * gout).to(dev), Gi2, Gd2)
    torch.cuda.synchronize()
    assert _close(Gi2[0].cpu().numpy(), 2 * gi_g, name="linearity")
    ctx.close()


def test_frame_backward_matches_oracle(torch, frame):
    import oracle
    fr = frame
    ctx = _gpu_context(torch, fr)
    _load_a0(torch, ctx, fr)
    dev = ctx.device
    e0 = fr.emission
    ctx.set_emission(torch.from_numpy(e0.astype(np.float32)).to(dev))
    ctx.set_differentiable(True)
    ctx.update_probes(fr.R)
    torch.cuda.synchronize()
    # the oracle's frame from the same A0
    E_o, A1_o, rec_o = fr.forward(e0, fr.A0)
    rec_g = ctx.ray_records(0)
    _, rep = flips(rec_g, rec_o)
    print(f"[adjoint] frame records: {rep}", flush=True)
    assert rep["unflagged_flips"] == 0
    # upstream: the oracle's dLoss/d(A1), rounded to float32, fed to both
    q = fr.w.queries
    gE = 2.0 * (E_o - fr.target) / E_o.size
    g1i, g1d = _zeros(A1_o)
    oracle.query_backward(A1_o, q.pos, q.nrm, q.view, gE, g1i, g1d)
    g1i = [g.astype(np.float32).astype(np.float64) for g in g1i]
    g1d = [g.astype(np.float32).astype(np.float64) for g in g1d]
    prev = oracle.copy_volumes(fr.A0)
    oracle.state_step(fr.sc, prev)
    for v in prev:
        v.irr_kappa[:] = 0.0      # the GPU reads the same float32 A0
        v.dist_kappa[:] = 0.0
    g0i, g0d = _zeros(prev)
    a0i, a0d = _zeros(prev)
    s0i, s0d = _zeros(prev)
    ge_o = np.zeros_like(e0)
    fr.sc.set_emission(e0)
    oracle.update_backward(fr.sc, prev, fr.R, rec_o, g1i, g1d, g0i, g0d, ge_o, a_prev_irr=a0i, a_prev_dist=a0d,
                           s_prev_irr=s0i, s_prev_dist=s0d)
    Gi, Gd = [], []
    for gv, a, b in zip(ctx.volumes, g1i, g1d):
        t = torch.zeros(gv.irradiance.shape, dtype=torch.float32)
        t[..., :3] = torch.from_numpy(a.astype(np.float32))
        Gi.append(t.to(dev))
        Gd.append(torch.from_numpy(b.astype(np.float32)).to(dev))
    P0i, P0d = _gpu_zeros(torch, ctx)
    ge = torch.zeros((e0.shape[0], 3), dtype=torch.float32, device=dev)
    ctx.update_backward(Gi, Gd, P0i, P0d, ge)
    torch.cuda.synchronize()
    # rays whose hit differs (oracle-flagged) and the probes they feed are
    # compared by validity only: none in this workload
    assert rep["flips"] == 0, rep
    assert _close(ge.cpu().numpy(), ge_o, name="dL/demission")
    assert _close(P0i[0].cpu().numpy()[..., :3], g0i[0], a0i[0], s0i[0], name="dL/dirr0")
    assert _close(P0d[0].cpu().numpy(), g0d[0], a0d[0], s0d[0], name="dL/ddist0")
    # backward needs a differentiable frame
    ctx.set_differentiable(False)
    from paper_2009_10796_amd import irf
    with pytest.raises(irf.IrfError):
        ctx.update_backward(Gi, Gd, P0i, P0d, ge)
    ctx.close()


def test_autograd_matches_directional_difference(torch, frame):
    """The autograd wrapper against the GPU's own forward: with hits fixed the
    loss is quadratic in the emitter radiance, so a central difference along
    a direction equals the directional derivative up to float32 rounding of
    the loss."""
    from paper_2009_10796_amd import diff
    fr = frame
    ctx = _gpu_context(torch, fr)
    dev = ctx.device
    q = fr.w.queries
    pos, nrm, view = (torch.from_numpy(a).to(dev) for a in (q.pos, q.nrm, q.view))
    A0 = []
    for o in fr.A0:
        irr = torch.zeros((o.irr.shape[0], 8, 8, 4), dtype=torch.float32)
        irr[..., :3] = torch.from_numpy(o.irr.astype(np.float32))
        A0 += [irr.to(dev), torch.from_numpy(o.dist.astype(np.float32)).to(dev)]
    states0 = [torch.from_numpy(o.states.copy()).to(dev) for o in fr.A0]
    target = torch.from_numpy(fr.target.astype(np.float32)).to(dev)

    def loss(e, grad=False):
        for gv, s0 in zip(ctx.volumes, states0):
            gv.states.copy_(s0)
        a = [t.clone().requires_grad_(grad) for t in A0]
        E = diff.frame_and_query(ctx, fr.R, pos, nrm, view, e, a)
        L = ((E.double() - target.double()) ** 2).mean()
        return L, a

    e = torch.from_numpy(fr.emission.astype(np.float32)).to(dev).requires_grad_(True)
    L, a = loss(e, grad=True)
    L.backward()
    ge = e.grad.double().cpu().numpy()
    assert np.abs(ge).max() > 0
    d = S.Stream(952, 3).uniform(ge.size, -1.0, 1.0).reshape(ge.shape)
    d *= (fr.emission != 0) | (np.arange(len(d)) == 0)[:, None]
    h = 0.05
    with torch.no_grad():
        dt = torch.from_numpy(d.astype(np.float32)).to(dev)
        Lp = float(loss(e.detach() + h * dt)[0])
        Lm = float(loss(e.detach() - h * dt)[0])
    fd = (Lp - Lm) / (2 * h)
    dd = float((ge * d).sum())
    print(f"[adjoint] directional: fd={fd:.6e} grad.d={dd:.6e}", flush=True)
    assert abs(fd - dd) <= 1e-3 * abs(dd) + 1e-6 * float(L.detach())
    # the texel gradients come back through autograd too
    assert a[0].grad is not None and a[1].grad is not None
    assert float(a[0].grad.abs().max()) > 0
    ctx.close()


def test_full_size_backward_matches_oracle(torch):
    """Full size: city volume 16x8x16 with 256 rays (2,048 probes), 64
    emissive quads, 65,536 surface points; every emitter value and every
    texel gradient is compared."""
    import oracle
    from paper_2009_10796_amd import irf
    from tests.adjoint_case import FullFrame
    fr = FullFrame()
    w = fr.w
    ctx = irf.build_workload(w)
    dev = ctx.device
    for gv, o in zip(ctx.volumes, fr.A0):
        gv.irradiance.zero_()
        gv.irradiance[..., :3].copy_(torch.from_numpy(o.irr.astype(np.float32)))
        gv.distance.copy_(torch.from_numpy(o.dist.astype(np.float32)))
        gv.states.copy_(torch.from_numpy(o.states.copy()))
    ctx.set_emission(torch.from_numpy(fr.emission.astype(np.float32)).to(dev))
    ctx.set_differentiable(True)
    ctx.update_probes(fr.R)
    torch.cuda.synchronize()
    E_o, A1_o, rec_o = fr.forward(fr.emission)
    rec_g = ctx.ray_records(0)
    flip, rep = flips(rec_g, rec_o)
    print(f"[adjoint-full] records: {rep}", flush=True)
    assert rep["unflagged_flips"] == 0
    if flip.any():
        # the oracle adopts the GPU's decisions on the flagged rays, so both
        # sides hold the same hits fixed and every gradient is compared
        E_o, A1_o, rec_o = fr.forward(fr.emission, force=(np.where(flip, 3, 0).astype(np.uint8), rec_g["tri"],
                                                           rec_g["vis"]))
        assert not flips(rec_g, rec_o)[0].any()
    q = w.queries
    pos, nrm, view = (torch.from_numpy(a).to(dev) for a in (q.pos, q.nrm, q.view))
    # query stage on the oracle's A1 (float32), upstream dLoss/dE
    gE = (2.0 * (E_o - fr.target) / E_o.size).astype(np.float32)
    for o in A1_o:
        o.irr[:] = o.irr.astype(np.float32)
        o.dist[:] = o.dist.astype(np.float32)
        o.irr_kappa[:] = 0.0
        o.dist_kappa[:] = 0.0
    g1i, g1d = _zeros(A1_o)
    a1i, a1d = _zeros(A1_o)
    s1i, s1d = _zeros(A1_o)
    oracle.query_backward(A1_o, q.pos, q.nrm, q.view, gE, g1i, g1d, a1i, a1d, s1i, s1d)
    saved = [(gv.irradiance.clone(), gv.distance.clone()) for gv in ctx.volumes]
    for gv, o in zip(ctx.volumes, A1_o):
        gv.irradiance[..., :3].copy_(torch.from_numpy(o.irr.astype(np.float32)))
        gv.distance.copy_(torch.from_numpy(o.dist.astype(np.float32)))
    Gi, Gd = _gpu_zeros(torch, ctx)
    ctx.query_backward(pos, nrm, view, torch.from_numpy(gE).to(dev), Gi, Gd)
    torch.cuda.synchronize()
    assert _close(Gi[0].cpu().numpy()[..., :3], g1i[0], a1i[0], s1i[0], name="full query dE/dirr")
    assert _close(Gd[0].cpu().numpy(), g1d[0], a1d[0], s1d[0], name="full query dE/ddist")
    for gv, (a, b) in zip(ctx.volumes, saved):
        gv.irradiance.copy_(a)
        gv.distance.copy_(b)
    # update stage from the oracle's upstream (float32)
    g1i = [g.astype(np.float32).astype(np.float64) for g in g1i]
    g1d = [g.astype(np.float32).astype(np.float64) for g in g1d]
    prev = oracle.copy_volumes(fr.A0)
    oracle.state_step(fr.sc, prev)
    g0i, g0d = _zeros(prev)
    a0i, a0d = _zeros(prev)
    s0i, s0d = _zeros(prev)
    ge_o = np.zeros_like(fr.emission)
    fr.sc.set_emission(fr.emission)
    oracle.update_backward(fr.sc, prev, fr.R, rec_o, g1i, g1d, g0i, g0d, ge_o, a_prev_irr=a0i, a_prev_dist=a0d,
                           s_prev_irr=s0i, s_prev_dist=s0d)
    Gi, Gd = [], []
    for gv, a, b in zip(ctx.volumes, g1i, g1d):
        t = torch.zeros(gv.irradiance.shape, dtype=torch.float32)
        t[..., :3] = torch.from_numpy(a.astype(np.float32))
        Gi.append(t.to(dev))
        Gd.append(torch.from_numpy(b.astype(np.float32)).to(dev))
    P0i, P0d = _gpu_zeros(torch, ctx)
    ge = torch.zeros((fr.emission.shape[0], 3), dtype=torch.float32, device=dev)
    ctx.update_backward(Gi, Gd, P0i, P0d, ge)
    torch.cuda.synchronize()
    ge_g = ge.cpu().numpy().astype(np.float64)
    gi_g = P0i[0].cpu().numpy()[..., :3].astype(np.float64)
    gd_g = P0d[0].cpu().numpy().astype(np.float64)
    assert _close(ge_g, ge_o, name="full dL/demission")
    assert _close(gi_g, g0i[0], a0i[0], s0i[0], name="full dL/dirr0")
    assert _close(gd_g, g0d[0], a0d[0], s0d[0], name="full dL/ddist0")
    # the sums run in a fixed order: a second backward gives the same bits
    Q2i, Q2d = _gpu_zeros(torch, ctx)
    ctx.query_backward(pos, nrm, view, torch.from_numpy(gE).to(dev), Q2i, Q2d)
    P2i, P2d = _gpu_zeros(torch, ctx)
    ge2 = torch.zeros_like(ge)
    ctx.update_backward(Gi, Gd, P2i, P2d, ge2)
    torch.cuda.synchronize()
    assert torch.equal(ge2, ge) and torch.equal(P2i[0], P0i[0]) and torch.equal(P2d[0], P0d[0])
    ctx.close()


def test_backward_is_deterministic(torch, frame):
    """Query and frame backward, run three times into fresh buffers: every
    gradient (texels and emitters) is the same bit for bit."""
    fr = frame
    ctx = _gpu_context(torch, fr)
    _load_a0(torch, ctx, fr)
    dev = ctx.device
    ctx.set_emission(torch.from_numpy(fr.emission.astype(np.float32)).to(dev))
    ctx.set_differentiable(True)
    ctx.update_probes(fr.R)
    q = fr.w.queries
    pos, nrm, view = (torch.from_numpy(a).to(dev) for a in (q.pos, q.nrm, q.view))
    gout = torch.from_numpy(S.Stream(953, 1).uniform(3 * len(q.pos), -1.0, 1.0)
                            .reshape(-1, 3).astype(np.float32)).to(dev)
    runs = []
    for _ in range(3):
        Qi, Qd = _gpu_zeros(torch, ctx)
        ctx.query_backward(pos, nrm, view, gout, Qi, Qd)
        Pi, Pd = _gpu_zeros(torch, ctx)
        ge = torch.zeros((fr.emission.shape[0], 3), dtype=torch.float32, device=dev)
        ctx.update_backward(Qi, Qd, Pi, Pd, ge)
        torch.cuda.synchronize()
        runs.append([t.cpu() for t in Qi + Qd + Pi + Pd + [ge]])
    assert float(runs[0][-1].abs().max()) > 0 and float(runs[0][0].abs().max()) > 0
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            assert torch.equal(a, b)
    ctx.close()


def test_cascade_backward_matches_oracle(torch):
    """Two cascaded volumes (Section "Multiple Probe Volumes"): a 6x4x6 volume
    at 1 m inside a 6x4x6 volume at 2.5 m, 64 rays each, in the city with 64
    emitters; 2,000 surface points spread over the inner volume, its
    fall-off band and the outer volume alone, so each query's gradient splits
    between the volumes by the cascade weights.  Frame 1 (oracle, rounded to
    float32) is A0; frame 2 is differentiated.  Query backward on the
    oracle's A1 and frame backward from the oracle's upstream gradient are
    compared per volume; rays the GPU decided otherwise are substituted in
    the oracle's frame (parity protocol), so both hold the same hits."""
    import oracle
    from paper_2009_10796_amd import irf
    from tests import parity as P
    w = S.config4(n_points=20000)
    w.volumes = [S.VolumeDesc(origin=(5.5, 0.5, 5.5), spacing=(1.0, 1.0, 1.0), counts=(6, 4, 6), rays_per_probe=64),
                 S.VolumeDesc(origin=(1.5, 0.5, 1.5), spacing=(2.5, 2.5, 2.5), counts=(6, 4, 6), rays_per_probe=64)]
    q = w.queries
    sel = np.all((q.pos >= [4.5, 0.0, 4.5]) & (q.pos <= [11.5, 4.5, 11.5]), axis=1)
    q = S.Queries(q.pos[sel][:2000], q.nrm[sel][:2000], q.view[sel][:2000])
    assert len(q.pos) == 2000
    osc = oracle.Scene(w.scene)
    A0 = [oracle.Volume(d) for d in w.volumes]
    oracle.classify(osc, A0, w.classify_rotations)
    oracle.update_frame(osc, w.lights, A0, w.frame_rotation(1), records=False)
    for v in A0:
        v.irr[:] = v.irr.astype(np.float32)
        v.dist[:] = v.dist.astype(np.float32)
        v.irr_kappa[:] = 0.0
        v.dist_kappa[:] = 0.0
    ctx = irf.build_workload(w)
    dev = ctx.device
    _load_a0(torch, ctx, SimpleNamespace(A0=A0))
    ctx.set_differentiable(True)
    R = w.frame_rotation(2)
    ctx.update_probes(R)
    torch.cuda.synchronize()
    rec_g = np.concatenate([ctx.ray_records(v) for v in range(2)])
    A1 = oracle.copy_volumes(A0)
    rec_o, rep = P.oracle_frame(osc, w.lights, A1, R, rec_g["tri"], rec_g["vis"])
    print(f"[adjoint-cascade] frame: {rep.line()}", flush=True)
    assert rep.unflagged_flips == 0
    # query backward on the oracle's A1 rounded to float32
    for o in A1:
        o.irr[:] = o.irr.astype(np.float32)
        o.dist[:] = o.dist.astype(np.float32)
        o.irr_kappa[:] = 0.0
        o.dist_kappa[:] = 0.0
    gE = S.Stream(955, 1).uniform(3 * len(q.pos), -1.0, 1.0).reshape(-1, 3).astype(np.float32)
    g1i, g1d = _zeros(A1)
    a1i, a1d = _zeros(A1)
    s1i, s1d = _zeros(A1)
    oracle.query_backward(A1, q.pos, q.nrm, q.view, gE.astype(np.float64), g1i, g1d, a1i, a1d, s1i, s1d)
    saved = [(gv.irradiance.clone(), gv.distance.clone()) for gv in ctx.volumes]
    for gv, o in zip(ctx.volumes, A1):
        gv.irradiance[..., :3].copy_(torch.from_numpy(o.irr.astype(np.float32)))
        gv.distance.copy_(torch.from_numpy(o.dist.astype(np.float32)))
    pos, nrm, view = (torch.from_numpy(a).to(dev) for a in (q.pos, q.nrm, q.view))
    Gi, Gd = _gpu_zeros(torch, ctx)
    ctx.query_backward(pos, nrm, view, torch.from_numpy(gE).to(dev), Gi, Gd)
    torch.cuda.synchronize()
    for v in range(2):
        assert np.abs(g1i[v]).max() > 0 and np.abs(g1d[v]).max() > 0, v    # both volumes take gradient
        assert _close(Gi[v].cpu().numpy()[..., :3], g1i[v], a1i[v], s1i[v], name=f"cascade query dE/dirr v{v}")
        assert _close(Gd[v].cpu().numpy(), g1d[v], a1d[v], s1d[v], name=f"cascade query dE/ddist v{v}")
    for gv, (a, b) in zip(ctx.volumes, saved):
        gv.irradiance.copy_(a)
        gv.distance.copy_(b)
    # frame backward from the oracle's upstream (float32)
    g1i = [g.astype(np.float32).astype(np.float64) for g in g1i]
    g1d = [g.astype(np.float32).astype(np.float64) for g in g1d]
    prev = oracle.copy_volumes(A0)
    oracle.state_step(osc, prev)
    g0i, g0d = _zeros(prev)
    a0i, a0d = _zeros(prev)
    s0i, s0d = _zeros(prev)
    ge_o = np.zeros_like(w.scene.emission, dtype=np.float64)
    osc.set_emission(w.scene.emission.astype(np.float64))
    oracle.update_backward(osc, prev, R, rec_o, g1i, g1d, g0i, g0d, ge_o, a_prev_irr=a0i, a_prev_dist=a0d,
                           s_prev_irr=s0i, s_prev_dist=s0d)
    Ui, Ud = [], []
    for gv, a, b in zip(ctx.volumes, g1i, g1d):
        t = torch.zeros(gv.irradiance.shape, dtype=torch.float32)
        t[..., :3] = torch.from_numpy(a.astype(np.float32))
        Ui.append(t.to(dev))
        Ud.append(torch.from_numpy(b.astype(np.float32)).to(dev))
    P0i, P0d = _gpu_zeros(torch, ctx)
    ge = torch.zeros((w.scene.emission.shape[0], 3), dtype=torch.float32, device=dev)
    ctx.update_backward(Ui, Ud, P0i, P0d, ge)
    torch.cuda.synchronize()
    assert np.abs(ge_o).max() > 0
    assert _close(ge.cpu().numpy(), ge_o, name="cascade dL/demission")
    for v in range(2):
        assert _close(P0i[v].cpu().numpy()[..., :3], g0i[v], a0i[v], s0i[v], name=f"cascade dL/dirr0 v{v}")
        assert _close(P0d[v].cpu().numpy(), g0d[v], a0d[v], s0d[v], name=f"cascade dL/ddist0 v{v}")
    ctx.close()


def test_batched_backward_matches_oracle(torch):
    """The adjoint's batches: the reduced terrain cascades (four 8x4x8
    volumes) with 1,024 rays per probe trace 344,064 rays in the
    differentiated frame, and 300,000 surface points are queried, so both
    backward passes run in three batches of 2^22 terms (33 per ray, 32 per
    point).  Every texel and emitter gradient is compared with the oracle's
    adjoint."""
    import oracle
    from paper_2009_10796_amd import irf
    from tests import parity as P
    w = S.config3(grid_vertices=97, size=48.0, n_buildings=12, cascade_counts=(8, 4, 8),
                  spacings=(1.0, 2.0, 4.0, 8.0), rays=1024, center_height=3.0)
    q = S.surface_points(w.scene, 300000, 7)
    osc = oracle.Scene(w.scene)
    A0 = [oracle.Volume(d) for d in w.volumes]
    oracle.classify(osc, A0, w.classify_rotations)
    oracle.update_frame(osc, S.sun_for_frame(1), A0, w.frame_rotation(1), records=False)
    for v in A0:
        v.irr[:] = v.irr.astype(np.float32)
        v.dist[:] = v.dist.astype(np.float32)
        v.irr_kappa[:] = 0.0
        v.dist_kappa[:] = 0.0
    ctx = irf.build_workload(w)
    dev = ctx.device
    _load_a0(torch, ctx, SimpleNamespace(A0=A0))
    L2, R = S.sun_for_frame(2), w.frame_rotation(2)
    ctx.set_lights(L2)
    ctx.set_differentiable(True)
    ctx.update_probes(R)
    torch.cuda.synchronize()
    rec_g = np.concatenate([ctx.ray_records(v) for v in range(len(w.volumes))])
    assert len(rec_g) > 2 * (1 << 22) // 33, len(rec_g)           # three batches of rays
    A1 = oracle.copy_volumes(A0)
    rec_o, rep = P.oracle_frame(osc, L2, A1, R, rec_g["tri"], rec_g["vis"])
    print(f"[adjoint-batched] frame: {rep.line()}", flush=True)
    assert rep.unflagged_flips == 0
    for o in A1:
        o.irr[:] = o.irr.astype(np.float32)
        o.dist[:] = o.dist.astype(np.float32)
        o.irr_kappa[:] = 0.0
        o.dist_kappa[:] = 0.0
    gE = S.Stream(956, 1).uniform(3 * len(q.pos), -1.0, 1.0).reshape(-1, 3).astype(np.float32)
    g1i, g1d = _zeros(A1)
    a1i, a1d = _zeros(A1)
    s1i, s1d = _zeros(A1)
    oracle.query_backward(A1, q.pos, q.nrm, q.view, gE.astype(np.float64), g1i, g1d, a1i, a1d, s1i, s1d)
    for gv, o in zip(ctx.volumes, A1):
        gv.irradiance[..., :3].copy_(torch.from_numpy(o.irr.astype(np.float32)))
        gv.distance.copy_(torch.from_numpy(o.dist.astype(np.float32)))
    pos, nrm, view = (torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev) for a in (q.pos, q.nrm, q.view))
    Gi, Gd = _gpu_zeros(torch, ctx)
    ctx.query_backward(pos, nrm, view, torch.from_numpy(gE).to(dev), Gi, Gd)
    torch.cuda.synchronize()
    for v in range(len(w.volumes)):
        assert _close(Gi[v].cpu().numpy()[..., :3], g1i[v], a1i[v], s1i[v], name=f"batched query dE/dirr v{v}")
        assert _close(Gd[v].cpu().numpy(), g1d[v], a1d[v], s1d[v], name=f"batched query dE/ddist v{v}")
    g1i = [g.astype(np.float32).astype(np.float64) for g in g1i]
    g1d = [g.astype(np.float32).astype(np.float64) for g in g1d]
    prev = oracle.copy_volumes(A0)
    oracle.state_step(osc, prev)
    g0i, g0d = _zeros(prev)
    a0i, a0d = _zeros(prev)
    s0i, s0d = _zeros(prev)
    ge_o = np.zeros_like(w.scene.emission, dtype=np.float64)
    oracle.update_backward(osc, prev, R, rec_o, g1i, g1d, g0i, g0d, ge_o, a_prev_irr=a0i, a_prev_dist=a0d,
                           s_prev_irr=s0i, s_prev_dist=s0d)
    Ui, Ud = [], []
    for gv, a, b in zip(ctx.volumes, g1i, g1d):
        t = torch.zeros(gv.irradiance.shape, dtype=torch.float32)
        t[..., :3] = torch.from_numpy(a.astype(np.float32))
        Ui.append(t.to(dev))
        Ud.append(torch.from_numpy(b.astype(np.float32)).to(dev))
    P0i, P0d = _gpu_zeros(torch, ctx)
    ge = torch.zeros((w.scene.emission.shape[0], 3), dtype=torch.float32, device=dev)
    ctx.update_backward(Ui, Ud, P0i, P0d, ge)
    torch.cuda.synchronize()
    assert _close(ge.cpu().numpy(), ge_o, name="batched dL/demission")
    for v in range(len(w.volumes)):
        assert _close(P0i[v].cpu().numpy()[..., :3], g0i[v], a0i[v], s0i[v], name=f"batched dL/dirr0 v{v}")
        assert _close(P0d[v].cpu().numpy(), g0d[v], a0d[v], s0d[v], name=f"batched dL/ddist0 v{v}")
    ctx.close()
