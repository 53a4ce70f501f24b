"""GPU second-order glossy pass (Section "Second Order Glossy") against the
FP64 oracle.

Stage parity: both sides read the oracle's atlases after two update frames,
rounded to float32 (oracle -> GPU input).  Points: the city's G-buffer (every
4th pixel, as the paper traces glossy rays at reduced resolution) with a
mirror-reflective ground and slightly reflective buildings; the room.  Per
point: the mirror ray's hit and shadow visibility (a difference must be an
oracle-flagged ray), its hit distance within the float32 rounding of the
ray's origin and direction, and its radiance within the parity rule."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests import gpu_helpers as G
from tests import parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _with_specular(w, ground, other):
    M = w.scene.albedo.shape[0]
    spec = np.full((M, 3), other, np.float32)
    spec[0] = ground
    w.scene.specular = spec
    return w


@pytest.mark.parametrize("name", ["room", "city"])
def test_glossy_parity(torch, name):
    import oracle
    from paper_2009_10796_amd import irf
    if name == "room":
        w = _with_specular(S.config0(), 0.5, 0.2)
        q = w.queries
        pos, nrm = q.pos, q.nrm
        st = S.Stream(985, 1)
        view = st.unit_vectors(len(pos)).astype(np.float32)
        view = np.where((np.sum(view * nrm, 1) < 0)[:, None], -view, view).astype(np.float32)
    else:
        w = _with_specular(S.config1(), 0.3, 0.1)
        q = w.queries
        sel = np.arange(0, q.n, 4)[:200000]
        pos, nrm, view = q.pos[sel], q.nrm[sel], q.view[sel]
    osc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    oracle.classify(osc, ov, w.classify_rotations)
    for f in (1, 2):
        oracle.update_frame(osc, w.lights, ov, w.frame_rotation(f), records=False)
    ctx = irf.build_workload(w)
    for gv, o in zip(ctx.volumes, ov):
        o.irr[:] = o.irr.astype(np.float32)
        o.dist[:] = o.dist.astype(np.float32)
        o.irr_kappa[:] = 0.0
        o.dist_kappa[:] = 0.0
        gv.irradiance[..., :3].copy_(torch.from_numpy(o.irr.astype(np.float32)))
        gv.distance.copy_(torch.from_numpy(o.dist.astype(np.float32)))
        gv.states.copy_(torch.from_numpy(o.states.copy()))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    out, rec_g = ctx.glossy(t(pos), t(nrm), t(view), records=True)
    rec_o = oracle.glossy(osc, w.lights, ov, pos, nrm, view)
    out = out.cpu().numpy()
    assert np.array_equal(out, rec_g["rgb"])
    flip = (rec_g["tri"] != rec_o["tri"]) | (rec_g["vis"] != rec_o["vis"])
    unflagged = flip & ((rec_o["flags"] & oracle.F_AMBIGUOUS) == 0)
    hit = rec_o["tri"] >= 0
    verdict = P.compare(f"glossy {name} radiance", out[~flip], rec_o["rgb"][~flip], rec_o["kappa"][~flip])
    same_hit = ~flip & hit
    # hit distance: the ray direction's and the lifted origin's float32
    # rounding (about u |o| per coordinate), over the cosine of incidence
    o_mag = np.abs(pos[same_hit]).max(1) + 1e-3
    t_ok = np.abs(rec_g["t"][same_hit] - rec_o["t"][same_hit]) <= 2e-6 * rec_o["t"][same_hit] + (
        8 * 2.0 ** -24 * (rec_o["t"][same_hit] + 4 * o_mag) / np.maximum(rec_o["cosi"][same_hit], 1e-6))
    if not t_ok.all():
        idx = np.nonzero(same_hit)[0][~t_ok]
        err = np.abs(rec_g["t"][idx] - rec_o["t"][idx]) / rec_o["t"][idx]
        for k in idx[np.argsort(-err)][:6]:
            print(f"[glossy] t mismatch point {k}: t_gpu {rec_g['t'][k]:.9g} t_orc {rec_o['t'][k]:.9g} "
                  f"rel {abs(rec_g['t'][k] - rec_o['t'][k]) / rec_o['t'][k]:.2e} cosi {rec_o['cosi'][k]:.3g} "
                  f"tri {rec_o['tri'][k]} n.v {float(np.dot(nrm[k], view[k])):.3g} pos {pos[k]}", flush=True)
    spec_share = np.mean(np.abs(out[~flip]).sum(1) > 0)
    print(f"[glossy] {name}: points {len(pos)}, hits {int(hit.sum())}, flips {int(flip.sum())} "
          f"(unflagged {int(unflagged.sum())}), t fail {int((~t_ok).sum())}, nonzero {spec_share:.3f}", flush=True)
    assert unflagged.sum() == 0
    assert flip.mean() <= 0.01
    G.check([verdict])
    assert t_ok.all()
    assert hit.sum() > 0.2 * len(pos)
    ctx.close()
