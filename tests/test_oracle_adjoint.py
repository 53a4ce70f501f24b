"""Pins of the oracle's adjoint (reverse pass of query -> blend -> hit
shading with ray hits fixed) against central finite differences in FP64 of
the oracle's forward, which is pinned by the other oracle tests.  With hits
and shadow decisions fixed the loss is quadratic in the emitter radiances, so
central differences are exact up to rounding; texels are checked where the
loss is smooth (the Chebyshev weight has a kink where mu2 = mu^2)."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests.adjoint_case import OracleFrame, workload


@pytest.fixture(scope="module")
def frame():
    return OracleFrame(workload())


def test_emitter_gradients_match_central_differences(frame):
    e0 = frame.emission
    ge, _, _ = frame.gradients(e0, frame.A0)
    assert np.abs(ge).max() > 0
    h = 1e-3
    worst = 0.0
    checked = 0
    for m in range(e0.shape[0]):
        for c in range(3):
            if frame.w.scene.emission[m, c] == 0 and m != 0:
                continue
            ep, em = e0.copy(), e0.copy()
            ep[m, c] += h
            em[m, c] -= h
            fd = (frame.loss(ep, frame.A0) - frame.loss(em, frame.A0)) / (2 * h)
            err = abs(fd - ge[m, c]) / max(abs(ge).max(), 1e-30)
            worst = max(worst, err)
            checked += 1
    print(f"emitters checked {checked}, worst error relative to max gradient {worst:.2e}")
    assert checked >= 64
    assert worst < 1e-7


def test_texel_gradients_match_central_differences(frame):
    _, g0i, g0d = frame.gradients(frame.emission, frame.A0)
    st = S.Stream(950, 1)
    P = frame.A0[0].irr.shape[0]
    active = np.nonzero(np.isin(frame.A0[0].states, [4, 5]))[0]
    worst_i = worst_d = 0.0
    n_i = n_d = n_big = 0
    scale_i = max(np.abs(g0i[0]).max(), 1e-30)
    d = frame.A0[0].dist
    smooth = (d[..., 1] - d[..., 0] ** 2) > 10 * 1e-4 * (2 * np.abs(d[..., 0]) + 1)
    scale_d = max(np.abs(g0d[0][smooth]).max(), 1e-30)   # kink texels excluded
    for t in range(60):
        q = int(active[int(st.uniform(1, 0, len(active))[0])])
        y, x = int(st.uniform(1, 1, 7)[0]), int(st.uniform(1, 1, 7)[0])
        c = int(st.uniform(1, 0, 3)[0])
        h = 1e-4
        A = [frame.o.copy_volumes(frame.A0) for _ in range(2)]
        A[0][0].irr[q, y, x, c] += h
        A[1][0].irr[q, y, x, c] -= h
        fd = (frame.loss(frame.emission, A[0]) - frame.loss(frame.emission, A[1])) / (2 * h)
        worst_i = max(worst_i, abs(fd - g0i[0][q, y, x, c]) / scale_i)
        n_i += 1
        # distance texels (half of them among those with a non-negligible
        # gradient); skip points where the loss is not smooth at this h
        if t % 2 == 0:
            y, x = int(st.uniform(1, 1, 15)[0]), int(st.uniform(1, 1, 15)[0])
            c = int(st.uniform(1, 0, 2)[0])
        else:
            # texels whose own variance mu2 - mu^2 is far from the clamp at 0
            # (sky texels sit on it: mu = d_max, mu2 = d_max^2)
            big = np.argwhere((np.abs(g0d[0]) > 1e-3 * scale_d) & smooth[..., None])
            q, y, x, c = (int(v) for v in big[int(st.uniform(1, 0, len(big))[0])])
        def one_sided(hh):
            A = [frame.o.copy_volumes(frame.A0) for _ in range(2)]
            A[0][0].dist[q, y, x, c] += hh
            A[1][0].dist[q, y, x, c] -= hh
            lp, lm = frame.loss(frame.emission, A[0]), frame.loss(frame.emission, A[1])
            return (lp - l0) / hh, (l0 - lm) / hh, (lp - lm) / (2 * hh)

        l0 = frame.loss(frame.emission, frame.A0)
        f1, b1, c1 = one_sided(h)
        f2, b2, c2 = one_sided(h / 2)
        # curvature makes forward and backward slopes differ by O(h); a kink of
        # max(mu2 - mu^2, 0) within h of the point leaves an O(1) gap
        if abs(f2 - b2) > 0.75 * abs(f1 - b1) and abs(f1 - b1) > 1e-6 * scale_d:
            continue
        vals = [c1, (4.0 * c2 - c1) / 3.0]     # Richardson: O(h^4)
        worst_d = max(worst_d, abs(vals[1] - g0d[0][q, y, x, c]) / scale_d)
        n_d += 1
        n_big += int(t % 2 == 1)
    print(f"irradiance texels {n_i}: worst {worst_i:.2e}; distance texels {n_d} ({n_big} with large gradient): "
          f"worst {worst_d:.2e}")
    assert n_i == 60 and n_d >= 20 and n_big >= 10
    assert worst_i < 1e-6 and worst_d < 1e-6


def test_gradient_is_linear_in_the_residual(frame):
    # the loss gradient is linear in the residual E - T: a target that doubles
    # the residual doubles every gradient
    ge1, gi1, _ = frame.gradients(frame.emission, frame.A0)
    t0 = frame.target
    frame.target = 2 * t0 - frame.forward(frame.emission, frame.A0)[0]
    ge2, gi2, _ = frame.gradients(frame.emission, frame.A0)
    frame.target = t0
    assert np.allclose(ge2, 2 * ge1, rtol=1e-9, atol=1e-18)
    assert np.allclose(gi2[0], 2 * gi1[0], rtol=1e-9, atol=1e-18)


def test_full_size_emitter_gradient_directional_differences():
    """Full-size differentiable frame: the loss is quadratic in the emitter
    radiances (hits fixed), so a central difference along any direction
    equals the directional derivative up to FP64 rounding."""
    from tests.adjoint_case import FullFrame
    fr = FullFrame()
    o = fr.o
    E, A1, rec = fr.forward(fr.emission)
    q = fr.w.queries
    gE = 2.0 * (E - fr.target) / E.size
    g1i = [np.zeros_like(v.irr) for v in A1]
    g1d = [np.zeros_like(v.dist) for v in A1]
    o.query_backward(A1, q.pos, q.nrm, q.view, gE, g1i, g1d)
    prev = o.copy_volumes(fr.A0)
    o.state_step(fr.sc, prev)
    g0i = [np.zeros_like(v.irr) for v in prev]
    g0d = [np.zeros_like(v.dist) for v in prev]
    ge = np.zeros_like(fr.emission)
    fr.sc.set_emission(fr.emission)
    o.update_backward(fr.sc, prev, fr.R, rec, g1i, g1d, g0i, g0d, ge)
    assert np.count_nonzero(ge[-64:]) >= 150     # the 64 emissive quads (the last materials)
    st = S.Stream(953, 1)
    for k in range(3):
        d = st.uniform(ge.size, -1.0, 1.0).reshape(ge.shape)
        h = 0.1
        fd = (fr.loss(fr.emission + h * d) - fr.loss(fr.emission - h * d)) / (2 * h)
        dd = float((ge * d).sum())
        print(f"direction {k}: fd={fd:.12e} grad.d={dd:.12e}")
        assert abs(fd - dd) <= 1e-8 * abs(dd) + 1e-14
