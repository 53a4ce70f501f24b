"""The seeded input generators: deterministic, and of the stated shape."""
import numpy as np

from paper_2009_10796_amd import scenes as S


def test_splitmix64_reference_values():
    # SplitMix64 seeded with 0: the first outputs of the published generator
    out = S.splitmix64(0, 0, 3)
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_rotations_are_orthonormal_and_deterministic():
    R = S.rotations(1, 8).reshape(-1, 3, 3).astype(np.float64)
    for r in R:
        assert np.allclose(r @ r.T, np.eye(3), atol=1e-6)
        assert np.linalg.det(r) > 0
    assert np.array_equal(S.rotations(1, 8), S.rotations(1, 8))
    assert np.array_equal(S.rotations(1, 3, start_frame=5), S.rotations(1, 8)[5:8])


def test_config0_shape():
    w = S.config0()
    assert w.scene.n_triangles == 38
    assert w.queries.n == 4096 and w.volumes[0].n_probes == 64
    assert np.all((w.queries.pos >= 0) & (w.queries.pos <= 8))
    assert np.allclose(np.linalg.norm(w.queries.nrm, axis=1), 1, atol=1e-6)
    assert w.scene.tri_object.max() == 1        # box B is dynamic
    w2 = S.config0()
    assert np.array_equal(w.scene.vertices, w2.scene.vertices)


def test_config1_shape_without_gbuffer():
    w = S.config1(gbuffer=False)
    assert abs(w.scene.n_triangles - 100_000) < 5000
    assert w.lights.point_pos.shape == (8, 3)
    assert (w.scene.emission.max(axis=1) > 0).sum() == 32
    assert w.volumes[0].n_probes == 2048 and w.volumes[0].rays_per_probe == 256
