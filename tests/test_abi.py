"""The C ABI library: it loads, exports every function its header declares,
and its host-side logic (validation, BVH build) behaves without a GPU."""
import os
import re

import numpy as np
import pytest

from paper_2009_10796_amd import irf, scenes as S

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "irf.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(irf_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = irf.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(irf.SIGNATURES), set(names) ^ set(irf.SIGNATURES)


def test_header_is_plain_c_and_links(tmp_path):
    """The header compiles as C99 with every declaration used, and a C
    program links against the library (no GPU needed: nothing is called)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    names = _declared()
    src = tmp_path / "use.c"
    src.write_text('#include "irf.h"\n#include <stdio.h>\nint main(void) {\n'
                   + "".join(f'  printf("%p\\n", (void*)&{n});\n' for n in names) + "  return 0;\n}\n")
    lib = irf.LIB_PATH
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", f"-I{os.path.dirname(HEADER)}", str(src), "-o",
                        str(tmp_path / "use"), lib, f"-Wl,-rpath,{os.path.dirname(lib)}"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_status_strings_and_version():
    lib = irf.load()
    assert lib.irf_status_str(0) == b"IRF_OK"
    assert lib.irf_status_str(4) == b"IRF_E_STATE"
    assert lib.irf_version().startswith(b"irf")


def _good():
    return S.VolumeDesc(origin=(0, 0, 0), spacing=(1, 1, 1), counts=(4, 4, 4), rays_per_probe=64)


@pytest.mark.parametrize("field,value", [
    ("counts", (1, 4, 4)), ("spacing", (1, 0, 1)), ("spacing", (1, float("nan"), 1)),
    ("rays_per_probe", 48), ("rays_per_probe", 0), ("rays_per_probe", 2048),
    ("hysteresis_irr", 1.5), ("hysteresis_dist", -0.1), ("cos_power", 0.0),
    ("self_shadow_bias", -1.0), ("cheb_power", 0), ("cheb_power", 5), ("max_distance", float("inf")),
    ("origin", (0, float("inf"), 0)), ("irradiance_gamma", 0.5), ("irradiance_gamma", 17.0),
    ("irradiance_gamma", float("nan")),
])
def test_volume_validation_rejects(field, value):
    d = _good()
    setattr(d, field, value)
    with pytest.raises(irf.IrfError) as e:
        irf.validate_volume_desc(d)
    assert e.value.status == irf.E_INVALID


def test_volume_validation_accepts():
    irf.validate_volume_desc(_good())
    d = _good()
    d.rays_per_probe, d.atlas_f16, d.blend = 1024, True, "bf16"
    irf.validate_volume_desc(d)
    d.irradiance_gamma, d.texel_thresholds = 5.0, True
    irf.validate_volume_desc(d)


@pytest.mark.parametrize("make", [lambda: S.config0().scene, lambda: S.random_triangle_soup(3000),
                                  lambda: S.sphere_scene(3.0, 2), lambda: S.config1(gbuffer=False).scene])
def test_host_bvh_is_valid_and_shallow(make):
    st = irf.bvh_stats(make())
    assert st["valid"]
    assert 1 <= st["depth"] <= 48
    assert st["leaves"] >= 1


def test_host_bvh_single_triangle_and_empty():
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    sc = S.Scene(verts, np.array([[0, 1, 2]], np.uint32), np.zeros(1, np.uint32), np.zeros(1, np.uint32),
                 np.full((1, 3), 0.5, np.float32), np.zeros((1, 3), np.float32))
    assert irf.bvh_stats(sc)["valid"]
    assert irf.bvh_stats(S.empty_scene())["valid"]


def test_scene_validation_rejects_bad_indices_and_materials():
    sc = S.config0().scene
    bad = S.Scene(sc.vertices, sc.indices.copy(), sc.tri_material, sc.tri_object, sc.albedo, sc.emission)
    bad.indices[3, 1] = 10_000
    with pytest.raises(irf.IrfError):
        irf.bvh_stats(bad)
    bad = S.Scene(sc.vertices, sc.indices, sc.tri_material.copy(), sc.tri_object, sc.albedo, sc.emission)
    bad.tri_material[0] = 99
    with pytest.raises(irf.IrfError):
        irf.bvh_stats(bad)
    bad = S.Scene(sc.vertices.copy(), sc.indices, sc.tri_material, sc.tri_object, sc.albedo, sc.emission)
    bad.vertices[0, 0] = np.nan
    with pytest.raises(irf.IrfError):
        irf.bvh_stats(bad)


def test_tracking_volume_needs_five_probes_per_axis():
    d = _good()
    d.tracking = True
    with pytest.raises(irf.IrfError) as e:
        irf.validate_volume_desc(d)
    assert e.value.status == irf.E_INVALID
    d.counts = (5, 5, 6)
    irf.validate_volume_desc(d)


def test_library_built_from_other_sources_is_refused(monkeypatch):
    """The loaders compare each library's build stamp with the sources beside
    it and refuse a library built from other sources."""
    import oracle
    from oracle import build as obuild
    from paper_2009_10796_amd import build as lbuild
    monkeypatch.setattr(irf, "_lib", None)
    monkeypatch.setattr(lbuild, "source_hash", lambda: "0" * 64)
    with pytest.raises(RuntimeError, match="not built from the sources"):
        irf.load()
    monkeypatch.setattr(oracle, "_lib", None)
    monkeypatch.setattr(obuild, "source_hash", lambda extra: "0" * 64)
    with pytest.raises(RuntimeError, match="not built from the oracle's sources"):
        oracle.lib()
