"""Host logic of bench.py (CPU): the committed counter figures are used only
while the kernel sources are the ones they were measured on; the counter
summary parses rocprofv3 CSVs and scales byte counters by the calibration
copy; the roofline takes the bound that binds; the query's algorithmic bytes
follow their definition (36 B in + 12 B out + 8 state bytes per point, 80 B
per sampled probe of its cage); the host CPU report has its fields."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2009_10796_amd import scenes as S  # noqa: E402


def _counter_file(tmp_path, sha):
    data = {"workload": "city", "kernel_source_sha256": sha,
            "per_launch": {"shadow": {"dram_bytes": 123.0, "valu_insts": 10.0}}}
    p = tmp_path / "counters.md"
    p.write_text("# t\n\ntext\n\n```json\n" + json.dumps(data) + "\n```\n")
    return str(p)


def test_counters_used_only_for_the_measured_sources(tmp_path, monkeypatch):
    files = dict(bench.COUNTER_FILES)
    monkeypatch.setattr(bench, "COUNTER_FILES", files)
    files["city"] = _counter_file(tmp_path, bench.kernel_source_hash())
    assert bench.load_counters("city") == {"shadow": {"dram_bytes": 123.0, "valu_insts": 10.0}}
    files["city"] = _counter_file(tmp_path, "0" * 64)
    assert bench.load_counters("city") == {}
    files["city"] = str(tmp_path / "missing.md")
    assert bench.load_counters("city") == {}


def test_kernel_source_hash_covers_the_frame_and_query_kernels():
    d = os.path.join(ROOT, "paper_2009_10796_amd", "csrc")
    for name in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(d, name))
    assert len(bench.kernel_source_hash()) == 64


def test_summary_scales_by_the_copy_and_averages_dispatches(tmp_path):
    rows = ["Dispatch_Id,Grid_Size,Kernel_Name,Counter_Name,Counter_Value"]
    # calibration copy (the largest copy grid): FETCH_SIZE reads half the
    # bytes, WRITE_SIZE all of them; a small runtime copy is not calibration
    for d in (1, 2, 3):
        rows.append(f"{d},131072,__amd_rocclr_copyBuffer,FETCH_SIZE,{128 * 1024}")
        rows.append(f"{d},131072,__amd_rocclr_copyBuffer,WRITE_SIZE,{256 * 1024}")
    rows.append("4,512,__amd_rocclr_copyBuffer,FETCH_SIZE,3")
    # two dispatches of the shadow kernel, a counter split over two rows of one dispatch
    rows += ["10,1,irf::k_shadow(irf::VolumeSet),FETCH_SIZE,100", "10,1,irf::k_shadow(irf::VolumeSet),FETCH_SIZE,100",
             "11,1,irf::k_shadow(irf::VolumeSet),FETCH_SIZE,400",
             "10,1,irf::k_shadow(irf::VolumeSet),WRITE_SIZE,10", "11,1,irf::k_shadow(irf::VolumeSet),WRITE_SIZE,30",
             "12,1,void irf::k_blend_mma<0>(irf::VolumeSet),SQ_VALU_MFMA_BUSY_CYCLES,7"]
    p = tmp_path / "c.csv"
    p.write_text("\n".join(rows) + "\n")
    d = bench.summarize("city", [str(p)])
    assert abs(d["copy_scale"]["FETCH_SIZE"] - 2.0) < 1e-12 and abs(d["copy_scale"]["WRITE_SIZE"] - 1.0) < 1e-12
    sh = d["per_launch"]["shadow"]
    assert sh["fetch_bytes"] == 300 * 1024 * 2.0 and sh["write_bytes"] == 20 * 1024
    assert sh["dram_bytes"] == sh["fetch_bytes"] + sh["write_bytes"]
    assert d["per_launch"]["blend_mma"]["mfma_busy_cycles"] == 7
    assert "```json" in bench.summary_markdown("city", [str(p)])


def test_roofline_takes_the_binding_bound():
    us = 50.0
    cyc = bench.SIMDS * bench.CLOCK_GHZ * 1e3 * us
    c = {"k": {"dram_bytes": 0.25 * bench.HBM_PEAK_GBS * 1e9 * us * 1e-6, "valu_insts": 0.6 * cyc / 4.0}}
    r = bench.binding_roofline("k", us, c)
    assert r["bound"] == "alu" and abs(r["frac"] - 0.6) < 1e-9 and abs(r["fractions"]["hbm"] - 0.25) < 1e-9
    assert r["frac"] <= 1.0 and r["traffic"] == int(c["k"]["dram_bytes"])
    assert bench.binding_roofline("k", us, {})["frac"] is None


def test_query_bytes_follow_the_definition():
    w = S.config0(n_queries=1000)
    d = w.volumes[0]
    n = d.n_probes
    none = np.zeros(n, np.uint8)
    all_sampled = np.full(n, S.VIGILANT, np.uint8)
    b0, m0 = bench.query_bytes(w, none)
    b8, m8 = bench.query_bytes(w, all_sampled)
    q = w.queries.n
    assert (b0, m0) == (q * (36 + 12 + 8), 0.0)
    assert m8 == 8.0 and b8 == q * (36 + 12 + 8) + q * 8 * (4 * 12 + 4 * 8)
    # awake probes are sampled too; probes still in a Newly state are not
    mixed = np.where(np.arange(n) % 2 == 0, S.AWAKE, S.NEWLY_VIGILANT).astype(np.uint8)
    _, mm = bench.query_bytes(w, mixed)
    assert 0.0 < mm < 8.0


def test_host_cpu_report():
    r = bench.host_cpu()
    assert set(r) == {"cpu_model", "nproc", "affinity"}
    assert r["nproc"] >= 1 and 1 <= r["affinity"] <= r["nproc"]
