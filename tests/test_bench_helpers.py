"""Host logic of bench.py (CPU): the committed DRAM-traffic figures are used
only while the kernel sources are the ones they were measured on; the
query's algorithmic bytes follow their definition (36 B in + 12 B out + 8
state bytes per point, 80 B per sampled probe of its cage); the host CPU
report has its fields."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2009_10796_amd import scenes as S  # noqa: E402


def _traffic_file(tmp_path, sha):
    data = {"workload": "x", "kernel_source_sha256": sha, "bytes_per_launch": {"shadow": 123, "query": 456}}
    p = tmp_path / "traffic.md"
    p.write_text("# t\n\ntext\n\n```json\n" + json.dumps(data) + "\n```\n")
    return str(p)


def test_traffic_used_only_for_the_measured_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, bench.kernel_source_hash()))
    assert bench.measured_traffic() == {"shadow": 123, "query": 456}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, "0" * 64))
    assert bench.measured_traffic() == {}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() == {}


def test_kernel_source_hash_sees_every_source():
    d = os.path.join(ROOT, "paper_2009_10796_amd", "csrc")
    names = sorted(n for n in os.listdir(d) if n.endswith((".hip", ".h", ".cpp")))
    assert names and len(bench.kernel_source_hash()) == 64


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
