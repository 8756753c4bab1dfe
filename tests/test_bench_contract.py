"""Host-side checks of bench.py: the one-GPU guard, the algorithmic byte
counts, and the committed HBM byte records of the three hot kernels (a
kernel changed since its counters were taken reports null traffic)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_records_follow_the_sources(tmp_path, monkeypatch):
    """Each committed record parses; it yields bytes exactly when the
    SHA-256 of the kernel's sources matches, and None once they change."""
    import json
    import re
    for prof, src in ((bench.PASS1_PROFILE, bench.PASS1_SOURCES),
                      (bench.SELECT_PROFILE, bench.SELECT_SOURCES),
                      (bench.PASS2_PROFILE, bench.PASS2_SOURCES)):
        text = open(os.path.join(ROOT, prof)).read()
        m = re.search(r"^traffic-record: (\{.*\})\s*$", text, re.M)
        assert m, prof
        rec = json.loads(m.group(1))
        for key in ("fetch_kib", "write_kib", "fetch_scale", "write_scale",
                    "source_sha256"):
            assert key in rec, (prof, key)
        t = bench.kernel_traffic(prof, src)
        if rec["source_sha256"] == bench.sources_digest(src):
            want = 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"]
                             + rec["write_kib"] * rec["write_scale"])
            assert t == want and t > 0
        else:
            assert t is None
    # a record whose digest does not match reports no traffic
    rec = {"kernel": "k", "fetch_kib": 1.0, "write_kib": 1.0, "fetch_scale": 2.0,
           "write_scale": 1.0, "source_sha256": "0" * 64}
    f = tmp_path / "p.md"
    f.write_text("traffic-record: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_traffic("p.md", []) is None
    rec["source_sha256"] = bench.sources_digest([])
    f.write_text("traffic-record: " + json.dumps(rec) + "\n")
    assert bench.kernel_traffic("p.md", []) == 3072.0


def test_algorithmic_bytes_per_particle():
    # 24 + 4 + 4 L + 24 + L + 12 + 32 with L = 77.5 list entries
    assert abs(bench.SELECT_BYTES_PER_PARTICLE - 483.5) < 1e-9
    assert bench.PASS2_BYTES_PER_PARTICLE == 629


def test_adjoint_flop_record_follows_the_sources(tmp_path, monkeypatch):
    """The committed float64 flop record of the adjoint step parses and is
    used exactly while the adjoint's sources are unchanged."""
    import json
    import re
    text = open(os.path.join(ROOT, bench.ADJOINT_PROFILE)).read()
    m = re.search(r"^flop-record: (\{.*\})\s*$", text, re.M)
    assert m
    rec = json.loads(m.group(1))
    assert rec["flop_per_particle"] > 1e4 and rec["particles"] == 131072
    got = bench.flop_record(bench.ADJOINT_PROFILE, bench.ADJOINT_SOURCES)
    if rec["source_sha256"] == bench.sources_digest(bench.ADJOINT_SOURCES):
        assert got == rec["flop_per_particle"]
    else:
        assert got is None
    f = tmp_path / "a.md"
    f.write_text("flop-record: " + json.dumps({"flop_per_particle": 5.0,
                                                "source_sha256": "0" * 64}) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.flop_record("a.md", []) is None
    f.write_text("flop-record: " + json.dumps({"flop_per_particle": 5.0,
                                                "source_sha256": bench.sources_digest([])})
                 + "\n")
    assert bench.flop_record("a.md", []) == 5.0
