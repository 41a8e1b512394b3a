"""Host-side checks of bench.py: the one-GPU guard, the algorithmic byte counts its
roofline uses, and the rule that the measured traffic is reported only for the
hop source it was measured on.  No GPU is touched."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("prec,recon,expect", [
    # per output site: 8 links + one input and one output spinor (18 / 12 / 10 / 8 reals per link)
    (0, 0, 8 * 18 * 8 + 2 * 24 * 8), (0, 1, 8 * 12 * 8 + 2 * 24 * 8),
    (0, 2, 8 * 10 * 8 + 2 * 24 * 8), (0, 3, 8 * 8 * 8 + 2 * 24 * 8),
    (1, 0, 8 * 18 * 4 + 2 * 24 * 4), (1, 1, 8 * 12 * 4 + 2 * 24 * 4),
    # FP16 spinors carry one FP32 scale per site
    (2, 0, 8 * 18 * 2 + 2 * (24 * 2 + 4)), (2, 1, 8 * 12 * 2 + 2 * (24 * 2 + 4)),
])
def test_algorithmic_bytes_per_site(prec, recon, expect):
    assert bench.BYTES_PER_SITE[(prec, recon)] == expect


def test_headline_bytes_per_launch():
    vh = 24 ** 3 * 48 // 2
    assert vh * bench.BYTES_PER_SITE[(0, 0)] == 509_607_936


def test_traffic_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    vh = 331_776
    rec = {"source_sha": bench.hop_source_hash(), "vh": vh, "bytes_per_launch": 123}
    (prof / "hop_f64_24x24x24x48_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash reads the sources under ROOT: point it back at the repository's
    sha = rec["source_sha"]
    monkeypatch.setattr(bench, "hop_source_hash", lambda: sha)
    assert bench.traffic_from_profile(vh) == 123
    assert bench.traffic_from_profile(vh + 1) is None            # another lattice
    rec["source_sha"] = "0" * 16
    (prof / "hop_f64_24x24x24x48_traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_from_profile(vh) is None                # another kernel source


def test_hop_source_hash_is_stable():
    assert bench.hop_source_hash() == bench.hop_source_hash()
    assert len(bench.hop_source_hash()) == 16
