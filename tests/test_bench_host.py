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
    rec = {"source_sha": bench.hop_source_hash(), "vh": vh,
           "shapes": {"128/2": {"bytes_per_launch": 123}, "256/4": {"bytes_per_launch": 456}}}
    (prof / "hop_f64_24x24x24x48_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash reads the sources under ROOT: point it back at the repository's
    sha = rec["source_sha"]
    monkeypatch.setattr(bench, "hop_source_hash", lambda: sha)
    assert bench.traffic_from_profile(vh, 128, 2) == 123
    assert bench.traffic_from_profile(vh, 256, 4) == 456          # the launch shape the bench tuned
    assert bench.traffic_from_profile(vh, 128, 4) is None         # a shape without counters
    assert bench.traffic_from_profile(vh + 1, 128, 2) is None     # another lattice
    rec["source_sha"] = "0" * 16
    (prof / "hop_f64_24x24x24x48_traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_from_profile(vh, 128, 2) is None         # another kernel source


def test_traffic_from_counters_groups_the_pinned_shapes(tmp_path, monkeypatch):
    """The counter rows of the 12 x 10 pinned hop launches are attributed to their shapes in order."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    shapes = [[b, o] for b in (128, 256) for o in range(6)]
    info = {"copy_bytes": 1 << 30, "hop_launches": 10, "shapes": shapes, "hop_block": 128, "hop_order": 2,
            "hop_algorithmic_bytes": 331_776 * 1536, "hop_source_sha": "abc"}
    log = tmp_path / "k.log"
    log.write_text("rocprofv3 noise\n" + json.dumps(info) + "\n")
    hop = "void tmqcd::(anonymous namespace)::hop_kernel<0, 0, false, false, 0, 0, {}>(tmqcd::stencil::HopK)"
    for counter, copy_kib, per in (("FETCH_SIZE", 524288.0, 1.0), ("WRITE_SIZE", 1048576.0, 0.5)):
        lines = ["Dispatch_Id,Kernel_Name,Workgroup_Size,Counter_Name,Counter_Value",
                 f"1,__amd_rocclr_copyBuffer,256,{counter},{copy_kib}"]
        d = 2
        for k in range(7):   # tuner launches before the pinned ones are ignored
            lines.append(f'{d},"{hop.format(128)}",128,{counter},9999')
            d += 1
        for i, (b, o) in enumerate(shapes):
            for _ in range(10):
                lines.append(f'{d},"{hop.format(b)}",{b},{counter},{(1000 + i) * per}')
                d += 1
        (tmp_path / f"{counter}.csv").write_text("\n".join(lines) + "\n")
    bench.traffic_from_counters(str(tmp_path / "FETCH_SIZE.csv"), str(tmp_path / "WRITE_SIZE.csv"), str(log))
    rec = json.loads((tmp_path / "profiles" / "hop_f64_24x24x24x48_traffic.json").read_text())
    assert rec["calibration"]["FETCH_SIZE"]["factor"] == 2.0 and rec["calibration"]["WRITE_SIZE"]["factor"] == 1.0
    for i, (b, o) in enumerate(shapes):
        r = rec["shapes"][f"{b}/{o}"]
        assert r["FETCH_SIZE"] == round((1000 + i) * 1024 * 2.0)
        assert r["WRITE_SIZE"] == round((1000 + i) * 0.5 * 1024)
        assert r["bytes_per_launch"] == r["FETCH_SIZE"] + r["WRITE_SIZE"]


def test_hop_source_hash_is_stable():
    assert bench.hop_source_hash() == bench.hop_source_hash()
    assert len(bench.hop_source_hash()) == 16


def test_mrhs_shapes_from_counters_attributes_launches(tmp_path, capsys):
    """The 18 x 3 pinned 12-RHS launches are attributed to their shapes in order, the 10 before them to
    the tuned shape, and the spinors' share of the fetch is what remains after the link reads of each
    sweep."""
    vh = 1000
    shapes = [[o, g] for o in range(6) for g in (0, 6, 4)]
    info = {"copy_bytes": 1 << 30, "launches": 10, "f64_shapes": shapes, "f64_shape_launches": 3, "vh": vh,
            "f64": {"order": 3, "group": 6}}
    log = tmp_path / "k.log"
    log.write_text(json.dumps(info) + "\n")
    name = "void tmqcd::stencil::(anonymous namespace)::hop_mrhs_kernel<0, 0, false, false, 0>(tmqcd::stencil::HopK)"
    links, spinors = vh * 1152, 12 * vh * 192
    for counter, copy_kib in (("FETCH_SIZE", 524288.0), ("WRITE_SIZE", 1048576.0)):
        lines = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value", f"1,__amd_rocclr_copyBuffer,{counter},{copy_kib}"]
        d = 2
        for _ in range(4):    # the tuner's own trial launches
            lines.append(f'{d},"{name}",{counter},77')
            d += 1
        for _ in range(10):   # the tuned launches before the pinned ones: shape 3/6, two sweeps
            kib = (2 * links + 2.0 * spinors) / 1024.0 / 2.0 if counter == "FETCH_SIZE" else 12 * vh * 192 / 1024.0
            lines.append(f'{d},"{name}",{counter},{kib}')
            d += 1
        for i, (o, g) in enumerate(shapes):
            sweeps = 1 if g == 0 else 12 // g
            fetch = sweeps * links + (1.5 + 0.1 * i) * spinors      # bytes
            for _ in range(3):
                kib = fetch / 1024.0 / 2.0 if counter == "FETCH_SIZE" else 12 * vh * 192 / 1024.0
                lines.append(f'{d},"{name}",{counter},{kib}')
                d += 1
        (tmp_path / f"{counter}.csv").write_text("\n".join(lines) + "\n")
    bench.mrhs_shapes_from_counters(str(tmp_path / "FETCH_SIZE.csv"), str(tmp_path / "WRITE_SIZE.csv"), str(log))
    out = [json.loads(l) for l in capsys.readouterr().out.splitlines()]
    assert [r["shape"] for r in out] == [f"{o}/{g}" for o, g in shapes] + ["tuned 3/6"]
    for i, r in enumerate(out[:-1]):
        assert r["spinor_fetch_ratio"] == round(1.5 + 0.1 * i, 2)
        assert r["WRITE_SIZE"] == 12 * vh * 192
    assert out[-1]["spinor_fetch_ratio"] == 2.0 and out[-1]["WRITE_SIZE"] == 12 * vh * 192
