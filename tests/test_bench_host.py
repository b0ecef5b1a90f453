"""Host-side checks of bench.py (no GPU): the one-GPU guard, the roofline byte models of the
SAP phase kernel and of the operator, and the lookup of counter traffic by source hash."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr and not p.stdout.strip()


def test_phase_byte_models_at_6x6x6x12_blocks():
    """Once-each bytes per site of a phase launch (FP32): own v, gathered neighbours and their
    links, clover blocks, x, y, r; the re-streamed model adds U, F and v per half-sweep."""
    import bench

    B, V = (6, 6, 6, 12), 24 ** 3 * 48
    f = sum(2.0 / b for b in B)
    once, flops = bench.phase_model(B, 4, 4)
    assert abs(once - 4 * (24 + 24 * f + 48 + 6 * f + 72 + 72 + 24)) < 1e-9
    assert abs(once * V / 2 - 364953600.0) < 1.0            # 365 MB per launch
    assert abs(bench.phase_stream_model(B, 4, 4) * V / 2 - 1893777408.0) < 1.0  # 1.89 GB per launch
    assert flops > 0
    d_bytes, _ = bench.dslash_model(8)
    assert d_bytes == 8 * (24 + 48 + 72 + 24)  # 1344 B per site in FP64


def test_counter_traffic_is_used_only_for_its_sources_and_workload(tmp_path, monkeypatch):
    import bench

    rec = {"workload": "24^3x48", "csrc_sha256": bench.csrc_sha256(), "fetch_scale": 2.0, "write_scale": 1.0,
           "kernels": {"k_sap_phase_parts": {"bytes_per_launch": 123.0}}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "counters.json").write_text(json.dumps(rec))
    csrc = tmp_path / "paper_1210_7398_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.PHASE_KERNEL_SOURCES:
        (csrc / name).write_bytes(open(os.path.join(ROOT, "paper_1210_7398_amd", "csrc", name), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("k_sap_phase_parts", "24^3x48") == 123.0
    assert bench.traffic_from_profiles("k_sap_phase_parts", "32^3x64") is None
    assert bench.traffic_from_profiles("k_other", "24^3x48") is None
    with open(csrc / "sap_parts.hip", "a") as fh:  # a changed kernel source voids the record
        fh.write("\n// changed\n")
    assert bench.traffic_from_profiles("k_sap_phase_parts", "24^3x48") is None
