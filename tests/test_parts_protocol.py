"""Host logic of the two-workgroup SAP phase kernel: the split tables and the halo
exchange protocol, emulated on the CPU (tests/host/parts_protocol.cpp) against an
unsplit hyperplane-order SSOR of a scalar toy operator, bit for bit, under random
interleavings of the two workgroups, including a launch after one whose waits timed out
(no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_parts_protocol(tmp_path):
    exe = tmp_path / "parts_protocol"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", str(exe), os.path.join(HERE, "host", "parts_protocol.cpp")])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all protocol cases agree" in out.stdout
