"""Host-side check of the grouped batch launches' block decode (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_grouped_batch_decode_covers_every_member_once(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "batch_check")
    subprocess.run(["hipcc", "-O1", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2511_21031_amd", "csrc"),
                    os.path.join(ROOT, "tests", "batch_index_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    res = subprocess.run([exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout
