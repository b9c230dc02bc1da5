"""The 16-byte-slot quotient map's key mix is a bijection onto (home slot, remainder) fields of
the right widths (host build of tests/qmix2_check.cpp against the library's header)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2511_14955_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_qmix2_is_injective_and_fits_its_fields():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "qmix2_check")
        subprocess.run(["hipcc", "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC,
                        os.path.join(HERE, "qmix2_check.cpp"), "-o", exe],
                       check=True, capture_output=True, timeout=600)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    lines = out.stdout.strip().splitlines()
    assert lines[-1] == "bad=0"
    for ln in lines[:-1]:
        f = dict(kv.split("=") for kv in ln.split())
        assert f["keys"] == f["images"], ln
