"""No step of the GPU path computes in FP64: every HIP source, compiled for
gfx950 to device assembly, holds no FP64 vector instruction (v_*_f64).
Runs on the CPU (hipcc cross-compiles); skipped where hipcc is missing."""
import os
import re
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2211_08506_amd"))
import build  # noqa: E402  (the library's own compile flags)

F64 = re.compile(r"^\s+v_\w+_f64\b", re.M)


def _device_asm(src: str, out_dir: str) -> str:
    out = os.path.join(out_dir, os.path.basename(src) + ".s")
    cmd = [build.HIPCC] + build.COMMON + ["-x", "hip", "--cuda-device-only", "-S",
                                          os.path.join(build.CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    with open(out) as f:
        return f.read()


@pytest.mark.skipif(not os.path.exists(build.HIPCC), reason="hipcc not available")
def test_device_code_has_no_fp64():
    hips = [s for s in build.SOURCES if s.endswith(".hip")]
    with tempfile.TemporaryDirectory() as d, ThreadPoolExecutor(4) as ex:
        asm = dict(zip(hips, ex.map(lambda s: _device_asm(s, d), hips)))
    bad = {s: F64.findall(a)[:3] for s, a in asm.items() if F64.search(a)}
    assert not bad, bad
