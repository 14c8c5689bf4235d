"""CPU check of the generated gfx950 code of the counting kernels: every LDS access is a
DS instruction (no generic/FLAT addressing), so a helper the compiler keeps out of line
cannot turn an LDS address into a global one."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_10047_amd", "csrc")


@pytest.mark.parametrize("unit", ["count_d1.hip", "count_d4.hip"])
def test_count_kernels_have_no_flat_accesses(tmp_path, unit):
    from paper_2002_10047_amd import build
    out = tmp_path / "k.s"
    cmd = [build.hipcc(), *build.FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, unit), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    asm = out.read_text()
    assert "k_count" in asm
    flat = re.findall(r"^\s+flat_\w+", asm, flags=re.M)
    assert not flat, flat[:5]
