"""Wait states around the inline-asm DPP FMAs of the covariance sweeps.

The register sweeps of ``csrc/cov.hip`` issue ``v_fmac_f64_dpp`` (a 64-bit
FMA whose first source is read through a DPP row broadcast) from inline asm,
which the compiler's hazard recognizer does not see into.  The asm carries
the two wait states a DPP read needs after a vector write of its source; a
write of EXEC needs five, and the sweeps rely on EXEC not changing right
before these FMAs.  This test builds the kernels for gfx950 and checks that,
counting back five wait states from every such FMA (an instruction is one,
``s_nop N`` is N + 1), no instruction writes EXEC.  No GPU needed.
"""
from __future__ import annotations

import os
import re
import subprocess

import pytest

from paper_1402_2518_amd import build as B

EXEC_WRITE = re.compile(r"^(s_\w+\s+exec\b|s_\w*saveexec\w*|v_cmpx_)")


def _instructions(asm: str) -> list[str]:
    out = []
    for line in asm.splitlines():
        t = line.strip()
        if not t or t.startswith((";", ".")) or t.endswith(":"):
            continue
        out.append(t.split(";")[0].strip())
    return out


def test_no_exec_write_within_five_wait_states_of_a_dpp_fma(tmp_path):
    if not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path / "cov.s"
    r = subprocess.run([B.HIPCC, *B.FLAGS, "--cuda-device-only", "-S", os.path.join(B.CSRC, "cov.hip"),
                        "-o", str(out)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    ins = _instructions(out.read_text())
    sites = 0
    for i, op in enumerate(ins):
        if not op.startswith("v_fmac_f64_dpp"):
            continue
        sites += 1
        waits, j = 0, i - 1
        while j >= 0 and waits < 5:
            prev = ins[j]
            assert not EXEC_WRITE.match(prev), (i, ins[max(0, i - 8):i + 1])
            m = re.match(r"^s_nop\s+(\d+)", prev)
            waits += int(m.group(1)) + 1 if m else 1
            j -= 1
    assert sites > 1000, sites  # the sweeps of both register paths, every kernel
