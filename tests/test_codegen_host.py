"""Code-generation checks of the fp32 cell kernel (host only: hipcc
cross-compiles for gfx950, nothing runs on a GPU).

The fp32 predictor's lane exchanges are the DPP source operands of
`v_fmac_f32_dpp` instructions written as inline assembly, each preceded by
`s_nop 1`. That covers the two wait states a DPP read needs after a VALU
write of its source. It does not cover the five wait states after a VALU
write of EXEC, which the compiler does not insert ahead of inline assembly;
the kernels rely on containing no such write (`v_cmpx*`). These tests
compile the cell kernels to assembly and check both facts.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1212_3585_amd import build

CSRC = build.CSRC


def _asm(src, tmp_path):
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        pytest.skip("hipcc not available")
    out = tmp_path / (os.path.splitext(src)[0] + ".s")
    flags = [f for f in build.compile_flags() if f not in ("-fPIC",)]
    cmd = [exe] + flags + ["-x", "hip", "--cuda-device-only", "-S",
                           os.path.join(CSRC, src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


def _kernel_bodies(asm, pattern):
    """Assembly text of each kernel whose symbol matches pattern."""
    bodies = {}
    for m in re.finditer(r"^(_Z\S+):\s*;", asm, re.M):
        name = m.group(1)
        if not re.search(pattern, name):
            continue
        end = asm.find("s_endpgm", m.end())
        bodies[name] = asm[m.end():end]
    return bodies


@pytest.mark.parametrize("src", ["cell2d_rows8.hip", "batch2d.hip"])
def test_fp32_cell_kernel_dpp_fmas_and_no_valu_exec_writes(src, tmp_path):
    asm = _asm(src, tmp_path)
    f32 = _kernel_bodies(asm, r"k_cell2d\w*ILi3ELi1ELi\d+EfE|k_cell2d_batch\w*ILi3ELi1ELi\d+EfE")
    assert f32, "no fp32 Euler M = 3 cell kernel found"
    for name, body in f32.items():
        assert "v_fmac_f32_dpp" in body, name
        # every DPP FMA directly follows its s_nop
        lines = [l.strip() for l in body.splitlines() if l.strip() and not l.strip().startswith(";")]
        for i, l in enumerate(lines):
            if l.startswith("v_fmac_f32_dpp"):
                assert lines[i - 1].startswith("s_nop"), (name, lines[i - 1])
    # no VALU write of EXEC anywhere in the translation unit's kernels
    assert not re.search(r"^\s*v_cmpx", asm, re.M)
    assert not re.search(r"^\s*v_\S+\s+exec\b", asm, re.M)
