"""Checks on the gfx950 assembly of the FP64 trilinear kernel, compiled here
from source with the flags of the build.  Its FMAs read their pair products
through a DPP row broadcast behind a two-wait-state s_nop; that is enough only
while no VALU instruction of the kernel writes EXEC (v_cmpx), which would
need five."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2110_13735_amd"))

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def kernel_asm(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    import build_lib

    out = tmp_path_factory.mktemp("isa") / "t1_pairs.s"
    cmd = [HIPCC, *build_lib.FLAGS, "-I", build_lib.CSRC, "--cuda-device-only", "-S",
           os.path.join(build_lib.CSRC, "t1_pairs.hip"), "-o", str(out)]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    s = out.read_text()
    m = re.search(r"^(_Z\w*trilinear_kernel\w*):", s, flags=re.M)
    assert m, "trilinear kernel not found in the assembly"
    end = s.index(".Lfunc_end", m.end())
    return s[m.end():end]


def _instructions(body):
    for line in body.splitlines():
        t = line.strip()
        if t and not t.startswith((";", ".")) and not t.endswith(":"):
            yield t


def test_no_valu_write_of_exec(kernel_asm):
    ops = [t.split()[0] for t in _instructions(kernel_asm)]
    assert not [o for o in ops if o.startswith("v_cmpx")]


def test_every_dpp_group_is_behind_a_wait(kernel_asm):
    ins = list(_instructions(kernel_asm))
    n = 0
    for i, t in enumerate(ins):
        if t.startswith("v_fmac_f64_dpp") and not ins[i - 1].startswith("v_fmac_f64_dpp"):
            assert ins[i - 1].startswith("s_nop"), ins[i - 1]
            assert int(ins[i - 1].split()[1]) >= 1
            n += 1
    assert n > 0
