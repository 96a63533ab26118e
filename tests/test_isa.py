"""Checks on the gfx950 assembly of the FP64 trilinear kernel, compiled here
from source with the flags of the build.  Its FMAs read their pair products
through a DPP row broadcast with no wait written before them: that is correct
only while no VALU instruction writes a DPP source register less than two
wait states before the read, and no VALU instruction writes EXEC (v_cmpx),
which would need five."""
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


def _vregs(tok):
    m = re.match(r"v\[(\d+):(\d+)\]$", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def dpp_hazards(asm):
    """(DPP reads checked, violations): walk back from every DPP read,
    counting wait states (one per instruction, n + 1 for s_nop n), until two
    have passed; a VALU write of the DPP source, or a block boundary (label),
    inside that distance is a violation."""
    ins = []
    for line in asm.splitlines():
        t = line.strip()
        if t and not t.startswith((";", ".")):
            ins.append(t)
    n, bad = 0, []
    for i, t in enumerate(ins):
        if not t.startswith("v_fmac_f64_dpp"):
            continue
        n += 1
        src0 = _vregs(t.split(None, 1)[1].split(",")[1].strip())
        waits, j = 0, i - 1
        while waits < 2:
            if j < 0 or ins[j].endswith(":"):
                bad.append(("block boundary", t))
                break
            op = ins[j].split()[0]
            if op == "s_nop":
                waits += int(ins[j].split()[1], 0) + 1
            else:
                if op.startswith("v_") and len(ins[j].split(None, 1)) > 1:
                    if _vregs(ins[j].split(None, 1)[1].split(",")[0].strip()) & src0:
                        bad.append((ins[j], t))
                waits += 1
            j -= 1
    return n, bad


def test_dpp_hazard_check_finds_a_planted_write():
    dpp = "v_fmac_f64_dpp v[10:11], v[122:123], v[4:5] row_newbcast:3 row_mask:0xf bank_mask:0xf"
    assert dpp_hazards(f"v_mov_b32 v123, 0\n{dpp}")[1]
    assert dpp_hazards(f"v_mov_b32 v122, 0\ns_nop 0\n{dpp}")[1]
    assert not dpp_hazards(f"v_mov_b32 v122, 0\ns_nop 1\n{dpp}")[1]
    assert not dpp_hazards(f"v_mov_b32 v122, 0\nv_add_f64 v[0:1], v[2:3], v[4:5]\ns_nop 0\n{dpp}")[1]
    assert not dpp_hazards(f"ds_read_b128 v[120:123], v1\ns_waitcnt lgkmcnt(0)\nv_mov_b32 v0, 1\n{dpp}")[1]
    assert dpp_hazards(f"label:\n{dpp}")[1]


def test_no_valu_write_of_a_dpp_source_within_two_wait_states(kernel_asm):
    n, bad = dpp_hazards(kernel_asm)
    assert n > 0
    assert not bad, bad[:3]
