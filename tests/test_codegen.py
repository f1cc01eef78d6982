"""Guard against a code-generation hazard seen with this toolchain on gfx950.

A wave-uniform value moved into scalar registers (a lane broadcast) and then compared in
floating point was compiled into `v_cmp_* vcc, ...` followed by `s_cselect`, where the select
reads the scalar condition code SCC, last written by an unrelated address addition (its carry
bit), instead of the compare's result in VCC.  The HRSS walk then saw every candidate as
outside the slice.  The kernels keep decision data in vector registers; this test compiles
them to gfx950 assembly and fails if the pattern reappears: an s_cselect (or SCC branch) whose
last SCC writer is an arithmetic scalar op while a VCC compare sits in between.
"""
import os
import re
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2601_23252_amd", "csrc")

ARITH = re.compile(r"^\s*s_(add|addc|sub|subb|lshl|lshr|ashr|mul|bfe|abs|absdiff|min|max)[_a-z0-9]*\b")
LOGIC = re.compile(r"^\s*s_(cmp|cmpk|and|or|xor|andn2|orn2|nand|nor|xnor|not|bitcmp)[_a-z0-9]*\b")
VCMP = re.compile(r"^\s*v_cmpx?_\S+_e32\s+vcc")
USE = re.compile(r"^\s*s_(cselect_b(32|64)|cbranch_scc[01]|cmovk|cmov)\b")
LABEL = re.compile(r"^\S+:")


def suspicious_selects(asm: str):
    hits = []
    last, last_i, last_vcmp = None, -1, -1
    lines = asm.splitlines()
    for i, ln in enumerate(lines):
        if LABEL.match(ln):
            last, last_vcmp = None, -1
        if USE.match(ln) and last == "arith" and last_vcmp > last_i:
            hits.append((i + 1, ln.strip()))
        if VCMP.match(ln):
            last_vcmp = i
        if ARITH.match(ln):
            last, last_i = "arith", i
        elif LOGIC.match(ln):
            last, last_i = "logic", i
    return hits


def test_scanner_flags_the_pattern():
    bad = "\n".join(["bb:", "\ts_add_i32 s6, s59, s79", "\tv_cmp_lg_f64_e32 vcc, s[6:7], v[4:5]",
                     "\ts_nop 1", "\ts_cselect_b32 s7, s7, 0xfff00000"])
    good = "\n".join(["bb:", "\ts_add_i32 s6, s59, s79", "\tv_cmp_lg_f64_e32 vcc, s[6:7], v[4:5]",
                      "\ts_and_b64 s[0:1], vcc, exec", "\ts_cselect_b32 s7, s7, 0xfff00000"])
    assert len(suspicious_selects(bad)) == 1
    assert suspicious_selects(good) == []


@pytest.mark.parametrize("src", ["nss_kernels.hip", "nss_hrss_plan.hip", "nss_gp.hip",
                                 "nss_post.hip"])
def test_no_select_on_stale_condition_code(src, tmp_path):
    out = tmp_path / "k.s"
    cmd = ["hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", "-o", str(out),
           os.path.join(CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    hits = suspicious_selects(out.read_text())
    assert hits == [], hits[:5]
