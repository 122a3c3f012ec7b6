"""Host check of the inline-assembly blocks that fuse a DPP broadcast into an
FP64 multiply-add (v_fmac_f64_dpp): a DPP instruction needs two wait states
after the write of any VGPR it reads (sources and accumulator), and the
compiler inserts none inside inline assembly.  Each block must start with at
least `s_nop 1` and keep two wait states between a write and every later read
of the same operand inside the block."""
import os
import re

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1901_06919_amd", "csrc", "fdl_device.h")


def _blocks():
    src = open(HDR).read()
    out = []
    for m in re.finditer(r'asm\((.*?)\s*:\s*"\+v"', src, re.S):
        text = "".join(re.findall(r'"((?:[^"\\]|\\.)*)"', m.group(1)))
        ins = [s.strip() for s in text.replace("\\t", "").split("\\n") if s.strip()]
        if any(i.startswith("v_fmac_f64_dpp") for i in ins):
            out.append(ins)
    return out


def _operands(ins):
    return re.findall(r"%(\d+)", ins.split("row_newbcast")[0])


def _violations(block):
    bad = []
    if not block[0].startswith("s_nop") or int(block[0].split()[1]) < 1:
        bad.append("block does not start with s_nop 1")
    slot = 0
    written = {}   # operand -> slot just after its write
    for ins in block:
        if ins.startswith("s_nop"):
            slot += int(ins.split()[1]) + 1
            continue
        ops = _operands(ins)
        for o in ops:          # every operand is read (the first is the accumulator)
            if o in written and slot - written[o] < 2:
                bad.append(f"{ins!r} reads %{o} {slot - written[o]} wait states after its write")
        slot += 1
        written[ops[0]] = slot
    return bad


def test_every_fused_dpp_block_keeps_two_wait_states():
    blocks = _blocks()
    assert len(blocks) >= 8
    for b in blocks:
        assert _violations(b) == [], b


def test_checker_flags_back_to_back_accumulation():
    # the pattern that broke the solver: two updates of one accumulator in a row
    b = ["s_nop 1", "v_fmac_f64_dpp %0, -%2, %4 row_newbcast:%c6", "v_fmac_f64_dpp %0, -%3, %5 row_newbcast:%c6"]
    assert _violations(b)
    assert _violations(["v_fmac_f64_dpp %0, %1, %2 row_newbcast:%c3"])
    ok = ["s_nop 1", "v_fmac_f64_dpp %0, -%2, %4 row_newbcast:%c6", "v_fmac_f64_dpp %1, -%2, %5 row_newbcast:%c6",
          "s_nop 0", "v_fmac_f64_dpp %0, -%3, %5 row_newbcast:%c6"]
    assert _violations(ok) == []
