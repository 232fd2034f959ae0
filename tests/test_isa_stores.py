"""Generated device code of the row passes: wide buffer stores keep their data registers safe.

A store of more than 64 bits reads its data registers after it issues.  The compiler keeps a
VALU write of those registers one wait state behind the store only when the store's scalar
offset is not a register, so the buffer-store helper always passes a constant zero there.
This test compiles the row-pass source to gfx950 assembly with the library's flags and checks
both that invariant and its consequence: no 96/128-bit store is followed directly by an
instruction that writes one of its data registers.
"""
import os
import re
import subprocess

import pytest

from paper_1403_7394_amd import build

STORE = re.compile(r"^\s*(buffer|global|flat)_store_dwordx[34]\s+(.*)$")
REGS = re.compile(r"^v\[(\d+):(\d+)\]$")


def _data_regs(kind, ops):
    data = ops[1] if kind in ("global", "flat") else ops[0]
    m = REGS.match(data)
    return (int(m.group(1)), int(m.group(2))) if m else None


def _writes(line, lo, hi):
    m = re.match(r"^\s*v_\w+\s+(v(\d+)|v\[(\d+):(\d+)\])", line)
    if not m:
        return False
    a, b = (int(m.group(2)), int(m.group(2))) if m.group(2) else (int(m.group(3)), int(m.group(4)))
    return not (b < lo or a > hi)


def test_wide_buffer_stores_in_generated_code(tmp_path):
    try:
        cc = build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    out = tmp_path / "sweep.s"
    flags = [f for f in build.flags() if f not in ("-shared", "-fPIC")]
    cmd = [cc, *flags, "-S", "--cuda-device-only", os.path.join(build.CSRC, "sweep.hip"), "-o", str(out)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-2000:]
    lines = out.read_text().splitlines()
    buffer_stores, bad_offset, hazards = 0, [], []
    for k, line in enumerate(lines):
        m = STORE.match(line)
        if not m:
            continue
        kind = m.group(1)
        ops = [o.strip() for o in m.group(2).split(",")]
        if kind == "buffer":
            buffer_stores += 1
            soffset = ops[3].split()[0]
            if not re.fullmatch(r"-?\d+", soffset):
                bad_offset.append(line.strip())
        regs = _data_regs(kind, ops)
        if regs is None:
            continue
        j = k + 1
        while j < len(lines) and (not lines[j].strip() or lines[j].strip().startswith(";")
                                  or lines[j].strip().endswith(":")):
            j += 1
        if j < len(lines) and _writes(lines[j], *regs):
            hazards.append((line.strip(), lines[j].strip()))
    assert buffer_stores > 0
    assert bad_offset == []
    assert hazards == []
