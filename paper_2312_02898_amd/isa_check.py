"""Checks of the gfx950 assembly the build produces (build tooling).

The device compiler of this toolchain can spill a 64-bit value held in a
register pair by writing only one 32-bit half to a 4-byte scratch slot
(the other half moved to a register that is never read), and later reload
only that half before using the pair as a 64-bit operand: the other half of
the operand is then whatever the register held before, and the kernel
computes wrong values without any fault.  It was found in a part kernel of
g g > t t~ g g g whose C++ is exact on the host; the same source compiled
with scratch-only spills is exact.

`half_reloads` finds that signature: a 4-byte reload into register r_N
that is not accompanied by a restore of its mate in the even-aligned pair
(r_{N xor 1}: no write to it among the few instructions before the reload,
where the compiler puts the restore of a pair saved half to scratch and half
to a spare register), followed, before the mate is written, by a read of a
register range that holds both.  Straight-line
scan per function (branches are not followed), so it can report a case that
control flow rules out; the build treats every report as an error.
"""
from __future__ import annotations

import re

_RELOAD = re.compile(r"^\s*scratch_load_dword ([va])(\d+),")
_RANGE = re.compile(r"([va])\[(\d+):(\d+)\]")
_SINGLE = re.compile(r"\b([va])(\d+)\b")
# instructions whose first operand is read, not written
_NO_DEST = ("scratch_store", "global_store", "buffer_store", "flat_store", "ds_write", "ds_store",
            "s_", "exp ", "v_cmp", "v_cmpx")


def _operands(line: str):
    code = line.split(";", 1)[0].strip()
    if not code or code.endswith(":") or code.startswith("."):
        return None, [], []
    parts = code.split(None, 1)
    op = parts[0]
    ops = [x.strip() for x in parts[1].split(",")] if len(parts) > 1 else []
    if op.startswith(_NO_DEST) or not ops:
        return op, [], ops
    return op, ops[:1], ops[1:]


def _regs(tokens):
    out = []
    for t in tokens:
        for m in _RANGE.finditer(t):
            out.append((m[1], int(m[2]), int(m[3])))
        t2 = _RANGE.sub("", t)
        for m in _SINGLE.finditer(t2):
            out.append((m[1], int(m[2]), int(m[2])))
    return out


def _mate_restored_before(lines, i, kind, mate, window=8):
    """True if one of the `window` instructions before line i writes the mate
    register: the compiler restores a pair whose halves were saved in two
    places (scratch and a spare register) with adjacent instructions."""
    seen = 0
    for j in range(i - 1, -1, -1):
        op, dst, _ = _operands(lines[j])
        if op is None:
            if re.match(r"^[A-Za-z_.][\w.$]*:", lines[j]):
                break   # block boundary
            continue
        if any(r[0] == kind and r[1] <= mate <= r[2] for r in _regs(dst)):
            return True
        seen += 1
        if seen >= window:
            break
    return False


def half_reloads(asm: str) -> list[str]:
    """Reports (function, line number, text) of every half reload."""
    lines = asm.split("\n")
    found = []
    func = "?"
    for i, line in enumerate(lines):
        if re.match(r"^[A-Za-z_][\w.$]*:", line) and not line.startswith(".L"):
            func = line.split(":", 1)[0]
        m = _RELOAD.match(line)
        if not m:
            continue
        kind, n = m[1], int(m[2])
        mate = n ^ 1   # 64-bit register tuples are even-aligned
        if _mate_restored_before(lines, i, kind, mate):
            continue   # a pair spilled half to scratch, half to a register, and restored whole
        for j in range(i + 1, len(lines)):
            l2 = lines[j]
            if re.match(r"^[A-Za-z_][\w.$]*:", l2) and not l2.startswith(".L"):
                break   # next function
            op, dst, src = _operands(l2)
            if op is None:
                continue
            bad = [r for r in _regs(src) if r[0] == kind and r[1] <= n <= r[2] and r[1] <= mate <= r[2]]
            if bad:
                found.append(f"{func}: line {i + 1} `{line.strip()}` then line {j + 1} `{l2.strip()}`")
                break
            w = [r for r in _regs(dst) if r[0] == kind]
            if any(r[1] <= n <= r[2] for r in w):
                break   # r_N overwritten: the reloaded half is dead
            if any(r[1] <= mate <= r[2] for r in w):
                break   # the other half written first: the pair is defined
    return found
