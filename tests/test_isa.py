"""Machine code of the built library (gfx950 code objects inside libtl.so).

A vector-memory store of more than 64 bits reads its data registers after it
has issued, so an ALU instruction that rewrites them must come at least two
wait states later.  The compiler inserts that gap for stores whose scalar
offset operand is not a register, but not for buffer stores with the offset in
a scalar register; measured on gfx950, such a store followed at once by a
rewrite of its data stored the new value now and then.  The library's 16-byte
stores therefore carry the component offset in the vector offset and a zero
scalar offset, and this test checks the disassembly of every kernel for a
rewrite that comes too early.  It also checks the other hazard a buffer access
can meet: a scalar register written by a vector instruction must not be read
by a memory instruction within five wait states.
"""
import os
import re
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1804_10120_amd", "libtl.so")
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"
WAIT_STATES = 2
BUNDLE = b"__CLANG_OFFLOAD_BUNDLE__"


def code_objects(path):
    """The gfx950 code objects of the offload bundles embedded in a HIP library."""
    data = open(path, "rb").read()
    out, i = [], 0
    while (i := data.find(BUNDLE, i)) >= 0:
        count = struct.unpack_from("<Q", data, i + len(BUNDLE))[0]
        pos = i + len(BUNDLE) + 8
        for _ in range(count):
            off, size, tlen = struct.unpack_from("<QQQ", data, pos)
            pos += 24
            triple = data[pos:pos + tlen].decode()
            pos += tlen
            if "gfx950" in triple and size > 0:
                out.append(data[i + off:i + off + size])
        i += 1
    return out


def vgprs(tok):
    m = re.fullmatch(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.fullmatch(r"v(\d+)", tok)
    return {int(m.group(1))} if m else set()


WIDE_STORE = re.compile(r"(buffer|global|flat|scratch)_store_dword(x3|x4)\b")


def early_rewrites(lines):
    """(function, store, rewrite) for every ALU write of a wide store's data
    registers fewer than WAIT_STATES wait states after the store."""
    bad = []
    ins = _instructions(lines)
    for j, (func, text) in enumerate(ins):
        m = WIDE_STORE.match(text)
        if not m:
            continue
        ops = [o.strip() for o in text.split(None, 1)[1].split(",")]
        data = vgprs(ops[0] if m.group(1) in ("buffer", "scratch") else ops[1])
        waited = 0
        for f2, nxt in ins[j + 1:]:
            if waited >= WAIT_STATES or f2 != func:
                break
            mnem, _, rest = nxt.partition(" ")
            if mnem.startswith("v_") and rest and vgprs(rest.split(",")[0].strip()) & data:
                bad.append((func, text, nxt))
                break
            waited += int(rest.strip()) + 1 if mnem == "s_nop" else 1
    return bad


def _instructions(lines):
    func, ins = None, []
    for line in lines:
        m = re.match(r"^[0-9a-f]+ <(\S+)>:", line)
        if m:
            func = m.group(1)
            continue
        text = line.split("//")[0].strip()
        if text and not text.endswith(":"):
            ins.append((func, text))
    return ins


def sgprs(tok):
    m = re.fullmatch(r"s\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.fullmatch(r"s(\d+)", tok)
    return {int(m.group(1))} if m else set()


SGPR_WAIT_STATES = 5


def early_sgpr_reads(lines):
    """(function, writer, memory instruction) for every buffer instruction that
    reads a scalar register a vector instruction wrote fewer than
    SGPR_WAIT_STATES wait states before."""
    bad = []
    ins = _instructions(lines)
    for j, (func, text) in enumerate(ins):
        if not text.startswith("buffer_"):
            continue
        ops = [o.strip().split()[0] for o in text.split(None, 1)[1].split(",") if o.strip()]
        read = set().union(*(sgprs(o) for o in ops))
        waited = 0
        for k in range(j - 1, -1, -1):
            f2, prev = ins[k]
            if waited >= SGPR_WAIT_STATES or f2 != func:
                break
            mnem, _, rest = prev.partition(" ")
            if mnem.startswith("v_") and rest and sgprs(rest.split(",")[0].strip()) & read:
                bad.append((func, prev, text))
                break
            waited += int(rest.strip()) + 1 if mnem == "s_nop" else 1
    return bad


def test_scan_finds_an_early_rewrite():
    lines = ["0000000000001000 <k>:",
             "\tbuffer_store_dwordx4 v[4:7], v1, s[0:3], s8 offen nt // 1000: 0",
             "\tv_mov_b32_e32 v5, 0 // 1008: 0",
             "\tbuffer_store_dwordx4 v[4:7], v1, s[0:3], s9 offen nt // 1010: 0",
             "\ts_nop 1 // 1018: 0",
             "\tv_mov_b32_e32 v5, 0 // 101c: 0",
             "\tglobal_store_dwordx4 v[8:9], v[4:7], off // 1020: 0",
             "\ts_nop 0 // 1028: 0",
             "\tv_cndmask_b32_e32 v6, v1, v2, vcc // 102c: 0"]
    bad = early_rewrites(lines)
    assert [b[2] for b in bad] == ["v_mov_b32_e32 v5, 0", "v_cndmask_b32_e32 v6, v1, v2, vcc"]


def test_scan_finds_an_early_sgpr_read():
    lines = ["0000000000001000 <k>:",
             "\tv_readlane_b32 s4, v9, 3 // 1000: 0",
             "\tbuffer_store_dwordx4 v[4:7], v1, s[0:3], s4 offen nt // 1008: 0",
             "\tv_readlane_b32 s5, v9, 4 // 1010: 0",
             "\ts_nop 4 // 1018: 0",
             "\tbuffer_store_dwordx4 v[4:7], v1, s[0:3], s5 offen nt // 1020: 0",
             "\tv_readfirstlane_b32 s2, v3 // 1028: 0",
             "\ts_nop 2 // 1030: 0",
             "\tbuffer_load_dwordx2 v[4:5], v1, s[0:3], 0 offen // 1038: 0"]
    bad = early_sgpr_reads(lines)
    assert [b[1] for b in bad] == ["v_readlane_b32 s4, v9, 3", "v_readfirstlane_b32 s2, v3"]


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtl.so is not built")
@pytest.mark.skipif(not os.path.exists(OBJDUMP), reason="llvm-objdump is not installed")
def test_memory_hazards_are_padded(tmp_path):
    objs = code_objects(LIB)
    assert objs, "no gfx950 code object in libtl.so"
    stores, bad, sbad = 0, [], []
    for k, co in enumerate(objs):
        path = tmp_path / f"co{k}.elf"
        path.write_bytes(co)
        asm = subprocess.run([OBJDUMP, "-d", "--mcpu=gfx950", str(path)], check=True,
                             capture_output=True, text=True).stdout.splitlines()
        stores += sum(1 for line in asm if WIDE_STORE.search(line))
        bad += early_rewrites(asm)
        sbad += early_sgpr_reads(asm)
    assert stores > 0
    assert not bad, f"{len(bad)} early rewrites, e.g. {bad[:3]}"
    assert not sbad, f"{len(sbad)} early scalar reads, e.g. {sbad[:3]}"
