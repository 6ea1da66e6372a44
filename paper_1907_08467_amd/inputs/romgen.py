"""Seeded synthetic Atari 2600 cartridges that stand in for the game suite.

The paper measures on the Atari game ROMs of its evaluation suite (Section 4,
"Experiments"); those cartridges are not available here, so every workload is
a cartridge produced by this generator from a seed.  The cartridges keep the
shape of a real game's frame loop:

* reset vector -> init code that clears RAM $80-$FF, seeds a few bytes, sets
  player colours, strobes RESP0/RESP1 once and seeds an LFSR byte at $D2;
* per frame: 3 VSYNC lines, 37 VBLANK lines, 192 visible lines, 30 overscan
  lines, every line ending in ``STA WSYNC`` (262 lines, 19,912 CPU cycles);
* one VBLANK line reads SWCHA/INPT4: right/left move the player-position byte
  $D3 and set HMP0, fire adds 1 to the BCD score at $D0 (decimal mode);
* one VBLANK line counts frames in $D4/$D5 and sets the terminal flag $D1 once
  the count reaches a seeded T in [500, 3000];
* one VBLANK line strobes HMOVE;
* the visible lines run bands of a generated body: 3-8 LDA/ADC/EOR/AND on RAM
  bytes interleaved with stores to COLUBK/COLUPF/PF0-2/GRP0/GRP1 and an
  optional store back to RAM.

"Divergent" cartridges also step the LFSR every visible line, branch on it with
a per-branch taken probability p ~ U(0.1, 0.9), XOR it with SWCHA on the input
line and add a random score event.  F8 cartridges (8 KB, two 4 KB banks)
carry the same skeleton at identical offsets in both banks; the bodies differ
in operands, and ``LDA $1FF8``/``LDA $1FF9`` on branch paths swap banks.

This module is input tooling only: it contains no emulator arithmetic.
"""

from __future__ import annotations

import dataclasses
import json

import numpy as np

from .asm6502 import assemble_with_symbols

SCORE, TERM, LFSR, PPOS, CNT_LO, CNT_HI = 0xD0, 0xD1, 0xD2, 0xD3, 0xD4, 0xD5
RAM_SRC_LO, RAM_SRC_HI = 0x80, 0xD5     # bytes the visible ops may read
RAM_DST_LO, RAM_DST_HI = 0x80, 0xCF     # bytes the visible ops may write
STORE_REGS = ["COLUBK", "COLUPF", "PF0", "PF1", "PF2", "GRP0", "GRP1"]
OPS = ["adc", "eor", "and", "lda"]

# worst-case cycles of the instructions this generator emits (zp ops, stores,
# immediates, implied) -- used only to assert the per-line budget.
_C = dict(zp=3, st=3, imm=2, imp=2, abs=4, br=4, inc_zp=5, jmp=3)
LINE_BUDGET = 73          # STA WSYNC must start by cycle 73 of its line


@dataclasses.dataclass
class RomSpec:
    seed: int
    kind: str = "4k"            # "4k" or "f8"
    divergent: bool = False
    n_bands: int | None = None  # visible bands (192 lines split evenly)


@dataclasses.dataclass
class Rom:
    spec: RomSpec
    data: bytes
    scheme: int                 # 0 = 4 KB flat, 1 = F8
    manifest: dict


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


class _Body:
    """One visible-line body: a list of statements and its worst-case cycles."""

    def __init__(self):
        self.lines: list[str] = []
        self.cycles = 0


def _gen_shape(rng, divergent: bool, f8: bool):
    """Item kinds of a band body.  The shape is shared by both F8 banks so that
    every instruction sits at the same offset in both; operands differ."""
    if divergent:
        n_ops = int(rng.integers(2, 5))
        n_st = 5
    else:
        n_ops = int(rng.integers(3, 9))
        n_st = 7
    store_back = bool(rng.integers(0, 2))
    items = ["op"] * (n_ops - 1) + ["st"] * n_st
    rng.shuffle(items)
    items = ["op"] + items
    if store_back:
        pos = int(rng.integers(1, len(items) + 1))
        items.insert(pos, "sb")
    shape = dict(items=items)
    if divergent:
        shape["thr"] = int(np.floor(rng.uniform(0.1, 0.9) * 256))
        shape["path_a"] = int(rng.integers(1, 3))
        shape["path_b"] = int(rng.integers(1, 3))
        shape["swap"] = f8 and bool(rng.integers(0, 2))
        shape["where"] = int(rng.integers(0, len(items) + 1))
    return shape


def _fill_body(rng, shape, label: str, bank: int) -> _Body:
    b = _Body()
    st_regs = list(STORE_REGS)
    rng.shuffle(st_regs)
    n_st = sum(1 for it in shape["items"] if it == "st")
    st_regs = st_regs[:n_st]

    def op_line(first=False):
        op = "lda" if first else OPS[int(rng.integers(0, 4))]
        a = int(rng.integers(RAM_SRC_LO, RAM_SRC_HI + 1))
        b.cycles += _C["zp"]
        return f"    {op} ${a:02X}"

    def emit_items(items, start_first):
        first = start_first
        for it in items:
            if it == "op":
                b.lines.append(op_line(first))
                first = False
            elif it == "st":
                b.lines.append(f"    sta {st_regs.pop()}")
                b.cycles += _C["st"]
            elif it == "sb":
                a = int(rng.integers(RAM_DST_LO, RAM_DST_HI + 1))
                b.lines.append(f"    sta ${a:02X}")
                b.cycles += _C["st"]

    items = shape["items"]
    if "thr" not in shape:
        emit_items(items, True)
        return b
    # divergent: LFSR step, a branch on it, two paths of different length
    w = shape["where"]
    emit_items(items[:w], True)
    b.lines += [f"    lda ${LFSR:02X}", "    lsr", f"    bcc {label}_nf",
                "    eor #$B8", f"{label}_nf:", f"    sta ${LFSR:02X}",
                f"    cmp #${shape['thr']:02X}", f"    bcc {label}_b"]
    # lda 3, lsr 2, max(bcc taken across a page 4, not taken 2 + eor 2), sta 3, cmp 2, bcc 4
    b.cycles += 3 + 2 + 4 + 3 + 2 + 4
    ca = 0
    for _ in range(shape["path_a"]):
        b.lines.append(op_line())
        ca += 3
    b.lines.append(f"    jmp {label}_j")
    ca += 3
    b.lines.append(f"{label}_b:")
    cb = 0
    for _ in range(shape["path_b"]):
        b.lines.append(op_line())
        cb += 3
    if shape["swap"]:
        # the same offset in both banks: bank 0 selects bank 1 and vice versa
        b.lines.append("    lda $1FF9" if bank == 0 else "    lda $1FF8")
        cb += 4
    b.lines.append(f"{label}_j:")
    # op_line already added 3 per op to b.cycles; keep only the longer path
    b.cycles -= 3 * (shape["path_a"] + shape["path_b"])
    b.cycles += max(ca, cb)
    emit_items(items[w:], False)
    return b


def _band_split(n_bands):
    per = 192 // n_bands
    assert per * n_bands == 192
    return [per] * n_bands


def generate(spec: RomSpec) -> Rom:
    rng = _rng(spec.seed)
    f8 = spec.kind == "f8"
    banks = 2 if f8 else 1
    n_bands = spec.n_bands or int(rng.choice([8, 12, 16]))
    T = int(rng.integers(500, 3001))
    colup0, colup1 = (int(x) for x in rng.integers(0, 256, 2))
    ctrlpf = int(rng.integers(0, 8))                  # reflect / score / priority
    hmp1 = int(rng.integers(0, 16)) << 4
    lfsr0 = int(rng.integers(1, 256))
    seeds = [(0x80 + int(i), int(v)) for i, v in zip(rng.choice(0x50, 8, replace=False),
                                                       rng.integers(0, 256, 8))]
    resp_delay = [int(x) for x in rng.integers(10, 34, 2)]
    score_thr = int(rng.integers(8, 48))
    shapes = [_gen_shape(rng, spec.divergent, f8) for _ in range(n_bands)]
    body_seeds = [int(x) for x in rng.integers(0, 2**31, (banks, n_bands)).ravel()]
    lines_per_band = _band_split(n_bands)

    def bank_source(bank: int) -> str:
        s: list[str] = [f"    .bank {bank}", "    .org $1000", "reset:"]
        s += ["    sei", "    cld", "    ldx #$FF", "    txs", "    lda #0", "    ldx #$7F",
              "clr:", "    sta $80,x", "    dex", "    bpl clr"]
        s += [f"    lda #${colup0:02X}", "    sta COLUP0", f"    lda #${colup1:02X}", "    sta COLUP1",
              f"    lda #${ctrlpf:02X}", "    sta CTRLPF", f"    lda #${hmp1:02X}", "    sta HMP1",
              f"    lda #${lfsr0:02X}", f"    sta ${LFSR:02X}"]
        for a, v in seeds:
            s += [f"    lda #${v:02X}", f"    sta ${a:02X}"]
        for i, d in enumerate(resp_delay):
            s += ["    sta WSYNC"] + ["    nop"] * d + [f"    sta RESP{i}"]
        s += ["    sta WSYNC", "    jmp frame"]
        # ---- frame loop ----
        s += ["frame:", "    lda #2", "    sta VSYNC", "    sta WSYNC", "    sta WSYNC", "    sta WSYNC",
              "    lda #0", "    sta VSYNC", "    lda #2", "    sta VBLANK"]
        # input line (VBLANK line 0)
        cyc = 2 + 3 + 2 + 3
        s += ["    ldy #0", "    lda SWCHA", "    bmi in_nr", f"    inc ${PPOS:02X}", "    ldy #$F0",
              "in_nr:", "    asl", "    bmi in_nl", f"    dec ${PPOS:02X}", "    ldy #$10", "in_nl:",
              "    sty HMP0", "    lda INPT4", "    bmi in_nf", "    sed", "    clc",
              f"    lda ${SCORE:02X}", "    adc #1", f"    sta ${SCORE:02X}", "    cld", "in_nf:"]
        cyc += 2 + 4 + 3 + 5 + 2 + 2 + 3 + 5 + 2 + 3 + 3 + 3 + 2 + 2 + 3 + 2 + 3 + 2
        if spec.divergent:
            s += [f"    lda ${LFSR:02X}", "    eor SWCHA", f"    sta ${LFSR:02X}"]
            cyc += 3 + 4 + 3
        s += ["    sta WSYNC"]
        assert cyc <= LINE_BUDGET, cyc
        # frame counter / terminal line
        s += [f"    inc ${CNT_LO:02X}", "    bne cn_nc", f"    inc ${CNT_HI:02X}", "cn_nc:",
              f"    lda ${CNT_HI:02X}", f"    cmp #${T >> 8:02X}", "    bcc cn_no", "    bne cn_t",
              f"    lda ${CNT_LO:02X}", f"    cmp #${T & 0xFF:02X}", "    bcc cn_no",
              "cn_t:", "    lda #1", f"    sta ${TERM:02X}", "cn_no:", "    sta WSYNC"]
        # HMOVE line (+ random score event on divergent cartridges)
        s += ["    sta HMOVE"]
        if spec.divergent:
            s += [f"    lda ${LFSR:02X}", f"    cmp #${score_thr:02X}", "    bcs sc_no", "    sed", "    clc",
                  f"    lda ${SCORE:02X}", "    adc #1", f"    sta ${SCORE:02X}", "    cld", "sc_no:"]
        s += ["    sta WSYNC", "    ldx #34", "vbl:", "    sta WSYNC", "    dex", "    bne vbl",
              "    lda #0", "    sta VBLANK"]
        # visible bands
        for k in range(n_bands):
            brng = _rng(body_seeds[bank * n_bands + k])
            body = _fill_body(brng, shapes[k], f"b{k}", bank)
            prefix = 2 + 2 + 2 + 3 + 2 if k == 0 else 2 + 3 + 2 + 2
            assert prefix + body.cycles <= LINE_BUDGET, (k, prefix + body.cycles)
            s += [f"    ldx #{lines_per_band[k]}", f"band{k}:"] + body.lines
            s += ["    sta WSYNC", "    dex", f"    bne band{k}"]
        # overscan
        s += ["    lda #2", "    sta VBLANK", "    ldx #30", "ovs:", "    sta WSYNC", "    dex",
              "    bne ovs", "    jmp frame"]
        s += ["    .org $1FFA", "    .word reset, reset, reset"]
        return "\n".join(s)

    srcs = [bank_source(b) for b in range(banks)]
    src = "\n".join(srcs)
    # labels repeat across banks: assemble each bank on its own
    images = []
    syms = []
    for b in range(banks):
        img, sy = assemble_with_symbols(srcs[b].replace(f".bank {b}", ".bank 0"), banks=1)
        images.append(img)
        syms.append(sy)
    if f8:
        # the skeleton must sit at identical offsets in both banks
        for lab in ["reset", "frame", "vbl", "ovs"] + [f"band{k}" for k in range(n_bands)]:
            assert syms[0][lab] == syms[1][lab], lab
    data = b"".join(images)
    manifest = dict(seed=spec.seed, kind=spec.kind, divergent=spec.divergent, n_bands=n_bands,
                    T=T, ctrlpf=ctrlpf, lfsr0=lfsr0, resp_delay=resp_delay,
                    thresholds=[sh.get("thr") for sh in shapes], frame_label=syms[0]["frame"])
    return Rom(spec=spec, data=data, scheme=1 if f8 else 0, manifest=manifest)


def manifest_json(rom: Rom) -> str:
    return json.dumps(rom.manifest, sort_keys=True)
