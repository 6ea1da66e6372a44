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

"Objects" cartridges also set NUSIZ modes and missile sizes, a ball size, turn
both missiles and the ball on and strobe their positions once, give them
motion (moved by every frame's HMOVE), let the visible stores also reach
ENAM0/ENAM1/ENABL, and read the collision latches in the first overscan line:
a frame in which the players met scores a point, a missile-1 hit on player 0
changes the ball's motion, then CXCLR.

"Divergent" cartridges also step the LFSR every visible line, branch on it with
a per-branch taken probability p ~ U(0.1, 0.9), XOR it with SWCHA on the input
line and add a random score event.  Bank-switched cartridges (F8, F6, F4: 2,
4 or 8 banks of 4 KB) carry the same skeleton at identical offsets in every
bank; the bodies differ in operands, and hotspot reads on branch paths swap
to another bank.  Superchip forms (F8SC, F6SC, F4SC) start their code at
$1100, read some body operands from the extra RAM ($1080+) and store some
results into it ($1000+).  E0 and 3F cartridges keep the skeleton in the
fixed segment and run each visible band as a position-independent routine in
a switched slice: the frame loop selects the band's slice (an E0 hotspot
read, or a write of the slice number to $3F) and calls it; 3F cartridges
write the TIA through its $40-$7F mirror, as the write to $00-$3F switches
slices.

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
OBJECT_STORE_REGS = STORE_REGS + ["ENAM0", "ENAM1", "ENABL"]
HITS = 0xD6               # objects cartridges: frames in which the players met
OPS = ["adc", "eor", "and", "lda"]

# worst-case cycles of the instructions this generator emits (zp ops, stores,
# immediates, implied) -- used only to assert the per-line budget.
_C = dict(zp=3, st=3, imm=2, imp=2, abs=4, br=4, inc_zp=5, jmp=3)
LINE_BUDGET = 73          # STA WSYNC must start by cycle 73 of its line


# cartridge kinds -> (scheme number of the library and oracle, 4 KB banks)
KINDS = {"4k": (0, 1), "f8": (1, 2), "f6": (2, 4), "f4": (3, 8), "f8sc": (4, 2), "f6sc": (5, 4), "f4sc": (6, 8),
         "e0": (7, 2), "3f": (8, 2)}
HOTSPOT0 = {2: 0xFF8, 4: 0xFF6, 8: 0xFF4}


@dataclasses.dataclass
class RomSpec:
    seed: int
    kind: str = "4k"            # a key of KINDS
    divergent: bool = False
    n_bands: int | None = None  # visible bands (192 lines split evenly)
    objects: bool = False       # missiles, ball, NUSIZ, object motion, collision reads


@dataclasses.dataclass
class Rom:
    spec: RomSpec
    data: bytes
    scheme: int                 # KINDS[kind][0]
    manifest: dict


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


class _Body:
    """One visible-line body: a list of statements and its worst-case cycles."""

    def __init__(self):
        self.lines: list[str] = []
        self.cycles = 0


def _gen_shape(rng, divergent: bool, f8: bool, sc: bool = False, routine: bool = False):
    """Item kinds of a band body.  The shape is shared by all banks so that
    every instruction sits at the same offset in each; operands differ.
    `routine`: the body runs as a called routine, whose first line also pays
    for the call, so divergent bodies are shorter."""
    if divergent:
        n_ops = int(rng.integers(2, 4 if routine else 5))
        n_st = 3 if routine else 5
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
    if sc:      # Superchip RAM: some operand reads ("xr") and the store back ("xw")
        items = [("xr" if it == "op" and i > 0 and rng.random() < 0.3 else it) for i, it in enumerate(items)]
        items = [("xw" if it == "sb" else it) for it in items]
    shape = dict(items=items)
    if divergent:
        shape["thr"] = int(np.floor(rng.uniform(0.1, 0.9) * 256))
        shape["path_a"] = int(rng.integers(1, 3))
        shape["path_b"] = int(rng.integers(1, 3))
        shape["swap"] = f8 and bool(rng.integers(0, 2))
        shape["where"] = int(rng.integers(0, len(items) + 1))
    return shape


def _fill_body(rng, shape, label: str, bank: int, n_banks: int = 2, tia_off: int = 0,
               store_regs=STORE_REGS) -> _Body:
    b = _Body()
    st_regs = list(store_regs)
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
                b.lines.append(f"    sta {st_regs.pop()}+{tia_off}")
                b.cycles += _C["st"]
            elif it == "sb":
                a = int(rng.integers(RAM_DST_LO, RAM_DST_HI + 1))
                b.lines.append(f"    sta ${a:02X}")
                b.cycles += _C["st"]
            elif it == "xr":
                op = OPS[int(rng.integers(0, 4))]
                b.lines.append(f"    {op} ${0x1080 + int(rng.integers(0, 128)):04X}")
                b.cycles += _C["abs"]
            elif it == "xw":
                b.lines.append(f"    sta ${0x1000 + int(rng.integers(0, 128)):04X}")
                b.cycles += _C["abs"]

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
        # the same offset in every bank: a hotspot read selects another bank
        tgt = 1 - bank if n_banks == 2 else (bank + 1 + int(rng.integers(0, n_banks - 1))) % n_banks
        b.lines.append(f"    lda ${0x1000 | (HOTSPOT0[n_banks] + tgt):04X}")
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
    scheme, banks = KINDS[spec.kind]
    segmented = spec.kind in ("e0", "3f")
    sc = spec.kind.endswith("sc")
    banked = banks > 1 and not segmented      # hotspot swaps inside the bodies
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
    shapes = [_gen_shape(rng, spec.divergent, banked, sc, segmented) for _ in range(n_bands)]
    body_seeds = [int(x) for x in rng.integers(0, 2**31, (1 if segmented else banks, n_bands)).ravel()]
    lines_per_band = _band_split(n_bands)
    tia = 0x40 if spec.kind == "3f" else 0            # 3F: TIA writes through the $40 mirror
    org = 0x1100 if sc else (0x1C00 if spec.kind == "e0" else 0x1800 if spec.kind == "3f" else 0x1000)

    def T_(name):
        return f"{name}+{tia}"

    def skeleton(visible: list[str]) -> list[str]:
        s: list[str] = [f"    .org ${org:04X}", "reset:"]
        s += ["    sei", "    cld", "    ldx #$FF", "    txs", "    lda #0", "    ldx #$7F",
              "clr:", "    sta $80,x", "    dex", "    bpl clr"]
        s += [f"    lda #${colup0:02X}", f"    sta {T_('COLUP0')}", f"    lda #${colup1:02X}", f"    sta {T_('COLUP1')}",
              f"    lda #${ctrlpf:02X}", f"    sta {T_('CTRLPF')}", f"    lda #${hmp1:02X}", f"    sta {T_('HMP1')}",
              f"    lda #${lfsr0:02X}", f"    sta ${LFSR:02X}"]
        for a, v in seeds:
            s += [f"    lda #${v:02X}", f"    sta ${a:02X}"]
        for i, d in enumerate(resp_delay):
            s += [f"    sta {T_('WSYNC')}"] + ["    nop"] * d + [f"    sta {T_(f'RESP{i}')}"]
        if spec.objects:
            s += objects_init()
        s += [f"    sta {T_('WSYNC')}", "    jmp frame"]
        # ---- frame loop ----
        s += ["frame:", "    lda #2", f"    sta {T_('VSYNC')}", f"    sta {T_('WSYNC')}", f"    sta {T_('WSYNC')}",
              f"    sta {T_('WSYNC')}", "    lda #0", f"    sta {T_('VSYNC')}", "    lda #2", f"    sta {T_('VBLANK')}"]
        # input line (VBLANK line 0)
        cyc = 2 + 3 + 2 + 3
        s += ["    ldy #0", "    lda SWCHA", "    bmi in_nr", f"    inc ${PPOS:02X}", "    ldy #$F0",
              "in_nr:", "    asl", "    bmi in_nl", f"    dec ${PPOS:02X}", "    ldy #$10", "in_nl:",
              f"    sty {T_('HMP0')}", "    lda INPT4", "    bmi in_nf", "    sed", "    clc",
              f"    lda ${SCORE:02X}", "    adc #1", f"    sta ${SCORE:02X}", "    cld", "in_nf:"]
        cyc += 2 + 4 + 3 + 5 + 2 + 2 + 3 + 5 + 2 + 3 + 3 + 3 + 2 + 2 + 3 + 2 + 3 + 2
        if spec.divergent:
            s += [f"    lda ${LFSR:02X}", "    eor SWCHA", f"    sta ${LFSR:02X}"]
            cyc += 3 + 4 + 3
        s += [f"    sta {T_('WSYNC')}"]
        assert cyc <= LINE_BUDGET, cyc
        # frame counter / terminal line
        s += [f"    inc ${CNT_LO:02X}", "    bne cn_nc", f"    inc ${CNT_HI:02X}", "cn_nc:",
              f"    lda ${CNT_HI:02X}", f"    cmp #${T >> 8:02X}", "    bcc cn_no", "    bne cn_t",
              f"    lda ${CNT_LO:02X}", f"    cmp #${T & 0xFF:02X}", "    bcc cn_no",
              "cn_t:", "    lda #1", f"    sta ${TERM:02X}", "cn_no:", f"    sta {T_('WSYNC')}"]
        # HMOVE line (+ random score event on divergent cartridges)
        s += [f"    sta {T_('HMOVE')}"]
        if spec.divergent:
            s += [f"    lda ${LFSR:02X}", f"    cmp #${score_thr:02X}", "    bcs sc_no", "    sed", "    clc",
                  f"    lda ${SCORE:02X}", "    adc #1", f"    sta ${SCORE:02X}", "    cld", "sc_no:"]
        s += [f"    sta {T_('WSYNC')}", "    ldx #34", "vbl:", f"    sta {T_('WSYNC')}", "    dex", "    bne vbl",
              "    lda #0", f"    sta {T_('VBLANK')}"]
        s += visible
        # overscan
        s += ["    lda #2", f"    sta {T_('VBLANK')}"]
        if spec.objects:
            s += objects_overscan()
        s += ["    ldx #30", "ovs:", f"    sta {T_('WSYNC')}", "    dex",
              "    bne ovs", "    jmp frame"]
        s += ["    .org $1FFA", "    .word reset, reset, reset"]
        return s

    # objects cartridges: drawn from a generator of their own, so the other
    # kinds stay byte-identical
    orng = _rng(spec.seed + 0x0B1EC7)
    o_nusiz = [int(x) for x in orng.integers(0, 8, 2) | (orng.integers(0, 4, 2) << 4)]
    o_ball = int(orng.integers(0, 4)) << 4
    o_delay = [int(x) for x in orng.integers(10, 34, 3)]
    o_hm = [int(x) << 4 for x in orng.integers(0, 16, 3)]

    def objects_init() -> list[str]:
        """NUSIZ modes and missile sizes, ball size, missiles and ball on,
        their positions strobed on lines of their own, their motion."""
        s = [f"    lda #${o_nusiz[0]:02X}", f"    sta {T_('NUSIZ0')}", f"    lda #${o_nusiz[1]:02X}",
             f"    sta {T_('NUSIZ1')}", f"    lda #${(ctrlpf | o_ball):02X}", f"    sta {T_('CTRLPF')}",
             "    lda #2", f"    sta {T_('ENAM0')}", f"    sta {T_('ENAM1')}", f"    sta {T_('ENABL')}"]
        for reg, d in zip(("RESM0", "RESM1", "RESBL"), o_delay):
            s += [f"    sta {T_('WSYNC')}"] + ["    nop"] * d + [f"    sta {T_(reg)}"]
        for reg, v in zip(("HMM0", "HMM1", "HMBL"), o_hm):
            s += [f"    lda #${v:02X}", f"    sta {T_(reg)}"]
        return s

    def objects_overscan() -> list[str]:
        """First overscan line: a frame in which the players met scores a
        point (BCD) and counts at $D6; a missile hit on player 0 moves the
        ball's motion; then CXCLR."""
        s = ["    lda CXPPMM", "    bpl cx_np", "    sed", "    clc", f"    lda ${SCORE:02X}", "    adc #1",
             f"    sta ${SCORE:02X}", "    cld", f"    inc ${HITS:02X}", "cx_np:", "    lda CXM1P", "    bpl cx_nm",
             f"    lda ${HITS:02X}", f"    sta {T_('HMBL')}", "cx_nm:", f"    sta {T_('CXCLR')}"]
        # lda 2, sta 3, then 3+2+2+2+3+2+3+2+5 + 3+2+3+3 + 3, ldx 2, sta WSYNC 3
        assert 2 + 3 + 32 + 11 + 3 + 2 + 3 <= LINE_BUDGET + 3
        return s

    def band_lines(bank: int, k: int, prefix: int) -> list[str]:
        brng = _rng(body_seeds[bank * n_bands + k])
        body = _fill_body(brng, shapes[k], f"b{k}", bank, banks, tia,
                          OBJECT_STORE_REGS if spec.objects else STORE_REGS)
        assert prefix + body.cycles <= LINE_BUDGET, (k, prefix + body.cycles)
        return [f"band{k}:"] + body.lines + [f"    sta {T_('WSYNC')}", "    dex", f"    bne band{k}"]

    if not segmented:
        srcs = []
        for bank in range(banks):
            vis = []
            for k in range(n_bands):
                prefix = 2 + 2 + 2 + 3 + 2 if k == 0 else 2 + 3 + 2 + 2
                vis += [f"    ldx #{lines_per_band[k]}"] + band_lines(bank, k, prefix)
            srcs.append("\n".join(skeleton(vis)))
        # labels repeat across banks: assemble each bank on its own
        images, syms = [], []
        for b in range(banks):
            img, sy = assemble_with_symbols(srcs[b], banks=1)
            images.append(img)
            syms.append(sy)
        # the skeleton must sit at identical offsets in every bank
        for b in range(1, banks):
            for lab in ["reset", "frame", "vbl", "ovs"] + [f"band{k}" for k in range(n_bands)]:
                assert syms[0][lab] == syms[b][lab], lab
        data = b"".join(images)
        frame_label = syms[0]["frame"]
    else:
        # bands as routines in switched slices: E0 slices 0-6 into segments 0-2,
        # 3F slices 0-2 into the lower 2 KB; routine k at offset 256 (k // n_sl)
        e0 = spec.kind == "e0"
        n_sl = 7 if e0 else 3
        vis, routines = [], []
        for k in range(n_bands):
            sl, off = k % n_sl, 0x100 * (k // n_sl)
            seg = k % 3 if e0 else 0
            entry = 0x1000 + 0x400 * seg + off
            if e0:
                select = [f"    lda ${0x1FE0 + 8 * seg + sl:04X}"]      # 4 cycles
                sel_c = 4
            else:
                select = [f"    lda #{sl}", "    sta $3F"]               # 5 cycles
                sel_c = 5
            vis += select + [f"    ldx #{lines_per_band[k]}", f"    jsr ${entry:04X}"]
            # first line: the previous routine's dex/bne/rts (or the VBLANK end), select, ldx, jsr
            prefix = (2 + 3 if k == 0 else 2 + 2 + 6) + sel_c + 2 + 6
            lines = band_lines(0, k, prefix) + ["    rts", "r_end:"]
            img, rs = assemble_with_symbols(f"    .org ${entry:04X}\n" + "\n".join(lines))
            size = rs["r_end"] - entry
            assert size <= 0x100, size
            routines.append((sl, off, img[entry - 0x1000: entry - 0x1000 + size]))
        fixed, syms0 = assemble_with_symbols("\n".join(skeleton(vis)), banks=1)
        sl_bytes = 1024 if e0 else 2048
        n_total = 8 if e0 else 4
        fill = _rng(spec.seed + 1)
        slices = [bytearray(fill.integers(0, 256, sl_bytes).astype(np.uint8).tobytes()) for _ in range(n_total - 1)]
        for sl, off, code in routines:
            slices[sl][off: off + len(code)] = code
        fixed_part = fixed[4096 - sl_bytes:] if e0 else fixed[2048:]
        data = b"".join(bytes(x) for x in slices) + fixed_part
        frame_label = syms0["frame"]
    manifest = dict(seed=spec.seed, kind=spec.kind, divergent=spec.divergent, objects=spec.objects, n_bands=n_bands,
                    T=T, ctrlpf=ctrlpf, lfsr0=lfsr0, resp_delay=resp_delay,
                    thresholds=[sh.get("thr") for sh in shapes], frame_label=frame_label)
    return Rom(spec=spec, data=data, scheme=scheme, manifest=manifest)


def manifest_json(rom: Rom) -> str:
    return json.dumps(rom.manifest, sort_keys=True)
