"""Random cartridges for differential testing of the GPU interpreter against
the oracle.  Every documented opcode appears with every addressing mode, on
RAM, TIA, RIOT (ports and timer) and cartridge operands, in decimal and
binary mode, with forward branches, subroutines, BRK/RTI and page crossings;
optionally the stable undocumented opcodes too.  Control flow stays
structured so that frames keep ending (VSYNC) and the cartridge never
executes a JAM or an unstable opcode.

Cartridge schemes: linear ones (4K, F8, F6, F4 and their Superchip forms)
carry the same code in every bank so a switch continues in place, with
different data per bank, and the data accesses hit the hotspots and the
Superchip RAM ports; E0 and 3F keep the code in the fixed segment and read
data from the switched ones, switch them at random, and call a routine that
straddles the last switched segment and the fixed one.
"""
import numpy as np

from paper_1907_08467_amd.inputs.asm6502 import OPCODES, UNDOC_OPCODES, assemble_with_symbols

S_4K, S_F8, S_F6, S_F4, S_F8SC, S_F6SC, S_F4SC, S_E0, S_3F = range(9)
LINEAR_BANKS = {S_4K: 1, S_F8: 2, S_F6: 4, S_F4: 8, S_F8SC: 2, S_F6SC: 4, S_F4SC: 8}
HOTSPOTS = {S_F8: range(0x1FF8, 0x1FFA), S_F6: range(0x1FF6, 0x1FFA), S_F4: range(0x1FF4, 0x1FFC),
            S_F8SC: range(0x1FF8, 0x1FFA), S_F6SC: range(0x1FF6, 0x1FFA), S_F4SC: range(0x1FF4, 0x1FFC),
            S_E0: range(0x1FE0, 0x1FF8)}
UNDOC_RMW = ["slo", "rla", "sre", "rra", "dcp", "isc"]

RAM = [a for a in range(0x80, 0xF8) if a not in (0xD0, 0xD1, 0xD4, 0xD5, 0xE0, 0xE1)]   # $F8-$FF: stack
TIA_W = [0x01, 0x06, 0x07, 0x08, 0x09, 0x0A, 0x0B, 0x0C, 0x0D, 0x0E, 0x0F, 0x10, 0x11, 0x1B, 0x1C,
         0x20, 0x21, 0x2A, 0x2B, 0x04, 0x05, 0x15, 0x19, 0x1D, 0x25, 0x2C,
         0x12, 0x13, 0x14, 0x1E, 0x1F, 0x22, 0x23, 0x24, 0x26, 0x27, 0x28, 0x29, 0x1B, 0x1C, 0x1D, 0x1F]
TIA_W_CX = [a for a in TIA_W if a != 0x01]       # no VBLANK: the objects stay drawn
TIA_R = list(range(0x00, 0x10))
# objects on at every frame start, then down to the visible rows (collision
# cartridges)
CX_FRAME = ["    lda #0", "    sta VBLANK", "    lda #$FF", "    sta GRP0", "    sta GRP1", "    lda #2",
            "    sta ENAM0", "    sta ENAM1", "    sta ENABL", "    sta PF1",
            "    ldx #36", "cxw:", "    sta WSYNC", "    dex", "    bne cxw"]
RIOT_R = [0x280, 0x281, 0x282, 0x283, 0x284, 0x285, 0x286, 0x287]
RIOT_W = [0x294, 0x295, 0x296, 0x297, 0x280, 0x281]
CART_R = list(range(0x1E00, 0x1F00))

READ_MN = ["lda", "ldx", "ldy", "adc", "sbc", "and", "ora", "eor", "cmp", "cpx", "cpy", "bit"]
STORE_MN = ["sta", "stx", "sty"]
RMW_MN = ["asl", "lsr", "rol", "ror", "inc", "dec"]
IMPLIED = ["clc", "sec", "cli", "sei", "clv", "cld", "sed", "nop", "tax", "tay", "txa", "tya", "tsx",
           "inx", "iny", "dex", "dey"]
BRANCHES = ["bpl", "bmi", "bvc", "bvs", "bcc", "bcs", "bne", "beq"]


class Gen:
    def __init__(self, seed, scheme=S_4K, undoc=False, cx=False):
        self.r = np.random.default_rng(seed)
        self.scheme = scheme
        self.undoc = undoc
        self.cx = cx
        self.n = 0
        self.lines = []
        self.hot = list(HOTSPOTS.get(scheme, []))
        self.sc = scheme in (S_F8SC, S_F6SC, S_F4SC)
        if scheme == S_E0:
            self.cart_r = list(range(0x1000, 0x1C00, 7))     # the switched segments
        elif scheme == S_3F:
            self.cart_r = list(range(0x1000, 0x1800, 5))
        else:
            self.cart_r = CART_R
        self.n_slices = 4

    def pick(self, seq):
        return seq[int(self.r.integers(0, len(seq)))]

    def label(self):
        self.n += 1
        return f"L{self.n}"

    def emit(self, s):
        self.lines.append("    " + s)

    def target(self, kind):
        """An address for a data access of `kind` ('r' or 'w')."""
        x = self.r.random()
        if kind == "r":
            if x < 0.55:
                return self.pick(RAM)
            if x < 0.7:
                return self.pick(TIA_R)
            if x < 0.8:
                return self.pick(RIOT_R)
            if self.hot and x < 0.84:
                return self.pick(self.hot)
            if self.sc and x < 0.9:
                return 0x1000 + int(self.r.integers(0, 256))    # both Superchip ports
            return self.pick(self.cart_r)
        if x < 0.55:
            return self.pick(RAM)
        if x < 0.8:
            return self.pick(TIA_W_CX if self.cx else TIA_W)
        if self.hot and x < 0.86:
            return self.pick(self.hot)
        if self.sc and x < 0.93:
            return 0x1000 + int(self.r.integers(0, 256))
        return self.pick(RIOT_W)

    def mem_op(self, mn, kind):
        modes = [m for m in {**UNDOC_OPCODES.get(mn, {}), **OPCODES.get(mn, {})} if m not in ("imp", "acc", "rel")]
        mode = self.pick(modes)
        if mode == "imm":
            self.emit(f"{mn} #${int(self.r.integers(0, 256)):02X}")
            return
        t = self.target(kind)
        if mode in ("zp", "zpx", "zpy") and t >= 0x100:
            t = self.pick(RAM)
        if mode == "zp":
            self.emit(f"{mn} ${t:02X}")
        elif mode == "abs":
            self.emit(f"{mn}.w ${t:04X}")
        elif mode in ("zpx", "zpy"):
            reg = mode[-1]
            k = int(self.r.integers(0, 256))
            self.emit(f"ld{reg} #${k:02X}")
            self.emit(f"{mn} ${(t - k) & 0xFF:02X},{reg}")
        elif mode in ("absx", "absy"):
            reg = mode[-1]
            k = int(self.r.integers(0, 256))
            base = (t - k) & 0xFFFF
            if base < 0x100:
                base += 0x2000       # a 13-bit mirror of the same address, forced absolute
            self.emit(f"ld{reg} #${k:02X}")
            self.emit(f"{mn}.w ${base:04X},{reg}")
        elif mode == "indx":
            k = int(self.r.integers(0, 256))
            self.emit(f"lda #${t & 0xFF:02X}")
            self.emit("sta $E0")
            self.emit(f"lda #${t >> 8:02X}")
            self.emit("sta $E1")
            if mn in ("sta", "sax"):
                self.emit(f"lda #${int(self.r.integers(0, 256)):02X}")
            self.emit(f"ldx #${k:02X}")
            self.emit(f"{mn} (${(0xE0 - k) & 0xFF:02X},x)")
        elif mode == "indy":
            k = int(self.r.integers(0, 256))
            base = (t - k) & 0xFFFF
            self.emit(f"lda #${base & 0xFF:02X}")
            self.emit("sta $E0")
            self.emit(f"lda #${base >> 8:02X}")
            self.emit("sta $E1")
            if mn in ("sta", "sax"):
                self.emit(f"lda #${int(self.r.integers(0, 256)):02X}")
            self.emit(f"ldy #${k:02X}")
            self.emit(f"{mn} ($E0),y")

    def instr(self):
        x = self.r.random()
        if self.undoc and x < 0.2:
            self.undoc_op()
            return
        if self.scheme == S_E0 and x > 0.985:
            # a data slice into segment 2, then a call that straddles it and the fixed segment
            self.emit(f"lda $1FF{int(self.r.integers(0, 7)):X}")
            self.emit("jsr $1BFE")
            return
        if self.scheme == S_3F and x > 0.985:
            v = int(self.r.integers(0, 256 // self.n_slices)) * self.n_slices + int(self.r.integers(0, self.n_slices - 1))
            self.emit(f"lda #${v:02X}")         # any slice but the fixed one
            self.emit("sta $3F")
            self.emit("jsr $17FE")
            return
        if self.scheme == S_3F and x > 0.96:
            self.emit(f"lda #${int(self.r.integers(0, 256)):02X}")
            self.emit("sta $3F")                  # selects slice v mod S
            return
        x = self.r.random()
        if x < 0.35:
            self.mem_op(self.pick(READ_MN), "r")
        elif x < 0.55:
            mn = self.pick(STORE_MN)
            self.mem_op(mn, "w")
        elif x < 0.65:
            mn = self.pick(RMW_MN)
            if self.r.random() < 0.3 and mn in ("asl", "lsr", "rol", "ror"):
                self.emit(f"{mn}")
            else:
                self.mem_op(mn, "w")
        elif x < 0.82:
            self.emit(self.pick(IMPLIED))
        elif x < 0.9:
            lab = self.label()
            self.emit(f"{self.pick(BRANCHES)} {lab}")
            for _ in range(int(self.r.integers(1, 4))):
                self.simple()
            self.lines.append(f"{lab}:")
        elif x < 0.94:
            self.emit("pha" if self.r.random() < 0.5 else "php")
            self.simple()
            self.emit("pla" if self.r.random() < 0.5 else "plp")
        elif x < 0.97:
            self.emit(f"jsr sub{int(self.r.integers(0, 4))}")
        else:
            self.emit("brk")
            self.emit(".byte $EA")

    def undoc_op(self):
        """One stable undocumented opcode (every mode, every encoding kind)."""
        x = self.r.random()
        imm = int(self.r.integers(0, 256))
        if x < 0.4:
            self.mem_op(self.pick(UNDOC_RMW), "w")
        elif x < 0.5:
            self.mem_op("sax", "w")
        elif x < 0.62:
            self.mem_op("lax", "r")
        elif x < 0.76:
            self.emit(self.pick([f"anc #${imm:02X}", f"alr #${imm:02X}", f"arr #${imm:02X}", f"sbx #${imm:02X}",
                                 f".byte $2B, ${imm:02X}", f".byte $EB, ${imm:02X}"]))
        elif x < 0.8:
            k = int(self.r.integers(0, 256))
            t = self.pick(RAM)
            self.emit(f"ldy #${k:02X}")
            self.emit(f"las ${(t - k) & 0xFFFF | 0x2000:04X},y")
            self.emit("ldx #$FB")                 # keep the stack where the code expects it
            self.emit("txs")
        elif x < 0.9:
            self.mem_op("nop", "r")               # the NOPs read their operand
        else:
            self.emit(self.pick([".byte $1A", ".byte $3A", ".byte $5A", ".byte $7A", ".byte $DA", ".byte $FA",
                                 f".byte $82, ${imm:02X}", f".byte $89, ${imm:02X}", f".byte $C2, ${imm:02X}",
                                 f".byte $E2, ${imm:02X}", f".byte $44, ${self.pick(RAM):02X}",
                                 f".byte $D4, ${self.pick(RAM):02X}", f".byte $FC, $00, $1E"]))

    def simple(self):
        x = self.r.random()
        if x < 0.5:
            self.mem_op(self.pick(READ_MN), "r")
        elif x < 0.75:
            self.emit(self.pick(IMPLIED))
        else:
            self.mem_op(self.pick(RMW_MN), "w")

    def source(self, lines_per_frame=60, T=None):
        T = T or int(self.r.integers(120, 300))
        head = ["reset:", "    ldx #$FF", "    txs", "    cld"]
        frame = ["frame:", "    lda #2", "    sta VSYNC", "    lda #0", "    sta VSYNC",
                 "    inc $D4", "    bne fc1", "    inc $D5", "fc1:", "    lda $D5", f"    cmp #${T >> 8:02X}",
                 "    bcc fc2", "    bne fc3", "    lda $D4", f"    cmp #${T & 0xFF:02X}", "    bcc fc2",
                 "fc3:", "    lda #1", "    sta $D1", "fc2:", "    lda INPT4", "    bmi fc4", "    sed", "    clc",
                 "    lda $D0", "    adc #1", "    sta $D0", "fc4:", "    cld", "    sta WSYNC"]
        if self.cx:
            frame += CX_FRAME
        self.lines = []
        for _ in range(lines_per_frame):
            for _ in range(int(self.r.integers(2, 7))):
                self.instr()
            self.emit("sta WSYNC")
        body = self.lines
        self.lines = []
        subs = []
        for k in range(4):
            self.lines = []
            for _ in range(int(self.r.integers(1, 5))):
                self.simple()
            subs += [f"sub{k}:"] + self.lines + ["    rts"]
        self.lines = []
        for _ in range(int(self.r.integers(1, 4))):
            self.simple()
        handler = ["brkh:"] + self.lines + ["    rti"]
        data = ["    .org $1E00"] + ["    .byte " + ", ".join(f"${int(v):02X}" for v in self.r.integers(0, 256, 16))
                                     for _ in range(16)]
        tail = ["    jmp frame"]
        return "\n".join(head + frame + body + tail + subs + handler), "\n".join(data)


VECTORS = "\n    .org $1FFA\n    .word reset, reset, brkh\n"


def _segmented(seed, scheme, undoc, lines_per_frame, size, cx):
    """E0 (8 KB) or 3F (`size`): code in the fixed segment, data slices."""
    g = Gen(seed, scheme, undoc, cx)
    if scheme == S_E0:
        n_sl, sl, fixed_at = 8, 1024, 0x1C00
    else:
        n_sl, sl, fixed_at = size // 2048, 2048, 0x1800
    g.n_slices = n_sl
    code, _ = g.source(lines_per_frame)
    r = np.random.default_rng(seed + 7)
    # fixed segment: byte 0 = $1E (the high byte of the straddling LDA), RTS, the
    # code, then (3F only) a data block at $1E00
    data = "" if scheme == S_E0 else "\n    .org $1E00\n" + "\n".join(
        "    .byte " + ", ".join(f"${int(v):02X}" for v in r.integers(0, 256, 16)) for _ in range(16))
    src = f"    .org ${fixed_at:04X}\n    .byte $1E\n    rts\n" + code + "\ncode_end:" + data + VECTORS
    img, syms = assemble_with_symbols(src)
    assert syms["code_end"] <= (0x1FE0 if scheme == S_E0 else 0x1E00), hex(syms["code_end"])
    fixed = img[fixed_at - 0x1000:]
    out = bytearray()
    for s_ in range(n_sl - 1):
        part = bytearray(r.integers(0, 256, sl).astype(np.uint8).tobytes())
        part[-2:] = bytes([0xAD, int(r.integers(0, 256))])    # LDA $1Exx across the boundary
        out += part
    out += fixed
    assert len(out) == n_sl * sl
    return bytes(out), scheme


def fuzz_cart(seed, f8=False, lines_per_frame=60, scheme=None, undoc=False, size=8192, cx=False):
    """cx: the objects are switched on at every frame start and VBLANK is
    never written, so that they collide."""
    scheme = (S_F8 if f8 else S_4K) if scheme is None else scheme
    if scheme in (S_E0, S_3F):
        return _segmented(seed, scheme, undoc, min(lines_per_frame, (12 if cx else 14) if scheme == S_E0 else 40), size, cx)
    nb = LINEAR_BANKS[scheme]
    org = "$1100" if scheme in (S_F8SC, S_F6SC, S_F4SC) else "$1000"
    g = Gen(seed, scheme, undoc, cx)
    code, data = g.source(lines_per_frame)
    # the same code in every bank (so a switch continues in place), different data
    g2 = Gen(seed + 1, scheme, undoc)
    images = []
    for b in range(nb):
        d = data if b == 0 else "\n".join(["    .org $1E00"] + [
            "    .byte " + ", ".join(f"${int(v):02X}" for v in g2.r.integers(0, 256, 16)) for _ in range(16)])
        img, _ = assemble_with_symbols(f"    .org {org}\n" + code + "\n" + d + VECTORS)
        images.append(img)
    return b"".join(images), scheme
