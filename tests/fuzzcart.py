"""Random cartridges for differential testing of the GPU interpreter against
the oracle.  Every documented opcode appears with every addressing mode, on
RAM, TIA, RIOT (ports and timer) and cartridge operands, in decimal and
binary mode, with forward branches, subroutines, BRK/RTI and page crossings.
Control flow stays structured so that frames keep ending (VSYNC) and the
cartridge never executes an undocumented opcode.
"""
import numpy as np

from paper_1907_08467_amd.inputs.asm6502 import OPCODES, assemble_with_symbols

RAM = [a for a in range(0x80, 0xF8) if a not in (0xD0, 0xD1, 0xD4, 0xD5, 0xE0, 0xE1)]   # $F8-$FF: stack
TIA_W = [0x01, 0x06, 0x07, 0x08, 0x09, 0x0A, 0x0B, 0x0C, 0x0D, 0x0E, 0x0F, 0x10, 0x11, 0x1B, 0x1C,
         0x20, 0x21, 0x2A, 0x2B, 0x04, 0x05, 0x15, 0x19, 0x1D, 0x25, 0x2C]
TIA_R = list(range(0x00, 0x10))
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
    def __init__(self, seed, f8=False):
        self.r = np.random.default_rng(seed)
        self.f8 = f8
        self.n = 0
        self.lines = []

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
            if x < 0.85:
                return self.pick(RIOT_R)
            if self.f8 and x < 0.88:
                return self.pick([0x1FF8, 0x1FF9])
            return self.pick(CART_R)
        if x < 0.6:
            return self.pick(RAM)
        if x < 0.85:
            return self.pick(TIA_W)
        if self.f8 and x < 0.9:
            return self.pick([0x1FF8, 0x1FF9])
        return self.pick(RIOT_W)

    def mem_op(self, mn, kind):
        modes = [m for m in OPCODES[mn] if m not in ("imp", "acc", "rel")]
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
            if mn in ("sta",):
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
            if mn in ("sta",):
                self.emit(f"lda #${int(self.r.integers(0, 256)):02X}")
            self.emit(f"ldy #${k:02X}")
            self.emit(f"{mn} ($E0),y")

    def instr(self):
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
        return "\n".join(head + frame + body + tail + subs + handler + data)


def fuzz_cart(seed, f8=False, lines_per_frame=60):
    g = Gen(seed, f8)
    src = g.source(lines_per_frame)
    if not f8:
        rom, _ = assemble_with_symbols("    .org $1000\n" + src + "\n    .org $1FFA\n    .word reset, reset, brkh\n")
        return rom, 0
    # F8: the same code in both banks (so a switch continues in place), different data
    g2 = Gen(seed + 1, f8)
    images = []
    for b in range(2):
        data_src = src if b == 0 else src[:src.index("    .org $1E00")] + "\n".join(
            ["    .org $1E00"] + ["    .byte " + ", ".join(f"${int(v):02X}" for v in g2.r.integers(0, 256, 16))
                                for _ in range(16)])
        img, _ = assemble_with_symbols("    .org $1000\n" + data_src + "\n    .org $1FFA\n    .word reset, reset, brkh\n")
        images.append(img)
    return images[0] + images[1], 1
