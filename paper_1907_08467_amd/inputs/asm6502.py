"""A small two-pass assembler for the NMOS 6502 instruction set (documented
opcodes, plus the stable undocumented ones for test programs).

Input tooling only: it turns hand-written test programs and the generated
synthetic cartridges into bytes.  It holds no part of the emulator; both the
CPU oracle and the GPU path receive its output as plain ROM images.

Syntax (one statement per line, ``;`` starts a comment)::

    NAME = expr              constant
    label:                   label (may share a line with a statement)
    .bank n                  select cartridge bank n (4 KB each)
    .org expr                set the location counter ($1000-$1FFF in a bank)
    .byte e, e, ...          raw bytes
    .word e, e, ...          little-endian words
    .fill n, value           n copies of a byte
    lda #expr                immediate
    lda expr / lda.w expr    zero page if the value is known and < $100,
                             else absolute (``.w`` forces absolute)
    lda expr,x / expr,y      indexed
    lda (expr,x) / (expr),y  indirect
    jmp (expr)               indirect jump
    asl / asl a              accumulator
    bne label                relative branch

Expressions: ``$hex``, ``%bin``, decimal, symbols, ``*`` (location counter),
``+``/``-``, unary ``<`` (low byte) and ``>`` (high byte).

Documented opcode encodings follow the MOS MCS6500 programming manual's
instruction matrix; the undocumented ones the published NMOS opcode matrix.
"""

from __future__ import annotations

import re

# mnemonic -> {mode: opcode}.  Modes: imp acc imm zp zpx zpy abs absx absy
# indx indy ind rel.
OPCODES: dict[str, dict[str, int]] = {
    "adc": dict(imm=0x69, zp=0x65, zpx=0x75, abs=0x6D, absx=0x7D, absy=0x79, indx=0x61, indy=0x71),
    "and": dict(imm=0x29, zp=0x25, zpx=0x35, abs=0x2D, absx=0x3D, absy=0x39, indx=0x21, indy=0x31),
    "asl": dict(acc=0x0A, zp=0x06, zpx=0x16, abs=0x0E, absx=0x1E),
    "bcc": dict(rel=0x90), "bcs": dict(rel=0xB0), "beq": dict(rel=0xF0), "bmi": dict(rel=0x30),
    "bne": dict(rel=0xD0), "bpl": dict(rel=0x10), "bvc": dict(rel=0x50), "bvs": dict(rel=0x70),
    "bit": dict(zp=0x24, abs=0x2C),
    "brk": dict(imp=0x00),
    "clc": dict(imp=0x18), "cld": dict(imp=0xD8), "cli": dict(imp=0x58), "clv": dict(imp=0xB8),
    "cmp": dict(imm=0xC9, zp=0xC5, zpx=0xD5, abs=0xCD, absx=0xDD, absy=0xD9, indx=0xC1, indy=0xD1),
    "cpx": dict(imm=0xE0, zp=0xE4, abs=0xEC),
    "cpy": dict(imm=0xC0, zp=0xC4, abs=0xCC),
    "dec": dict(zp=0xC6, zpx=0xD6, abs=0xCE, absx=0xDE),
    "dex": dict(imp=0xCA), "dey": dict(imp=0x88),
    "eor": dict(imm=0x49, zp=0x45, zpx=0x55, abs=0x4D, absx=0x5D, absy=0x59, indx=0x41, indy=0x51),
    "inc": dict(zp=0xE6, zpx=0xF6, abs=0xEE, absx=0xFE),
    "inx": dict(imp=0xE8), "iny": dict(imp=0xC8),
    "jmp": dict(abs=0x4C, ind=0x6C),
    "jsr": dict(abs=0x20),
    "lda": dict(imm=0xA9, zp=0xA5, zpx=0xB5, abs=0xAD, absx=0xBD, absy=0xB9, indx=0xA1, indy=0xB1),
    "ldx": dict(imm=0xA2, zp=0xA6, zpy=0xB6, abs=0xAE, absy=0xBE),
    "ldy": dict(imm=0xA0, zp=0xA4, zpx=0xB4, abs=0xAC, absx=0xBC),
    "lsr": dict(acc=0x4A, zp=0x46, zpx=0x56, abs=0x4E, absx=0x5E),
    "nop": dict(imp=0xEA),
    "ora": dict(imm=0x09, zp=0x05, zpx=0x15, abs=0x0D, absx=0x1D, absy=0x19, indx=0x01, indy=0x11),
    "pha": dict(imp=0x48), "php": dict(imp=0x08), "pla": dict(imp=0x68), "plp": dict(imp=0x28),
    "rol": dict(acc=0x2A, zp=0x26, zpx=0x36, abs=0x2E, absx=0x3E),
    "ror": dict(acc=0x6A, zp=0x66, zpx=0x76, abs=0x6E, absx=0x7E),
    "rti": dict(imp=0x40), "rts": dict(imp=0x60),
    "sbc": dict(imm=0xE9, zp=0xE5, zpx=0xF5, abs=0xED, absx=0xFD, absy=0xF9, indx=0xE1, indy=0xF1),
    "sec": dict(imp=0x38), "sed": dict(imp=0xF8), "sei": dict(imp=0x78),
    "sta": dict(zp=0x85, zpx=0x95, abs=0x8D, absx=0x9D, absy=0x99, indx=0x81, indy=0x91),
    "stx": dict(zp=0x86, zpy=0x96, abs=0x8E),
    "sty": dict(zp=0x84, zpx=0x94, abs=0x8C),
    "tax": dict(imp=0xAA), "tay": dict(imp=0xA8), "tsx": dict(imp=0xBA),
    "txa": dict(imp=0x8A), "txs": dict(imp=0x9A), "tya": dict(imp=0x98),
}

# The stable undocumented NMOS opcodes (one encoding each; the duplicate
# encodings such as ANC $2B, SBC $EB and the other NOPs are emitted with
# .byte).  Mnemonics as in the common unintended-opcode tables.
UNDOC_OPCODES: dict[str, dict[str, int]] = {
    "slo": dict(zp=0x07, zpx=0x17, abs=0x0F, absx=0x1F, absy=0x1B, indx=0x03, indy=0x13),
    "rla": dict(zp=0x27, zpx=0x37, abs=0x2F, absx=0x3F, absy=0x3B, indx=0x23, indy=0x33),
    "sre": dict(zp=0x47, zpx=0x57, abs=0x4F, absx=0x5F, absy=0x5B, indx=0x43, indy=0x53),
    "rra": dict(zp=0x67, zpx=0x77, abs=0x6F, absx=0x7F, absy=0x7B, indx=0x63, indy=0x73),
    "sax": dict(zp=0x87, zpy=0x97, abs=0x8F, indx=0x83),
    "lax": dict(zp=0xA7, zpy=0xB7, abs=0xAF, absy=0xBF, indx=0xA3, indy=0xB3),
    "dcp": dict(zp=0xC7, zpx=0xD7, abs=0xCF, absx=0xDF, absy=0xDB, indx=0xC3, indy=0xD3),
    "isc": dict(zp=0xE7, zpx=0xF7, abs=0xEF, absx=0xFF, absy=0xFB, indx=0xE3, indy=0xF3),
    "anc": dict(imm=0x0B), "alr": dict(imm=0x4B), "arr": dict(imm=0x6B), "sbx": dict(imm=0xCB),
    "las": dict(absy=0xBB),
    "nop": dict(imm=0x80, zp=0x04, zpx=0x14, abs=0x0C, absx=0x1C),
}


def _modes(mnem: str) -> dict[str, int]:
    return {**UNDOC_OPCODES.get(mnem, {}), **OPCODES.get(mnem, {})}


MODE_LEN = dict(imp=1, acc=1, imm=2, zp=2, zpx=2, zpy=2, abs=3, absx=3, absy=3,
                indx=2, indy=2, ind=3, rel=2)

# Standard Atari 2600 register names (hardware addresses), for convenience.
VCS_SYMBOLS = {
    "VSYNC": 0x00, "VBLANK": 0x01, "WSYNC": 0x02, "RSYNC": 0x03, "NUSIZ0": 0x04, "NUSIZ1": 0x05,
    "COLUP0": 0x06, "COLUP1": 0x07, "COLUPF": 0x08, "COLUBK": 0x09, "CTRLPF": 0x0A,
    "REFP0": 0x0B, "REFP1": 0x0C, "PF0": 0x0D, "PF1": 0x0E, "PF2": 0x0F,
    "RESP0": 0x10, "RESP1": 0x11, "RESM0": 0x12, "RESM1": 0x13, "RESBL": 0x14,
    "AUDC0": 0x15, "AUDC1": 0x16, "AUDF0": 0x17, "AUDF1": 0x18, "AUDV0": 0x19, "AUDV1": 0x1A,
    "GRP0": 0x1B, "GRP1": 0x1C, "ENAM0": 0x1D, "ENAM1": 0x1E, "ENABL": 0x1F,
    "HMP0": 0x20, "HMP1": 0x21, "HMM0": 0x22, "HMM1": 0x23, "HMBL": 0x24,
    "VDELP0": 0x25, "VDELP1": 0x26, "VDELBL": 0x27, "RESMP0": 0x28, "RESMP1": 0x29,
    "HMOVE": 0x2A, "HMCLR": 0x2B, "CXCLR": 0x2C,
    "CXM0P": 0x00, "CXM1P": 0x01, "CXP0FB": 0x02, "CXP1FB": 0x03, "CXM0FB": 0x04, "CXM1FB": 0x05,
    "CXBLPF": 0x06, "CXPPMM": 0x07, "INPT4": 0x0C, "INPT5": 0x0D,
    "SWCHA": 0x280, "SWACNT": 0x281, "SWCHB": 0x282, "SWBCNT": 0x283,
    "INTIM": 0x284, "TIMINT": 0x285,
    "TIM1T": 0x294, "TIM8T": 0x295, "TIM64T": 0x296, "T1024T": 0x297,
}


class AsmError(Exception):
    pass


_TOKEN = re.compile(r"\s*(\$[0-9A-Fa-f]+|%[01]+|\d+|[A-Za-z_.][A-Za-z0-9_.]*|\*|[<>+\-])")


class Assembler:
    def __init__(self, symbols: dict[str, int] | None = None, bank_size: int = 4096):
        self.base_symbols = dict(VCS_SYMBOLS)
        if symbols:
            self.base_symbols.update(symbols)
        self.bank_size = bank_size

    # -- expressions -------------------------------------------------------
    def _eval(self, expr: str, syms: dict[str, int], pc: int, strict: bool) -> int | None:
        toks = []
        pos = 0
        expr = expr.strip()
        while pos < len(expr):
            m = _TOKEN.match(expr, pos)
            if not m:
                raise AsmError(f"bad expression {expr!r}")
            toks.append(m.group(1))
            pos = m.end()
            while pos < len(expr) and expr[pos].isspace():
                pos += 1
        val = 0
        sign = 1
        i = 0
        unknown = False
        expect_term = True
        while i < len(toks):
            t = toks[i]
            if expect_term:
                unary = None
                if t in ("<", ">"):
                    unary = t
                    i += 1
                    t = toks[i]
                if t == "-":
                    sign = -sign
                    i += 1
                    continue
                if t.startswith("$"):
                    v = int(t[1:], 16)
                elif t.startswith("%"):
                    v = int(t[1:], 2)
                elif t.isdigit():
                    v = int(t)
                elif t == "*":
                    v = pc
                else:
                    key = t.upper() if t.upper() in VCS_SYMBOLS and t not in syms else t
                    if key in syms:
                        v = syms[key]
                    elif t in syms:
                        v = syms[t]
                    else:
                        if strict:
                            raise AsmError(f"undefined symbol {t!r}")
                        unknown = True
                        v = 0
                if unary == "<":
                    v &= 0xFF
                elif unary == ">":
                    v = (v >> 8) & 0xFF
                val += sign * v
                sign = 1
                expect_term = False
            else:
                if t == "+":
                    sign = 1
                elif t == "-":
                    sign = -1
                else:
                    raise AsmError(f"bad operator {t!r} in {expr!r}")
                expect_term = True
            i += 1
        return None if unknown else val

    # -- parsing ------------------------------------------------------------
    @staticmethod
    def _split(line: str):
        line = line.split(";", 1)[0].rstrip()
        label = None
        m = re.match(r"^\s*([A-Za-z_][A-Za-z0-9_]*)\s*:(.*)$", line)
        if m:
            label, line = m.group(1), m.group(2)
        return label, line.strip()

    def _operand_mode(self, mnem: str, opnd: str, force_abs: bool, syms, pc, strict):
        modes = _modes(mnem)
        o = opnd.strip()
        if o == "" or o.lower() == "a":
            if "acc" in modes:
                return "acc", None
            if "imp" in modes and o == "":
                return "imp", None
            raise AsmError(f"{mnem} needs an operand")
        if "rel" in modes:
            return "rel", o
        if o.startswith("#"):
            return "imm", o[1:]
        m = re.match(r"^\((.*),\s*[xX]\s*\)$", o)
        if m:
            return "indx", m.group(1)
        m = re.match(r"^\((.*)\)\s*,\s*[yY]$", o)
        if m:
            return "indy", m.group(1)
        m = re.match(r"^\((.*)\)$", o)
        if m:
            return "ind", m.group(1)
        idx = None
        m = re.match(r"^(.*),\s*([xXyY])$", o)
        if m:
            o, idx = m.group(1), m.group(2).lower()
        v = self._eval(o, syms, pc, strict=False)
        zp_ok = (not force_abs) and v is not None and 0 <= v < 256
        if idx is None:
            mode = "zp" if zp_ok and "zp" in modes else "abs"
        else:
            mode = ("zp" + idx) if zp_ok and ("zp" + idx) in modes else ("abs" + idx)
        return mode, o

    def assemble(self, src: str, banks: int = 1) -> bytes:
        """Assemble ``src`` into ``banks`` x bank_size bytes (unused = $FF)."""
        lines = src.splitlines()
        sizing: dict[int, str] = {}
        syms = dict(self.base_symbols)
        for pass_no in (1, 2):
            out = [bytearray([0xFF] * self.bank_size) for _ in range(banks)]
            bank = 0
            pc = 0x1000
            for ln, raw in enumerate(lines):
                try:
                    label, stmt = self._split(raw)
                    if label:
                        if pass_no == 1 and label in syms and label not in self.base_symbols:
                            raise AsmError(f"duplicate label {label}")
                        syms[label] = pc
                    if not stmt:
                        continue
                    m = re.match(r"^([A-Za-z_][A-Za-z0-9_]*)\s*=\s*(.+)$", stmt)
                    if m:
                        v = self._eval(m.group(2), syms, pc, strict=(pass_no == 2))
                        if v is not None:
                            syms[m.group(1)] = v
                        continue
                    parts = stmt.split(None, 1)
                    op = parts[0].lower()
                    arg = parts[1] if len(parts) > 1 else ""
                    strict = pass_no == 2
                    if op == ".bank":
                        bank = self._eval(arg, syms, pc, True)
                        if not 0 <= bank < banks:
                            raise AsmError("bank out of range")
                        continue
                    if op == ".org":
                        pc = self._eval(arg, syms, pc, True)
                        continue
                    if op in (".byte", ".word", ".fill"):
                        vals = [a for a in arg.split(",")]
                        data = []
                        if op == ".fill":
                            n = self._eval(vals[0], syms, pc, True)
                            fv = self._eval(vals[1], syms, pc, strict) if len(vals) > 1 else 0
                            data = [(fv or 0) & 0xFF] * n
                        for a in (vals if op != ".fill" else []):
                            v = self._eval(a, syms, pc, strict) or 0
                            if op == ".byte":
                                data.append(v & 0xFF)
                            else:
                                data += [v & 0xFF, (v >> 8) & 0xFF]
                        self._emit(out, bank, pc, data)
                        pc += len(data)
                        continue
                    force_abs = op.endswith(".w")
                    mnem = op[:-2] if force_abs else op
                    if mnem not in OPCODES and mnem not in UNDOC_OPCODES:
                        raise AsmError(f"unknown mnemonic {op!r}")
                    if pass_no == 1:
                        mode, expr = self._operand_mode(mnem, arg, force_abs, syms, pc, False)
                        sizing[ln] = mode
                    else:
                        mode = sizing[ln]
                        _, expr = self._operand_mode(mnem, arg, force_abs, syms, pc, False)
                    opc = _modes(mnem).get(mode)
                    if opc is None:
                        raise AsmError(f"{mnem} has no {mode} mode")
                    data = [opc]
                    if mode == "rel":
                        tgt = self._eval(expr, syms, pc, strict)
                        if tgt is None:
                            data.append(0)
                        else:
                            off = tgt - (pc + 2)
                            if strict and not -128 <= off <= 127:
                                raise AsmError(f"branch out of range ({off})")
                            data.append(off & 0xFF)
                    elif MODE_LEN[mode] >= 2:
                        v = self._eval(expr, syms, pc, strict)
                        v = 0 if v is None else v
                        if MODE_LEN[mode] == 2:
                            if strict and not 0 <= v <= 0xFF:
                                raise AsmError(f"operand {v:#x} does not fit one byte")
                            data.append(v & 0xFF)
                        else:
                            data += [v & 0xFF, (v >> 8) & 0xFF]
                    self._emit(out, bank, pc, data)
                    pc += len(data)
                except AsmError as e:
                    raise AsmError(f"line {ln + 1}: {raw.strip()!r}: {e}") from None
        self.symbols = syms
        return b"".join(bytes(b) for b in out)

    def _emit(self, out, bank, pc, data):
        for i, b in enumerate(data):
            a = pc + i
            if not 0x1000 <= a <= 0x1FFF:
                raise AsmError(f"address {a:#x} outside the cartridge window")
            out[bank][a - 0x1000] = b


def assemble(src: str, banks: int = 1, symbols: dict[str, int] | None = None) -> bytes:
    return Assembler(symbols).assemble(src, banks)


def assemble_with_symbols(src: str, banks: int = 1, symbols: dict[str, int] | None = None):
    a = Assembler(symbols)
    rom = a.assemble(src, banks)
    return rom, a.symbols
