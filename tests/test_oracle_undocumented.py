"""Pins of the oracle's undocumented opcodes.

* Length and cycles of every undocumented opcode against the published NMOS
  matrix in golden/nmos6502_undocumented.txt; the JAMs and unstable opcodes
  listed there fault.
* Each read-modify-write + ALU pair against the two documented instructions
  it combines (SLO = ASL + ORA, RLA = ROL + AND, SRE = LSR + EOR, RRA = ROR +
  ADC, DCP = DEC + CMP, ISC = INC + SBC), LAX against LDA + TAX and ALR against
  AND # + LSR A, over random registers and flags in binary and decimal mode;
  the other ones against their closed forms (SAX, LAS, ANC, SBX, binary ARR)
  and hand-derived decimal ARR cases.
* The NOPs with a memory operand perform their read: NOP $1FF8 switches an
  F8 cartridge's bank.
"""
import os

import numpy as np
import pytest

import oracle
from helpers import decode, set_fields
from paper_1907_08467_amd.inputs.asm6502 import assemble

GOLDEN_UNDOC = os.path.join(os.path.dirname(__file__), "golden", "nmos6502_undocumented.txt")
C, Z, D, V, N = 0x01, 0x02, 0x08, 0x40, 0x80


def undoc_rows():
    rows = []
    for line in open(GOLDEN_UNDOC):
        line = line.strip()
        if line and not line.startswith("#"):
            op, mn, mode, nb, cyc = line.split()
            rows.append((int(op, 16), mn, mode, int(nb), cyc))
    return rows


ROWS = undoc_rows()


def exec_code(code, n, at=0x1000, **state):
    rom = bytearray([0xEA] * 4096)
    off = at - 0x1000
    rom[off:off + len(code)] = bytes(code)
    rom[0xFFC:0xFFE] = bytes([at & 0xFF, at >> 8])
    st = set_fields(oracle.power_on(bytes(rom)), **state)
    out, done = oracle.run_instructions(st, bytes(rom), n)
    return decode(out), done


def operands(mode, cross):
    ram = {0x80: 0x90, 0x81: 0x00, 0x82: 0xF0 if cross else 0x90, 0x83: 0x00}
    st = dict(ram=ram, x=0x20 if cross else 0, y=0x20 if cross else 0)
    return {"zp": [0x90], "zpx": [0x90], "zpy": [0x90], "abs": [0x90, 0x00],
            "absx": [0xF0, 0x00] if cross else [0x90, 0x00], "absy": [0xF0, 0x00] if cross else [0x90, 0x00],
            "indx": [0x80], "indy": [0x82], "imm": [0x01], "imp": []}[mode], st


def test_golden_covers_105_opcodes():
    assert len(ROWS) == 105 and len({r[0] for r in ROWS}) == 105
    assert sum(1 for r in ROWS if r[4] == "fault") == 19


@pytest.mark.parametrize("row", ROWS, ids=[f"{r[0]:02X}_{r[1]}_{r[2]}" for r in ROWS])
def test_undocumented_cycles_and_faults(row):
    op, mn, mode, nb, cyc = row
    opnd, st = operands(mode, cross=False)
    d, done = exec_code([op] + opnd, 1, **st)
    if cyc == "fault":
        assert done == 0 and d["err"] == oracle.ERR_ILLEGAL
        return
    base = int(cyc.split("+")[0])
    assert done == 1 and d["err"] == 0
    assert d["cycle"] == base and d["pc"] == 0x1000 + nb
    if mode in ("absx", "absy", "indy"):
        opnd, st = operands(mode, cross=True)
        d, _ = exec_code([op] + opnd, 1, **st)
        assert d["cycle"] == base + (1 if cyc.endswith("+p") else 0)


PAIRS = {"slo": ("asl", "ora"), "rla": ("rol", "and"), "sre": ("lsr", "eor"), "rra": ("ror", "adc"),
         "dcp": ("dec", "cmp"), "isc": ("inc", "sbc")}


def run_prog(src, n, **state):
    rom = assemble("    .org $1000\nreset:\n" + src + "\n    .org $1FFC\n    .word reset\n")
    st = set_fields(oracle.power_on(rom), **state)
    out, done = oracle.run_instructions(st, rom, n)
    assert done == n
    return decode(out)


def state_key(d):
    return (d["a"], d["x"], d["y"], d["sp"], d["p"], bytes(d["ram"]))


@pytest.mark.parametrize("mn", sorted(PAIRS))
def test_combo_equals_documented_pair(mn):
    first, second = PAIRS[mn]
    rng = np.random.default_rng(sum(map(ord, mn)))
    for _ in range(300):
        a, x, m = (int(v) for v in rng.integers(0, 256, 3))
        p = 0x20 | int(rng.integers(0, 256)) & (C | Z | V | N | D)
        st = dict(a=a, x=x, p=p, ram={0xA0: m})
        got = run_prog(f"    {mn} $A0", 1, **st)
        want = run_prog(f"    {first} $A0\n    {second} $A0", 2, **st)
        assert state_key(got) == state_key(want), (mn, hex(a), hex(m), hex(p))


def test_lax_alr_sbc_eb_equal_documented_sequences():
    rng = np.random.default_rng(11)
    for _ in range(200):
        a, x, m, imm = (int(v) for v in rng.integers(0, 256, 4))
        p = 0x20 | int(rng.integers(0, 256)) & (C | Z | V | N | D)
        st = dict(a=a, x=x, p=p, ram={0xA0: m})
        assert state_key(run_prog("    lax $A0", 1, **st)) == state_key(run_prog("    lda $A0\n    tax", 2, **st))
        assert state_key(run_prog(f"    alr #${imm:02X}", 1, **st)) == \
            state_key(run_prog(f"    and #${imm:02X}\n    lsr a", 2, **st))
        assert state_key(run_prog(f"    .byte $EB, ${imm:02X}", 1, **st)) == \
            state_key(run_prog(f"    sbc #${imm:02X}", 1, **st))


def test_closed_forms():
    rng = np.random.default_rng(12)
    for _ in range(300):
        a, x, m, imm, sp = (int(v) for v in rng.integers(0, 256, 5))
        p = 0x20 | int(rng.integers(0, 256)) & (C | Z | V | N)
        st = dict(a=a, x=x, p=p, sp=sp, ram={0xA0: m})
        d = run_prog("    sax $A0", 1, **st)                      # M = A & X, flags untouched
        assert d["ram"][0x20] == a & x and d["p"] == p and (d["a"], d["x"]) == (a, x)
        d = run_prog("    ldy #0\n    las $00A0,y", 2, **st)        # A = X = SP = M & SP
        v = m & sp
        assert (d["a"], d["x"], d["sp"]) == (v, v, v)
        assert d["p"] & (N | Z) == (v & N) | (Z if v == 0 else 0)
        d = run_prog(f"    anc #${imm:02X}", 1, **st)            # A &= imm; C = N
        v = a & imm
        assert d["a"] == v and d["p"] == (p & ~(N | Z | C)) | (v & N) | (Z if v == 0 else 0) | (v >> 7)
        d = run_prog(f"    sbx #${imm:02X}", 1, **st)            # X = (A & X) - imm, C = no borrow
        t = a & x
        r = (t - imm) & 0xFF
        assert d["x"] == r and d["a"] == a
        assert d["p"] == (p & ~(N | Z | C)) | (r & N) | (Z if r == 0 else 0) | (C if t >= imm else 0)
        d = run_prog(f"    arr #${imm:02X}", 1, **st)            # binary ARR
        r = ((a & imm) >> 1) | ((p & C) << 7)
        want_p = (p & ~(N | Z | C | V)) | (r & N) | (Z if r == 0 else 0) | (C if r & 0x40 else 0) | \
            (V if ((r >> 6) ^ (r >> 5)) & 1 else 0)
        assert d["a"] == r and d["p"] == want_p


@pytest.mark.parametrize("a,imm,cin,want_a,want_p", [
    # t = A & imm; r = t >> 1 | C << 7; N = C in; Z from r; V = bit 6 of t ^ r;
    # low nibble + 6 when (t & $0F) + (t & 1) > 5; + $60 and C when (t & $F0) + (t & $10) > $50
    (0xFF, 0xFF, 0, 0xD5, C),            # r $7F -> $75 -> $D5, C
    (0x00, 0xFF, 1, 0x80, N),            # r $80, no correction
    (0x22, 0xFF, 0, 0x11, 0),            # r $11: low 2+0, high $20+0: none
    (0x0B, 0xFF, 0, 0x0B, 0),            # r $05: low $B+1 = 12 > 5 -> $0B
    (0x60, 0xFF, 0, 0x90, C | V),        # r $30, V (bit 6: t 1, r 0), high $60 > $50 -> $90, C
    (0x01, 0x01, 0, 0x00, Z),            # r 0: Z; low 1+1 = 2
])
def test_arr_decimal_hand_cases(a, imm, cin, want_a, want_p):
    d = run_prog(f"    arr #${imm:02X}", 1, a=a, p=0x20 | D | cin)
    assert d["a"] == want_a and d["p"] == 0x20 | D | want_p


def test_nops_perform_their_read():
    src = """
    .bank 0
    .org $1000
r0:
    .byte $0C, $F9, $1F        ; NOP $1FF9 (absolute): selects bank 1
    lda $1800
    .org $1800
    .byte $A0
    .org $1FFC
    .word r0
    .bank 1
    .org $1000
r1:
    .byte $0C, $F9, $1F
    lda $1800
    .org $1800
    .byte $B1
    .org $1FFC
    .word r1
"""
    rom = assemble(src, banks=2)
    st = set_fields(oracle.power_on(rom, 1), bank=0, pc=0x1000)
    out, _ = oracle.run_instructions(st, rom, 2, scheme=1)
    d = decode(out)
    assert d["bank"] == 1 and d["a"] == 0xB1 and d["cycle"] == 4 + 4
