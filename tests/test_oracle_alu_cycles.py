"""Exhaustive ADC/SBC tables and the datasheet cycle matrix, run through the
oracle's instruction path.

* Binary ADC/SBC: all 256 x 256 x 2 carry inputs against the signed/unsigned
  arithmetic definition of the result and of C, V, N, Z.
* Decimal ADC/SBC on valid BCD operands: the textbook result
  (dec(A) +/- dec(M) +/- carry) mod 100 with the decimal carry.
* Decimal ADC/SBC on every operand (valid or not) against B. Clark's NMOS
  algorithm ("Decimal Mode", 6502.org, Appendix A), written out here a second
  time, independently of the oracle's C.
* Every documented opcode executed alone: length and cycles against the
  datasheet matrix in golden/mos6502_opcodes.txt (MOS programming manual).
"""
import os

import numpy as np
import pytest

import oracle
from helpers import decode, set_fields
from paper_1907_08467_amd.inputs.asm6502 import assemble

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mos6502_opcodes.txt")
GOLDEN_UNDOC = os.path.join(os.path.dirname(__file__), "golden", "nmos6502_undocumented.txt")
C, Z, D, V, N = 0x01, 0x02, 0x08, 0x40, 0x80


def sx(b):
    return b - 256 if b >= 128 else b


def _run_alu(opcode):
    """Run `<op> $80` once on every (A, M, C, D): returns A_out, P_out arrays."""
    rom = bytearray([0xFF] * 4096)
    rom[0:2] = bytes([opcode, 0x80])
    rom[0xFFC:0xFFE] = bytes([0x00, 0x10])
    base = oracle.power_on(bytes(rom))
    a, m, c, d = np.meshgrid(np.arange(256), np.arange(256), np.arange(2), np.arange(2), indexing="ij")
    a, m, c, d = a.ravel(), m.ravel(), c.ravel(), d.ravel()
    st = np.repeat(base[None, :], a.size, axis=0)
    st[:, 0] = a
    st[:, 32] = m
    st[:, 4] = 0x20 | c | (d * D)
    out = oracle.batch_instructions(st, bytes(rom), 1)
    return a, m, c, d, out[:, 0].astype(int), out[:, 4].astype(int)


def dec(b):
    return 10 * (b >> 4) + (b & 15)


def bcd(v):
    return ((v // 10) << 4) | (v % 10)


def clark_adc(a, m, c):
    """NMOS decimal ADC: sequences 1 (A, C) and 2 (N, V) of Clark's Appendix A."""
    al = (a & 0x0F) + (m & 0x0F) + c
    if al >= 0x0A:
        al = ((al + 0x06) & 0x0F) + 0x10
    s = (a & 0xF0) + (m & 0xF0) + al
    if s >= 0xA0:
        s += 0x60
    res, carry = s & 0xFF, int(s >= 0x100)
    al2 = (a & 0x0F) + (m & 0x0F) + c
    if al2 >= 0x0A:
        al2 = ((al2 + 0x06) & 0x0F) + 0x10
    s2 = sx(a & 0xF0) + sx(m & 0xF0) + al2
    n = int(bool(s2 & 0x80))
    v = int(s2 < -128 or s2 > 127)
    return res, carry, n, v


def clark_sbc(a, m, c):
    """NMOS decimal SBC: accumulator by sequence 3 of Clark's Appendix A."""
    al = (a & 0x0F) - (m & 0x0F) + c - 1
    if al < 0:
        al = ((al - 0x06) & 0x0F) - 0x10
    s = (a & 0xF0) - (m & 0xF0) + al
    if s < 0:
        s -= 0x60
    return s & 0xFF


@pytest.fixture(scope="module")
def adc():
    return _run_alu(0x65)


@pytest.fixture(scope="module")
def sbc():
    return _run_alu(0xE5)


def test_adc_binary_exhaustive(adc):
    a, m, c, d, ao, po = adc
    sel = d == 0
    a, m, c, ao, po = a[sel], m[sel], c[sel], ao[sel], po[sel]
    s = a + m + c
    assert np.array_equal(ao, s & 0xFF)
    assert np.array_equal(po & C, (s > 0xFF).astype(int))
    signed = np.array([sx(x) for x in range(256)])[a] + np.array([sx(x) for x in range(256)])[m] + c
    assert np.array_equal((po & V) != 0, (signed < -128) | (signed > 127))
    assert np.array_equal((po & Z) != 0, (s & 0xFF) == 0)
    assert np.array_equal((po & N) != 0, (s & 0x80) != 0)


def test_sbc_binary_exhaustive(sbc):
    a, m, c, d, ao, po = sbc
    sel = d == 0
    a, m, c, ao, po = a[sel], m[sel], c[sel], ao[sel], po[sel]
    s = a - m - (1 - c)
    assert np.array_equal(ao, s & 0xFF)
    assert np.array_equal(po & C, (s >= 0).astype(int))
    sxt = np.array([sx(x) for x in range(256)])
    signed = sxt[a] - sxt[m] - (1 - c)
    assert np.array_equal((po & V) != 0, (signed < -128) | (signed > 127))
    assert np.array_equal((po & Z) != 0, (s & 0xFF) == 0)
    assert np.array_equal((po & N) != 0, (s & 0x80) != 0)


def _valid_bcd(x):
    return ((x >> 4) <= 9) & ((x & 15) <= 9)


def test_adc_decimal_valid_bcd_textbook(adc):
    a, m, c, d, ao, po = adc
    sel = (d == 1) & _valid_bcd(a) & _valid_bcd(m)
    assert sel.sum() == 100 * 100 * 2
    for ai, mi, ci, aoi, poi in zip(a[sel], m[sel], c[sel], ao[sel], po[sel]):
        tot = dec(ai) + dec(mi) + ci
        assert aoi == bcd(tot % 100) and (poi & C) == int(tot >= 100), (hex(ai), hex(mi), ci)
        assert bool(poi & Z) == (((ai + mi + ci) & 0xFF) == 0)      # NMOS: Z of the binary sum


def test_sbc_decimal_valid_bcd_textbook(sbc):
    a, m, c, d, ao, po = sbc
    sel = (d == 1) & _valid_bcd(a) & _valid_bcd(m)
    for ai, mi, ci, aoi, poi in zip(a[sel], m[sel], c[sel], ao[sel], po[sel]):
        tot = dec(ai) - dec(mi) - (1 - ci)
        assert aoi == bcd(tot % 100) and (poi & C) == int(tot >= 0), (hex(ai), hex(mi), ci)


def test_adc_decimal_all_inputs_clark(adc):
    a, m, c, d, ao, po = adc
    sel = d == 1
    for ai, mi, ci, aoi, poi in zip(a[sel], m[sel], c[sel], ao[sel], po[sel]):
        res, carry, n, v = clark_adc(int(ai), int(mi), int(ci))
        assert aoi == res and (poi & C) == carry
        assert bool(poi & N) == bool(n) and bool(poi & V) == bool(v)
        assert bool(poi & Z) == (((ai + mi + ci) & 0xFF) == 0)


def test_sbc_decimal_all_inputs_clark(sbc):
    a, m, c, d, ao, po = sbc
    sel = d == 1
    for ai, mi, ci, aoi, poi in zip(a[sel], m[sel], c[sel], ao[sel], po[sel]):
        s = int(ai) - int(mi) - (1 - int(ci))
        assert aoi == clark_sbc(int(ai), int(mi), int(ci))
        assert (poi & C) == int(s >= 0) and bool(poi & Z) == ((s & 0xFF) == 0)
        assert bool(poi & N) == bool(s & 0x80)


# ------------------------------------------------------------ cycle matrix

def golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        op, mn, mode, nbytes, cyc = line.split()
        rows.append((int(op, 16), mn, mode, int(nbytes), cyc))
    return rows


ROWS = golden_rows()


def test_golden_has_151_opcodes():
    assert len(ROWS) == 151 and len({r[0] for r in ROWS}) == 151


BRANCH_FLAGS = {"BPL": (N, 0), "BMI": (N, 1), "BVC": (V, 0), "BVS": (V, 1),
                "BCC": (C, 0), "BCS": (C, 1), "BNE": (Z, 0), "BEQ": (Z, 1)}


def _exec_one(code, at=0x1000, **state):
    rom = bytearray([0xEA] * 4096)
    off = at - 0x1000
    rom[off:off + len(code)] = bytes(code)
    rom[0xFFC:0xFFE] = bytes([at & 0xFF, at >> 8])
    rom[0xFFE:0x1000] = bytes([0x00, 0x15])            # BRK vector -> $1500
    st = oracle.power_on(bytes(rom))
    st = set_fields(st, **state)
    out, n = oracle.run_instructions(st, bytes(rom), 1)
    assert n == 1
    return decode(out)


def _operands(mode, cross):
    """operand bytes and machine state for a mode; `cross` forces a page cross."""
    ram = {0x80: 0x80, 0x81: 0x01, 0x82: 0xF0 if cross else 0x80, 0x83: 0x01}
    st = dict(ram=ram, x=0x20 if cross else 0, y=0x20 if cross else 0)
    if mode in ("zp", "zpx", "zpy"):
        return [0x80], st
    if mode == "abs":
        return [0x80, 0x01], st
    if mode in ("absx", "absy"):
        return ([0xF0, 0x01] if cross else [0x80, 0x01]), st
    if mode == "indx":
        st["x"] = 0
        return [0x80], st
    if mode == "indy":
        return [0x82], st
    if mode == "imm":
        return [0x01], st
    return [], st


@pytest.mark.parametrize("row", ROWS, ids=[f"{r[1]}_{r[2]}" for r in ROWS])
def test_cycle_matrix(row):
    op, mn, mode, nbytes, cyc = row
    if mode == "rel":
        flag, want = BRANCH_FLAGS[mn]
        p_not = 0x20 | (0 if want else flag)
        p_yes = 0x20 | (flag if want else 0)
        d = _exec_one([op, 0x10], p=p_not)
        assert d["cycle"] == 2 and d["pc"] == 0x1002
        d = _exec_one([op, 0x10], p=p_yes)
        assert d["cycle"] == 3 and d["pc"] == 0x1012
        d = _exec_one([op, 0x20], at=0x10F0, p=p_yes)
        assert d["cycle"] == 4 and d["pc"] == 0x1112
        return
    base = int(cyc.split("+")[0])
    if mn in ("JMP", "JSR"):
        d = _exec_one([op, 0x80, 0x01] if mode == "ind" else [op, 0x34, 0x12], ram={0x80: 0x78, 0x81: 0x16})
        assert d["cycle"] == base
        assert d["pc"] == (0x1678 if mode == "ind" else 0x1234)
        return
    if mn == "RTS":
        d = _exec_one([op], sp=0xFD, ram={0xFE: 0x33, 0xFF: 0x12})
        assert d["cycle"] == base and d["pc"] == 0x1234
        return
    if mn == "RTI":
        d = _exec_one([op], sp=0xFC, ram={0xFD: 0x00, 0xFE: 0x34, 0xFF: 0x12})
        assert d["cycle"] == base and d["pc"] == 0x1234
        return
    if mn == "BRK":
        d = _exec_one([op])
        assert d["cycle"] == base and d["pc"] == 0x1500
        return
    opnd, st = _operands(mode, cross=False)
    d = _exec_one([op] + opnd, **st)
    assert d["cycle"] == base, (mn, mode, d["cycle"])
    assert d["pc"] == 0x1000 + nbytes
    if mode in ("absx", "absy", "indy"):
        opnd, st = _operands(mode, cross=True)
        d = _exec_one([op] + opnd, **st)
        assert d["cycle"] == base + (1 if cyc.endswith("+p") else 0), (mn, mode, "cross")


def test_every_opcode_is_documented_or_in_the_undocumented_table():
    undoc = {int(line.split()[0], 16) for line in open(GOLDEN_UNDOC) if line.strip() and not line.startswith("#")}
    documented = {r[0] for r in ROWS}
    assert len(undoc) == 105 and not (undoc & documented) and (undoc | documented) == set(range(256))


def test_assembler_encodings_match_golden():
    from paper_1907_08467_amd.inputs.asm6502 import OPCODES
    table = {(mn.lower(), mode): op for op, mn, mode, _, _ in ROWS}
    ours = {(mn, mode): op for mn, modes in OPCODES.items() for mode, op in modes.items()}
    assert ours == table
