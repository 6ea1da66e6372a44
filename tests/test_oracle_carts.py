"""Pins of the oracle's cartridge schemes, each against the scheme's
definition (hotspot addresses, slice layout, Superchip RAM ports): every
expected byte below is the tag the test wrote into the ROM image at the
place the definition says the access must reach.

Scheme numbers: 0 4K (2 or 4 KB), 1 F8, 2 F6, 3 F4, 4-6 their Superchip
forms, 7 E0, 8 3F.
"""
import numpy as np
import pytest

import oracle
from helpers import decode, set_fields
from paper_1907_08467_amd.inputs.asm6502 import assemble

F8, F6, F4, F8SC, F6SC, F4SC, E0, TF = 1, 2, 3, 4, 5, 6, 7, 8


def run_bytes(rom, scheme, code, n, bank=None, pc=None, **state):
    """Put `code` at the reset address of every 4 KB bank image position
    $1100 (linear schemes) and run n instructions."""
    st = oracle.power_on(bytes(rom), scheme)
    kw = dict(state)
    if bank is not None:
        kw["bank"] = bank
    if pc is not None:
        kw["pc"] = pc
    st = set_fields(st, **kw)
    out, done = oracle.run_instructions(st, bytes(rom), n, scheme=scheme)
    return decode(out), done


def linear_rom(n_banks, code, at=0x1100):
    """n_banks x 4 KB: the same code at `at` in every bank, tag byte b at
    $1800 + 0 of bank b, reset vector -> at."""
    rom = bytearray([0xEA] * (4096 * n_banks))
    for b in range(n_banks):
        base = b * 4096
        rom[base + at - 0x1000: base + at - 0x1000 + len(code)] = bytes(code)
        rom[base + 0x800] = 0xB0 + b
        rom[base + 0xFFC: base + 0xFFE] = bytes([at & 0xFF, at >> 8])
    return rom


@pytest.mark.parametrize("scheme,nb,first", [(F8, 2, 0xFF8), (F6, 4, 0xFF6), (F4, 8, 0xFF4),
                                             (F8SC, 2, 0xFF8), (F6SC, 4, 0xFF6), (F4SC, 8, 0xFF4)])
def test_linear_hotspots(scheme, nb, first):
    # power-on in the last bank
    rom = linear_rom(nb, [0xAD, 0x00, 0x18])             # LDA $1800
    d, _ = run_bytes(rom, scheme, None, 1)
    assert d["bank"] == nb - 1 and d["a"] == 0xB0 + nb - 1
    for b in range(nb):
        hs = 0x1000 | (first + b)
        # a read of the hotspot switches first, then reads the new bank
        code = [0xAD, hs & 0xFF, hs >> 8, 0xAD, 0x00, 0x18]  # LDA hotspot; LDA $1800
        rom = linear_rom(nb, code)
        for i in range(nb):                                  # hotspot bytes of bank i hold $F0 + i
            rom[i * 4096 + first: i * 4096 + first + nb] = bytes([0xF0 + i] * nb)
        d, _ = run_bytes(rom, scheme, None, 2)
        assert d["bank"] == b and d["a"] == 0xB0 + b
        d1, _ = run_bytes(rom, scheme, None, 1)
        assert d1["a"] == 0xF0 + b                           # read from the bank it selected
        # a write to the hotspot switches too
        code = [0x8D, hs & 0xFF, hs >> 8, 0xAD, 0x00, 0x18]  # STA hotspot; LDA $1800
        d, _ = run_bytes(linear_rom(nb, code), scheme, None, 2)
        assert d["bank"] == b and d["a"] == 0xB0 + b
    # the addresses just outside the hotspot range do nothing
    for a in (first - 1, first + nb):
        hs = 0x1000 | a
        d, _ = run_bytes(linear_rom(nb, [0xAD, hs & 0xFF, hs >> 8]), scheme, None, 1)
        assert d["bank"] == nb - 1


@pytest.mark.parametrize("scheme,nb", [(F8SC, 2), (F6SC, 4), (F4SC, 8)])
def test_superchip_ram(scheme, nb):
    src_code = [0xA9, 0x5A,              # LDA #$5A
                0x8D, 0x10, 0x10,        # STA $1010   (write port)
                0xAD, 0x90, 0x10,        # LDA $1090   (read port: $5A)
                0xAA,                    # TAX
                0xAD, 0x10, 0x10,        # LDA $1010   (the write port reads 0)
                0xA8,                    # TAY
                0xA9, 0x77,              # LDA #$77
                0x8D, 0x91, 0x10,        # STA $1091   (a write to the read port does nothing)
                0xAD, 0x91, 0x10]        # LDA $1091
    rom = linear_rom(nb, src_code)
    d, done = run_bytes(rom, scheme, None, 9)
    assert done == 9
    assert d["x"] == 0x5A and d["y"] == 0x00 and d["a"] == 0x00
    assert d["xram"][0x10] == 0x5A and d["xram"][0x11] == 0 and d["xram"].sum() == 0x5A
    # without the Superchip the same program reads ROM
    plain = {F8SC: F8, F6SC: F6, F4SC: F4}[scheme]
    d, _ = run_bytes(rom, plain, None, 3)
    assert d["a"] == rom[(nb - 1) * 4096 + 0x090] and not d["xram"].any()


def test_superchip_ram_survives_a_state_round_trip_and_fetch_sees_rom():
    rom = linear_rom(2, [0xA9, 0x33, 0x8D, 0x7F, 0x10, 0x4C, 0x7F, 0x10])   # LDA #$33; STA $107F; JMP $107F
    rom[4096 + 0x07F: 4096 + 0x081] = bytes([0xA2, 0x44])                    # ROM at $107F: LDX #$44
    d, _ = run_bytes(rom, F8SC, None, 4)
    assert d["xram"][0x7F] == 0x33 and d["x"] == 0x44                       # fetched the ROM, not the RAM
    st = oracle.power_on(bytes(rom), F8SC)
    st, _ = oracle.run_instructions(st, bytes(rom), 2, scheme=F8SC)
    st2, _ = oracle.run_instructions(st.copy(), bytes(rom), 0, scheme=F8SC)
    assert np.array_equal(st, st2) and decode(st)["xram"][0x7F] == 0x33


def e0_rom():
    """8 x 1 KB slices; byte 0 of slice s is $C0 + s, byte 1 is $D0 + s."""
    rom = bytearray([0xEA] * 8192)
    for s in range(8):
        rom[s * 1024] = 0xC0 + s
        rom[s * 1024 + 1] = 0xD0 + s
    return rom


def test_e0_segments():
    rom = e0_rom()
    # code in segment 3 (fixed slice 7) at $1C10; reset vector there
    code = [0xAD, 0x00, 0x10,      # LDA $1000 (segment 0)
            0xAA,                  # TAX
            0xAD, 0x00, 0x14,      # LDA $1400 (segment 1)
            0xA8,                  # TAY
            0xAD, 0x00, 0x18]      # LDA $1800 (segment 2)
    rom[7 * 1024 + 0x10: 7 * 1024 + 0x10 + len(code)] = bytes(code)
    rom[8190 - 2: 8190] = bytes([0x10, 0x1C])            # $1FFC -> $1C10
    d, _ = run_bytes(rom, E0, None, 5)
    assert d["bank"] == 4 | (5 << 3) | (6 << 6)
    assert (d["x"], d["y"], d["a"]) == (0xC4, 0xC5, 0xC6)  # power-on slices 4, 5, 6
    # select slice n into segment k with an access to $1FE0 + 8k + n, then read the segment
    for k in range(3):
        for n in range(8):
            hs = 0x1FE0 + 8 * k + n
            prog = [0xAD, hs & 0xFF, hs >> 8, 0xAD, 0x00, 0x10 + 4 * k]
            r = bytearray(rom)
            r[7 * 1024 + 0x10: 7 * 1024 + 0x10 + len(prog)] = bytes(prog)
            d, _ = run_bytes(r, E0, None, 2)
            assert d["a"] == 0xC0 + n, (k, n)
            assert (d["bank"] >> (3 * k)) & 7 == n
    # segment 3 always shows slice 7
    prog = [0xAD, 0xE0, 0x1F, 0xAD, 0x00, 0x1C]
    r = bytearray(rom)
    r[7 * 1024 + 0x10: 7 * 1024 + 0x10 + len(prog)] = bytes(prog)
    d, _ = run_bytes(r, E0, None, 2)
    assert d["a"] == 0xC7


def test_e0_instruction_across_segments():
    """LDA abs at $1BFE: opcode and low byte from segment 2's slice, the high
    byte from segment 3 (slice 7)."""
    rom = e0_rom()
    for s in range(7):
        rom[s * 1024 + 0x3FE: s * 1024 + 0x400] = bytes([0xAD, 0x20 + s])   # LDA $??(20+s)
    rom[7 * 1024] = 0x1E                                                     # high byte: $1E
    rom[7 * 1024 + 0x220: 7 * 1024 + 0x228] = bytes(range(0x60, 0x68))     # $1E20.. in slice 7
    d, _ = run_bytes(rom, E0, None, 1, pc=0x1BFE)                            # segment 2 = slice 6
    assert d["a"] == 0x60 + 6 and d["pc"] == 0x1C01


def tf_rom(size):
    """2 KB slices; byte 0 of slice s is $A0 + s; code in the last slice."""
    rom = bytearray([0xEA] * size)
    for s in range(size // 2048):
        rom[s * 2048] = 0xA0 + s
    return rom


@pytest.mark.parametrize("size", [4096, 8192, 16384, 32768])
def test_3f_slices(size):
    S = size // 2048
    rom = tf_rom(size)
    last = size - 2048
    for v in (0, 1, S - 1, S, 0x3F, 0xFF):
        prog = [0xA9, v,               # LDA #v
                0x85, 0x3F,            # STA $3F   (selects slice v mod S; also a TIA write)
                0xAD, 0x00, 0x10,      # LDA $1000 (lower half)
                0xAA,                  # TAX
                0xAD, 0x00, 0x18]      # LDA $1800 (upper half: the last slice)
        r = bytearray(rom)
        r[last + 0x100: last + 0x100 + len(prog)] = bytes(prog)
        r[size - 4: size - 2] = bytes([0x00, 0x19])        # $1FFC -> $1900
        d, _ = run_bytes(r, TF, None, 5)
        assert d["bank"] == v % S and d["x"] == 0xA0 + v % S and d["a"] == 0xA0 + S - 1
    # power-on slice 0; a write to a mirror ($7F) or a read of $3F selects nothing
    prog = [0xA9, 1, 0x85, 0x7F, 0xA5, 0x3F, 0xAD, 0x00, 0x10]
    r = bytearray(rom)
    r[last + 0x100: last + 0x100 + len(prog)] = bytes(prog)
    r[size - 4: size - 2] = bytes([0x00, 0x19])
    d, _ = run_bytes(r, TF, None, 4)
    assert d["bank"] == 0 and d["a"] == 0xA0


def test_2k_rom_is_mirrored():
    rom = bytearray([0xEA] * 2048)
    rom[0x100] = 0x5C
    rom[0x7FC:0x7FE] = bytes([0x00, 0x18])                     # reset vector at $1FFC = $17FC mirrored
    prog = [0xAD, 0x00, 0x11, 0xAA, 0xAD, 0x00, 0x19]          # LDA $1100; TAX; LDA $1900
    rom[0x000:len(prog)] = bytes(prog)
    d, _ = run_bytes(rom, 0, None, 3)
    assert d["pc"] == 0x1807 and d["x"] == 0x5C and d["a"] == 0x5C


def test_rom_sizes_checked():
    for size, scheme in [(8192, 0), (4096, F8), (8192, F6), (16384, F4), (4096, E0), (2048, TF), (6144, TF)]:
        with pytest.raises(RuntimeError):
            oracle.power_on(bytes(size), scheme)
