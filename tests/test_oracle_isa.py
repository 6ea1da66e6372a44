"""Pins of the oracle's 6507 core against the MOS 6502 definition.

Every expected value below is derived by hand from the MOS MCS6500
programming manual (instruction semantics, flag rules, cycle counts), not by
running the oracle.  These programs cover every addressing mode, the stack,
subroutines, BRK/RTI, the JMP ($xxFF) page bug, branch timing, the RIOT
timer, F8 bank switching, WSYNC and the input ports.
"""
import numpy as np
import pytest

import oracle
from helpers import cart, decode, set_fields
from paper_1907_08467_amd.inputs.asm6502 import assemble

N, V, U, B, D, I, Z, C = 0x80, 0x40, 0x20, 0x10, 0x08, 0x04, 0x02, 0x01


def run(src, n, action=0, state_kw=None, banks=1, scheme=0):
    rom, syms = cart(src, banks=banks)
    st = oracle.power_on(rom, scheme)
    if state_kw:
        st = set_fields(st, **state_kw)
    st2, done = oracle.run_instructions(st, rom, n, scheme=scheme, action=action)
    return decode(st2), done, syms


def test_power_on_state():
    rom, _ = cart("reset:\n    nop\n")
    d = decode(oracle.power_on(rom))
    assert (d["a"], d["x"], d["y"], d["sp"], d["p"], d["pc"], d["cycle"]) == (0, 0, 0, 0xFD, 0x24, 0x1000, 0)
    assert d["interval"] == 1024 and d["intim"] == 0 and d["expired"] == 0
    assert not d["ram"].any()


def test_loads_transfers_flags():
    d, n, _ = run("""
reset:
    lda #$80
    ldx #$00
    ldy #$7F
    tax
    tya
    tsx
""", 6)
    assert n == 6
    assert (d["a"], d["x"], d["y"], d["sp"]) == (0x7F, 0xFD, 0x7F, 0xFD)
    assert d["p"] == 0x24 | N
    assert d["pc"] == 0x1009 and d["cycle"] == 12


def test_adc_sbc_binary_flags():
    d, _, _ = run("reset:\n    clc\n    lda #$50\n    adc #$50\n", 3)
    assert d["a"] == 0xA0 and d["p"] == 0x24 | N | V and d["cycle"] == 6
    d, _, _ = run("reset:\n    sec\n    lda #$FF\n    adc #$00\n", 3)
    assert d["a"] == 0x00 and d["p"] == 0x24 | C | Z
    d, _, _ = run("reset:\n    sec\n    lda #$50\n    sbc #$F0\n", 3)
    assert d["a"] == 0x60 and d["p"] == 0x24
    d, _, _ = run("reset:\n    sec\n    lda #$50\n    sbc #$B0\n", 3)
    assert d["a"] == 0xA0 and d["p"] == 0x24 | N | V


def test_decimal_examples():
    d, _, _ = run("reset:\n    sed\n    clc\n    lda #$19\n    adc #$28\n", 4)
    assert d["a"] == 0x47 and not d["p"] & C
    d, _, _ = run("reset:\n    sed\n    sec\n    lda #$50\n    sbc #$01\n", 4)
    assert d["a"] == 0x49 and d["p"] & C
    # 99 + 01: A = 00, C = 1; NMOS takes Z from the binary sum $9A and N from
    # the intermediate $A0 of the decimal adjustment
    d, _, _ = run("reset:\n    sed\n    clc\n    lda #$99\n    adc #$01\n", 4)
    assert d["a"] == 0x00 and d["p"] == 0x24 | D | C | N


def test_addressing_modes_and_page_cross():
    src = """
reset:
    ldx #$20
    lda $18F0,x
    sta $80
    ldy #$01
    lda $1800,y
    sta $81
    lda #$10
    sta $82
    lda #$19
    sta $83
    ldx #$02
    lda ($80,x)
    sta $84
    ldy #$F0
    lda ($82),y
    sta $85
    .org $1800
    .byte $11, $C3
    .org $1910
    .byte $5A
    .org $1A00
    .byte $77
"""
    d, n, _ = run(src, 16)
    assert n == 16
    assert list(d["ram"][:6]) == [0x5A, 0xC3, 0x10, 0x19, 0x5A, 0x77]
    # 2 + (4+1) + 3 + 2 + 4 + 3 + 2 + 3 + 2 + 3 + 2 + 6 + 3 + 2 + (5+1) + 3
    assert d["cycle"] == 51
    assert d["pc"] == 0x1022 and d["a"] == 0x77 and d["p"] == 0x24


def test_zero_page_indexed():
    d, _, _ = run("""
reset:
    ldx #$05
    lda #$AA
    sta $80,x
    ldy #$03
    ldx $82,y
""", 5)
    assert d["ram"][5] == 0xAA and d["x"] == 0xAA and d["p"] == 0x24 | N
    assert d["cycle"] == 2 + 2 + 4 + 2 + 4


def test_stack_jsr_rts():
    d, n, _ = run("""
reset:
    ldx #$FF
    txs
    lda #$42
    pha
    php
    jsr sub
    lda #$01
    plp
    pla
sub:
    lda #$99
    rts
""", 11)
    # order: ldx txs lda pha php jsr | lda#$99 rts | lda#$01 plp pla
    assert d["a"] == 0x42 and d["sp"] == 0xFF and d["p"] == 0x24
    assert d["ram"][0x7F] == 0x42 and d["ram"][0x7E] == 0x34
    assert d["ram"][0x7D] == 0x10 and d["ram"][0x7C] == 0x09   # JSR at $1007 pushes $1009
    assert d["cycle"] == 2 + 2 + 2 + 3 + 3 + 6 + 2 + 6 + 2 + 4 + 4
    assert d["pc"] == 0x100E


def test_brk_rti():
    src = """
reset:
    ldx #$FF
    txs
    sed
    brk
    .byte $EA
    lda #$55
handler:
    cld
    rti
    .org $1FFC
    .word reset
    .word handler
"""
    d, n, _ = run(src, 7)
    assert d["a"] == 0x55 and d["p"] == 0x2C and d["sp"] == 0xFF
    assert list(d["ram"][0x7D:0x80]) == [0xBC, 0x06, 0x10]     # P = N|U|D|I after LDX #$FF, SED
    assert d["cycle"] == 2 + 2 + 2 + 7 + 2 + 6 + 2
    assert d["pc"] == 0x1008


def test_jmp_indirect_page_bug():
    src = """
reset:
    sei
    jmp ($10FF)
    .org $10FF
    .byte $34
    .org $1100
    .byte $12
    .org $1234
    lda #$11
    .org $1834
    lda #$99
"""
    # the pointer's high byte comes from $1000 (the SEI opcode, $78), not $1100
    d, _, _ = run(src, 3)
    assert d["a"] == 0x99 and d["pc"] == 0x7836 and d["cycle"] == 2 + 5 + 2


def test_branch_timing():
    src = """
reset:
    ldx #$00
    bne reset
    beq near
    nop
near:
    jmp $10FA
    .org $10FA
    ldy #$01
    bne ahead
    .org $1102
ahead:
    lda #$33
"""
    d, _, _ = run(src, 7)
    assert d["a"] == 0x33 and d["pc"] == 0x1104
    assert d["cycle"] == 2 + 2 + 3 + 3 + 2 + 4 + 2


def test_compare_bit_shifts_incdec():
    d, _, _ = run("""
reset:
    lda #$C0
    sta $80
    lda #$40
    cmp #$41
    bit $80
""", 5)
    assert d["p"] == 0x24 | N | V
    d, _, _ = run("""
reset:
    lda #$81
    asl
    ror
    lsr
    rol
""", 5)
    assert d["a"] == 0x81 and d["p"] == 0x24 | N
    d, _, _ = run("""
reset:
    lda #$FF
    sta $80
    inc $80
    ldx $80
    dec $80
""", 5)
    assert d["ram"][0] == 0xFF and d["x"] == 0 and d["p"] == 0x24 | N
    assert d["cycle"] == 2 + 3 + 5 + 3 + 5


def test_undocumented_opcode_faults():
    rom, _ = cart("reset:\n    nop\n    .byte $02\n")
    st, n = oracle.run_instructions(oracle.power_on(rom), rom, 5)
    d = decode(st)
    assert n == 1 and d["err"] == oracle.ERR_ILLEGAL and d["pc"] == 0x1001 and d["cycle"] == 2


ACTION_PORTS = [  # (SWCHA, INPT4) for the 18 actions, ALE order
    (0xFF, 0x80), (0xFF, 0x00), (0xEF, 0x80), (0x7F, 0x80), (0xBF, 0x80), (0xDF, 0x80),
    (0x6F, 0x80), (0xAF, 0x80), (0x5F, 0x80), (0x9F, 0x80),
    (0xEF, 0x00), (0x7F, 0x00), (0xBF, 0x00), (0xDF, 0x00), (0x6F, 0x00), (0xAF, 0x00),
    (0x5F, 0x00), (0x9F, 0x00)]


@pytest.mark.parametrize("action", range(18))
def test_input_ports(action):
    d, _, _ = run("""
reset:
    lda SWCHA
    sta $80
    lda INPT4
    sta $81
    lda SWCHB
    sta $82
    lda INPT5
    sta $83
    lda $0281
    sta $84
""", 10, action=action)
    assert (d["ram"][0], d["ram"][1]) == ACTION_PORTS[action]
    assert d["ram"][2] == 0x0B and d["ram"][3] == 0x80 and d["ram"][4] == 0


def timer_closed_form(t, w, v, n):
    """INTIM / TIMINT of a read at cycle t after TIMnT <- v written at cycle w."""
    e = t - w - 1
    if e < (v + 1) * n:
        return v - e // n, 0x00
    return (0xFF - (e - (v + 1) * n)) & 0xFF, 0x80


@pytest.mark.parametrize("v,reg,n", [(3, "TIM8T", 8), (1, "TIM1T", 1), (2, "TIM64T", 64), (0, "T1024T", 1024)])
def test_timer_against_closed_form(v, reg, n):
    src = f"""
reset:
    lda #${v:02X}
    sta {reg}
    ldx #$00
loop:
    lda INTIM
    sta $80,x
    lda TIMINT
    sta $A0,x
    inx
    cpx #$10
    bne loop
"""
    d, _, _ = run(src, 3 + 16 * 7)
    w = 5                                  # lda #v (0-1), sta abs (2-5)
    for i in range(16):
        start = 8 + 23 * i                 # loop body: 4 + 4 + 4 + 4 + 2 + 2 + 3 cycles
        intim, _ = timer_closed_form(start + 3, w, v, n)
        _, timint = timer_closed_form(start + 8 + 3, w, v, n)
        assert d["ram"][i] == intim, (i, d["ram"][i], intim)
        assert d["ram"][0x20 + i] == timint, (i, d["ram"][0x20 + i], timint)


def test_timer_runs_through_wsync():
    d, _, _ = run("""
reset:
    lda #$10
    sta TIM64T
    sta WSYNC
    lda INTIM
    sta $80
""", 5)
    # write at 5; WSYNC written at 8 resumes at 76; LDA INTIM reads at 79
    assert d["ram"][0] == timer_closed_form(79, 5, 0x10, 64)[0] == 15


@pytest.mark.parametrize("k,expect", [(36, 76), (37, 152)])
def test_wsync_resume(k, expect):
    # k NOPs (2 cycles each) then STA WSYNC (3 cycles, write on its last)
    d, _, _ = run("reset:\n" + "    nop\n" * k + "    sta WSYNC\n", k + 1)
    assert d["cycle"] == expect


def test_wsync_on_last_cycle_of_line():
    # 35 NOPs + LDA zp (3): STA WSYNC starts at 73 and writes at 75 -> 76
    d, _, _ = run("reset:\n" + "    nop\n" * 35 + "    lda $80\n    sta WSYNC\n", 37)
    assert d["cycle"] == 76


def test_f8_switch_then_read():
    src = """
    .bank 1
    .org $1000
    lda $1FF8
    lda #$B1
    sta $80
    lda $1FF9
    lda #$C1
    sta $81
    .org $1FF8
    .byte $D8, $D9
    .word $1000, $1000, $1000
    .bank 0
    .org $1000
    lda $1FF8
    lda #$B0
    sta $80
    lda $1FF9
    lda #$C0
    sta $81
    .org $1FF8
    .byte $E0, $E9
    .word $1000, $1000, $1000
"""
    rom = assemble(src, banks=2)
    st0 = oracle.power_on(rom, 1)
    assert decode(st0)["bank"] == 1
    st, _ = oracle.run_instructions(st0, rom, 1, scheme=1)
    d = decode(st)
    assert d["bank"] == 0 and d["a"] == 0xE0          # switched first, then read bank 0
    st, _ = oracle.run_instructions(st0, rom, 6, scheme=1)
    d = decode(st)
    assert d["ram"][0] == 0xB0 and d["ram"][1] == 0xC1 and d["bank"] == 1


def test_f8_write_hotspot():
    src = """
    .bank 1
    .org $1000
    sta $1FF8
    lda #$B1
    .org $1FFA
    .word $1000, $1000, $1000
    .bank 0
    .org $1000
    sta $1FF8
    lda #$B0
    .org $1FFA
    .word $1000, $1000, $1000
"""
    rom = assemble(src, banks=2)
    st, _ = oracle.run_instructions(oracle.power_on(rom, 1), rom, 2, scheme=1)
    d = decode(st)
    assert d["bank"] == 0 and d["a"] == 0xB0
