"""Exhaustive ADC, SBC, RRA and ISC tables on the GPU against the oracle.

Every env of one cartridge computes one row of a table: its RAM holds the
accumulator A, the carry C, the decimal flag D and the operation (ADC zp,
SBC zp, RRA zp = ROR + ADC, ISC zp = INC + SBC); each frame it applies the
operation to 32 memory operands M and stores the 32 results and the 32 flag
bytes (PHP) in RAM, so eight frames cover M = 0..255.  4096 envs cover all
(A, C, D, operation): 256 x 2 x 2 x 4 rows x 256 operands = 1,048,576 cases,
compared element by element through the full machine-state records after
every frame.

The first assignment gives the 64 envs of a wave the same operation, C and D
(and 64 values of A), so the wave runs on the wave-uniform path (ADC and SBC
in its binary or decimal form for the whole wave; RRA and ISC on the
per-lane path, which takes every undocumented opcode).  The second mixes all
16 (operation, C, D) combinations in every wave, so the lanes stand at
different places and the per-lane executor takes the arithmetic.
"""
import sys

import numpy as np
import pytest

from helpers import cart, diff_records
from parity import make_pair

pytestmark = pytest.mark.gpu

IN_A, IN_C, IN_D, IN_OP, FRAME, BASE, OPND = 0xC0, 0xC1, 0xC2, 0xC3, 0xC5, 0xC6, 0xC7
RES, FLG = 0x80, 0xA0        # 32 results, 32 flag bytes


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def table_rom():
    def op_path(name, insn):
        return f"""
{name}:
    lda ${IN_D:02X}
    beq {name}_b
    sed
    jmp {name}_d
{name}_b:
    cld
{name}_d:
    lda ${IN_C:02X}
    beq {name}_nc
    sec
    jmp {name}_c
{name}_nc:
    clc
{name}_c:
    lda ${IN_A:02X}
    {insn} ${OPND:02X}
    jmp store
"""
    src = f"""
reset:
    ldx #$FF
    txs
frame:
    lda #2
    sta VSYNC
    lda #0
    sta VSYNC
    lda ${FRAME:02X}
    and #7
    asl
    asl
    asl
    asl
    asl
    sta ${BASE:02X}
    ldx #0
loop:
    txa
    ora ${BASE:02X}
    sta ${OPND:02X}
    lda ${IN_OP:02X}
    beq do_adc
    cmp #1
    beq do_sbc_j
    cmp #2
    beq do_rra_j
    jmp do_isc
do_sbc_j:
    jmp do_sbc
do_rra_j:
    jmp do_rra
{op_path("do_adc", "adc")}
{op_path("do_sbc", "sbc")}
{op_path("do_rra", "rra")}
{op_path("do_isc", "isc")}
store:
    sta ${RES:02X},x
    php
    pla
    sta ${FLG:02X},x
    cld
    inx
    cpx #32
    beq done
    jmp loop
done:
    inc ${FRAME:02X}
    jmp frame
"""
    rom, _ = cart(src)
    return rom


def assignments(kind):
    e = np.arange(4096)
    if kind == "uniform":
        combo, a = e // 256, e % 256
    else:
        combo, a = e % 16, e // 16
    return a, combo // 4, combo % 2, (combo // 2) % 2     # A, operation, C, D


@pytest.mark.parametrize("kind", ["uniform", "mixed"])
def test_alu_tables(kind):
    import torch
    rom = table_rom()
    n = 4096
    say(f"case: ALU tables, {kind} waves, {n} envs")
    o, g = make_pair([(rom, 0)], np.zeros(n, np.uint16), seed=1, frameskip=1, render_mode=1)
    a, op, cin, dec = assignments(kind)
    for env in range(n):
        rec = o.get_state(env)
        assert np.array_equal(rec, g.get_state(env)), f"env {env} differs before the tables"
        rec = rec.copy()
        ram = rec[32:160]
        ram[:] = 0
        ram[IN_A - 0x80], ram[IN_C - 0x80], ram[IN_D - 0x80], ram[IN_OP - 0x80] = a[env], cin[env], dec[env], op[env]
        o.set_state(env, rec)
        g.set_state(env, rec)
    zero = np.zeros(n, np.uint8)
    for frame in range(8):
        go, gr, gd, _ = g.step(torch.from_numpy(zero).cuda(), want_obs=False)
        _, orr, od, _ = o.step(zero, render=False)
        torch.cuda.synchronize()
        assert np.array_equal(gd.cpu().numpy(), od) and not od.any(), f"frame {frame}: done flags"
        if kind == "uniform" and frame == 0:
            instr, uni = g.last_step_stats()
            frac = uni / instr
            say(f"wave-uniform fraction of the first frame: {frac:.3f}")
            assert frac > 0.5
        for env in range(n):
            ga, ob = g.get_state(env), o.get_state(env)
            assert np.array_equal(ga, ob), (f"{kind}: frame {frame} env {env} (A={a[env]} op={op[env]} C={cin[env]} "
                                            f"D={dec[env]}): {diff_records(ga, ob)}")
    assert g.poll_errors() == o.poll_errors()
    g.close()
    o.close()
