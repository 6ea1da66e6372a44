"""Pins of the oracle's fuller TIA: NUSIZ copies and widths, missiles, the
ball, vertical delay, RESMP, HMOVE of every object and its blank, priority
with missiles and ball, and the collision latches.  Every expected pixel and
latch is derived by hand from the register definitions and the timing
conventions: a write at access cycle c takes effect at colour clock
3(c+1); a player reset at clock h >= 68 lands at h - 68 + 5, a missile or
ball reset at h - 68 + 4; frame row r is scanline 34 + r.
"""
import numpy as np
import pytest

import oracle
from helpers import cart, decode

ROW = 60                                   # a visible row every test looks at


def rom_with(setup, per_frame_end=""):
    """`setup` runs once on a line of its own (after a WSYNC, so its first
    instruction starts at cycle 0); frames are 1 + 255 WSYNC lines, then
    `per_frame_end` runs in the VSYNC line."""
    src = f"""
reset:
    sta WSYNC
{setup}
frame:
    sta WSYNC
    lda #2
    sta VSYNC
    lda #0
    sta VSYNC
{per_frame_end}
    ldx #0
lines:
    sta WSYNC
    dex
    bne lines
    jmp frame
"""
    rom, _ = cart(src)
    return rom


def run(rom, n=3, track=False):
    st = oracle.power_on(rom)
    st[230] = 1 if track else 0
    st, frames, ends, got = oracle.run_frames(st, rom, n, actions=np.zeros(n, np.uint8))
    assert got == n and decode(st)["err"] == 0
    return frames[-1], decode(st)


def lit(row):
    return set(np.nonzero(row)[0].tolist())


# 20 NOPs after the WSYNC: the next store's access cycle is 40 + 2 = 42 ->
# clock 129 -> player position 66, missile / ball position 65
AT42 = "    nop\n" * 20


@pytest.mark.parametrize("mode,want", [(0, {66}), (1, {66, 82}), (2, {66, 98}), (3, {66, 82, 98}),
                                       (4, {66, 130}), (5, {66, 67}), (6, {66, 98, 130}),
                                       (7, {66, 67, 68, 69})])
def test_player_copies_and_widths(mode, want):
    f, _ = run(rom_with(f"    lda #${mode:02X}\n    sta NUSIZ0\n    lda #$80\n    sta GRP0\n"
                        f"    lda #$36\n    sta COLUP0\n    sta WSYNC\n" + AT42 + "    sta RESP0"))
    assert lit(f[ROW]) == want and f[ROW][66] == 0x36


@pytest.mark.parametrize("nusiz,want", [(0x00, {65}), (0x10, {65, 66}), (0x20, set(range(65, 69))),
                                        (0x30, set(range(65, 73))), (0x11, {65, 66, 81, 82}),
                                        (0x05, {65}), (0x16, {65, 66, 97, 98, 129, 130})])
def test_missile_sizes_and_copies(nusiz, want):
    f, _ = run(rom_with(f"    lda #${nusiz:02X}\n    sta NUSIZ0\n    lda #2\n    sta ENAM0\n"
                        f"    lda #$36\n    sta COLUP0\n    sta WSYNC\n" + AT42 + "    sta RESM0"))
    assert lit(f[ROW]) == want and f[ROW][65] == 0x36


@pytest.mark.parametrize("ctrlpf,want", [(0x00, {65}), (0x10, {65, 66}), (0x20, set(range(65, 69))),
                                         (0x30, set(range(65, 73)))])
def test_ball_sizes_in_playfield_colour(ctrlpf, want):
    f, _ = run(rom_with(f"    lda #${ctrlpf | 2:02X}\n    sta CTRLPF\n    lda #2\n    sta ENABL\n"
                        f"    lda #$44\n    sta COLUPF\n    lda #$36\n    sta COLUP0\n    sta WSYNC\n" + AT42 +
                        "    sta RESBL"))
    # score mode (CTRLPF D1) colours the playfield, not the ball
    assert lit(f[ROW]) == want and f[ROW][65] == 0x44


def test_vertical_delay():
    base = "    lda #1\n    sta VDELP0\n    lda #$FF\n    sta GRP0\n    lda #$36\n    sta COLUP0\n" \
           "    sta WSYNC\n" + AT42 + "    sta RESP0\n"
    f, _ = run(rom_with(base))
    assert lit(f[ROW]) == set()                       # the delayed copy is still 0
    f, _ = run(rom_with(base + "    sta GRP1\n    lda #0\n    sta GRP0"))
    assert lit(f[ROW]) == set(range(66, 74))          # GRP1 copied GRP0 ($FF); a new GRP0 waits
    f, _ = run(rom_with("    lda #2\n    sta ENABL\n    lda #1\n    sta VDELBL\n    sta WSYNC\n" + AT42 +
                        "    sta RESBL\n    lda #$44\n    sta COLUPF"))
    assert lit(f[ROW]) == set()
    f, _ = run(rom_with("    lda #2\n    sta ENABL\n    lda #1\n    sta VDELBL\n    sta GRP1\n"
                        "    lda #0\n    sta ENABL\n    sta WSYNC\n" + AT42 + "    sta RESBL\n    lda #$44\n    sta COLUPF"))
    assert lit(f[ROW]) == {65}                        # GRP1 copied ENABL (2) before it was cleared


@pytest.mark.parametrize("nusiz,pos", [(0, 69), (5, 72), (7, 76)])
def test_resmp_release_centres_missile(nusiz, pos):
    setup = f"    lda #${nusiz:02X}\n    sta NUSIZ0\n    lda #2\n    sta ENAM0\n    sta RESMP0\n" \
            "    lda #$36\n    sta COLUP0\n    sta WSYNC\n" + AT42 + "    sta RESP0\n"
    f, _ = run(rom_with(setup))
    assert lit(f[ROW]) == set()                       # hidden while RESMP0 D1 is set
    f, _ = run(rom_with(setup + "    lda #0\n    sta RESMP0"))
    assert lit(f[ROW]) == {pos}


def test_hmove_moves_missiles_and_ball():
    setup = "    lda #2\n    sta ENAM0\n    sta ENABL\n    lda #$36\n    sta COLUP0\n    lda #$44\n    sta COLUPF\n" \
            "    sta WSYNC\n" + AT42 + "    sta RESM0\n" + "    sta WSYNC\n" + "    nop\n" * 24 + "    sta RESBL\n" \
            "    lda #$F0\n    sta HMM0\n    lda #$20\n    sta HMBL\n    sta WSYNC\n    sta HMOVE\n"
    # RESBL: 24 NOPs -> access cycle 50 -> clock 153 -> position 89; an HMOVE at the start of the
    # blank (clock 9): HMM0 $F0 moves +1, HMBL $20 moves -2
    f, _ = run(rom_with(setup))
    assert lit(f[ROW]) == {66, 87} and f[ROW][66] == 0x36 and f[ROW][87] == 0x44
    f, _ = run(rom_with(setup + "    sta HMCLR\n    sta WSYNC\n    sta HMOVE"))
    assert lit(f[ROW]) == {66, 87}                    # HMCLR: an early second HMOVE moves nothing
    # the first HMOVE late instead (no WSYNC before it: access cycle 63, clock 192): of the pulses
    # at clocks 196, 200, ..., those from 228 on (the 9th and later) reach the next line's blank:
    # HMM0 $F0 (7 pulses) moves nothing, HMBL $20 (10 pulses) moves 2 left
    late = setup.replace("    sta WSYNC\n    sta HMOVE\n", "    sta HMOVE\n")
    f, _ = run(rom_with(late))
    assert lit(f[ROW]) == {65, 87}
    # then HMCLR and a second late HMOVE (access cycle 69, clock 210): pulses 5-8 of the 8 that
    # cleared registers let through land in the next blank: both move 4 left
    f, _ = run(rom_with(late + "    sta HMCLR\n    sta HMOVE"))
    assert lit(f[ROW]) == {61, 83}


def pulse_rom(nops):
    """HMP0 $70, HMP1 $80, HMM0 $00, HMM1 $30, HMBL $F0; P0 and P1 placed at 66,
    M0, M1 and the ball at 65; then one line: `nops` NOPs and STA HMOVE,
    whose write is at access cycle 2 nops + 2, clock h = 6 nops + 9."""
    setup = "    lda #$70\n    sta HMP0\n    lda #$80\n    sta HMP1\n    lda #$00\n    sta HMM0\n" \
            "    lda #$30\n    sta HMM1\n    lda #$F0\n    sta HMBL\n"
    for reg in ("RESP0", "RESP1", "RESM0", "RESM1", "RESBL"):
        setup += "    sta WSYNC\n" + AT42 + f"    sta {reg}\n"
    setup += "    sta WSYNC\n" + "    nop\n" * nops + "    sta HMOVE\n"
    return rom_with(setup)


# Positions (P0, P1, M0, M1, BL) after one HMOVE at clock h = 6 nops + 9.  The objects take
# n = 15, 0, 8, 11, 7 pulses (HM nibble XOR 8), at clocks h + 4, h + 8, ...; a pulse moves its
# object one pixel left only in horizontal blank (clocks 0-67, 0-75 on a line whose blank an
# HMOVE before clock 68 extended, which also holds it 8 pixels right).  Derived by hand:
#  h =   9: blank to 76, pulses up to h + 64 = 73 count: all n   -> n - 8 left: 59 74 65 62 66
#  h =  21: pulses up to 21 + 52 = 73: min(n, 13)                -> 61 74 65 62 66
#  h =  39: pulses up to 39 + 36 = 75: min(n, 9)                 -> 65 74 65 64 66
#  h =  63: pulses up to 63 + 12 = 75: min(n, 3)                 -> 71 74 70 70 70
#  h =  69: no extension; every pulse (73 .. 129) in the visible part: none   -> 66 66 65 65 65
#  h = 189: pulses from the 10th (189 + 40 = 229) in the next blank: n - 9    -> 60 66 65 63 65
#  h = 207: from the 6th (207 + 24 = 231): n - 5                              -> 56 66 62 59 63
#  h = 225: all (225 + 4 = 229): n                                            -> 51 66 57 54 58
@pytest.mark.parametrize("nops,want", [(0, (59, 74, 65, 62, 66)), (2, (61, 74, 65, 62, 66)),
                                       (5, (65, 74, 65, 64, 66)), (9, (71, 74, 70, 70, 70)),
                                       (10, (66, 66, 65, 65, 65)), (30, (60, 66, 65, 63, 65)),
                                       (33, (56, 66, 62, 59, 63)), (36, (51, 66, 57, 54, 58))])
def test_hmove_pulse_timing(nops, want):
    rom = pulse_rom(nops)
    st, _, _, got_frames = oracle.run_frames(oracle.power_on(rom), rom, 2, actions=np.zeros(2, np.uint8))
    assert got_frames == 2 and decode(st)["err"] == 0
    st = np.asarray(st, np.uint8)
    got = (int(st[176]), int(st[177]), int(st[221]), int(st[222]), int(st[223]))
    assert got == want


def test_hmove_blank():
    # per line: STA HMOVE right after the WSYNC (access cycle 2, clock 9 < 68)
    # blanks pixels 0-7 of the line; one at access cycle 42 does not
    early = f"""
reset:
    lda #$1E
    sta COLUBK
frame:
    sta WSYNC
    lda #2
    sta VSYNC
    lda #0
    sta VSYNC
    ldx #0
lines:
    sta WSYNC
    sta HMOVE
    dex
    bne lines
    jmp frame
"""
    rom, _ = cart(early)
    f, _ = run(rom)
    assert (f[ROW][:8] == 0).all() and (f[ROW][8:] == 0x1E).all()
    late = early.replace("    sta HMOVE\n", "    nop\n" * 20 + "    sta HMOVE\n")
    rom, _ = cart(late)
    f, _ = run(rom)
    assert (f[ROW] == 0x1E).all()


def test_priority_with_missiles_and_ball():
    # M0 at 65 over P1 (66-73, $FF), ball at 65 under both; PF (PF2 bit 0 -> pixels 32-35) far away
    setup = "    lda #2\n    sta ENAM0\n    sta ENABL\n    lda #$FF\n    sta GRP1\n    lda #$36\n    sta COLUP0\n" \
            "    lda #$58\n    sta COLUP1\n    lda #$44\n    sta COLUPF\n    lda #$10\n    sta NUSIZ0\n" \
            "    sta WSYNC\n" + AT42 + "    sta RESM0\n    sta WSYNC\n" + AT42 + "    sta RESP1\n" + \
            "    sta WSYNC\n" + AT42 + "    sta RESBL\n"
    f, _ = run(rom_with(setup))
    row = f[ROW]
    assert row[65] == 0x36 and row[66] == 0x36 and row[67] == 0x58 and row[73] == 0x58 and row[74] == 0
    f, _ = run(rom_with(setup + "    lda #4\n    sta CTRLPF"))     # PF/BL first: the ball shows at 65
    row = f[ROW]
    assert row[65] == 0x44 and row[66] == 0x36 and row[67] == 0x58


CX_READ = "\n".join(f"    lda ${r:02X}\n    sta ${0x90 + r:02X}" for r in range(8)) + "\n    sta CXCLR"


def cx_regs(d):
    return [int(d["ram"][0x10 + r]) for r in range(8)]


def test_all_collisions_at_one_pixel():
    # every object on pixel 66: players 66-73, missiles and ball 2 wide from 65,
    # playfield block 16 (PF2 D4) = pixels 64-67
    setup = "    lda #$10\n    sta PF2\n    lda #2\n    sta ENAM0\n    sta ENAM1\n    sta ENABL\n" \
            "    lda #$FF\n    sta GRP0\n    sta GRP1\n    lda #$10\n    sta NUSIZ0\n    sta NUSIZ1\n" \
            "    lda #$10\n    sta CTRLPF\n" + \
            "".join("    sta WSYNC\n" + AT42 + f"    sta {r}\n" for r in ("RESP0", "RESP1", "RESM0", "RESM1", "RESBL"))
    _, d = run(rom_with(setup, per_frame_end=CX_READ), track=True)
    assert cx_regs(d) == [0xC0, 0xC0, 0xC0, 0xC0, 0xC0, 0xC0, 0x80, 0xC0]
    _, d = run(rom_with(setup, per_frame_end=CX_READ), track=False)
    assert cx_regs(d) == [0] * 8                        # untracked latches read 0


@pytest.mark.parametrize("pair,reg,bit", [(("RESP0", "RESP1"), 7, 0x80), (("RESM0", "RESP1"), 0, 0x80),
                                          (("RESM0", "RESP0"), 0, 0x40), (("RESM1", "RESP0"), 1, 0x80),
                                          (("RESM1", "RESP1"), 1, 0x40), (("RESM0", "RESM1"), 7, 0x40),
                                          (("RESP0", "RESBL"), 2, 0x40), (("RESP1", "RESBL"), 3, 0x40),
                                          (("RESM0", "RESBL"), 4, 0x40), (("RESM1", "RESBL"), 5, 0x40)])
def test_single_collision_pairs(pair, reg, bit):
    """Only two objects are enabled and placed together: exactly one latch."""
    enable = {"RESP0": "    lda #$FF\n    sta GRP0\n", "RESP1": "    lda #$FF\n    sta GRP1\n",
              "RESM0": "    lda #$32\n    sta ENAM0\n    lda #$30\n    sta NUSIZ0\n",
              "RESM1": "    lda #$32\n    sta ENAM1\n    lda #$30\n    sta NUSIZ1\n",
              "RESBL": "    lda #2\n    sta ENABL\n    lda #$30\n    sta CTRLPF\n"}
    setup = enable[pair[0]] + enable[pair[1]] + "".join("    sta WSYNC\n" + AT42 + f"    sta {r}\n" for r in pair)
    _, d = run(rom_with(setup, per_frame_end=CX_READ), track=True)
    want = [0] * 8
    want[reg] = bit
    assert cx_regs(d) == want


def test_collision_read_timing_and_vblank():
    # P0 (66-73) and P1 (66-73) meet at clocks 134-141 of every line; on the
    # read line CXCLR (access cycle 2) clears the earlier rows' latches, then
    # after n NOPs LDA CXPPMM (zero page, 3 cycles) reads at access cycle
    # 2n + 5, seeing clocks up to 3(2n + 5) + 2: n = 19 -> clock 131 (none
    # yet), n = 20 -> clock 137
    def prog(nops, vblank=False):
        return f"""
reset:
    lda #$FF
    sta GRP0
    sta GRP1
    sta WSYNC
{AT42}    sta RESP0
    sta WSYNC
{AT42}    sta RESP1
frame:
    sta WSYNC
    lda #2
    sta VSYNC
    lda #0
    sta VSYNC
    lda #{2 if vblank else 0}
    sta VBLANK
    ldx #59
lines:
    sta WSYNC
    dex
    bne lines
    sta WSYNC
    sta CXCLR
""" + "    nop\n" * nops + """    lda CXPPMM
    sta $A0
    ldx #0
rest:
    sta WSYNC
    dex
    bne rest
    jmp frame
"""
    for nops, want in [(19, 0), (20, 0x80)]:
        rom, _ = cart(prog(nops))
        _, d = run(rom, track=True)
        assert d["ram"][0x20] == want, nops
    rom, _ = cart(prog(20, vblank=True))
    _, d = run(rom, track=True)
    assert d["ram"][0x20] == 0                     # nothing is drawn, so nothing collides, in VBLANK


# Fetches that read the latches.  The TIA drives D7/D6 of a collision
# register on every read cycle of it, whoever reads: zero-page pointer bytes
# and instruction bytes fetched from $00-$07 (and mirrors) see the latches as
# a data read would.  Fetches happen at the instruction's first cycle t and,
# like a data read at cycle t, see the pixels through colour clock 3t+2.

# P0 on pixels 66-73 over playfield PF2 (pixels 48-79): CXP0FB D7 on every
# visible row; with the ball (2 wide from 65) over P0 too: CXP0FB D7 and D6
P0_OVER_PF = "    lda #$FF\n    sta PF2\n    sta GRP0\n    lda #$36\n    sta COLUP0\n" \
             "    sta WSYNC\n" + AT42 + "    sta RESP0\n"
BALL_ON_P0 = "    lda #2\n    sta ENABL\n    lda #$10\n    sta CTRLPF\n    sta WSYNC\n" + AT42 + "    sta RESBL\n"
# markers at the RAM bytes a latch-valued pointer can name
MARKS = "    lda #$5A\n    sta $80\n    lda #$A5\n    sta $C0\n"
PTR_READS = MARKS + "    ldy #0\n    lda ($02),y\n    sta $A0\n    ldx #4\n    lda ($FE,x)\n    sta $A1\n"


@pytest.mark.parametrize("setup,want", [("", 0x00), (P0_OVER_PF, 0x5A), (P0_OVER_PF + BALL_ON_P0, 0xA5)])
def test_pointer_bytes_read_latches(setup, want):
    """LDA ($02),Y and LDA ($FE,X) with X = 4 take their pointer from
    CXP0FB/CXP1FB: low byte $80 (P0-PF) names RAM $80, $C0 (P0-PF and P0-BL)
    names RAM $C0, $00 names TIA register $00 (CXM0P, 0 here); the high
    byte ($00 or $80, CXP1FB) only sets address bits that the 13-bit bus
    drops."""
    _, d = run(rom_with(setup, per_frame_end=PTR_READS), track=True)
    assert int(d["ram"][0x20]) == want and int(d["ram"][0x21]) == want
    _, d = run(rom_with(setup, per_frame_end=PTR_READS), track=False)
    assert int(d["ram"][0x20]) == 0 and int(d["ram"][0x21]) == 0     # untracked: the pointer is $0000


def fetch_rom(setup):
    """LDY #imm with its opcode at $00FF (RAM) and its operand at $0100, which
    the 13-bit bus maps to TIA read register 0 (CXM0P); the next opcode
    comes from $0101 (CXM1P, 0 here: BRK), whose handler stores Y."""
    src = f"""
reset:
    sta WSYNC
{setup}
frame:
    sta WSYNC
    lda #2
    sta VSYNC
    lda #0
    sta VSYNC
    lda #$A0
    sta $FF
    jmp $00FF
back:
    ldx #0
lines:
    sta WSYNC
    dex
    bne lines
    jmp frame
brkh:
    sty $A2
    tsx
    lda $0102,x
    sta $A3
    pla
    pla
    pla
    jmp back
    .org $1FFC
    .word reset
    .word brkh
"""
    rom, _ = cart(src)
    return rom


M0_ON_P0 = "    lda #$FF\n    sta GRP0\n    lda #2\n    sta ENAM0\n    lda #$10\n    sta NUSIZ0\n" \
           "    sta WSYNC\n" + AT42 + "    sta RESP0\n    sta WSYNC\n" + AT42 + "    sta RESM0\n"
P1_ON_M0 = "    lda #$FF\n    sta GRP1\n    sta WSYNC\n" + AT42 + "    sta RESP1\n"


@pytest.mark.parametrize("setup,want", [("", 0x00), (M0_ON_P0, 0x40), (M0_ON_P0 + P1_ON_M0, 0xC0)])
def test_operand_fetch_reads_latches(setup, want):
    """The operand byte of LDY # fetched from $0100 is CXM0P: D6 = M0-P0,
    D7 = M0-P1 (M0 2 wide from 65 meets the players on 66).  BRK at $0101
    pushes the return address $0103: its low byte lands at $0102 + S."""
    _, d = run(fetch_rom(setup), track=True)
    assert int(d["ram"][0x22]) == want and int(d["ram"][0x23]) == 0x03
    _, d = run(fetch_rom(setup), track=False)
    assert int(d["ram"][0x22]) == 0


def timing_rom(nops):
    """On the read line: CXCLR (cycles 0-2), LDA zp (3-5), `nops` NOPs, then
    LDA ($07),Y (Y = 0) at t = 6 + 2 nops; the result goes to RAM $A0."""
    src = f"""
reset:
    lda #$FF
    sta GRP0
    sta GRP1
    lda #$5A
    sta $80
    sta WSYNC
{AT42}    sta RESP0
    sta WSYNC
{AT42}    sta RESP1
frame:
    sta WSYNC
    lda #2
    sta VSYNC
    lda #0
    sta VSYNC
    ldx #59
    ldy #0
lines:
    sta WSYNC
    dex
    bne lines
    sta WSYNC
    sta CXCLR
    lda $F0
""" + "    nop\n" * nops + """    lda ($07),y
    sta $A0
    ldx #0
rest:
    sta WSYNC
    dex
    bne rest
    jmp frame
"""
    rom, _ = cart(src)
    return rom


@pytest.mark.parametrize("nops,want", [(18, 0x00), (19, 0x5A)])
def test_pointer_fetch_timing(nops, want):
    """P0 and P1 (both on 66-73) meet from colour clock 68 + 66 = 134.  The
    pointer low byte (CXPPMM) is fetched at t = 6 + 2 nops and sees clocks
    through 3t+2: t = 42 -> 128 (pointer $00, A = CXM0P = 0), t = 44 -> 134
    (pointer $80, A = RAM $80 = $5A).  A pointer read at the access cycle
    t+4 would latch already at t = 42; one that saw only the cycles before t
    would not latch at t = 44."""
    _, d = run(timing_rom(nops), track=True)
    assert int(d["ram"][0x20]) == want
