"""The fuller TIA on the GPU against the oracle, with the collision latches
tracked: fuzz cartridges write every object register (NUSIZ, ENAM/ENABL,
RESP/RESM/RESBL, HMxx, VDELxx, RESMPx, CXCLR, HMOVE at any cycle) and read
CXM0P..CXPPMM at any cycle of any line, so a latch read in mid-line needs the
pixels drawn so far; full machine-state records (latches included) and
frames are compared every step, with every frame rendered and with only the
last two (the unrendered frames still feed the latches).  A hand-written
cartridge moves all five objects with HMOVE and branches on the latches, so
a wrong latch changes the control flow that follows.
"""
import sys

import numpy as np
import pytest

from fuzzcart import S_3F, S_E0, S_F8, S_F6SC, S_4K, fuzz_cart
from helpers import cart, decode, diff_records
from parity import make_pair, step_both

pytestmark = pytest.mark.gpu

CASES = [(S_4K, False, 0), (S_4K, True, 0), (S_4K, False, 1), (S_F8, True, 1), (S_F8, False, 0), (S_F6SC, False, 1), (S_E0, True, 0),
         (S_3F, True, 1)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_all(o, g, n, tag):
    for e in range(n):
        a, b = g.get_state(e), o.get_state(e)
        assert np.array_equal(a, b), f"{tag}: env {e}: {diff_records(a, b)}"


@pytest.mark.parametrize("scheme,undoc,mode", CASES, ids=[f"s{c[0]}_u{int(c[1])}_r{c[2]}" for c in CASES])
def test_fuzz_collisions(scheme, undoc, mode):
    seed = 5100 + 13 * scheme + (1 if undoc else 0) + 5 * mode
    say(f"case: collisions, scheme {scheme} undoc {undoc} render_mode {mode} seed {seed}")
    rom, sch = fuzz_cart(seed, scheme=scheme, undoc=undoc, cx=True)
    n = 48
    o, g = make_pair([(rom, sch)], np.zeros(n, np.uint16), seed=seed, frameskip=4, render_mode=mode,
                     collisions=True)
    rng = np.random.default_rng(seed)
    latched = 0
    for s in range(20):
        step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"collisions step {s}")
        compare_all(o, g, n, f"collisions scheme {scheme} step {s}")
        latched += sum(int(o.get_state(e)[228:230].any()) for e in range(n))
    assert latched > 0                       # the cartridges do collide
    assert g.poll_errors() == o.poll_errors()
    g.close()
    o.close()


MOVER = """
reset:
    ldx #$FF
    txs
    lda #$FF
    sta GRP0
    lda #$3C
    sta GRP1
    lda #2
    sta ENAM0
    sta ENAM1
    sta ENABL
    lda #$15
    sta NUSIZ0
    lda #$27
    sta NUSIZ1
    lda #$21
    sta CTRLPF
    lda #$10
    sta HMP0
    lda #$F0
    sta HMP1
    lda #$20
    sta HMM0
    lda #$E0
    sta HMM1
    lda #$70
    sta HMBL
    sta WSYNC
    nop
    nop
    sta RESP0
    nop
    sta RESM1
    sta RESP1
    nop
    nop
    nop
    sta RESBL
    sta RESM0
frame:
    sta WSYNC
    lda #2
    sta VSYNC
    lda #0
    sta VSYNC
    sta HMOVE
    inc $80
    lda $80
    and #$0F
    sta PF1
    ldx #80
top:
    sta WSYNC
    dex
    bne top
    lda CXPPMM
    bpl nopp
    inc $81
    lda $81
    sta COLUP0
nopp:
    sta WSYNC
    lda CXM0P
    asl
    bcc nom0
    inc $82
    sta HMCLR
    sta HMOVE
nom0:
    lda CXBLPF
    bpl nobl
    inc $83
    lda $83
    sta COLUBK
nobl:
    lda CXM0FB
    ora CXM1FB
    ora CXP0FB
    ora CXP1FB
    sta $84
    sta CXCLR
    ldx #120
bottom:
    sta WSYNC
    dex
    bne bottom
    lda INPT4
    bmi noreset
    lda $82
    and #7
    sta RESMP0
noreset:
    lda #0
    sta RESMP0
    jmp frame
"""


def test_moving_objects_branch_on_latches():
    rom, _ = cart(MOVER)
    n = 32
    say(f"case: moving objects, {n} envs")
    o, g = make_pair([(rom, 0)], np.zeros(n, np.uint16), seed=9, frameskip=4, collisions=True)
    rng = np.random.default_rng(9)
    for s in range(30):
        step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"mover step {s}")
        compare_all(o, g, n, f"mover step {s}")
    assert g.poll_errors() == o.poll_errors()
    g.close()
    o.close()


def test_untracked_latches_read_zero():
    """The same cartridge without tracking: the latches read 0 on both sides."""
    rom, _ = cart(MOVER)
    n = 8
    o, g = make_pair([(rom, 0)], np.zeros(n, np.uint16), seed=9, frameskip=4)
    for s in range(5):
        step_both(o, g, np.zeros(n, np.uint8), want_frames=True, tag=f"untracked step {s}")
        compare_all(o, g, n, f"untracked step {s}")
    assert not o.get_state(0)[228:230].any()
    g.close()
    o.close()


OBJ_CASES = [(7000, "4k", 0, True), (7001, "4k", 1, True), (7002, "f8", 0, True), (7003, "4k", 0, False)]


@pytest.mark.parametrize("seed,kind,mode,track", OBJ_CASES, ids=[f"{c[0]}_{c[1]}_r{c[2]}_t{int(c[3])}" for c in OBJ_CASES])
def test_objects_cartridges(seed, kind, mode, track):
    """Generated objects cartridges (missiles, ball, NUSIZ copies, motion,
    latch reads that score) with several ROMs per launch: rewards, frames and
    states every step."""
    from paper_1907_08467_amd.inputs.romgen import RomSpec, generate
    roms = [generate(RomSpec(seed + 10 * k, kind, k == 1, objects=True)) for k in range(3)]
    n = 3 * 32
    env_rom = (np.arange(n) % 3).astype(np.uint16)
    say(f"case: objects cartridges seed {seed} kind {kind} render_mode {mode} collisions {track}")
    o, g = make_pair([(r.data, r.scheme) for r in roms], env_rom, seed=seed, frameskip=4, render_mode=mode,
                     collisions=track)
    rng = np.random.default_rng(seed)
    for s in range(30):
        step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"objects step {s}")
        if s % 10 == 9:
            compare_all(o, g, n, f"objects step {s}")
    hits = sum(int(decode(o.get_state(e))["ram"][0x56]) for e in range(n))     # $D6: frames the players met
    assert (hits > 0) == track
    assert g.poll_errors() == o.poll_errors()
    g.close()
    o.close()
