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


def objects_roms():
    from paper_1907_08467_amd.inputs.romgen import RomSpec, generate
    return [(r.data, r.scheme) for r in (generate(RomSpec(7100 + k, "4k" if k % 2 == 0 else "f8", k >= 2, objects=True))
                                         for k in range(4))]


@pytest.mark.parametrize("pipes", [1, 2])
def test_collisions_graph_replays(pipes):
    """Captured steps with tracked latches and only the last two frames
    rendered (the other frames log to the pipelines' scratch logs): every
    replay equals the oracle's steps, with eager steps and other device work
    between replays."""
    import torch
    n = 160
    say(f"case: collisions, captured 3-step graph, {n} envs, pipelines {pipes}")
    env_rom = (np.arange(n) % 4).astype(np.uint16)
    o, g = make_pair(objects_roms(), env_rom, gpu_kw={"pipelines": pipes}, seed=31, render_mode=1,
                     collisions=True)
    g.set_launch(16, 0, 256)
    rng = np.random.default_rng(8)
    graph = g.capture(n=n, steps=3, want_frames=True)
    side = torch.zeros(1 << 20, device="cuda")
    for rep in range(4):
        acts = rng.integers(0, 18, (3, n)).astype(np.uint8)
        obs, rew, done, frames = graph.launch(torch.from_numpy(acts).cuda())
        side.add_(1.0)
        torch.cuda.synchronize()
        for j in range(3):
            oo, orr, od, of = o.step(acts[j], want_frames=True)
            tag = f"collisions graph replay {rep} step {j}"
            assert np.array_equal(done[j].cpu().numpy(), od), tag + ": done"
            assert np.array_equal(rew[j].cpu().numpy(), orr), tag + ": reward"
            assert np.array_equal(obs[j].cpu().numpy(), oo), tag + ": obs"
            assert np.array_equal(frames[j].cpu().numpy(), of), tag + ": frames"
        compare_all(o, g, n, f"after replay {rep}")
        step_both(o, g, rng.integers(0, 18, n), want_frames=False, tag=f"eager step after replay {rep}")
    graph.close()
    assert g.poll_errors() == o.poll_errors()
    g.close()
    o.close()


def test_collisions_pipelines_overlap():
    """Two pipelines on two streams step disjoint env sets of objects
    cartridges with tracked latches at the same time."""
    import torch
    n = 192
    say(f"case: collisions, 2 pipelines on 2 streams, {n} envs")
    env_rom = (np.arange(n) % 4).astype(np.uint16)
    o, g = make_pair(objects_roms(), env_rom, gpu_kw={"pipelines": 2}, seed=6, render_mode=1, collisions=True)
    g.set_launch(8, 0, 256)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    rng = np.random.default_rng(19)
    for k in range(6):
        perm = rng.permutation(n).astype(np.int32)
        ids_a, ids_b = perm[:90], perm[90:180]
        act_a, act_b = rng.integers(0, 18, 90), rng.integers(0, 18, 90)
        ra = g.step(torch.from_numpy(act_a.astype(np.uint8)).cuda(), env_ids=ids_a, pipe=0, stream=s1,
                    want_frames=True)
        rb = g.step(torch.from_numpy(act_b.astype(np.uint8)).cuda(), env_ids=ids_b, pipe=1, stream=s2,
                    want_frames=True)
        torch.cuda.synchronize()
        for ids, act, res, name in ((ids_a, act_a, ra, "a"), (ids_b, act_b, rb, "b")):
            oo, orr, od, of = o.step(act, env_ids=ids, want_frames=True)
            tag = f"collisions pipelines step {k} half {name}"
            assert np.array_equal(res[2].cpu().numpy(), od), tag + ": done"
            assert np.array_equal(res[1].cpu().numpy(), orr), tag + ": reward"
            assert np.array_equal(res[0].cpu().numpy(), oo), tag + ": obs"
            assert np.array_equal(res[3].cpu().numpy(), of), tag + ": frames"
    compare_all(o, g, n, "after pipelined steps")
    assert g.poll_errors() == o.poll_errors()
    g.close()
    o.close()


# ---------------------------------------------------------------- fetches
# Bytes fetched with an instruction (pointer bytes, operand bytes, opcodes)
# from the TIA read registers show the collision latches, as the oracle's
# pins define it (the latches through the fetch cycle's pixels, 3t+2).

def fetch_programs():
    from test_oracle_tia_objects import (BALL_ON_P0, M0_ON_P0, P0_OVER_PF, P1_ON_M0, PTR_READS, fetch_rom,
                                         rom_with, timing_rom)
    return [("pointer P0-PF", rom_with(P0_OVER_PF, per_frame_end=PTR_READS), 0x20, 0x5A),
            ("pointer P0-PF+BL", rom_with(P0_OVER_PF + BALL_ON_P0, per_frame_end=PTR_READS), 0x20, 0xA5),
            ("operand M0-P0", fetch_rom(M0_ON_P0), 0x22, 0x40),
            ("operand M0-P0/P1", fetch_rom(M0_ON_P0 + P1_ON_M0), 0x22, 0xC0),
            ("pointer timing 18", timing_rom(18), 0x20, 0x00),
            ("pointer timing 19", timing_rom(19), 0x20, 0x5A)]


@pytest.mark.parametrize("mode", [0, 1])
def test_fetches_read_latches(mode):
    """Each program on the GPU and the oracle, latches tracked: states,
    frames and the RAM byte the fetch decided, every step."""
    for name, rom, addr, want in fetch_programs():
        n = 8
        say(f"case: fetch reads latches, {name}, render_mode {mode}")
        o, g = make_pair([(rom, 0)], np.zeros(n, np.uint16), seed=3, frameskip=4, render_mode=mode,
                         collisions=True)
        rng = np.random.default_rng(3)
        for s in range(3):
            step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"{name} step {s}")
            compare_all(o, g, n, f"{name} step {s}")
        assert int(decode(o.get_state(0))["ram"][addr & 0x7F]) == want, name
        ge, oe = g.poll_errors(), o.poll_errors()
        assert ge == oe and ge[1] == 0, (name, ge, oe)
        g.close()
        o.close()


# ---------------------------------------------------------------- row log
# Rows with as many logged writes as a program can make: 24 back-to-back
# STA HMOVE (18 land in the visible part, each moving all five objects),
# RESMP set/release toggles on both missiles, a chain of 8 JSRs whose
# pushes walk down the TIA registers from RESBL to NUSIZ1, and a BRK
# pushing into REFP0, CTRLPF and COLUBK (its handler continues the frame:
# a stack in the TIA cannot be pulled back).

def storm_cart():
    hm = "    sta WSYNC\n" + "    sta HMOVE\n" * 24
    resmp = "    sta WSYNC\n    lda #2\n    ldy #0\n" + \
            "    sta RESMP0\n    sty RESMP0\n    sta RESMP1\n    sty RESMP1\n" * 5
    jsr = "    sta WSYNC\n    ldx #$14\n    txs\n" + "".join(f"    jsr j{k}_%d\nj{k}_%d:\n" for k in range(8)) + \
          "    ldx #$FF\n    txs\n"
    body = []
    for i in range(48):
        body.append([hm, resmp, jsr.replace("%d", str(i))][i % 3])
    body.append("    sta WSYNC\n    ldx #$0B\n    txs\n" + "    nop\n" * 12 + "    brk\n    .byte $EA\nafter_brk:\n")
    src = f"""
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
frame:
    sta WSYNC
    lda #2
    sta VSYNC
    lda #0
    sta VSYNC
    sta VBLANK
    ldx #40
top:
    sta WSYNC
    dex
    bne top
{"".join(body)}    ldx #170
bottom:
    sta WSYNC
    dex
    bne bottom
    jmp frame
brkh:
    ldx #$FF
    txs
    jmp after_brk
    .org $1FFC
    .word reset
    .word brkh
"""
    rom, _ = cart(src)
    return rom


@pytest.mark.parametrize("mode,track", [(0, False), (1, False), (0, True), (1, True)])
def test_row_log_storms(mode, track):
    """Parity on rows far past the old per-row capacity (7 HMOVEs), with no
    error bit: frames, rewards, states every step."""
    rom = storm_cart()
    n = 16
    say(f"case: row-log storms, render_mode {mode}, collisions {track}")
    o, g = make_pair([(rom, 0)], np.zeros(n, np.uint16), seed=4, frameskip=4, render_mode=mode,
                     collisions=track)
    rng = np.random.default_rng(4)
    for s in range(6):
        step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"storm step {s}")
        compare_all(o, g, n, f"storm step {s}")
    ge, oe = g.poll_errors(), o.poll_errors()
    assert ge == oe and ge[1] == 0, (ge, oe)
    g.close()
    o.close()
