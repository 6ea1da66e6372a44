"""Pins of the oracle's frame timing, TIA rendering and preprocessing.

Frame invariants: every generated cartridge runs 262-line frames of exactly
76 x 262 = 19,912 CPU cycles (NTSC), with the frame boundary at a fixed cycle
of its line.  Render special cases are derived by hand from the TIA register
definitions (playfield bit order, reflection, players, priority, score mode)
and the timing conventions of the oracle.  The preprocessing is checked
against a brute-force exact-area average in rational arithmetic.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from helpers import cart, decode
from paper_1907_08467_amd.inputs.palette import GRAY
from paper_1907_08467_amd.inputs.romgen import RomSpec, generate


@pytest.mark.parametrize("spec", [RomSpec(1000), RomSpec(2000), RomSpec(3000, "4k", True),
                                  RomSpec(3004, "f8", True), RomSpec(4001, "f8", True), RomSpec(7000, objects=True),
                                  RomSpec(7001, "f8", True, objects=True)],
                         ids=lambda s: f"{s.seed}-{s.kind}-{'div' if s.divergent else 'plain'}{'-obj' if s.objects else ''}")
def test_generated_rom_frame_invariants(spec):
    rom = generate(spec)
    rng = np.random.default_rng(spec.seed)
    st = oracle.power_on(rom.data, rom.scheme)
    st, _, ends, got = oracle.run_frames(st, rom.data, 80, rom.scheme,
                                         actions=rng.integers(0, 18, 80).astype(np.uint8), render=False)
    d = decode(st)
    assert got == 80 and d["err"] == 0
    diffs = np.diff(ends.astype(np.int64))[1:]
    assert (diffs == 19912).all(), set(diffs.tolist())          # 262 lines x 76 cycles
    assert len({int(e) % 76 for e in ends[1:]}) == 1             # boundary at a fixed cycle of its line
    assert d["frame_line0"] == int(ends[-1]) // 76


def frame_rom(setup, per_line="", lines=0):
    """A cartridge that runs `setup` once, then frames of 1 + `lines` (0 = 256)
    WSYNC lines; `per_line` runs at the start of every line."""
    src = f"""
reset:
{setup}
frame:
    sta WSYNC
    lda #2
    sta VSYNC
    lda #0
    sta VSYNC
    ldx #{lines}
lines:
    sta WSYNC
{per_line}
    dex
    bne lines
    jmp frame
"""
    rom, _ = cart(src)
    return rom


def frames_of(rom, n=3, action=0):
    st = oracle.power_on(rom)
    st, frames, ends, got = oracle.run_frames(st, rom, n, actions=np.full(n, action, np.uint8))
    assert got == n and decode(st)["err"] == 0
    return frames


def test_constant_background():
    f = frames_of(frame_rom("    lda #$1F\n    sta COLUBK"))
    assert (f[-1] == 0x1E).all()


def test_vblank_blanks():
    f = frames_of(frame_rom("    lda #$1E\n    sta COLUBK\n    lda #2\n    sta VBLANK"))
    assert (f[-1] == 0).all()


def test_row_mapping_y0_34():
    # line L+j of the frame (j >= 1) gets COLUBK = (1 - j) & $FF at its start;
    # row r shows line L + 34 + r
    f = frames_of(frame_rom("", per_line="    stx COLUBK"))[-1]
    for r in range(210):
        assert (f[r] == ((1 - (34 + r)) & 0xFF) & 0xFE).all(), r


def test_playfield_blocks_and_reflection():
    setup = "    lda #$F0\n    sta PF0\n    lda #$44\n    sta COLUPF\n    lda #$02\n    sta COLUBK"
    row = frames_of(frame_rom(setup))[-1][100]
    want = np.full(160, 0x02)
    want[0:16] = 0x44
    want[80:96] = 0x44
    assert np.array_equal(row, want)
    row = frames_of(frame_rom(setup + "\n    lda #1\n    sta CTRLPF"))[-1][100]
    want = np.full(160, 0x02)
    want[0:16] = 0x44
    want[144:160] = 0x44
    assert np.array_equal(row, want)


def test_playfield_bit_order():
    # PF1 D7 -> playfield bit 4 (pixels 16..19); PF2 D0 -> bit 12 (48..51)
    setup = "    lda #$80\n    sta PF1\n    lda #$01\n    sta PF2\n    lda #$44\n    sta COLUPF"
    row = frames_of(frame_rom(setup))[-1][50]
    on = set(np.nonzero(row)[0].tolist())
    assert on == set(range(16, 20)) | set(range(48, 52)) | set(range(96, 100)) | set(range(128, 132))


@pytest.mark.parametrize("seed", range(4))
def test_random_playfield_symmetries(seed):
    r = np.random.default_rng(seed)
    pf = [int(x) for x in r.integers(0, 256, 3)]
    setup = (f"    lda #${pf[0]:02X}\n    sta PF0\n    lda #${pf[1]:02X}\n    sta PF1\n"
             f"    lda #${pf[2]:02X}\n    sta PF2\n    lda #$C6\n    sta COLUPF\n    lda #$0A\n    sta COLUBK")
    row = frames_of(frame_rom(setup))[-1][120]
    assert np.array_equal(row[:80], row[80:])                           # repeated
    row = frames_of(frame_rom(setup + "\n    lda #1\n    sta CTRLPF"))[-1][120]
    assert np.array_equal(row, row[::-1])                               # mirrored


@pytest.mark.parametrize("k", [10, 20, 25])
def test_mid_line_split(k):
    # per line: COLUBK <- $0E written at cycle 4 (before the visible part),
    # then k NOPs, then COLUBK <- $84 written at cycle 9 + 2k: it shows from
    # colour clock 3 (10 + 2k), i.e. pixel 6k - 38
    per_line = "    lda #$0E\n    sta COLUBK\n" + "    nop\n" * k + "    lda #$84\n    sta COLUBK"
    row = frames_of(frame_rom("", per_line=per_line))[-1][100]
    x = 6 * k - 38
    want = np.array([0x0E] * x + [0x84] * (160 - x))
    assert np.array_equal(row, want)


def _player_rom(grp, refp=0, extra=""):
    return frame_rom(f"""
    lda #${grp:02X}
    sta GRP0
    lda #${refp:02X}
    sta REFP0
    lda #$36
    sta COLUP0
    sta WSYNC
""" + "    nop\n" * 20 + "    sta RESP0\n" + extra)


def test_player_position_and_reflection():
    # RESP0 written at cycle 42 of its line -> clock 129 -> position 66
    row = frames_of(_player_rom(0xC0))[-1][80]
    assert set(np.nonzero(row)[0].tolist()) == {66, 67} and row[66] == 0x36
    row = frames_of(_player_rom(0xC0, refp=8))[-1][80]
    assert set(np.nonzero(row)[0].tolist()) == {72, 73}


@pytest.mark.parametrize("hm,pos", [(0xF0, 67), (0x70, 59), (0x80, 74)])
def test_hmove(hm, pos):
    # one HMOVE at the start of a horizontal blank moves the player by -signed(high nibble)
    rom = _player_rom(0x80, extra=f"    lda #${hm:02X}\n    sta HMP0\n    sta WSYNC\n    sta HMOVE")
    row = frames_of(rom)[-1][80]
    assert set(np.nonzero(row)[0].tolist()) == {pos}


def test_resp_in_hblank_and_priority_score():
    base = """
    lda #$F0
    sta PF0
    lda #$44
    sta COLUPF
    lda #$36
    sta COLUP0
    lda #$58
    sta COLUP1
    lda #$FF
    sta GRP0
    sta WSYNC
    sta RESP0
"""
    # RESP0 written at cycle 2 (clock 9, horizontal blank) -> position 3
    row = frames_of(frame_rom(base))[-1][60]
    want = np.zeros(160, int)
    want[0:16] = 0x44
    want[80:96] = 0x44
    want[3:11] = 0x36                      # player over playfield
    assert np.array_equal(row, want)
    row = frames_of(frame_rom(base + "    lda #4\n    sta CTRLPF"))[-1][60]
    want[0:16] = 0x44                      # playfield priority
    want[3:11] = 0x36
    want[3:16] = 0x44
    assert np.array_equal(row, want)
    row = frames_of(frame_rom(base + "    lda #2\n    sta CTRLPF"))[-1][60]
    want = np.zeros(160, int)
    want[0:16] = 0x36                      # score mode: left half in COLUP0
    want[80:96] = 0x58                     # right half in COLUP1
    assert np.array_equal(row, want)


def test_rows_after_frame_end_are_black():
    # frames of 1 + 96 lines: lines at or after the next VSYNC line are not part of the frame
    f = frames_of(frame_rom("    lda #$1E\n    sta COLUBK", lines=0x60))[-1]
    last_line = 0x60 + 1                    # the next frame's VSYNC line, counted from this frame's
    for r in range(210):
        line = 34 + r
        assert (f[r] == (0x1E if line < last_line else 0)).all(), r


def test_frame_cap():
    rom, _ = cart("reset:\n    sta WSYNC\n    jmp reset\n")
    st, frames, ends, got = oracle.run_frames(oracle.power_on(rom), rom, 2)
    d = decode(st)
    assert got == 1 and d["err"] == oracle.ERR_FRAME_CAP
    assert int(ends[0]) == 320 * 76 - 1


# ------------------------------------------------------------ preprocess

def brute_obs(f_prev, f_last, lut):
    lut = np.frombuffer(bytes(lut), np.uint8).astype(int)
    g = lut[f_last >> 1]
    if f_prev is not None:
        g = np.maximum(g, lut[f_prev >> 1])
    out = np.zeros((84, 84), int)
    for i in range(84):
        y0, y1 = Fraction(210 * i, 84), Fraction(210 * (i + 1), 84)
        for j in range(84):
            x0, x1 = Fraction(160 * j, 84), Fraction(160 * (j + 1), 84)
            acc = Fraction(0)
            for r in range(int(y0), int(np.ceil(y1))):
                wy = min(y1, r + 1) - max(y0, r)
                for c in range(int(x0), int(np.ceil(x1))):
                    wx = min(x1, c + 1) - max(x0, c)
                    acc += wy * wx * int(g[r, c])
            mean = acc / ((y1 - y0) * (x1 - x0))
            out[i, j] = int(mean + Fraction(1, 2))          # round half up
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_preprocess_exact_area_bruteforce(seed):
    r = np.random.default_rng(seed)
    fa = r.integers(0, 256, (210, 160)).astype(np.uint8)
    fb = r.integers(0, 256, (210, 160)).astype(np.uint8)
    got = oracle.preprocess(fa, fb, GRAY)
    assert np.array_equal(got, brute_obs(fa, fb, GRAY))


def test_preprocess_single_frame_bruteforce():
    r = np.random.default_rng(7)
    fb = r.integers(0, 256, (210, 160)).astype(np.uint8)
    assert np.array_equal(oracle.preprocess(None, fb, GRAY), brute_obs(None, fb, GRAY))


def test_preprocess_constant_and_max():
    for c in (0, 0x1E, 0x86, 0xFE):
        f = np.full((210, 160), c, np.uint8)
        assert (oracle.preprocess(f, f, GRAY) == GRAY[c >> 1]).all()
    r = np.random.default_rng(3)
    a = r.integers(0, 256, (210, 160)).astype(np.uint8)
    b = r.integers(0, 256, (210, 160)).astype(np.uint8)
    assert np.array_equal(oracle.preprocess(a, a, GRAY), oracle.preprocess(None, a, GRAY))
    assert np.array_equal(oracle.preprocess(a, b, GRAY), oracle.preprocess(b, a, GRAY))


def test_all_workload_cartridges_keep_ntsc_frames():
    """Every cartridge of the workloads: 262-line frames, no faults."""
    from paper_1907_08467_amd.inputs.workloads import config
    seen = set()
    for c in (1, 2, 3, 4, 6, 7):
        for spec in config(c).rom_specs:
            if spec.seed in seen:
                continue
            seen.add(spec.seed)
            rom = generate(spec)
            st = oracle.power_on(rom.data, rom.scheme)
            acts = np.random.default_rng(spec.seed).integers(0, 18, 12).astype(np.uint8)
            st, _, ends, got = oracle.run_frames(st, rom.data, 12, rom.scheme, actions=acts, render=False)
            assert got == 12 and decode(st)["err"] == 0
            assert (np.diff(ends.astype(np.int64))[1:] == 19912).all(), spec


def test_objects_cartridge_collides_and_scores():
    """An objects cartridge with tracked latches: frames show missiles and
    the ball, the players meet in some frames (counted at $D6, each such
    frame scoring a point), and untracked the counter stays 0."""
    rom = generate(RomSpec(7001, objects=True))
    acts = np.random.default_rng(3).integers(0, 18, 40).astype(np.uint8)
    for track in (True, False):
        st = oracle.power_on(rom.data, rom.scheme)
        st[230] = 1 if track else 0
        st, frames, ends, got = oracle.run_frames(st, rom.data, 40, rom.scheme, actions=acts)
        d = decode(st)
        assert got == 40 and d["err"] == 0
        hits = int(d["ram"][0x56])
        assert (hits > 0) == track, hits
