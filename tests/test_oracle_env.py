"""Pins of the oracle's environment layer: frameskip, reward, done, eager
reset from the 30-entry cache of start-up + no-op states (paper, Section 3),
sticky actions, error handling and batch-composition invariance."""
import numpy as np
import pytest

import oracle
from helpers import decode, diff_records
from paper_1907_08467_amd.inputs.palette import GRAY
from paper_1907_08467_amd.inputs.romgen import RomSpec, generate

ROM = generate(RomSpec(1000))
F8 = generate(RomSpec(3004, "f8", True))


def make(n=8, roms=(ROM,), env_rom=None, **kw):
    o = oracle.Oracle(n, GRAY, **kw)
    o.load_roms([(r.data, r.scheme) for r in roms])
    o.assign(np.zeros(n, np.uint16) if env_rom is None else env_rom)
    return o


def dec(b):
    b = int(b)
    return 10 * (b >> 4) + (b & 15)


def test_cache_entries_follow_startup_and_noops():
    o = make(2, seed=11)
    ns = set()
    for k in range(30):
        st, obs = o.get_cache(0, k)
        d = decode(st)
        frames = d["ram"][0x54] | (d["ram"][0x55] << 8)     # the ROM's frame counter
        n_k = frames - 64                                  # frame 0 has no counter line
        assert n_k == (oracle.rng(11, 0, 3, k) >> 32) % 31
        ns.add(n_k)
        assert d["err"] == 0 and d["prev_action"] == 0
        assert obs.any()
    assert len(ns) > 10


def test_cache_obs_is_preprocess_of_last_two_frames():
    o = make(1, seed=5)
    st, obs = o.get_cache(0, 3)
    n_total = 1 + 64 + (oracle.rng(5, 0, 3, 3) >> 32) % 31
    _, frames, _, _ = oracle.run_frames(oracle.power_on(ROM.data), ROM.data, int(n_total))
    assert np.array_equal(obs, oracle.preprocess(frames[-2], frames[-1], GRAY))


def test_step_matches_bare_machine():
    o = make(4, seed=3)
    acts = np.array([1, 3, 4, 17], np.uint8)
    starts = [o.get_state(e) for e in range(4)]
    obs, rew, done, frames = o.step(acts, want_frames=True)
    for e in range(4):
        st, fr, _, got = oracle.run_frames(starts[e], ROM.data, 4, actions=np.full(4, acts[e], np.uint8))
        assert got == 4 and not done[e]
        assert np.array_equal(frames[e], fr)
        assert np.array_equal(obs[e], oracle.preprocess(fr[2], fr[3], GRAY))
        after = o.get_state(e)
        assert rew[e] == dec(after[32 + 0x50]) - dec(starts[e][32 + 0x50])
        d0, d1 = decode(starts[e]), decode(after)
        assert d1["step_idx"] == d0["step_idx"] + 1 and d1["prev_action"] == acts[e]
        # everything except the env bookkeeping equals the bare machine's run
        st = st.copy()
        st[184:196] = after[184:196]
        assert not diff_records(st, after), diff_records(st, after)


def test_frameskip_cycles_and_reward_stream():
    o = make(8, seed=1)
    rng = np.random.default_rng(0)
    prev = [o.get_state(e) for e in range(8)]
    for s in range(40):
        obs, rew, done, _ = o.step(rng.integers(0, 18, 8).astype(np.uint8))
        for e in range(8):
            cur = o.get_state(e)
            if not done[e]:
                assert decode(cur)["cycle"] - decode(prev[e])["cycle"] == 4 * 19912
                assert rew[e] == dec(cur[32 + 0x50]) - dec(prev[e][32 + 0x50])
            prev[e] = cur


def test_done_triggers_eager_reset_from_cache():
    o = make(2, seed=9)
    T = ROM.manifest["T"]
    st = o.get_state(1)
    st[32 + 0x54], st[32 + 0x55] = (T - 2) & 0xFF, (T - 2) >> 8   # terminal two frames ahead
    o.set_state(1, st)
    ep = decode(st)["episode_idx"]
    obs, rew, done, frames = o.step(np.array([0, 0], np.uint8), want_frames=True)
    assert done[1] == 1 and done[0] == 0
    assert frames[1][2:].max() == 0 and frames[1][1].any()            # stopped after frame 2
    k = (oracle.rng(9, 1, 2, ep) >> 32) % 30
    cst, cobs = o.get_cache(0, k)
    assert np.array_equal(obs[1], cobs)
    after = o.get_state(1)
    d = decode(after)
    assert d["episode_idx"] == ep + 1 and d["prev_action"] == 0 and d["err"] == 0
    cst = cst.copy()
    cst[184:196] = after[184:196]
    assert not diff_records(cst, after)


def test_sticky_always_equals_noop():
    a = make(4, sticky_threshold=0xFFFFFFFF, seed=21)
    b = make(4, sticky_threshold=0, seed=21)
    rng = np.random.default_rng(1)
    for _ in range(12):
        oa, ra, da, _ = a.step(rng.integers(0, 18, 4).astype(np.uint8))
        ob, rb, db, _ = b.step(np.zeros(4, np.uint8))
        assert np.array_equal(oa, ob) and np.array_equal(ra, rb) and np.array_equal(da, db)
    for e in range(4):
        sa, sb = a.get_state(e), b.get_state(e)
        sa[192] = sb[192]
        assert not diff_records(sa, sb)


def test_sticky_quarter_changes_trajectory_and_is_deterministic():
    runs = []
    for _ in range(2):
        o = make(4, sticky_threshold=0x40000000, seed=21)
        rng = np.random.default_rng(1)
        for _ in range(10):
            o.step(rng.integers(0, 18, 4).astype(np.uint8))
        runs.append(np.stack([o.get_state(e) for e in range(4)]))
    assert np.array_equal(runs[0], runs[1])


def test_batch_composition_invariance():
    full = make(8, roms=(ROM, F8), env_rom=np.array([0, 1] * 4, np.uint16), seed=4,
                sticky_threshold=0x40000000)
    solo = make(8, roms=(ROM, F8), env_rom=np.array([0, 1] * 4, np.uint16), seed=4,
                sticky_threshold=0x40000000)
    rng = np.random.default_rng(2)
    for s in range(6):
        acts = rng.integers(0, 18, 8).astype(np.uint8)
        of, rf, df, _ = full.step(acts)
        for e in [5, 2, 7, 0, 1, 3, 6, 4]:
            os_, rs, ds, _ = solo.step(acts[e:e + 1], env_ids=np.array([e], np.int32))
            assert np.array_equal(os_[0], of[e]) and rs[0] == rf[e] and ds[0] == df[e]
    for e in range(8):
        assert np.array_equal(full.get_state(e), solo.get_state(e))


def test_permuted_ids_step():
    a = make(8, seed=4)
    b = make(8, seed=4)
    acts = np.arange(8, dtype=np.uint8) + 3
    perm = np.array([3, 1, 7, 0, 5, 2, 6, 4], np.int32)
    oa, ra, da, _ = a.step(acts)
    ob, rb, db, _ = b.step(acts[perm], env_ids=perm)
    assert np.array_equal(oa[perm], ob) and np.array_equal(ra[perm], rb)


def test_bad_action_and_error_word():
    o = make(4, seed=2)
    ep = decode(o.get_state(2))["episode_idx"]
    obs, rew, done, _ = o.step(np.array([0, 0, 18, 0], np.uint8))
    assert list(done) == [0, 0, 1, 0] and rew[2] == 0
    first, bits = o.poll_errors()
    assert first == 2 and bits == oracle.ERR_BAD_ACTION
    assert decode(o.get_state(2))["episode_idx"] == ep + 1
    assert o.poll_errors() == (0xFFFFFFFF, 0)


def test_reset_api_and_duplicates():
    o = make(4, seed=2)
    obs = o.reset(np.array([3, 1], np.int32))
    for i, e in enumerate([3, 1]):
        d = decode(o.get_state(e))
        k = (oracle.rng(2, e, 2, d["episode_idx"] - 1) >> 32) % 30
        assert np.array_equal(obs[i], o.get_cache(0, k)[1])
    with pytest.raises(RuntimeError):
        o.reset(np.array([1, 1], np.int32))
    with pytest.raises(RuntimeError):
        o.step(np.zeros(2, np.uint8), env_ids=np.array([0, 4], np.int32))


def test_last2_frames_mode():
    a = make(3, seed=8, render_mode=oracle.RENDER_ALL)
    b = make(3, seed=8, render_mode=oracle.RENDER_LAST2)
    acts = np.array([2, 11, 16], np.uint8)
    oa, ra, da, fa = a.step(acts, want_frames=True)
    ob, rb, db, fb = b.step(acts, want_frames=True)
    assert fb.shape == (3, 2, 210, 160)
    assert np.array_equal(fa[:, 2:], fb) and np.array_equal(oa, ob)


def test_last2_frames_of_an_early_stop_are_zero():
    o = make(2, seed=9, render_mode=oracle.RENDER_LAST2)
    T = ROM.manifest["T"]
    st = o.get_state(0)
    st[32 + 0x54], st[32 + 0x55] = (T - 3) & 0xFF, (T - 3) >> 8    # ends after frame 3 of 4
    o.set_state(0, st)
    _, _, done, fr = o.step(np.array([0, 0], np.uint8), want_frames=True)
    assert done[0] == 1 and fr[0][0].any() and not fr[0][1].any()
    assert fr[1][0].any() and fr[1][1].any()


def bare_run(n_frames):
    """Power-on, then n_frames NOOP frames on the bare machine: the record and
    the last two frames."""
    st, frames, _, got = oracle.run_frames(oracle.power_on(ROM.data), ROM.data, n_frames)
    assert got == n_frames
    return st, frames


def same_machine(a, b):
    """Records equal but for the env bookkeeping (rom, step, episode, prev
    action, error byte)."""
    a, b = a.copy(), b.copy()
    a[180:196] = b[180:196]
    return not diff_records(a, b)


def test_noop_after_copy_assign_reset_and_cache():
    """No-ops after the copy: the cache holds the state two frames before the
    end of the start-up; each reset runs 2 + n NOOP frames, n drawn from
    R(seed, env, 4, episode) -- so an env holds exactly the bare machine after
    1 + 64 + n frames, and the reset's obs is made from that run's last two
    frames."""
    o = make(6, seed=13, noop_after_copy=True, noop_max=7)
    for k in range(30):                                      # all entries alike, 62 start-up frames in
        st, _ = o.get_cache(0, k)
        d = decode(st)
        assert d["ram"][0x54] | (d["ram"][0x55] << 8) == 62
    seen = set()
    for e in range(6):
        n = (oracle.rng(13, e, 4, 0) >> 32) % 8              # assign: episode 0 before the reset
        seen.add(n)
        st = o.get_state(e)
        assert decode(st)["ram"][0x54] == 64 + n
        ref, _ = bare_run(1 + 64 + n)
        assert same_machine(st, ref)
        assert decode(st)["step_idx"] == 0 and decode(st)["episode_idx"] == 1
    assert len(seen) > 1
    # an explicit reset: episode 1 -> 2, its own n, obs of the last two frames
    ids = np.array([2, 4], np.int32)
    obs = o.reset(ids)
    for i, e in enumerate(ids):
        n = (oracle.rng(13, int(e), 4, 1) >> 32) % 8
        ref, frames = bare_run(1 + 64 + n)
        assert same_machine(o.get_state(int(e)), ref)
        assert np.array_equal(obs[i], oracle.preprocess(frames[-2], frames[-1], GRAY))
        assert decode(o.get_state(int(e)))["episode_idx"] == 2


def test_noop_after_copy_eager_reset():
    o = make(2, seed=9, noop_after_copy=True)
    T = ROM.manifest["T"]
    o.step(np.array([0, 0], np.uint8))
    st = o.get_state(1)
    st[32 + 0x54], st[32 + 0x55] = (T - 2) & 0xFF, (T - 2) >> 8   # terminal two frames ahead
    o.set_state(1, st)
    ep = decode(st)["episode_idx"]
    obs, rew, done, _ = o.step(np.array([0, 0], np.uint8))
    assert done[1] == 1 and done[0] == 0
    n = (oracle.rng(9, 1, 4, ep) >> 32) % 31
    ref, frames = bare_run(1 + 64 + n)
    after = o.get_state(1)
    assert same_machine(after, ref)
    assert np.array_equal(obs[1], oracle.preprocess(frames[-2], frames[-1], GRAY))
    d = decode(after)
    assert d["episode_idx"] == ep + 1 and d["step_idx"] == 2 and d["prev_action"] == 0


def test_noop_after_copy_needs_two_startup_frames():
    with pytest.raises(RuntimeError):
        oracle.Oracle(2, GRAY, startup_frames=1, noop_after_copy=True)
