"""Reset no-ops after the copy (vcs_config.noop_after_copy) on the GPU
against the oracle: fuzz cartridges whose episodes end every 30-75 steps, so
eager resets run their 2 + n NOOP frames inside the step (state, reward,
done and the reset observation compared every step), explicit resets of
listed and of all envs, both render modes, sticky actions, tracked latches,
captured graphs on two pipelines, and assign-time no-ops with max_batch
below num_envs (several launches).
"""
import sys

import numpy as np
import pytest

from fuzzcart import S_4K, S_F8, fuzz_cart
from helpers import decode, diff_records
from parity import make_pair, step_both

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_all(o, g, n, tag):
    for e in range(n):
        a, b = g.get_state(e), o.get_state(e)
        assert np.array_equal(a, b), f"{tag}: env {e}: {diff_records(a, b)}"


CASES = [(S_4K, 0, 0, False, 7), (S_F8, 1, 0x40000000, False, 30), (S_4K, 1, 0, True, 12)]


@pytest.mark.parametrize("scheme,mode,sticky,cx,noop_max", CASES,
                         ids=[f"s{c[0]}_r{c[1]}_st{int(c[2] > 0)}_cx{int(c[3])}_m{c[4]}" for c in CASES])
def test_eager_resets_with_noops(scheme, mode, sticky, cx, noop_max):
    seed = 6100 + 7 * scheme + mode + noop_max
    say(f"case: no-ops after copy, scheme {scheme} render_mode {mode} sticky {sticky:#x} collisions {cx} "
        f"noop_max {noop_max} seed {seed}")
    rom, sch = fuzz_cart(seed, scheme=scheme, cx=cx)
    n = 48
    o, g = make_pair([(rom, sch)], np.zeros(n, np.uint16), seed=seed, frameskip=4, render_mode=mode,
                     sticky_threshold=sticky, collisions=cx, noop_after_copy=True, noop_max=noop_max,
                     startup_frames=8)
    compare_all(o, g, n, "after assign")
    rng = np.random.default_rng(seed)
    for s in range(60):
        step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"noops step {s}")
        if s % 10 == 9:
            compare_all(o, g, n, f"noops step {s}")
    assert max(int(decode(o.get_state(e))["episode_idx"]) for e in range(n)) > 1   # episodes did end
    assert g.poll_errors() == o.poll_errors()
    g.close()
    o.close()


def test_explicit_resets_with_noops():
    import torch
    rom, sch = fuzz_cart(6201, scheme=S_4K)
    n = 40
    o, g = make_pair([(rom, sch)], np.zeros(n, np.uint16), seed=77, frameskip=4, noop_after_copy=True,
                     noop_max=9, startup_frames=6)
    rng = np.random.default_rng(5)
    for s in range(3):
        step_both(o, g, rng.integers(0, 18, n), tag=f"step {s}")
    for rep, ids in enumerate([np.array([3, 17, 5, 39], np.int32), None]):
        go = g.reset(None if ids is None else torch.from_numpy(ids).cuda())
        oo = o.reset(ids)
        torch.cuda.synchronize()
        assert np.array_equal(go.cpu().numpy(), oo), f"reset {rep}: obs"
        compare_all(o, g, n, f"after reset {rep}")
        step_both(o, g, rng.integers(0, 18, n), tag=f"step after reset {rep}")
    compare_all(o, g, n, "end")
    g.close()
    o.close()


def test_noops_graph_replays_two_pipelines():
    import torch
    rom, sch = fuzz_cart(6301, scheme=S_F8)
    n = 64
    o, g = make_pair([(rom, sch)], np.zeros(n, np.uint16), gpu_kw={"pipelines": 2}, seed=8, frameskip=4,
                     noop_after_copy=True, noop_max=5, startup_frames=4)
    g.set_launch(16, 0, 256)
    rng = np.random.default_rng(2)
    graph = g.capture(n=n, steps=3, want_frames=True)
    for rep in range(8):
        acts = rng.integers(0, 18, (3, n)).astype(np.uint8)
        obs, rew, done, frames = graph.launch(torch.from_numpy(acts).cuda())
        torch.cuda.synchronize()
        for j in range(3):
            oo, orr, od, of = o.step(acts[j], want_frames=True)
            tag = f"noop graph replay {rep} step {j}"
            assert np.array_equal(done[j].cpu().numpy(), od), tag + ": done"
            assert np.array_equal(rew[j].cpu().numpy(), orr), tag + ": reward"
            assert np.array_equal(obs[j].cpu().numpy(), oo), tag + ": obs"
            assert np.array_equal(frames[j].cpu().numpy(), of), tag + ": frames"
    compare_all(o, g, n, "after replays")
    graph.close()
    g.close()
    o.close()


def test_assign_noops_in_several_launches():
    """max_batch below num_envs: the assign-time no-ops run in chunks."""
    from paper_1907_08467_amd.inputs.romgen import RomSpec, generate
    roms = [generate(RomSpec(2000)), generate(RomSpec(3005, "f8", True))]
    n = 200
    env_rom = (np.arange(n) % 2).astype(np.uint16)
    o, g = make_pair([(r.data, r.scheme) for r in roms], env_rom, gpu_kw={"max_batch": 64}, seed=4,
                     noop_after_copy=True, collisions=True)
    compare_all(o, g, n, "after assign")
    rng = np.random.default_rng(1)
    ids = rng.permutation(n)[:64].astype(np.int32)
    step_both(o, g, rng.integers(0, 18, 64), ids=ids, want_frames=True, tag="listed step")
    compare_all(o, g, n, "after a listed step")
    g.close()
    o.close()


SHAPED = [((8, 0, 128), S_4K, 0), ((16, 1, 512), S_F8, 1), ((1, 0, 64), S_4K, 1)]


@pytest.mark.parametrize("shape,scheme,mode", SHAPED, ids=[f"w{s[0][0]}-p{s[0][1]}-r{s[0][2]}_s{s[1]}_m{s[2]}"
                                                           for s in SHAPED])
def test_noops_collisions_under_launch_shapes(shape, scheme, mode):
    """No-ops after the copy together with tracked latches under narrow,
    persistent and one-env-per-wave launch shapes."""
    seed = 6400 + 3 * scheme + mode + shape[0]
    say(f"case: noops + collisions, launch {shape}, scheme {scheme}, render mode {mode}, seed {seed}")
    rom, sch = fuzz_cart(seed, scheme=scheme, cx=True)
    n = 40
    o, g = make_pair([(rom, sch)], np.zeros(n, np.uint16), seed=seed, frameskip=3, render_mode=mode,
                     collisions=True, noop_after_copy=True, noop_max=6, startup_frames=5)
    g.set_launch(*shape)
    rng = np.random.default_rng(seed)
    for s in range(110):                       # 330 frames: past every fuzz cartridge's episode length
        step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"shaped step {s}")
    compare_all(o, g, n, "end")
    assert max(int(decode(o.get_state(e))["episode_idx"]) for e in range(n)) > 1
    g.close()
    o.close()
