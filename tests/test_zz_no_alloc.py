"""vcs_step_noalloc (the step entry point that allocates nothing, for callers
that cannot allocate) against vcs_step through the C ABI: two contexts with
the same configuration, cartridges and env assignment; one steps with
vcs_step, the other with vcs_step_noalloc, on the same env ids and actions.
Observations, rewards, done flags and the full machine state of every
listed env must be identical (integer work: bit-exact), over consecutive
calls whose sizes shrink, so the second call runs on scratch the first one
left behind."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(roms, env_rom, **cfg):
    from paper_1907_08467_amd.env import VcsEnv
    from paper_1907_08467_amd.inputs.palette import GRAY
    a = VcsEnv(roms, env_rom, GRAY, **cfg)
    b = VcsEnv(roms, env_rom, GRAY, **cfg)
    return a, b


def _noalloc(env, ids, actions):
    import torch
    from paper_1907_08467_amd import binding as B
    n = actions.numel()
    obs = torch.empty((n, 84, 84), dtype=torch.uint8, device=env.device)
    rew = torch.empty(n, dtype=torch.int32, device=env.device)
    done = torch.empty(n, dtype=torch.uint8, device=env.device)
    B.vcs_step_noalloc(env._h, ids.data_ptr() if ids is not None else None, actions.data_ptr(), n,
                       obs.data_ptr(), rew.data_ptr(), done.data_ptr(), env._stream())
    return obs, rew, done


CASES = [("4k+f8, all frames", 0, False), ("4k+f8, last two frames", 1, False),
         ("objects, latches tracked, last two frames", 1, True)]


@pytest.mark.parametrize("name,mode,objects", CASES, ids=["all", "last2", "objects"])
def test_noalloc_equals_step(name, mode, objects):
    import torch
    from paper_1907_08467_amd.inputs.romgen import RomSpec, generate
    if objects:
        roms = [(r.data, r.scheme) for r in (generate(RomSpec(7000, objects=True)),
                                             generate(RomSpec(7101, "f8", True, objects=True)))]
    else:
        roms = [(r.data, r.scheme) for r in (generate(RomSpec(4011)), generate(RomSpec(4001, "f8", True)))]
    num = 700
    env_rom = (np.arange(num) % 2).astype(np.uint16)
    a, b = _pair(roms, env_rom, frameskip=4, seed=9, render_mode=mode, collisions=objects)
    rng = np.random.default_rng(17)
    dev = a.device
    for call, n in enumerate([480, 96, 512, 33, 300, 7]):
        say(f"case: no-alloc vs step, {name}, call {call}, {n} envs")
        ids_np = rng.choice(num, size=n, replace=False).astype(np.int32)
        ids = torch.from_numpy(ids_np).to(dev)
        act = torch.from_numpy(rng.integers(0, 18, n).astype(np.uint8)).to(dev)
        oa, ra, da, _ = a.step(act, env_ids=ids)
        ob, rb, db = _noalloc(b, ids, act)
        torch.cuda.synchronize()
        assert torch.equal(da, db), f"{name} call {call}: done differs"
        assert torch.equal(ra, rb), f"{name} call {call}: reward differs"
        assert torch.equal(oa, ob), f"{name} call {call}: obs differ"
        for e in ids_np[:64]:
            assert np.array_equal(a.get_state(int(e)), b.get_state(int(e))), f"{name} call {call}: env {e} state"
    # implicit ids 0..n-1
    n = 200
    act = torch.from_numpy(rng.integers(0, 18, n).astype(np.uint8)).to(dev)
    oa, ra, da, _ = a.step(act)
    ob, rb, db = _noalloc(b, None, act)
    torch.cuda.synchronize()
    assert torch.equal(da, db) and torch.equal(ra, rb) and torch.equal(oa, ob), f"{name}: implicit ids differ"
    for e in range(num):
        assert np.array_equal(a.get_state(e), b.get_state(e)), f"{name}: env {e} state at the end"
    assert a.poll_errors() == b.poll_errors()
    a.close()
    b.close()


def test_noalloc_rejects_beyond_its_limit():
    """More than 512 envs in one call: an argument error before any work."""
    import torch
    from paper_1907_08467_amd import binding as B
    from paper_1907_08467_amd.inputs.romgen import RomSpec, generate
    rom = generate(RomSpec(4011))
    a, _ = _pair([(rom.data, rom.scheme)], np.zeros(600, np.uint16), frameskip=4, seed=1)
    act = torch.zeros(513, dtype=torch.uint8, device=a.device)
    with pytest.raises(B.VcsError) as ei:
        _noalloc(a, None, act)
    assert ei.value.code == B.VCS_E_INVAL and "512" in str(ei.value)
    a.close()
