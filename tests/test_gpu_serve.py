"""Env server on the GPU: served results equal solo results, bit for bit.

Actors send overlapping requests while batches are on the device (two
pipelines).  Every request is then replayed alone, one step call per request
in arrival order, on a fresh GPU context, and its observations, rewards and
done flags must be identical; the oracle replays the same requests as well.
"""
import sys
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1907_08467_amd.env import VcsEnv
from paper_1907_08467_amd.inputs.palette import GRAY
from paper_1907_08467_amd.inputs.romgen import RomSpec, generate
from paper_1907_08467_amd.serve import ActorPool, EnvServer, GpuBackend, run_served

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_served_equals_solo_gpu():
    specs = [RomSpec(4000, "4k", True), RomSpec(4001, "f8", True), RomSpec(4002, "4k", True),
             RomSpec(4003, "f8", True)]
    roms = [(r.data, r.scheme) for r in map(generate, specs)]
    n_envs, cap = 2048, 512
    env_rom = (np.arange(n_envs) % 4).astype(np.uint16)
    cfg = dict(frameskip=4, render_mode=1, seed=13, sticky_threshold=0x40000000)
    say(f"case: served vs solo, {n_envs} envs, 2 pipelines, batch cap {cap}")
    g = VcsEnv(roms, env_rom, GRAY, max_batch=cap, pipelines=2, **cfg)
    g.set_launch(16, 0, 256)
    backend = GpuBackend(g, cap)
    served = {}

    def keep(req, obs, rew, done):
        served[req.seq] = (req, obs.cpu().numpy(), rew.cpu().numpy(), done.cpu().numpy())

    server = EnvServer(backend, cap, n_envs, on_result=keep)
    actors = ActorPool(8, n_envs, mean_wait_s=3e-4, size_lo=16, size_hi=256, seed0=900)
    t0 = time.perf_counter()
    stats = run_served(server, actors, seconds=1.5)
    say("served:", stats, f"deferred {server.deferred}", f"wall {time.perf_counter() - t0:.2f}s")
    assert stats["requests"] == len(served) > 20
    assert server.deferred > 0
    assert max(server.batch_sizes) <= cap

    solo = VcsEnv(roms, env_rom, GRAY, max_batch=cap, **cfg)
    o = oracle.Oracle(n_envs, GRAY, **cfg)
    o.load_roms(roms)
    o.assign(env_rom)
    for seq in sorted(served):
        req, obs, rew, done = served[seq]
        so, sr, sd, _ = solo.step(torch.from_numpy(req.actions).cuda(), env_ids=req.ids)
        tag = f"request {seq} ({req.ids.size} envs)"
        assert np.array_equal(sd.cpu().numpy(), done), tag + ": done, served vs solo"
        assert np.array_equal(sr.cpu().numpy(), rew), tag + ": reward, served vs solo"
        assert np.array_equal(so.cpu().numpy(), obs), tag + ": obs, served vs solo"
        oo, orr, od, _ = o.step(req.actions, env_ids=req.ids)
        assert np.array_equal(od, done) and np.array_equal(orr, rew) and np.array_equal(oo, obs), \
            tag + ": served vs oracle"
    for e in range(0, n_envs, 37):
        assert np.array_equal(g.get_state(e), o.get_state(e)), f"env {e} state"
    assert g.poll_errors()[1] == 0
