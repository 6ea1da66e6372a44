"""Batching form vs CPU oracle, bit-exact: every launch shape (envs per wave,
persistent interpreter, render workgroup size), the autotuner (results after
tuning are those without it) and HIP-graph-captured steps (each replay equals
the oracle's step, with other work on the device between replays).
"""
import sys

import numpy as np
import pytest
import torch

from parity import compare_states, make_pair, step_both
from paper_1907_08467_amd import binding as B
from paper_1907_08467_amd.inputs.romgen import RomSpec, generate

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_roms():
    """Two 4 KB and two F8 divergent cartridges."""
    specs = [RomSpec(3000, "4k", True), RomSpec(3005, "f8", True), RomSpec(3002, "4k", True),
             RomSpec(3006, "f8", True)]
    return [(r.data, r.scheme) for r in map(generate, specs)]


def uneven_assignment(n, seed):
    rng = np.random.default_rng(seed)
    counts = [n // 2, n // 4, n // 8]
    counts.append(n - sum(counts))
    return rng.permutation(np.repeat(np.arange(4, dtype=np.uint16), counts))


SHAPES = [(1, 0, 64), (4, 0, 128), (16, 8, 512), (64, 3, 256), (8, 1, 256), (32, 0, 512)]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"w{a}-p{b}-r{c}" for a, b, c in SHAPES])
def test_launch_shape_parity(shape):
    w, workers, blk = shape
    n = 203
    say(f"case: launch shape tile_envs={w} workers={workers} render_block={blk}, {n} envs")
    o, g = make_pair(mixed_roms(), uneven_assignment(n, w), seed=11, sticky_threshold=0x40000000)
    g.set_launch(w, workers, blk)
    assert g.get_launch() == {"tile_envs": w, "workers": workers, "render_block": blk}
    rng = np.random.default_rng(w)
    for s in range(10):
        step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"shape {shape} step {s}")
    compare_states(o, g, range(n), f"shape {shape}")
    # listed ids: a permuted subset with a ragged count
    ids = rng.permutation(n)[:77].astype(np.int32)
    for s in range(4):
        step_both(o, g, rng.integers(0, 18, ids.size), ids=ids, want_frames=True, tag=f"shape {shape} ids step {s}")
    compare_states(o, g, range(n), f"shape {shape} after listed steps")
    assert g.poll_errors() == o.poll_errors()


def test_bad_launch_rejected():
    say("case: invalid launch shapes")
    rom = generate(RomSpec(1000))
    _, g = make_pair([(rom.data, rom.scheme)], np.zeros(8, np.uint16))
    for bad in [(0, 0, 256), (3, 0, 256), (128, 0, 256), (64, 0, 100), (64, 0, 1024), (64, 1 << 21, 256)]:
        with pytest.raises(B.VcsError):
            g.set_launch(*bad)
    assert g.get_launch() == {"tile_envs": 64, "workers": 0, "render_block": 256}


def test_autotune_keeps_results():
    n = 640
    say(f"case: autotune in the middle of an episode stream, {n} envs")
    o, g = make_pair(mixed_roms(), uneven_assignment(n, 5), seed=3)
    rng = np.random.default_rng(9)
    for s in range(3):
        step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"pre-tune step {s}")
    best, ms = g.autotune(steps=2, want_frames=True, want_obs=True)
    say("autotune picked", best, f"{ms:.3f} ms/step")
    assert best == g.get_launch()
    assert ms > 0
    assert g.poll_errors() == o.poll_errors()
    compare_states(o, g, range(n), "right after autotune")
    for s in range(6):
        step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"post-tune step {s}")
    compare_states(o, g, range(n), "post-tune")


@pytest.mark.parametrize("listed,pipes,steps", [(False, 1, 2), (True, 1, 2), (False, 2, 3), (True, 2, 4)],
                         ids=["all-envs", "listed-ids", "all-envs-overlapped", "listed-ids-overlapped"])
def test_graph_replays(listed, pipes, steps):
    """With two pipelines the captured steps alternate pipelines and each
    step's render overlaps the next step's interpreter."""
    n_envs = 150
    say(f"case: captured {steps}-step graph, {n_envs} envs, listed={listed}, pipelines={pipes}")
    o, g = make_pair(mixed_roms(), uneven_assignment(n_envs, 2), gpu_kw={"pipelines": pipes}, seed=21,
                     sticky_threshold=0x20000000)
    g.set_launch(16, 0, 256)
    rng = np.random.default_rng(4)
    ids = rng.permutation(n_envs)[:97].astype(np.int32) if listed else None
    n = ids.size if listed else n_envs
    graph = g.capture(n=n, steps=steps, env_ids=ids, want_frames=True)
    side = torch.zeros(1 << 20, device="cuda")
    for rep in range(5):
        acts = rng.integers(0, 18, (steps, n)).astype(np.uint8)
        obs, rew, done, frames = graph.launch(torch.from_numpy(acts).cuda())
        side.add_(1.0)                      # unrelated device work between replays
        torch.cuda.synchronize()
        for j in range(steps):
            oo, orr, od, of = o.step(acts[j], env_ids=ids, want_frames=True)
            tag = f"graph replay {rep} step {j}"
            assert np.array_equal(done[j].cpu().numpy(), od), tag + ": done"
            assert np.array_equal(rew[j].cpu().numpy(), orr), tag + ": reward"
            assert np.array_equal(obs[j].cpu().numpy(), oo), tag + ": obs"
            assert np.array_equal(frames[j].cpu().numpy(), of), tag + ": frames"
        compare_states(o, g, range(n_envs), f"after replay {rep}")
        # an eager step between replays
        a = rng.integers(0, 18, n_envs)
        step_both(o, g, a, want_frames=False, tag=f"eager step after replay {rep}")
    assert float(side[0]) == 5.0
    g.set_launch(64, 0, 256)
    with pytest.raises(B.VcsError):
        graph.launch()
    graph.close()
    assert g.poll_errors() == o.poll_errors()


def test_pipelines_overlap():
    """Two pipelines on two streams step disjoint env sets at the same time."""
    n_envs = 256
    say(f"case: 2 pipelines on 2 streams, {n_envs} envs, disjoint random halves per step")
    o, g = make_pair(mixed_roms(), uneven_assignment(n_envs, 8), gpu_kw={"pipelines": 2}, seed=5)
    g.set_launch(8, 0, 256)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    rng = np.random.default_rng(17)
    for k in range(8):
        perm = rng.permutation(n_envs).astype(np.int32)
        ids_a, ids_b = perm[:120], perm[120:240]
        act_a, act_b = rng.integers(0, 18, 120), rng.integers(0, 18, 120)
        ra = g.step(torch.from_numpy(act_a.astype(np.uint8)).cuda(), env_ids=ids_a, pipe=0, stream=s1,
                    want_frames=True)
        rb = g.step(torch.from_numpy(act_b.astype(np.uint8)).cuda(), env_ids=ids_b, pipe=1, stream=s2,
                    want_frames=True)
        torch.cuda.synchronize()
        for ids, act, res, name in ((ids_a, act_a, ra, "a"), (ids_b, act_b, rb, "b")):
            oo, orr, od, of = o.step(act, env_ids=ids, want_frames=True)
            tag = f"pipelines step {k} half {name}"
            assert np.array_equal(res[2].cpu().numpy(), od), tag + ": done"
            assert np.array_equal(res[1].cpu().numpy(), orr), tag + ": reward"
            assert np.array_equal(res[0].cpu().numpy(), oo), tag + ": obs"
            assert np.array_equal(res[3].cpu().numpy(), of), tag + ": frames"
    compare_states(o, g, range(n_envs), "after pipelined steps")
    assert g.poll_errors() == o.poll_errors()
    with pytest.raises(B.VcsError):
        g.step(torch.zeros(4, dtype=torch.uint8, device="cuda"), env_ids=np.arange(4), pipe=2)
