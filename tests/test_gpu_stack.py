"""Frame stack on the GPU vs the oracle's frame stack fed with the oracle
env's observations: 8-bit and 4-bit storage, all envs and listed ids,
episode ends inside the run.
"""
import sys

import numpy as np
import pytest
import torch

from oracle.stack import FrameStack as OracleStack
from parity import make_pair
from paper_1907_08467_amd import binding as B
from paper_1907_08467_amd.env import FrameStack
from paper_1907_08467_amd.inputs.romgen import RomSpec, generate

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("bits,depth,listed", [(8, 4, False), (4, 4, False), (8, 3, True), (4, 2, True)])
def test_stack_parity(bits, depth, listed):
    n_envs = 96
    say(f"case: frame stack bits={bits} depth={depth} listed={listed}, {n_envs} envs")
    roms = [(r.data, r.scheme) for r in (generate(RomSpec(1000)), generate(RomSpec(3005, "f8", True)))]
    o, g = make_pair(roms, np.arange(n_envs, dtype=np.uint16) % 2, seed=31)
    gs = FrameStack(g, depth=depth, bits=bits)
    os_ = OracleStack(n_envs, depth=depth, bits=bits)
    rng = np.random.default_rng(bits + depth)
    ended = 0
    for s in range(40):
        if listed:
            ids = rng.permutation(n_envs)[:61].astype(np.int32)
        else:
            ids = None
        n = n_envs if ids is None else ids.size
        a = rng.integers(0, 18, n).astype(np.uint8)
        go, _, gd, _ = g.step(torch.from_numpy(a).cuda(), env_ids=ids)
        oo, _, od, _ = o.step(a, env_ids=ids)
        first = s == 0 and not listed
        gdone = torch.ones_like(gd) if first else gd
        odone = np.ones_like(od) if first else od
        gout = gs.push(go, gdone, env_ids=ids).cpu().numpy()
        oout = os_.push(oo, odone, env_ids=ids)
        ended += int(od.sum())
        bad = np.nonzero((gout != oout).reshape(n, -1).any(axis=1))[0]
        assert bad.size == 0, f"step {s}: stacks differ at positions {bad[:8].tolist()}"
    say(f"episodes ended during the run: {ended}")
    gs.close()


def test_stack_rejects_bad_arguments():
    rom = generate(RomSpec(1000))
    _, g = make_pair([(rom.data, rom.scheme)], np.zeros(4, np.uint16))
    for depth, bits in [(0, 8), (17, 8), (4, 6)]:
        with pytest.raises(B.VcsError):
            FrameStack(g, depth=depth, bits=bits)
    fs = FrameStack(g, depth=4)
    with pytest.raises(B.VcsError):
        B.vcs_stack_push(fs._s, None, 8, torch.zeros((8, 84, 84), dtype=torch.uint8, device="cuda").data_ptr(),
                         None, None, None)
    fs.close()
