"""Policy network on the GPU (bf16 MFMA) vs the float64 oracle.

Tolerance: the GPU rounds the output of each of the 4 hidden layers to bf16
(relative error at most 2^-9); the input pixels are exact in bf16, weights are
bf16 on both sides and the fp32 accumulation adds far less.  A logit is a sum
of terms larger than itself (the head's 512 products cancel), so these 4
roundings can move it by several times 4 * 2^-9 = 0.008 of the output RMS;
random stacks and random He-uniform weights measure up to 0.028.  The test
allows LOGIT_TOL = 0.04 of each env's output RMS.  A GPU action must be the
oracle's unless another logit lies within 2 * LOGIT_TOL of the oracle's
maximum, and must always be one of those near-maximal logits.
"""
import sys

import numpy as np
import pytest
import torch

from oracle.policy import forward, greedy
from oracle.stack import FrameStack as OracleStack
from parity import make_pair
from paper_1907_08467_amd import binding as B
from paper_1907_08467_amd.env import FrameStack, Policy
from paper_1907_08467_amd.inputs.policy_weights import policy_weights
from paper_1907_08467_amd.inputs.romgen import RomSpec, generate
from test_oracle_policy import delta_layers, delta_pixel

pytestmark = pytest.mark.gpu

LOGIT_TOL = 0.04


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_policy(g, layers):
    return Policy(g, [l[0] for l in layers], [l[2] for l in layers])


def check_outputs(glog, gact, ref):
    """Element-wise logits within tolerance; actions exact or near-tied."""
    scale = np.sqrt((ref ** 2).mean(axis=1, keepdims=True)) + 1e-6
    err = np.abs(glog[:, :19] - ref) / scale
    worst = float(err.max())
    assert worst <= LOGIT_TOL, f"logit error {worst:.4f} of the output RMS (env {int(err.max(axis=1).argmax())})"
    oact = greedy(ref)
    top = ref[:, :18].max(axis=1)
    gap_tol = 2 * LOGIT_TOL * scale[:, 0]
    for i in range(ref.shape[0]):
        near = np.nonzero(ref[i, :18] >= top[i] - gap_tol[i])[0]
        assert gact[i] in near, f"env {i}: action {gact[i]} not among near-maximal {near.tolist()}"
        if near.size == 1:
            assert gact[i] == oact[i]
    # the GPU's argmax is the first maximal of its own logits
    assert np.array_equal(gact, np.argmax(glog[:, :18], axis=1))
    return worst


def env_for(n):
    rom = generate(RomSpec(1000))
    _, g = make_pair([(rom.data, rom.scheme)], np.zeros(n, np.uint16))
    return g


@pytest.mark.parametrize("n", [1, 61, 130])
def test_policy_random_stacks(n):
    say(f"case: policy on {n} random stacks")
    g = env_for(max(n, 8))
    layers = policy_weights(7)
    P = make_policy(g, layers)
    rng = np.random.default_rng(n)
    stack = rng.integers(0, 256, (n, 4, 84, 84)).astype(np.uint8)
    act, lg = P.act(torch.from_numpy(stack).cuda(), want_logits=True)
    worst = check_outputs(lg.cpu().numpy().astype(np.float64), act.cpu().numpy(), forward(stack, layers))
    say(f"n={n}: worst logit error {worst:.5f} of the output RMS")
    P.close()


def test_policy_delta_network():
    """Single-weight selections: logit 7 is one input pixel / 255, the rest 0."""
    say("case: policy delta network")
    g = env_for(8)
    rng = np.random.default_rng(3)
    stack = rng.integers(0, 256, (8, 4, 84, 84)).astype(np.uint8)
    for args in [dict(), dict(ci=0, k1=(7, 7), k2=(3, 3), k3=(0, 2), yx4=(6, 4))]:
        P = make_policy(g, delta_layers(**args))
        act, lg = P.act(torch.from_numpy(stack).cuda(), want_logits=True)
        lg = lg.cpu().numpy()
        c, y, x = delta_pixel(**args)
        want = stack[:, c, y, x] / 255.0
        assert np.all(np.abs(lg[:, 7] - want) <= want * 2.0 ** -8)
        assert not np.delete(lg[:, :19], 7, axis=1).any()
        assert np.array_equal(act.cpu().numpy(), np.where(stack[:, c, y, x] > 0, 7, 0))
        P.close()


def test_policy_rejects_bad_arguments():
    g = env_for(8)
    layers = policy_weights(7)
    P = make_policy(g, layers)
    big = torch.zeros((g.num_envs + 1, 4, 84, 84), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.VcsError):
        P.act(big)
    with pytest.raises(B.VcsError):
        B.vcs_policy_act(P._p, big.data_ptr(), 4, None, None, None)
    empty = torch.zeros((0, 4, 84, 84), dtype=torch.uint8, device="cuda")
    a, _ = P.act(empty)
    assert a.numel() == 0
    with pytest.raises(ValueError):
        P.act(torch.zeros((2, 3, 84, 84), dtype=torch.uint8, device="cuda"))
    P.close()


def test_inference_loop_parity():
    """Emulation + frame stack + policy on the GPU, actions from the GPU's
    policy; the oracle env steps with the same actions (bit-exact emulation
    and stacks) and its policy checks the GPU's logits and actions."""
    n_envs = 64
    say(f"case: inference loop, {n_envs} envs")
    roms = [(r.data, r.scheme) for r in (generate(RomSpec(1000)), generate(RomSpec(3005, "f8", True)))]
    o, g = make_pair(roms, np.arange(n_envs, dtype=np.uint16) % 2, seed=17)
    layers = policy_weights(11)
    P = make_policy(g, layers)
    gs, os_ = FrameStack(g, depth=4, bits=8), OracleStack(n_envs, depth=4, bits=8)
    gobs = g.reset()
    oobs = o.reset()
    gst = gs.push(gobs, torch.ones(n_envs, dtype=torch.uint8, device="cuda"))
    ost = os_.push(oobs, np.ones(n_envs, np.uint8))
    worst, ended = 0.0, 0
    for s in range(24):
        assert np.array_equal(gst.cpu().numpy(), ost), f"step {s}: stacks differ"
        act, lg = P.act(gst, want_logits=True)
        a = act.cpu().numpy()
        worst = max(worst, check_outputs(lg.cpu().numpy().astype(np.float64), a, forward(ost, layers)))
        go, _, gd, _ = g.step(act)
        oo, _, od, _ = o.step(a)
        gst = gs.push(go, gd)
        ost = os_.push(oo, od)
        ended += int(od.sum())
    say(f"inference loop: 24 steps agree, worst logit error {worst:.5f}, episodes ended {ended}")
    P.close()
    gs.close()
