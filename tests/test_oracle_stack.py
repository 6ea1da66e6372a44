"""Pins of the frame-stack oracle against its definition (Section 5 of the
paper: the last four observations per env), checked with properties a wrong
order, a missing reset or a wrong quantisation would break."""
import numpy as np

from oracle.stack import FrameStack


def obs_seq(rng, k, n):
    return rng.integers(0, 256, (k, n, 84, 84)).astype(np.uint8)


def test_last_depth_in_order():
    rng = np.random.default_rng(0)
    fs = FrameStack(3, depth=4)
    seq = obs_seq(rng, 7, 3)
    for t in range(7):
        out = fs.push(seq[t])
    for d in range(4):                       # oldest first: frames 3, 4, 5, 6
        assert np.array_equal(out[:, d], seq[3 + d])


def test_fresh_stack_is_zero_then_fills():
    rng = np.random.default_rng(1)
    fs = FrameStack(2, depth=4)
    a = obs_seq(rng, 1, 2)[0]
    out = fs.push(a)
    assert not out[:, :3].any() and np.array_equal(out[:, 3], a)


def test_done_fills_every_slot():
    rng = np.random.default_rng(2)
    fs = FrameStack(4, depth=4)
    seq = obs_seq(rng, 6, 4)
    for t in range(5):
        fs.push(seq[t])
    done = np.array([1, 0, 1, 0], np.uint8)
    out = fs.push(seq[5], done=done)
    for d in range(4):
        assert np.array_equal(out[0, d], seq[5, 0]) and np.array_equal(out[2, d], seq[5, 2])
    assert np.array_equal(out[1, 0], seq[2, 1]) and np.array_equal(out[1, 3], seq[5, 1])


def test_ids_subset_and_permutation():
    rng = np.random.default_rng(3)
    full = FrameStack(5, depth=2)
    part = FrameStack(5, depth=2)
    seq = obs_seq(rng, 3, 5)
    for t in range(3):
        full.push(seq[t])
        perm = rng.permutation(5)
        part.push(seq[t][perm], env_ids=perm)
    assert all(np.array_equal(np.stack(full.frames[e]), np.stack(part.frames[e])) for e in range(5))


def test_four_bit_readback():
    fs = FrameStack(1, depth=1, bits=4)
    v = np.arange(256, dtype=np.uint8)
    img = np.resize(v, (84, 84))[None]
    out = fs.push(img)[0, 0]
    # q * 17: 0, 17, ..., 255 and the 16 levels cover 0..255 in steps of 16
    assert set(np.unique(out).tolist()) == {17 * q for q in range(16)}
    assert np.array_equal(out, (img[0] >> 4) * 17)
    assert (np.abs(out.astype(int) - img[0].astype(int)) <= 15).all()
