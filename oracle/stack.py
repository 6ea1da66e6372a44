"""Frame stack oracle (test infrastructure only; the library never uses it).

Follows the paper's Section 5 ("Memory limitations"): each env keeps its last
D observations (the paper's agents use D = 4).  Stated here as the plain
definition, one env at a time:

- the stack of an env is the list of its last D pushed observations, oldest
  first;
- a push with done set starts a new episode: the stack becomes D copies of
  the pushed observation;
- with 4-bit storage each stored pixel is the top nibble q = v // 16 of the
  gray level, and reads back as 17 * q (0..255); 8-bit storage reads back
  unchanged.
"""
from __future__ import annotations

import numpy as np


class FrameStack:
    def __init__(self, num_envs: int, depth: int = 4, bits: int = 8):
        assert bits in (4, 8) and depth >= 1
        self.depth, self.bits = depth, bits
        # before any push every slot is zero, like the library's fresh stack
        self.frames = [[np.zeros((84, 84), np.uint8) for _ in range(depth)] for _ in range(num_envs)]

    def stored(self, obs: np.ndarray) -> np.ndarray:
        """What a slot holds (read back in 8 bits) for observation obs."""
        if self.bits == 8:
            return obs.copy()
        return ((obs.astype(np.int32) // 16) * 17).astype(np.uint8)

    def push(self, obs, done=None, env_ids=None) -> np.ndarray:
        obs = np.asarray(obs, np.uint8)
        n = obs.shape[0]
        ids = range(n) if env_ids is None else [int(e) for e in env_ids]
        out = np.zeros((n, self.depth, 84, 84), np.uint8)
        for i, e in enumerate(ids):
            if not (0 <= e < len(self.frames)):
                continue
            v = self.stored(obs[i])
            if done is not None and done[i]:
                self.frames[e] = [v.copy() for _ in range(self.depth)]
            else:
                self.frames[e] = self.frames[e][1:] + [v]
            out[i] = np.stack(self.frames[e])
        return out
