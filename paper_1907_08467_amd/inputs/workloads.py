"""The workload configurations, as seeded synthetic inputs.

Each configuration stands in for the paper's emulation-only measurements on
its game suite (Section 4, Fig. 2a and Fig. 3) with synthetic cartridges from
``romgen``; shapes follow the paper (frameskip 4, 210x160 frames, 84x84
observations, 18 actions, a 30-entry reset cache, env counts around the
paper's 512 and 4096 points).  ROM r of configuration c uses seed 1000*c + r.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .romgen import RomSpec, generate

N_ACTIONS = 18
RENDER_ALL, RENDER_LAST2 = 0, 1


@dataclasses.dataclass
class Workload:
    name: str
    n_envs: int
    rom_specs: list
    steps: int
    frameskip: int = 4
    action_seed: int = 0
    sticky_threshold: int = 0       # floor(p * 2**32)
    render_mode: int = RENDER_ALL
    rng_seed: int = 0
    counts: list | None = None      # envs per ROM (None = even split)
    assign_seed: int | None = None  # shuffle env ids across ROMs
    collisions: bool = False        # collision latches tracked

    def roms(self):
        return [generate(s) for s in self.rom_specs]

    def env_rom(self) -> np.ndarray:
        n_roms = len(self.rom_specs)
        counts = self.counts or [self.n_envs // n_roms] * n_roms
        assert sum(counts) == self.n_envs
        lab = np.repeat(np.arange(n_roms, dtype=np.uint16), counts)
        if self.assign_seed is not None:
            lab = np.random.Generator(np.random.PCG64(self.assign_seed)).permutation(lab)
        return lab.astype(np.uint16)

    def actions(self, steps: int | None = None, n: int | None = None) -> np.ndarray:
        """uint8 [steps, n] uniform over the 18 actions, PCG64(action_seed)."""
        steps = self.steps if steps is None else steps
        n = self.n_envs if n is None else n
        g = np.random.Generator(np.random.PCG64(self.action_seed))
        return g.integers(0, N_ACTIONS, (steps, n), dtype=np.uint8)


def zipf_counts(n: int, k: int, s: float) -> list[int]:
    """Largest-remainder split of n over k ranks with weights 1/r^s."""
    w = np.array([1.0 / (r ** s) for r in range(1, k + 1)])
    q = w / w.sum() * n
    base = np.floor(q).astype(np.int64)
    rem = n - int(base.sum())
    order = np.argsort(-(q - base), kind="stable")
    base[order[:rem]] += 1
    return [int(x) for x in base]


def _mixed16(c):
    return [RomSpec(1000 * c + r, "4k" if r % 2 == 0 else "f8", True) for r in range(16)]


def config(c: int) -> Workload:
    if c == 1:
        return Workload("plain-c1: 8 envs, 1 ROM 4KB, 500 steps", 8, [RomSpec(1000)], 500,
                        action_seed=0, rng_seed=1)
    if c == 2:
        return Workload("plain-batch: 4096 envs, 1 ROM 4KB, frameskip 4, render all",
                        4096, [RomSpec(2000)], 10000, action_seed=1, rng_seed=2)
    if c == 3:
        specs = [RomSpec(3000 + r, "4k" if r < 4 else "f8", True) for r in range(8)]
        return Workload("divergent: 32768 envs, 8 ROMs (4x4KB, 4xF8), sticky 0.25", 32768, specs,
                        5000, action_seed=2, sticky_threshold=0x40000000, rng_seed=3)
    if c == 4:
        return Workload("batching: 65536 envs, 16 ROMs Zipf 1.2, render last 2", 65536, _mixed16(4),
                        2000, action_seed=3, render_mode=RENDER_LAST2, rng_seed=4,
                        counts=zipf_counts(65536, 16, 1.2), assign_seed=104)
    if c == 6:
        kinds = ["4k", "f8", "f6", "f4", "f8sc", "f6sc", "f4sc", "e0", "3f"]
        specs = [RomSpec(6000 + r, k, True) for r, k in enumerate(kinds)]
        return Workload("mixed schemes: 36864 envs, 9 ROMs (every cartridge scheme), sticky 0.25, render last 2",
                        36864, specs, 2000, action_seed=6, sticky_threshold=0x40000000,
                        render_mode=RENDER_LAST2, rng_seed=6, assign_seed=106)
    if c == 7:
        return Workload("objects: 4096 envs, 1 objects ROM 4KB (missiles, ball, NUSIZ, object motion, "
                        "collision reads), frameskip 4, render all, collisions tracked",
                        4096, [RomSpec(7000, objects=True)], 10000, action_seed=7, rng_seed=7, collisions=True)
    if c == 5:
        return Workload("serving: 131072 resident envs, 16 ROMs Zipf 1.2", 131072, _mixed16(4),
                        0, action_seed=5, render_mode=RENDER_LAST2, rng_seed=5,
                        counts=zipf_counts(131072, 16, 1.2), assign_seed=105)
    raise ValueError(c)
