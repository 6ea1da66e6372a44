"""Batched Atari 2600 envs on one GPU: a thin torch-facing wrapper of the C ABI.

Device memory comes from torch tensors and work is enqueued on torch's
current stream; every computation happens in the HIP library.
"""

from __future__ import annotations

import numpy as np
import torch

from . import binding as B


class VcsEnv:
    """`num_envs` consoles, each running one of `roms` ([(bytes, scheme)])."""

    def __init__(self, roms, env_rom, gray_lut, frameskip=4, sticky_threshold=0, reset_cache_k=30,
                 noop_max=30, startup_frames=64, seed=0, render_mode=B.VCS_RENDER_ALL, max_batch=0,
                 hbm_budget_bytes=0, device=0, pipelines=1, collisions=False, noop_after_copy=False):
        env_rom = np.ascontiguousarray(env_rom, dtype=np.uint16)
        cfg = B.VcsConfig()
        cfg.num_envs = int(env_rom.shape[0])
        cfg.frameskip = frameskip
        cfg.sticky_threshold = sticky_threshold
        cfg.reset_cache_k = reset_cache_k
        cfg.noop_max = noop_max
        cfg.startup_frames = startup_frames
        cfg.seed = seed
        cfg.render_mode = render_mode
        cfg.max_batch = max_batch
        cfg.hbm_budget_bytes = hbm_budget_bytes
        cfg.device = device
        cfg.pipelines = pipelines
        cfg.collisions = 1 if collisions else 0
        cfg.noop_after_copy = 1 if noop_after_copy else 0
        for i, g in enumerate(bytes(gray_lut)):
            cfg.gray_lut[i] = g
        self.num_envs = cfg.num_envs
        self.pipelines = max(1, pipelines)
        self.frameskip = frameskip
        self.render_mode = render_mode
        self.max_batch = max_batch or cfg.num_envs
        self.device = torch.device("cuda", device)
        self._h = B.vcs_create(cfg)
        B.vcs_load_roms(self._h, [r for r, _ in roms], [s for _, s in roms])
        B.vcs_assign(self._h, env_rom)

    def close(self):
        if getattr(self, "_h", None):
            B.vcs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_slots(self):
        return self.frameskip if self.render_mode == B.VCS_RENDER_ALL else 2

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def _ids(self, env_ids):
        if env_ids is None:
            return None, None
        ids = torch.as_tensor(env_ids, dtype=torch.int32, device=self.device).contiguous()
        return ids, ids.data_ptr()

    def reset(self, env_ids=None, n=None, obs=None):
        ids, ids_ptr = self._ids(env_ids)
        n = ids.numel() if ids is not None else (self.num_envs if n is None else n)
        if obs is None:
            obs = torch.empty((n, 84, 84), dtype=torch.uint8, device=self.device)
        B.vcs_reset(self._h, ids_ptr, n, obs.data_ptr(), self._stream())
        return obs

    def step(self, actions, env_ids=None, want_frames=False, want_obs=True, out=None, pipe=0, stream=None):
        """actions: uint8 cuda tensor [n].  Returns (obs, reward, done, frames).

        `pipe` selects the scratch pipeline and `stream` (a torch stream; default
        the current one) the stream: steps on different pipelines and streams
        may overlap when their env ids are disjoint."""
        if stream is not None:
            with torch.cuda.stream(stream):
                return self.step(actions, env_ids, want_frames, want_obs, out, pipe)
        actions = torch.as_tensor(actions, dtype=torch.uint8, device=self.device).contiguous()
        n = actions.numel()
        ids, ids_ptr = self._ids(env_ids)
        if out is None:
            obs = torch.empty((n, 84, 84), dtype=torch.uint8, device=self.device) if want_obs else None
            reward = torch.empty(n, dtype=torch.int32, device=self.device)
            done = torch.empty(n, dtype=torch.uint8, device=self.device)
            frames = (torch.empty((n, self.n_slots, 210, 160), dtype=torch.uint8, device=self.device)
                      if want_frames else None)
        else:
            obs, reward, done, frames = out
        B.vcs_step_pipe(self._h, pipe, ids_ptr, actions.data_ptr(), n, obs.data_ptr() if obs is not None else None,
                        reward.data_ptr(), done.data_ptr(), frames.data_ptr() if frames is not None else None,
                        self._stream())
        return obs, reward, done, frames

    def get_state(self, env):
        return np.frombuffer(B.vcs_get_state(self._h, env), dtype=np.uint8).copy()

    def set_state(self, env, rec):
        B.vcs_set_state(self._h, env, bytes(np.asarray(rec, dtype=np.uint8)))

    def get_cache(self, rom, k):
        st, ob = B.vcs_get_cache(self._h, rom, k)
        return np.frombuffer(st, np.uint8).copy(), np.frombuffer(ob, np.uint8).reshape(84, 84).copy()

    def poll_errors(self):
        return B.vcs_poll_errors(self._h)

    def last_step_instructions(self):
        return B.vcs_last_step_instructions(self._h)

    def last_step_stats(self):
        return B.vcs_last_step_stats(self._h)

    def last_step_counts(self):
        """(instructions, of them on the wave-uniform path, wave instruction
        passes, wave scheduling rounds) of the last step; lane utilisation =
        instr / (64 * passes)."""
        return B.vcs_last_step_counts(self._h)

    def timing(self, enable):
        B.vcs_timing(self._h, enable)

    def kernel_time(self, which):
        return B.vcs_kernel_time(self._h, which)

    # launch shape (results do not depend on it)
    def set_launch(self, tile_envs=64, workers=0, render_block=256):
        B.vcs_set_launch(self._h, tile_envs, workers, render_block)

    def get_launch(self):
        return B.vcs_get_launch(self._h)

    def autotune(self, n=0, steps=3, want_frames=False, want_obs=True):
        """Pick the fastest launch shape for steps over envs 0..n-1; states are restored."""
        return B.vcs_autotune(self._h, n, steps, want_frames, want_obs)

    def capture(self, n=None, steps=1, env_ids=None, want_frames=False, want_obs=True):
        return StepGraph(self, n, steps, env_ids, want_frames, want_obs)


class StepGraph:
    """`steps` consecutive step calls captured in one HIP graph with fixed
    buffers: write actions into `.actions` ([steps, n]) and call launch()."""

    def __init__(self, env, n=None, steps=1, env_ids=None, want_frames=False, want_obs=True):
        dev = env.device
        self.env = env
        self.ids = None if env_ids is None else torch.as_tensor(env_ids, dtype=torch.int32, device=dev).contiguous()
        n = self.ids.numel() if self.ids is not None else (env.num_envs if n is None else n)
        self.n, self.steps = n, steps
        self.actions = torch.zeros((steps, n), dtype=torch.uint8, device=dev)
        self.obs = torch.empty((steps, n, 84, 84), dtype=torch.uint8, device=dev) if want_obs else None
        self.reward = torch.empty((steps, n), dtype=torch.int32, device=dev)
        self.done = torch.empty((steps, n), dtype=torch.uint8, device=dev)
        self.frames = (torch.empty((steps, n, env.n_slots, 210, 160), dtype=torch.uint8, device=dev)
                       if want_frames else None)
        ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        self._g = B.vcs_graph_create(env._h, ptr(self.ids), self.actions.data_ptr(), n, steps, ptr(self.obs),
                                     self.reward.data_ptr(), self.done.data_ptr(), ptr(self.frames))

    def launch(self, actions=None):
        if actions is not None:
            self.actions.copy_(torch.as_tensor(actions, dtype=torch.uint8).reshape(self.steps, self.n))
        B.vcs_graph_launch(self._g, self.env._stream())
        return self.obs, self.reward, self.done, self.frames

    def close(self):
        if getattr(self, "_g", None):
            B.vcs_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FrameStack:
    """The last `depth` observations of every env of `env`, kept in device
    memory (8-bit, or 4-bit packed); push() after each step."""

    def __init__(self, env, depth=4, bits=8):
        self.env, self.depth, self.bits = env, depth, bits
        self._s = B.vcs_stack_create(env._h, depth, bits)

    def push(self, obs, done=None, env_ids=None, out=None, want_out=True):
        """obs: uint8 cuda [n, 84, 84]; done: uint8 cuda [n] or None.
        Returns the stacked observations [n, depth, 84, 84] (or None)."""
        ids, ids_ptr = self.env._ids(env_ids)
        n = obs.shape[0]
        if out is None and want_out:
            out = torch.empty((n, self.depth, 84, 84), dtype=torch.uint8, device=self.env.device)
        B.vcs_stack_push(self._s, ids_ptr, n, obs.data_ptr(), done.data_ptr() if done is not None else None,
                         out.data_ptr() if out is not None else None, self.env._stream())
        return out

    def close(self):
        if getattr(self, "_s", None):
            B.vcs_stack_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Policy:
    """The inference-path policy network of `env`'s context (bf16 weights,
    fp32 accumulation on the matrix cores).  weights/biases: the 5 layers in
    the library's layouts (bf16 bit patterns as uint16, float32 biases)."""

    def __init__(self, env, weights, biases):
        self.env = env
        self._p = B.vcs_policy_create(env._h, weights, biases)

    def act(self, stack, logits=None, actions=None, want_logits=False):
        """stack: uint8 cuda [n, 4, 84, 84].  Returns (actions uint8 [n],
        logits float32 [n, 32] or None); entries 0..17 of a logits row are
        the action logits, 18 the value."""
        if stack.dtype != torch.uint8 or stack.dim() != 4 or tuple(stack.shape[1:]) != (4, 84, 84) \
                or not stack.is_contiguous():
            raise ValueError("stack must be a contiguous uint8 tensor [n, 4, 84, 84]")
        n = stack.shape[0]
        dev = self.env.device
        if actions is None:
            actions = torch.empty(n, dtype=torch.uint8, device=dev)
        if logits is None and want_logits:
            logits = torch.empty((n, 32), dtype=torch.float32, device=dev)
        B.vcs_policy_act(self._p, stack.data_ptr(), n, logits.data_ptr() if logits is not None else None,
                         actions.data_ptr(), self.env._stream())
        return actions, logits

    def close(self):
        if getattr(self, "_p", None):
            B.vcs_policy_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
