"""Python access to the CPU oracle (liboracle.so) -- TEST INFRASTRUCTURE.

The oracle is the plain sequential emulator the GPU library is checked
against.  Only the tests, the smoke check and the bench's CPU-baseline leg
may import this package.  It shares no code with the GPU library.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

STATE_BYTES = 384
RENDER_ALL, RENDER_LAST2 = 0, 1
ERR_ILLEGAL, ERR_FRAME_CAP, ERR_BAD_ACTION = 1, 2, 4

_u8p = ctypes.POINTER(ctypes.c_uint8)


class OracleConfig(ctypes.Structure):
    _fields_ = [
        ("num_envs", ctypes.c_uint32),
        ("frameskip", ctypes.c_uint32),
        ("sticky_threshold", ctypes.c_uint32),
        ("reset_cache_k", ctypes.c_uint32),
        ("noop_max", ctypes.c_uint32),
        ("startup_frames", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("render_mode", ctypes.c_uint32),
        ("collisions", ctypes.c_uint32),
        ("noop_after_copy", ctypes.c_uint32),
        ("gray_lut", ctypes.c_uint8 * 128),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.oracle_create.argtypes = [ctypes.POINTER(OracleConfig), ctypes.POINTER(vp)]
        L.oracle_destroy.argtypes = [vp]
        L.oracle_destroy.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_get_threads.restype = ctypes.c_int
        L.oracle_load_roms.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(_u8p), vp, vp]
        L.oracle_assign.argtypes = [vp, vp]
        L.oracle_reset.argtypes = [vp, vp, ctypes.c_uint32, vp]
        L.oracle_step.argtypes = [vp, vp, vp, ctypes.c_uint32, vp, vp, vp, vp, ctypes.c_int]
        L.oracle_get_state.argtypes = [vp, ctypes.c_uint32, vp]
        L.oracle_set_state.argtypes = [vp, ctypes.c_uint32, vp]
        L.oracle_get_cache.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, vp, vp]
        L.oracle_poll_errors.argtypes = [vp, vp, vp]
        L.oracle_power_on.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, vp]
        L.oracle_run_instructions.argtypes = [vp, vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                              ctypes.c_uint32]
        L.oracle_batch_instructions.argtypes = [vp, ctypes.c_uint32, vp, ctypes.c_uint32, ctypes.c_uint32,
                                                ctypes.c_uint32]
        L.oracle_run_frames.argtypes = [vp, vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, vp, vp, vp]
        L.oracle_preprocess.argtypes = [vp, vp, vp, vp]
        L.oracle_preprocess.restype = None
        L.oracle_splitmix64_next.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        L.oracle_splitmix64_next.restype = ctypes.c_uint64
        L.oracle_rng.argtypes = [ctypes.c_uint64] * 4
        L.oracle_rng.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


def set_threads(n: int):
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return lib().oracle_get_threads()


class Oracle:
    """Batched env API of the oracle, host arrays in and out."""

    def __init__(self, num_envs, gray_lut, frameskip=4, sticky_threshold=0, reset_cache_k=30,
                 noop_max=30, startup_frames=64, seed=0, render_mode=RENDER_ALL, collisions=False,
                 noop_after_copy=False):
        cfg = OracleConfig()
        cfg.num_envs = num_envs
        cfg.frameskip = frameskip
        cfg.sticky_threshold = sticky_threshold
        cfg.reset_cache_k = reset_cache_k
        cfg.noop_max = noop_max
        cfg.startup_frames = startup_frames
        cfg.seed = seed
        cfg.render_mode = render_mode
        cfg.collisions = 1 if collisions else 0
        cfg.noop_after_copy = 1 if noop_after_copy else 0
        for i, g in enumerate(bytes(gray_lut)):
            cfg.gray_lut[i] = g
        self.cfg = cfg
        self.num_envs = num_envs
        self.frameskip = frameskip
        self.render_mode = render_mode
        h = ctypes.c_void_p()
        _check(lib().oracle_create(ctypes.byref(cfg), ctypes.byref(h)), "create")
        self._h = h

    def close(self):
        if self._h:
            lib().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_roms(self, roms):
        """roms: list of (bytes, scheme)."""
        self._rom_keep = [np.frombuffer(bytes(d), dtype=np.uint8).copy() for d, _ in roms]
        arr = (_u8p * len(roms))(*[r.ctypes.data_as(_u8p) for r in self._rom_keep])
        sizes = np.array([len(d) for d, _ in roms], dtype=np.uint32)
        schemes = np.array([s for _, s in roms], dtype=np.uint32)
        _check(lib().oracle_load_roms(self._h, len(roms), arr, _ptr(sizes), _ptr(schemes)), "load_roms")

    def assign(self, env_rom):
        er = np.ascontiguousarray(env_rom, dtype=np.uint16)
        assert er.shape == (self.num_envs,)
        _check(lib().oracle_assign(self._h, _ptr(er)), "assign")

    def reset(self, env_ids=None, n=None):
        ids = None if env_ids is None else np.ascontiguousarray(env_ids, dtype=np.int32)
        n = len(ids) if ids is not None else (self.num_envs if n is None else n)
        obs = np.zeros((n, 84, 84), dtype=np.uint8)
        _check(lib().oracle_reset(self._h, _ptr(ids), n, _ptr(obs)), "reset")
        return obs

    def n_slots(self):
        return 2 if self.render_mode == RENDER_LAST2 else self.frameskip

    def step(self, actions, env_ids=None, want_frames=False, render=True):
        act = np.ascontiguousarray(actions, dtype=np.uint8)
        n = act.shape[0]
        ids = None if env_ids is None else np.ascontiguousarray(env_ids, dtype=np.int32)
        obs = np.zeros((n, 84, 84), dtype=np.uint8) if render else None
        rew = np.zeros(n, dtype=np.int32)
        done = np.zeros(n, dtype=np.uint8)
        frames = np.zeros((n, self.n_slots(), 210, 160), dtype=np.uint8) if want_frames else None
        _check(lib().oracle_step(self._h, _ptr(ids), _ptr(act), n, _ptr(obs), _ptr(rew), _ptr(done),
                                 _ptr(frames), int(bool(render))), "step")
        return obs, rew, done, frames

    def get_state(self, env):
        out = np.zeros(STATE_BYTES, dtype=np.uint8)
        _check(lib().oracle_get_state(self._h, env, _ptr(out)), "get_state")
        return out

    def set_state(self, env, rec):
        rec = np.ascontiguousarray(rec, dtype=np.uint8)
        _check(lib().oracle_set_state(self._h, env, _ptr(rec)), "set_state")

    def get_cache(self, rom, k):
        st = np.zeros(STATE_BYTES, dtype=np.uint8)
        obs = np.zeros((84, 84), dtype=np.uint8)
        _check(lib().oracle_get_cache(self._h, rom, k, _ptr(st), _ptr(obs)), "get_cache")
        return st, obs

    def poll_errors(self):
        first = np.zeros(1, dtype=np.uint32)
        bits = np.zeros(1, dtype=np.uint32)
        _check(lib().oracle_poll_errors(self._h, _ptr(first), _ptr(bits)), "poll_errors")
        return int(first[0]), int(bits[0])


# ---------------------------------------------------------------- bare machine

def _rom_arr(rom):
    return np.frombuffer(bytes(rom), dtype=np.uint8).copy()


def power_on(rom, scheme=0):
    r = _rom_arr(rom)
    st = np.zeros(STATE_BYTES, dtype=np.uint8)
    _check(lib().oracle_power_on(_ptr(r), len(r), scheme, _ptr(st)), "power_on")
    return st


def run_instructions(state, rom, n, scheme=0, action=0):
    r = _rom_arr(rom)
    st = np.ascontiguousarray(state, dtype=np.uint8).copy()
    done = _check(lib().oracle_run_instructions(_ptr(st), _ptr(r), len(r), scheme, n, action), "run")
    return st, done


def batch_instructions(states, rom, n, scheme=0):
    r = _rom_arr(rom)
    st = np.ascontiguousarray(states, dtype=np.uint8).copy()
    assert st.ndim == 2 and st.shape[1] == STATE_BYTES
    _check(lib().oracle_batch_instructions(_ptr(st), st.shape[0], _ptr(r), len(r), scheme, n), "batch")
    return st


def run_frames(state, rom, n_frames, scheme=0, actions=None, render=True):
    r = _rom_arr(rom)
    st = np.ascontiguousarray(state, dtype=np.uint8).copy()
    acts = None if actions is None else np.ascontiguousarray(actions, dtype=np.uint8)
    frames = np.zeros((n_frames, 210, 160), dtype=np.uint8) if render else None
    ends = np.zeros(n_frames, dtype=np.uint64)
    got = _check(lib().oracle_run_frames(_ptr(st), _ptr(r), len(r), scheme, n_frames, _ptr(acts),
                                         _ptr(frames), _ptr(ends)), "run_frames")
    return st, frames, ends, got


def preprocess(f_prev, f_last, gray_lut):
    fl = np.ascontiguousarray(f_last, dtype=np.uint8)
    fp = None if f_prev is None else np.ascontiguousarray(f_prev, dtype=np.uint8)
    lut = np.frombuffer(bytes(gray_lut), dtype=np.uint8).copy()
    obs = np.zeros((84, 84), dtype=np.uint8)
    lib().oracle_preprocess(_ptr(fp), _ptr(fl), _ptr(lut), _ptr(obs))
    return obs


def splitmix64_stream(seed, n):
    s = ctypes.c_uint64(seed)
    return [lib().oracle_splitmix64_next(ctypes.byref(s)) for _ in range(n)]


def rng(seed, env_id, purpose, n):
    return lib().oracle_rng(seed, env_id, purpose, n)
