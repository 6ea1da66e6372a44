"""ctypes binding of libvcs355.so (include/vcs355.h): argument marshalling only.

Every step of the emulation runs in the library's HIP kernels.  Importing this
module loads the library and fails loudly if it has not been built; there is
no fallback.
"""

from __future__ import annotations

import ctypes
import os
import re

import torch  # noqa: F401  -- loads the HIP runtime the library links against

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvcs355.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vcs355.h")

VCS_OK, VCS_E_INVAL, VCS_E_NOMEM, VCS_E_ROM, VCS_E_HIP, VCS_E_STATE, VCS_E_BUDGET = 0, -1, -2, -3, -4, -5, -6
VCS_BANK_4K, VCS_BANK_F8, VCS_BANK_F6, VCS_BANK_F4, VCS_BANK_F8SC, VCS_BANK_F6SC, VCS_BANK_F4SC, VCS_BANK_E0, \
    VCS_BANK_3F = range(9)
VCS_RENDER_ALL, VCS_RENDER_LAST2 = 0, 1
ERR_ILLEGAL, ERR_FRAME_CAP, ERR_BAD_ACTION, ERR_BAD_ID, ERR_LOG = 1, 2, 4, 8, 16
STATE_BYTES = 384


class VcsConfig(ctypes.Structure):
    _fields_ = [
        ("num_envs", ctypes.c_uint32),
        ("frameskip", ctypes.c_uint32),
        ("sticky_threshold", ctypes.c_uint32),
        ("reset_cache_k", ctypes.c_uint32),
        ("noop_max", ctypes.c_uint32),
        ("startup_frames", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("render_mode", ctypes.c_uint32),
        ("max_batch", ctypes.c_uint32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("device", ctypes.c_int32),
        ("pipelines", ctypes.c_uint32),
        ("collisions", ctypes.c_uint32),
        ("noop_after_copy", ctypes.c_uint32),
        ("gray_lut", ctypes.c_uint8 * 128),
    ]


class VcsLaunch(ctypes.Structure):
    _fields_ = [
        ("tile_envs", ctypes.c_uint32),
        ("workers", ctypes.c_uint32),
        ("render_block", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {"tile_envs": self.tile_envs, "workers": self.workers, "render_block": self.render_block}


class VcsError(RuntimeError):
    def __init__(self, code, what, msg):
        super().__init__(f"{what} failed ({code}): {msg}")
        self.code = code


_vp = ctypes.c_void_p
_u8p = ctypes.POINTER(ctypes.c_uint8)


def _declare(L):
    L.vcs_create.argtypes = [ctypes.POINTER(VcsConfig), ctypes.POINTER(_vp)]
    L.vcs_destroy.argtypes = [_vp]
    L.vcs_destroy.restype = None
    L.vcs_load_roms.argtypes = [_vp, ctypes.c_uint32, ctypes.POINTER(_u8p), _vp, _vp]
    L.vcs_assign.argtypes = [_vp, _vp]
    L.vcs_reset.argtypes = [_vp, _vp, ctypes.c_uint32, _vp, _vp]
    L.vcs_step.argtypes = [_vp, _vp, _vp, ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp]
    L.vcs_step_pipe.argtypes = [_vp, ctypes.c_uint32, _vp, _vp, ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp]
    L.vcs_step_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_uint32, _vp, _vp, _vp, _vp]
    L.vcs_get_state.argtypes = [_vp, ctypes.c_uint32, _vp]
    L.vcs_set_state.argtypes = [_vp, ctypes.c_uint32, _vp]
    L.vcs_get_cache.argtypes = [_vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _vp]
    L.vcs_poll_errors.argtypes = [_vp, _vp, _vp]
    L.vcs_last_step_instructions.argtypes = [_vp, _vp]
    L.vcs_last_step_stats.argtypes = [_vp, _vp]
    L.vcs_last_step_counts.argtypes = [_vp, _vp]
    L.vcs_timing.argtypes = [_vp, ctypes.c_int]
    L.vcs_kernel_time.argtypes = [_vp, ctypes.c_int, _vp, _vp]
    L.vcs_set_launch.argtypes = [_vp, ctypes.POINTER(VcsLaunch)]
    L.vcs_get_launch.argtypes = [_vp, ctypes.POINTER(VcsLaunch)]
    L.vcs_autotune.argtypes = [_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(VcsLaunch), ctypes.POINTER(ctypes.c_double)]
    L.vcs_graph_create.argtypes = [_vp, _vp, _vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _vp, _vp, _vp,
                                   ctypes.POINTER(_vp)]
    L.vcs_graph_launch.argtypes = [_vp, _vp]
    L.vcs_graph_destroy.argtypes = [_vp]
    L.vcs_graph_destroy.restype = None
    L.vcs_stack_create.argtypes = [_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(_vp)]
    L.vcs_stack_push.argtypes = [_vp, _vp, ctypes.c_uint32, _vp, _vp, _vp, _vp]
    L.vcs_stack_destroy.argtypes = [_vp]
    L.vcs_stack_destroy.restype = None
    L.vcs_policy_create.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp)]
    L.vcs_policy_act.argtypes = [_vp, _vp, ctypes.c_uint32, _vp, _vp, _vp]
    L.vcs_policy_destroy.argtypes = [_vp]
    L.vcs_policy_destroy.restype = None
    L.vcs_last_error.argtypes = []
    L.vcs_last_error.restype = ctypes.c_char_p
    for name in ("vcs_create", "vcs_load_roms", "vcs_assign", "vcs_reset", "vcs_step", "vcs_step_pipe",
                 "vcs_step_noalloc", "vcs_get_state",
                 "vcs_set_state", "vcs_get_cache", "vcs_poll_errors", "vcs_last_step_instructions", "vcs_last_step_stats",
                 "vcs_last_step_counts",
                 "vcs_timing", "vcs_kernel_time", "vcs_set_launch", "vcs_get_launch", "vcs_autotune",
                 "vcs_graph_create", "vcs_graph_launch", "vcs_stack_create", "vcs_stack_push",
                 "vcs_policy_create", "vcs_policy_act"):
        getattr(L, name).restype = ctypes.c_int


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    _declare(L)
    return L


lib = load()


def header_functions():
    """Names of the functions include/vcs355.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(vcs_\w+)\s*\(", text, re.M)))


def check(rc, what):
    if rc != VCS_OK:
        raise VcsError(rc, what, lib.vcs_last_error().decode(errors="replace"))
    return rc


# thin wrappers with the C names -------------------------------------------

def vcs_create(cfg: VcsConfig):
    h = _vp()
    check(lib.vcs_create(ctypes.byref(cfg), ctypes.byref(h)), "vcs_create")
    return h


def vcs_destroy(h):
    lib.vcs_destroy(h)


def vcs_load_roms(h, roms, schemes):
    keep = [ctypes.create_string_buffer(bytes(r), len(r)) for r in roms]
    arr = (_u8p * len(roms))(*[ctypes.cast(k, _u8p) for k in keep])
    sizes = (ctypes.c_uint32 * len(roms))(*[len(r) for r in roms])
    sch = (ctypes.c_uint32 * len(roms))(*schemes)
    check(lib.vcs_load_roms(h, len(roms), arr, sizes, sch), "vcs_load_roms")


def vcs_assign(h, env_rom):
    import numpy as np
    er = np.ascontiguousarray(env_rom, dtype=np.uint16)
    check(lib.vcs_assign(h, er.ctypes.data_as(_vp)), "vcs_assign")


def vcs_reset(h, ids_ptr, n, obs_ptr, stream):
    check(lib.vcs_reset(h, ids_ptr, n, obs_ptr, stream), "vcs_reset")


def vcs_step(h, ids_ptr, actions_ptr, n, obs_ptr, reward_ptr, done_ptr, frames_ptr, stream):
    check(lib.vcs_step(h, ids_ptr, actions_ptr, n, obs_ptr, reward_ptr, done_ptr, frames_ptr, stream), "vcs_step")


def vcs_step_pipe(h, pipe, ids_ptr, actions_ptr, n, obs_ptr, reward_ptr, done_ptr, frames_ptr, stream):
    check(lib.vcs_step_pipe(h, pipe, ids_ptr, actions_ptr, n, obs_ptr, reward_ptr, done_ptr, frames_ptr, stream),
          "vcs_step_pipe")


def vcs_step_noalloc(h, ids_ptr, actions_ptr, n, obs_ptr, reward_ptr, done_ptr, stream):
    check(lib.vcs_step_noalloc(h, ids_ptr, actions_ptr, n, obs_ptr, reward_ptr, done_ptr, stream),
          "vcs_step_noalloc")


def vcs_get_state(h, env):
    buf = (ctypes.c_uint8 * STATE_BYTES)()
    check(lib.vcs_get_state(h, env, buf), "vcs_get_state")
    return bytes(buf)


def vcs_set_state(h, env, rec):
    buf = (ctypes.c_uint8 * STATE_BYTES).from_buffer_copy(bytes(rec))
    check(lib.vcs_set_state(h, env, buf), "vcs_set_state")


def vcs_get_cache(h, rom, k):
    st = (ctypes.c_uint8 * STATE_BYTES)()
    ob = (ctypes.c_uint8 * (84 * 84))()
    check(lib.vcs_get_cache(h, rom, k, st, ob), "vcs_get_cache")
    return bytes(st), bytes(ob)


def vcs_poll_errors(h):
    first = ctypes.c_uint32()
    bits = ctypes.c_uint32()
    check(lib.vcs_poll_errors(h, ctypes.byref(first), ctypes.byref(bits)), "vcs_poll_errors")
    return first.value, bits.value


def vcs_last_step_instructions(h):
    v = ctypes.c_uint64()
    check(lib.vcs_last_step_instructions(h, ctypes.byref(v)), "vcs_last_step_instructions")
    return v.value


def vcs_last_step_stats(h):
    v = (ctypes.c_uint64 * 2)()
    check(lib.vcs_last_step_stats(h, v), "vcs_last_step_stats")
    return v[0], v[1]


def vcs_last_step_counts(h):
    v = (ctypes.c_uint64 * 4)()
    check(lib.vcs_last_step_counts(h, v), "vcs_last_step_counts")
    return v[0], v[1], v[2], v[3]


def vcs_timing(h, enable):
    check(lib.vcs_timing(h, int(enable)), "vcs_timing")


def vcs_kernel_time(h, which):
    ms = ctypes.c_double()
    cnt = ctypes.c_uint32()
    check(lib.vcs_kernel_time(h, which, ctypes.byref(ms), ctypes.byref(cnt)), "vcs_kernel_time")
    return ms.value, cnt.value


def vcs_set_launch(h, tile_envs=64, workers=0, render_block=256):
    l = VcsLaunch(tile_envs, workers, render_block)
    check(lib.vcs_set_launch(h, ctypes.byref(l)), "vcs_set_launch")


def vcs_get_launch(h):
    l = VcsLaunch()
    check(lib.vcs_get_launch(h, ctypes.byref(l)), "vcs_get_launch")
    return l.as_dict()


def vcs_autotune(h, n, steps, want_frames, want_obs):
    l = VcsLaunch()
    ms = ctypes.c_double()
    check(lib.vcs_autotune(h, n, steps, int(bool(want_frames)), int(bool(want_obs)), ctypes.byref(l),
                           ctypes.byref(ms)), "vcs_autotune")
    return l.as_dict(), ms.value


def vcs_graph_create(h, ids_ptr, actions_ptr, n, steps, obs_ptr, reward_ptr, done_ptr, frames_ptr):
    g = _vp()
    check(lib.vcs_graph_create(h, ids_ptr, actions_ptr, n, steps, obs_ptr, reward_ptr, done_ptr, frames_ptr,
                               ctypes.byref(g)), "vcs_graph_create")
    return g


def vcs_graph_launch(g, stream):
    check(lib.vcs_graph_launch(g, stream), "vcs_graph_launch")


def vcs_graph_destroy(g):
    lib.vcs_graph_destroy(g)


def vcs_stack_create(h, depth, bits):
    st = _vp()
    check(lib.vcs_stack_create(h, depth, bits, ctypes.byref(st)), "vcs_stack_create")
    return st


def vcs_stack_push(st, ids_ptr, n, obs_ptr, done_ptr, out_ptr, stream):
    check(lib.vcs_stack_push(st, ids_ptr, n, obs_ptr, done_ptr, out_ptr, stream), "vcs_stack_push")


def vcs_stack_destroy(st):
    lib.vcs_stack_destroy(st)


def vcs_policy_create(h, weights, biases):
    """weights: 5 contiguous uint16 numpy arrays (bf16 bits), biases: 5 float32 arrays."""
    import numpy as np
    ws = [np.ascontiguousarray(w, np.uint16) for w in weights]
    bs = [np.ascontiguousarray(b, np.float32) for b in biases]
    if len(ws) != 5 or len(bs) != 5:
        raise ValueError("the policy has 5 layers")
    wp = (_vp * 5)(*[w.ctypes.data for w in ws])
    bp = (_vp * 5)(*[b.ctypes.data for b in bs])
    p = _vp()
    check(lib.vcs_policy_create(h, wp, bp, ctypes.byref(p)), "vcs_policy_create")
    return p


def vcs_policy_act(p, stack_ptr, n, logits_ptr, actions_ptr, stream):
    check(lib.vcs_policy_act(p, stack_ptr, n, logits_ptr, actions_ptr, stream), "vcs_policy_act")


def vcs_policy_destroy(p):
    lib.vcs_policy_destroy(p)


def vcs_last_error():
    return lib.vcs_last_error().decode(errors="replace")
