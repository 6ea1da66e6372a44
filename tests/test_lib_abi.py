"""The C-ABI library loads and exports every function include/vcs355.h
declares; host-side argument checks reject bad configs before any device
work.  No GPU is needed (no compute call is made)."""
import ctypes

import pytest

B = pytest.importorskip("paper_1907_08467_amd.binding")


def test_every_declared_function_is_exported():
    names = B.header_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(B.lib, n)]
    assert not missing


def test_header_struct_matches_binding():
    # vcs_config: 6 x u32, u64, 2 x u32, u64, i32, 3 x u32, 128 B -> 192 bytes with alignment
    assert ctypes.sizeof(B.VcsConfig) == 192
    assert B.VcsConfig.collisions.offset == 56 and B.VcsConfig.noop_after_copy.offset == 60
    assert B.VcsConfig.gray_lut.offset == 64


@pytest.mark.parametrize("field,value", [("num_envs", 0), ("frameskip", 0), ("render_mode", 2),
                                         ("reset_cache_k", 0), ("frameskip", 9)])
def test_create_rejects_bad_config(field, value):
    cfg = B.VcsConfig()
    cfg.num_envs = 4
    cfg.frameskip = 4
    cfg.reset_cache_k = 30
    cfg.render_mode = 0
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    rc = B.lib.vcs_create(ctypes.byref(cfg), ctypes.byref(h))
    assert rc == B.VCS_E_INVAL and not h.value
    assert B.vcs_last_error()


def test_null_arguments_rejected():
    assert B.lib.vcs_create(None, None) == B.VCS_E_INVAL
    assert B.lib.vcs_step(None, None, None, 0, None, None, None, None, None) == B.VCS_E_INVAL
    assert B.lib.vcs_reset(None, None, 0, None, None) == B.VCS_E_INVAL


@pytest.mark.parametrize("noop_after_copy,startup", [(1, 1), (1, 0), (2, 64)])
def test_create_rejects_bad_noop_after_copy(noop_after_copy, startup):
    cfg = B.VcsConfig()
    cfg.num_envs = 4
    cfg.frameskip = 4
    cfg.reset_cache_k = 30
    cfg.startup_frames = startup
    cfg.noop_after_copy = noop_after_copy
    h = ctypes.c_void_p()
    assert B.lib.vcs_create(ctypes.byref(cfg), ctypes.byref(h)) == B.VCS_E_INVAL and not h.value
