"""Helpers that run the GPU library and the CPU oracle side by side."""
import numpy as np

import oracle
from helpers import diff_records
from paper_1907_08467_amd.inputs.palette import GRAY


def make_pair(roms, env_rom, gpu_kw=None, **cfg):
    """roms: [(bytes, scheme)].  Returns (oracle, gpu env) with identical configs
    (gpu_kw: options of the GPU env only, such as pipelines)."""
    import torch  # noqa: F401
    from paper_1907_08467_amd.env import VcsEnv
    env_rom = np.ascontiguousarray(env_rom, np.uint16)
    o = oracle.Oracle(len(env_rom), GRAY, **cfg)
    o.load_roms(roms)
    o.assign(env_rom)
    g = VcsEnv(roms, env_rom, GRAY, **cfg, **(gpu_kw or {}))
    return o, g


def step_both(o, g, actions, ids=None, want_frames=False, tag=""):
    import torch
    a = np.ascontiguousarray(actions, np.uint8)
    gid = None if ids is None else torch.as_tensor(np.asarray(ids, np.int32), device="cuda")
    go, gr, gd, gf = g.step(torch.from_numpy(a).cuda(), env_ids=gid, want_frames=want_frames)
    oo, orr, od, of = o.step(a, env_ids=ids, want_frames=want_frames)
    torch.cuda.synchronize()
    go, gr, gd = go.cpu().numpy(), gr.cpu().numpy(), gd.cpu().numpy()
    bad = np.nonzero(gd != od)[0]
    assert bad.size == 0, f"{tag}: done differs at positions {bad[:8]}: gpu {gd[bad[:8]]} oracle {od[bad[:8]]}"
    bad = np.nonzero(gr != orr)[0]
    assert bad.size == 0, f"{tag}: reward differs at positions {bad[:8]}: gpu {gr[bad[:8]]} oracle {orr[bad[:8]]}"
    if want_frames:
        gf = gf.cpu().numpy()
        diff = np.nonzero((gf != of).reshape(gf.shape[0], -1).any(axis=1))[0]
        if diff.size:
            i = int(diff[0])
            where = np.argwhere(gf[i] != of[i])[:5]
            raise AssertionError(f"{tag}: frames differ for {diff.size} positions, first {i}; "
                                 f"(slot,row,col) {where.tolist()} gpu {gf[i][tuple(where.T)]} "
                                 f"oracle {of[i][tuple(where.T)]}")
    diff = np.nonzero((go != oo).reshape(go.shape[0], -1).any(axis=1))[0]
    assert diff.size == 0, f"{tag}: obs differ for positions {diff[:8]}"
    return go, gr, gd


def compare_states(o, g, envs, tag=""):
    for e in envs:
        a, b = g.get_state(int(e)), o.get_state(int(e))
        if not np.array_equal(a, b):
            raise AssertionError(f"{tag}: state of env {e} differs: {diff_records(a, b)}")
