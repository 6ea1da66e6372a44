"""Throughput of the batched emulation step on one MI355X.

Workload: the plain batched configuration -- 4096 envs of one seeded 4 KB
synthetic cartridge, frameskip 4, every frame rendered to 210x160 and kept in
HBM plus the 84x84 gray max-of-two observation, uniform random actions
(PCG64 seed 1), no sticky actions.  Actions for every timed step are resident
in HBM before the timed region starts.

Prints one JSON line: raw emulated frames/s (= env steps x frameskip / s), the
roofline of the dominant kernel (timed with HIP events on the launch stream)
and the CPU oracle's rate on the host cores for a bounded sample of the same
workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KERNELS = {0: "k_interp", 1: "k_render_frames", 2: "k_render_obs", 3: "k_reset"}
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz integer VALU lane-ops
ALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--envs", type=int, default=4096)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=16)
    p.add_argument("--launch", type=str, default="auto",
                   help="'auto' (autotuner) or tile_envs,workers,render_block, e.g. 64,0,256")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="only run a plain device-to-device copy of this many MiB (HBM counter calibration)")
    return p.parse_args()


def copy_calibration(mib):
    import torch
    a = torch.ones(mib << 18, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": mib << 20, "bytes_written": mib << 20}))


def cpu_baseline(w, roms, env_rom, steps):
    import oracle
    from paper_1907_08467_amd.inputs.palette import GRAY
    o = oracle.Oracle(w.n_envs, GRAY, frameskip=w.frameskip, seed=w.rng_seed)
    o.load_roms(roms)
    o.assign(env_rom)
    acts = w.actions(steps=steps)
    t0 = time.perf_counter()
    for s in range(steps):
        o.step(acts[s], want_frames=True)
    dt = time.perf_counter() - t0
    frames = w.n_envs * w.frameskip * steps
    return {"value": frames / dt, "unit": "raw frames/s", "cores": oracle.get_threads(), "kind": "oracle",
            "sample": f"{w.n_envs} envs x {steps} steps x frameskip {w.frameskip} ({frames} raw frames), "
                      f"every frame rendered + obs, same cartridge, seed and actions",
            "seconds": dt}


def main():
    args = parse()
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the envs are independent and "
              "shard by env id, but this build measures the single-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1907_08467_amd.env import VcsEnv
    from paper_1907_08467_amd.inputs.palette import GRAY
    from paper_1907_08467_amd.inputs.workloads import config

    w = config(2)
    if args.envs != w.n_envs:
        w.n_envs = args.envs
    roms = [(r.data, r.scheme) for r in w.roms()]
    env_rom = w.env_rom()
    dev = torch.device("cuda", 0)
    env = VcsEnv(roms, env_rom, GRAY, frameskip=w.frameskip, seed=w.rng_seed, render_mode=w.render_mode)
    n, K, W = w.n_envs, args.steps, args.warmup
    if args.launch == "auto":
        launch, tune_ms = env.autotune(steps=3, want_frames=True, want_obs=True)
        print(f"autotuner picked {launch} ({tune_ms:.3f} ms/step)", file=sys.stderr, flush=True)
    else:
        tw, wk, rb = (int(x) for x in args.launch.split(","))
        env.set_launch(tw, wk, rb)
        launch = env.get_launch()
    acts = torch.from_numpy(w.actions(steps=K + W)).to(dev)
    obs = torch.empty((n, 84, 84), dtype=torch.uint8, device=dev)
    rew = torch.empty(n, dtype=torch.int32, device=dev)
    done = torch.empty(n, dtype=torch.uint8, device=dev)
    frames = torch.empty((n, w.frameskip, 210, 160), dtype=torch.uint8, device=dev)
    out = (obs, rew, done, frames)
    for s in range(W):
        env.step(acts[s], out=out)
    torch.cuda.synchronize()
    instr_one = env.last_step_instructions()   # instructions of the last warmup step
    print(f"warmup done: {W} steps; instructions in one step {instr_one}", file=sys.stderr, flush=True)

    env.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        env.step(acts[W + s], out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    env.timing(False)
    instr_last, instr_uniform = env.last_step_stats()
    kern = {}
    for k, name in KERNELS.items():
        ms, cnt = env.kernel_time(k)
        kern[name] = {"mean_ms": ms, "launches": cnt}
    raw_frames = n * w.frameskip * K
    value = raw_frames / dt
    first, bits = env.poll_errors()
    print(f"timed {K} steps in {dt:.3f}s; errors {bits:#x}", file=sys.stderr, flush=True)

    # dominant kernel = the interpreter: emulated instructions per launch over its mean duration
    t_interp = kern["k_interp"]["mean_ms"] * 1e-3
    instr_rate = instr_last / t_interp if t_interp > 0 else 0.0
    roofline = {"bound": "alu", "kernel": "k_interp", "achieved": instr_rate / 1e9,
                "peak": ALU_LANE_OPS_PEAK / 1e9, "unit": "G emulated instr/s vs G lane-ops/s",
                "frac": instr_rate / ALU_LANE_OPS_PEAK, "traffic": None,
                "work_per_launch": f"{instr_last} emulated 6502 instructions ({n} envs x {w.frameskip} frames)"}
    # render + observation kernels against HBM
    fb = n * w.frameskip * 210 * 160 + n * 84 * 84
    t_render = (kern["k_render_frames"]["mean_ms"] + kern["k_render_obs"]["mean_ms"]) * 1e-3
    render = {"bound": "hbm", "algorithmic_bytes_written": fb,
              "achieved_GBs": fb / t_render / 1e9 if t_render > 0 else 0.0, "peak_GBs": HBM_PEAK_GBS}
    render["frac"] = render["achieved_GBs"] / HBM_PEAK_GBS

    cpu = None
    if not args.no_cpu_baseline:
        print(f"cpu baseline: oracle, {args.cpu_steps} steps", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, roms, env_rom, args.cpu_steps)
    line = {
        "metric": "raw emulated frames/s on 1 MI355X (p50/p99 step latency in served mode)",
        "value": value, "unit": "raw frames/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"plain batched step: {n} envs x 1 seeded 4 KB synthetic cartridge, frameskip "
                               f"{w.frameskip}, every 210x160 frame rendered to HBM + 84x84 max-of-two gray obs, "
                               "random actions (seed 1), no sticky actions",
                   "num_envs": n, "frameskip": w.frameskip, "render": "all frames",
                   "launch": launch, "launch_from": "autotuner" if args.launch == "auto" else "fixed"},
        "roofline": roofline,
        "render_roofline": render,
        "kernels_ms": {k: v["mean_ms"] for k, v in kern.items()},
        "emulated_instr_per_step": instr_last,
        "uniform_mode_fraction": instr_uniform / instr_last if instr_last else 0.0,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
