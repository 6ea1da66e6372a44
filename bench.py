"""Throughput of the batched emulation step on one MI355X.

Default (--workload metric): the configurations the metric is quoted on.
 - The value: the batching form, 65,536 envs over 16 seeded synthetic
   cartridges (8 x 4 KB, 8 x F8) in Zipf 1.2 populations, frameskip 4, the
   last two frames of each step rendered into the 84x84 gray max-of-two
   observation, launch shape from the autotuner, steps captured in HIP
   graphs on two pipelines; the plain kernel (64 envs per wave, eager calls)
   on the same inputs beside it.  Exactly --steps steps are timed.
 - The served form: 131,072 resident envs over the same cartridges behind
   the env server, 64 closed-loop actors, continuous batching; raw frames/s
   and p50/p99 request latency over --metric-serve-seconds, the fixed-batch
   reference and an open-loop overload curve.
 - The plain 4096-env step (one cartridge, every frame rendered to HBM) as
   the baseline, over --c2-steps eager steps and as many in graphs, a window
   that crosses the first episode ends and their resets.
Actions for every timed step are resident in HBM before the timed region
starts.  Per-kernel times come from HIP events on the launch stream.

Prints one JSON line: raw emulated frames/s (= env steps x frameskip / s), the
roofline of the dominant kernel, the interpreter's active-lane utilisation,
and the CPU oracle's rates on the host cores (configuration 1 in full and
bounded samples of the other two).  Other --workload values print the line
of one configuration.
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
# HBM bytes per launch, from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a
# 256 MiB copy's readings (read x2.000, write x1.000), on the plain 4096-env
# step and on the 65,536-env batching workload; reported only while the
# kernel source and the headers it includes are the ones they were taken on
# (sha256 prefix of the files concatenated), otherwise null.
_INTERP_SRC = ("interp.hip", "tia_draw.h", "vcs_device.h")
_RENDER_SRC = ("render.hip", "tia_draw.h", "vcs_device.h")
MEASURED_TRAFFIC = {
    ("k_interp", "plain_4096"): (_INTERP_SRC, "437de748e86a04c8", (1273.0 * 2.0 + 162348.0) * 1024),
    ("k_render_frames", "plain_4096"): (_RENDER_SRC, "f7363e502d223ad4", (41151.0 * 2.0 + 268800.0) * 1024),
    ("k_render_obs", "plain_4096"): (_RENDER_SRC, "f7363e502d223ad4", (41137.2 * 2.0 + 297222.0) * 1024),
    ("k_interp", "batching_65536"): (_INTERP_SRC, "437de748e86a04c8", (17241.2 * 2.0 + 1648190.0) * 1024),
    ("k_render_obs", "batching_65536"): (_RENDER_SRC, "f7363e502d223ad4", (606480.0 * 2.0 + 452608.0) * 1024),
}
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz integer VALU lane-ops
ALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
CLOCK_HZ = 2.4e9
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0
# policy CNN: output positions per env, output channels, reduction length
POLICY_GEMMS = [(400, 32, 256), (81, 64, 512), (49, 64, 576), (1, 512, 3136), (1, 19, 512)]
POLICY_FLOPS_PER_ENV = sum(2 * m * n * k for m, n, k in POLICY_GEMMS)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=8)
    p.add_argument("--envs", type=int, default=4096)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=16)
    p.add_argument("--cpu-c4-steps", type=int, default=2,
                   help="steps of the oracle's 65,536-env batching sample (metric workload)")
    p.add_argument("--c2-steps", type=int, default=600,
                   help="metric workload: timed steps of the plain 4096-env baseline (eager, then graphs); 600 "
                        "steps cross the first episode ends and their resets")
    p.add_argument("--metric-serve-seconds", type=float, default=20.0)
    p.add_argument("--metric-open-waits", type=float, nargs="*", default=[64.0, 32.0, 16.0])
    p.add_argument("--count-episodes", action="store_true",
                   help="plain workloads: count the episodes that end in each timed window")
    p.add_argument("--workload", choices=["metric", "plain", "batching", "serve", "divergent", "stack", "inference",
                                          "schemes", "objects", "noops"], default="metric",
                   help="metric (default): the batching form of 65536 envs over 16 ROMs (the value), the served "
                        "form of 131072 resident envs (p50/p99) and the plain 4096-env step; plain: 4096 envs, "
                        "1 ROM, every frame; batching: 65536 envs over 16 ROMs; serve: 131072 resident envs "
                        "behind the env server; divergent: 32768 envs over 8 branchy ROMs with sticky actions, "
                        "with the per-step rate over the run; stack: the frame stack of 16384 envs; inference: "
                        "4096 envs whose actions come from the policy CNN; schemes: 36864 envs over one ROM of "
                        "every cartridge scheme")
    p.add_argument("--serve-seconds", type=float, default=60.0)
    p.add_argument("--serve-pipelines", type=int, default=3)
    p.add_argument("--serve-open-waits", type=float, nargs="*", default=[128.0, 64.0, 32.0, 16.0],
                   help="open-loop mean gaps between a client's requests (ms), one curve point each")
    p.add_argument("--serve-open-seconds", type=float, default=3.0)
    p.add_argument("--graph", type=int, default=16,
                   help="plain workload: time steps captured G at a time in HIP graphs (two pipelines, each step's "
                        "render overlapping the next step's interpreter) after the eager steps, and report them as "
                        "the value; 0 = eager steps only")
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
    o = oracle.Oracle(w.n_envs, GRAY, frameskip=w.frameskip, seed=w.rng_seed, collisions=w.collisions)
    o.load_roms(roms)
    o.assign(env_rom)
    acts = w.actions(steps=steps)
    t0 = time.perf_counter()
    for s in range(steps):
        o.step(acts[s], want_frames=True)
    dt = time.perf_counter() - t0
    frames = w.n_envs * w.frameskip * steps
    cores = oracle.get_threads()
    # one core: the first 256 envs for the same steps, from the same states
    n1 = min(256, w.n_envs)
    o1 = oracle.Oracle(n1, GRAY, frameskip=w.frameskip, seed=w.rng_seed, collisions=w.collisions)
    o1.load_roms(roms)
    o1.assign(env_rom[:n1])
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        for s in range(steps):
            o1.step(acts[s][:n1], want_frames=True)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return {"value": frames / dt, "unit": "raw frames/s", "cores": cores, "kind": "oracle",
            "sample": f"{w.n_envs} envs x {steps} steps x frameskip {w.frameskip} ({frames} raw frames), "
                      f"every frame rendered + obs, same cartridge, seed and actions",
            "seconds": dt,
            "single_core": {"value": n1 * w.frameskip * steps / dt1, "sample": f"{n1} envs x {steps} steps",
                            "seconds": dt1},
            "cpu_model": cpu_model, "host_cpus": os.cpu_count()}


def measured_traffic(kernel, workload="plain_4096"):
    import hashlib
    srcs, sha, nbytes = MEASURED_TRAFFIC[(kernel, workload)]
    h = hashlib.sha256()
    for src in srcs:
        path = os.path.join(ROOT, "paper_1907_08467_amd", "csrc", src)
        if not os.path.exists(path):
            return None
        with open(path, "rb") as f:
            h.update(f.read())
    return nbytes if h.hexdigest()[:16] == sha else None


def graph_len(k, cap):
    """The longest graph of at most `cap` steps whose launches cover exactly
    k steps."""
    for g in range(min(cap, k), 0, -1):
        if k % g == 0:
            return g
    return 1


def episodes_ended(env):
    """Episodes ended so far, summed over every env (state record bytes
    188..191); synchronises."""
    return sum(int.from_bytes(bytes(env.get_state(e)[188:192]), "little") for e in range(env.num_envs))


def select_launch(env, args, n, want_frames, want_obs):
    if args.launch == "auto":
        launch, tune_ms = env.autotune(n=n, steps=3, want_frames=want_frames, want_obs=want_obs)
        print(f"autotuner picked {launch} ({tune_ms:.3f} ms/step)", file=sys.stderr, flush=True)
        return launch, "autotuner"
    tw, wk, rb = (int(x) for x in args.launch.split(","))
    env.set_launch(tw, wk, rb)
    return env.get_launch(), "fixed"


def kernel_table(env):
    kern = {}
    for k, name in KERNELS.items():
        ms, cnt = env.kernel_time(k)
        kern[name] = {"mean_ms": ms, "launches": cnt}
    return kern


def interp_roofline(kern, instr, n, frameskip):
    """The interpreter against the chip's integer lane-op issue rate."""
    t = kern["k_interp"]["mean_ms"] * 1e-3
    rate = instr / t if t > 0 else 0.0
    return {"bound": "alu", "kernel": "k_interp", "achieved": rate / 1e9, "peak": ALU_LANE_OPS_PEAK / 1e9,
            "unit": "G emulated instr/s vs G lane-ops/s", "frac": rate / ALU_LANE_OPS_PEAK, "traffic": None,
            "work_per_launch": f"{instr} emulated 6502 instructions ({n} envs x {frameskip} frames)"}


def interp_latency(kern, passes, rounds, env_rom, tile=64):
    """The interpreter's own bound, the latency of each wave's instruction
    stream: cycles per wave instruction pass if every wave lived the whole
    launch (an upper bound: waves that end early leave their SIMDs idle),
    next to the cost of a pass for a wave on the plain step (SQ counters:
    471 cycles, half of them issuing) and the scheduling rounds."""
    t = kern["k_interp"]["mean_ms"] * 1e-3
    counts = np.bincount(np.asarray(env_rom, dtype=np.int64))
    waves = int(sum((int(c) + tile - 1) // tile for c in counts if c))
    cyc = t * CLOCK_HZ * waves / passes if passes else None
    return {"bound": "latency", "waves": waves, "wave_passes": passes, "scheduling_rounds": rounds,
            "passes_per_round": passes / rounds if rounds else None,
            "cycles_per_pass_if_all_waves_lived_the_launch": cyc, "cycles_per_pass_plain_step_counters": 471}


def lane_util(instr, passes):
    """Active-lane utilisation of the interpreter: emulated instructions
    (summed over envs) over the lanes its waves' instruction passes offer."""
    return instr / (64.0 * passes) if passes else 0.0


def render_roofline(kern, n, frames_per_step, with_frames):
    fb = (n * frames_per_step * 210 * 160 if with_frames else 0) + n * 84 * 84
    t = (kern["k_render_frames"]["mean_ms"] + kern["k_render_obs"]["mean_ms"]) * 1e-3
    r = {"bound": "hbm", "algorithmic_bytes_written": fb, "achieved_GBs": fb / t / 1e9 if t > 0 else 0.0,
         "peak_GBs": HBM_PEAK_GBS}
    r["frac"] = r["achieved_GBs"] / HBM_PEAK_GBS
    return r


def gpu_env(w, **kw):
    from paper_1907_08467_amd.env import VcsEnv
    from paper_1907_08467_amd.inputs.palette import GRAY
    roms = [(r.data, r.scheme) for r in w.roms()]
    env_rom = w.env_rom()
    env = VcsEnv(roms, env_rom, GRAY, frameskip=w.frameskip, seed=w.rng_seed, render_mode=w.render_mode,
                 sticky_threshold=w.sticky_threshold, collisions=w.collisions, **kw)
    return env, roms, env_rom


def bench_plain(args, c=2):
    import torch
    from paper_1907_08467_amd.inputs.workloads import config
    w = config(c)
    if args.envs != w.n_envs:
        w.n_envs = args.envs
    K, W = args.steps, args.warmup
    G = graph_len(K, args.graph) if args.graph else 0
    env, roms, env_rom = gpu_env(w, pipelines=2 if G else 1)
    dev = torch.device("cuda", 0)
    n = w.n_envs
    launch, launch_from = select_launch(env, args, n, True, True)
    acts = torch.from_numpy(w.actions(steps=2 * K + W)).to(dev)
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

    ep0 = episodes_ended(env) if args.count_episodes else None
    env.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        env.step(acts[W + s], out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    env.timing(False)
    ep1 = episodes_ended(env) if args.count_episodes else None
    instr_last, instr_uniform, passes, rounds = env.last_step_counts()
    kern = kernel_table(env)
    value = eager_value = n * w.frameskip * K / dt
    eager_ms = dt / K * 1e3
    print(f"timed {K} eager steps in {dt:.3f}s", file=sys.stderr, flush=True)
    graph_res = None
    if G:
        graph = env.capture(n=n, steps=G, want_frames=True, want_obs=True)
        for s in range(0, 2 * G, G):        # two untimed launches
            graph.actions.copy_(acts[W + s:W + s + G])
            graph.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(0, K, G):
            graph.actions.copy_(acts[W + K + s:W + K + s + G])
            graph.launch()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        value = n * w.frameskip * K / dt
        graph_res = {"value": value, "ms_per_step": dt / K * 1e3, "steps_per_graph": G,
                     "steps": f"{W + K + 2 * G}..{W + 2 * K + 2 * G - 1}"}
        if args.count_episodes:
            graph_res["episodes_ended"] = episodes_ended(env) - ep1
        print(f"timed {K} graph steps in {dt:.3f}s", file=sys.stderr, flush=True)
    first, bits = env.poll_errors()
    print(f"errors {bits:#x}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print(f"cpu baseline: oracle, {args.cpu_steps} steps", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, roms, env_rom, args.cpu_steps)
    return {
        "metric": "raw emulated frames/s on 1 MI355X (p50/p99 step latency in served mode)",
        "value": value, "unit": "raw frames/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": n * w.frameskip / value * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": (f"plain batched step: {n} envs x 1 seeded 4 KB synthetic cartridge, frameskip "
                                f"{w.frameskip}, every 210x160 frame rendered to HBM + 84x84 max-of-two gray obs, "
                                "random actions (seed 1), no sticky actions") if c == 2 else
                               (f"objects step: {n} envs x 1 seeded 4 KB synthetic cartridge with missiles, ball, "
                                f"NUSIZ copies, object motion and collision reads, collision latches tracked, "
                                f"frameskip {w.frameskip}, every 210x160 frame rendered to HBM + 84x84 max-of-two "
                                f"gray obs, random actions (seed {w.action_seed}), no sticky actions"),
                   "num_envs": n, "frameskip": w.frameskip, "render": "all frames",
                   "launch": launch, "launch_from": launch_from,
                   "steps_as": f"HIP graphs of {G} steps, render overlapping the next interpreter" if G
                   else "eager step calls"},
        "eager": {"value": eager_value, "ms_per_step": eager_ms, "steps": f"{W}..{W + K - 1}",
                  "episodes_ended": None if ep0 is None else ep1 - ep0},
        "graph": graph_res,
        # counter figures of this workload exist for the 4096-env step
        "roofline": dict(interp_roofline(kern, instr_last, n, w.frameskip),
                         traffic=measured_traffic("k_interp") if (n == 4096 and c == 2) else None),
        "render_roofline": dict(render_roofline(kern, n, w.frameskip, True),
                                traffic={k: measured_traffic(k) if (n == 4096 and c == 2) else None
                                         for k in ("k_render_frames", "k_render_obs")}),
        "kernels_ms": {k: v["mean_ms"] for k, v in kern.items()},
        "emulated_instr_per_step": instr_last,
        "uniform_mode_fraction": instr_uniform / instr_last if instr_last else 0.0,
        "lane_utilisation": lane_util(instr_last, passes), "wave_passes": passes, "wave_rounds": rounds,
        "interp_latency": interp_latency(kern, passes, rounds, env_rom, launch["tile_envs"]),
        "errors": bits,
        "cpu_baseline": cpu,
    }


def bench_batching(args):
    """Uneven populations over 16 mixed ROMs, last two frames rendered, obs
    only: the plain kernel (64 envs per wave, eager steps) against the
    batching form (autotuned shape, graph-captured steps) on the same inputs."""
    import torch
    from paper_1907_08467_amd.inputs.workloads import config
    w = config(4)
    n = w.n_envs
    K, W = args.steps, args.warmup
    G = graph_len(K, 4)                      # steps per captured graph
    dev = torch.device("cuda", 0)
    acts = torch.from_numpy(w.actions(steps=K + W)).to(dev)
    res = {}
    finals = {}
    for form in ("plain", "batching"):
        env, roms, env_rom = gpu_env(w, pipelines=1 if form == "plain" else 2)
        if form == "plain":
            env.set_launch(64, 0, 256)
            launch, launch_from = env.get_launch(), "fixed"
        else:
            launch, launch_from = select_launch(env, args, n, False, True)
        obs = torch.empty((n, 84, 84), dtype=torch.uint8, device=dev)
        rew = torch.empty(n, dtype=torch.int32, device=dev)
        done = torch.empty(n, dtype=torch.uint8, device=dev)
        for s in range(W):
            env.step(acts[s], out=(obs, rew, done, None))
        torch.cuda.synchronize()
        print(f"{form}: warmup done ({W} steps)", file=sys.stderr, flush=True)
        if form == "plain":
            env.timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(K):
                env.step(acts[W + s], out=(obs, rew, done, None))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            env.timing(False)
            kern = kernel_table(env)
            last = (obs, rew, done)
        else:
            graph = env.capture(n=n, steps=G, want_obs=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(0, K, G):
                graph.actions.copy_(acts[W + s:W + s + G])
                graph.launch()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            last = (graph.obs[G - 1], graph.reward[G - 1], graph.done[G - 1])
            # kernel durations of the same shape, measured eagerly
            env.timing(True)
            for s in range(G):
                env.step(acts[s], out=(obs, rew, done, None))
            torch.cuda.synchronize()
            env.timing(False)
            kern = kernel_table(env)
        instr_last, instr_uniform, passes, rounds = env.last_step_counts()
        bits = env.poll_errors()[1]
        finals[form] = [t.cpu().numpy() for t in last]
        res[form] = {"value": n * w.frameskip * K / dt, "ms_per_step": dt / K * 1e3, "launch": launch,
                     "uniform_mode_fraction": instr_uniform / instr_last if instr_last else 0.0,
                     "lane_utilisation": lane_util(instr_last, passes), "wave_passes": passes,
                     "wave_rounds": rounds,
                     "interp_latency": interp_latency(kern, passes, rounds, env_rom, launch["tile_envs"]),
                     "launch_from": launch_from, "kernels_ms": {k: v["mean_ms"] for k, v in kern.items()},
                     "roofline": dict(interp_roofline(kern, instr_last, n, w.frameskip),
                                      traffic=measured_traffic("k_interp", "batching_65536") if n == 65536 else None),
                     "render_roofline": dict(render_roofline(kern, n, 2, False),
                                             traffic={"k_render_obs": measured_traffic("k_render_obs", "batching_65536")
                                                      if n == 65536 else None}),
                     "errors": bits}
        print(f"{form}: {res[form]['value']:.4g} raw frames/s", file=sys.stderr, flush=True)
        del env
        torch.cuda.empty_cache()
    same = all(np.array_equal(a, b) for a, b in zip(finals["plain"], finals["batching"]))
    b = res["batching"]
    return {
        "metric": "raw emulated frames/s on 1 MI355X (p50/p99 step latency in served mode)",
        "value": b["value"], "unit": "raw frames/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": b["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"batching form: {n} envs over 16 synthetic ROMs (8 x 4 KB, 8 x F8) in Zipf 1.2 "
                               "populations, frameskip 4, last two frames rendered into the 84x84 obs, "
                               f"random actions (seed 3); {G}-step HIP graphs on two pipelines (each step's render "
                               "overlapping the next interpreter), autotuned launch",
                   "num_envs": n, "frameskip": w.frameskip, "render": "last two", "launch": b["launch"],
                   "launch_from": b["launch_from"], "graph_steps": G},
        "roofline": b["roofline"], "render_roofline": b["render_roofline"], "kernels_ms": b["kernels_ms"],
        "uniform_mode_fraction": b["uniform_mode_fraction"], "lane_utilisation": b["lane_utilisation"],
        "wave_passes": b["wave_passes"], "wave_rounds": b["wave_rounds"], "interp_latency": b["interp_latency"],
        "plain_kernel": res["plain"], "speedup_vs_plain": b["value"] / res["plain"]["value"],
        "last_step_identical_to_plain": bool(same), "errors": b["errors"] | res["plain"]["errors"],
        "cpu_baseline": None,
    }


def bench_divergent(args, noop_after_copy=False, keep_step_ms=False):
    """32768 envs over 8 divergent ROMs (4 x 4 KB, 4 x F8), sticky actions
    p = 0.25, every frame rendered: raw frames/s and the per-step time over the
    run (the paper's FPS-against-step curve: envs start in step from the reset
    cache and drift apart)."""
    import torch
    from paper_1907_08467_amd.inputs.workloads import config
    w = config(3)
    n, K = w.n_envs, args.steps
    env, roms, env_rom = gpu_env(w, noop_after_copy=noop_after_copy)
    dev = torch.device("cuda", 0)
    launch, launch_from = select_launch(env, args, n, True, True)
    env.reset()                                # every env back to a cache state: the curve starts correlated
    acts = torch.from_numpy(w.actions(steps=K)).to(dev)
    obs = torch.empty((n, 84, 84), dtype=torch.uint8, device=dev)
    rew = torch.empty(n, dtype=torch.int32, device=dev)
    done = torch.empty(n, dtype=torch.uint8, device=dev)
    frames = torch.empty((n, w.frameskip, 210, 160), dtype=torch.uint8, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    pts = sorted(set([0, 1, 2, 5, 10, 20, 50, 100, 200, 500, 1000, 2000, 3000, 4000, K - 1]) & set(range(K)))
    util = {}
    torch.cuda.synchronize()
    ev[0].record()
    for s in range(K):
        env.step(acts[s], out=(obs, rew, done, frames))
        ev[s + 1].record()
        if s in pts:     # the step's counters (read after it: a sync at these few steps only)
            instr, _, passes, rounds = env.last_step_counts()
            util[str(s)] = {"lane_utilisation": lane_util(instr, passes), "instr": instr, "passes": passes,
                            "rounds": rounds}
        if s % 500 == 499:
            print(f"divergent: step {s + 1} of {K}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms = [ev[s].elapsed_time(ev[s + 1]) for s in range(K)]
    total = sum(ms) * 1e-3
    value = n * w.frameskip * K / total
    bits = env.poll_errors()[1]
    return {
        "metric": "raw emulated frames/s on 1 MI355X (p50/p99 step latency in served mode)",
        "value": value, "unit": "raw frames/s", "n_gpus": 1, "steps": K, "warmup": 0,
        "ms_per_step": total / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"divergent batch: {n} envs over 8 synthetic ROMs (4 x 4 KB, 4 x F8 bank-switched) "
                               "with data-dependent branches, sticky actions p = 0.25, frameskip 4, every frame "
                               "rendered + obs, eager steps from a fresh reset", "num_envs": n,
                   "launch": launch, "launch_from": launch_from},
        "fps_by_step": {str(s): n * w.frameskip / (ms[s] * 1e-3) for s in pts},
        "interp_by_step": util,
        "errors": bits, "roofline": None, "cpu_baseline": None,
        **({"step_ms": ms} if keep_step_ms else {}),
    }


def bench_noops(args):
    """The divergent workload with the reset no-ops run after each copy
    (every reset then emulates 2 + n, n <= 30, NOOP frames inside the step)
    against the same run with the no-ops baked into the cache (the paper's
    design): raw frames/s, mean and longest step time of both."""
    base = bench_divergent(args, keep_step_ms=True)
    res = bench_divergent(args, noop_after_copy=True, keep_step_ms=True)
    ms_b, ms_v = base.pop("step_ms"), res.pop("step_ms")
    res["config"]["workload"] = res["config"]["workload"].replace(
        "eager steps from a fresh reset", "eager steps from a fresh reset; reset no-ops (0-30 frames) run after "
        "each reset's cache copy instead of being baked into the cache")
    res["baked_noops"] = {"value": base["value"], "ms_per_step": base["ms_per_step"]}
    res["mean_step_ms"] = {"noops_after_copy": sum(ms_v) / len(ms_v), "baked": sum(ms_b) / len(ms_b)}
    res["max_step_ms"] = {"noops_after_copy": max(ms_v), "baked": max(ms_b)}
    return res


def cpu_baseline_sample(w, roms, env_rom, per_rom, steps):
    """The oracle on `per_rom` envs of every ROM of `w` for `steps` steps."""
    import oracle
    from paper_1907_08467_amd.inputs.palette import GRAY
    ids = np.concatenate([np.nonzero(env_rom == r)[0][:per_rom] for r in range(len(roms))])
    o = oracle.Oracle(ids.size, GRAY, frameskip=w.frameskip, seed=w.rng_seed, render_mode=w.render_mode,
                      sticky_threshold=w.sticky_threshold)
    o.load_roms(roms)
    o.assign(env_rom[ids])
    acts = w.actions(steps=steps)[:, ids]
    t0 = time.perf_counter()
    for s in range(steps):
        o.step(acts[s])
    dt = time.perf_counter() - t0
    frames = ids.size * w.frameskip * steps
    return {"value": frames / dt, "unit": "raw frames/s", "cores": oracle.get_threads(), "kind": "oracle",
            "sample": f"{per_rom} envs of each of the {len(roms)} ROMs x {steps} steps x frameskip {w.frameskip}, "
                      "same cartridges, sticky actions and render mode", "seconds": dt}


def bench_schemes(args):
    """36864 envs over one divergent ROM of every cartridge scheme (4K, F8,
    F6, F4, F8SC, F6SC, F4SC, E0, 3F), sticky actions p = 0.25, last two
    frames rendered: the interpreter with 32 KB of cartridge in LDS."""
    import torch
    from paper_1907_08467_amd.inputs.workloads import config
    w = config(6)
    n, K, W = w.n_envs, args.steps, args.warmup
    env, roms, env_rom = gpu_env(w)
    dev = torch.device("cuda", 0)
    launch, launch_from = select_launch(env, args, n, False, True)
    acts = torch.from_numpy(w.actions(steps=K + W)).to(dev)
    obs = torch.empty((n, 84, 84), dtype=torch.uint8, device=dev)
    rew = torch.empty(n, dtype=torch.int32, device=dev)
    done = torch.empty(n, dtype=torch.uint8, device=dev)
    for s in range(W):
        env.step(acts[s], out=(obs, rew, done, None))
    torch.cuda.synchronize()
    env.timing(True)
    t0 = time.perf_counter()
    for s in range(K):
        env.step(acts[W + s], out=(obs, rew, done, None))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    env.timing(False)
    instr_last, instr_uniform = env.last_step_stats()
    kern = kernel_table(env)
    value = n * w.frameskip * K / dt
    bits = env.poll_errors()[1]
    cpu = None
    if not args.no_cpu_baseline:
        print("cpu baseline: oracle on a sample of every ROM", file=sys.stderr, flush=True)
        cpu = cpu_baseline_sample(w, roms, env_rom, per_rom=64, steps=48)
    return {
        "metric": "raw emulated frames/s on 1 MI355X (p50/p99 step latency in served mode)",
        "value": value, "unit": "raw frames/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"mixed cartridge schemes: {n} envs over 9 synthetic divergent ROMs, one per scheme "
                               "(4K, F8, F6, F4, F8SC, F6SC, F4SC, E0, 3F), sticky actions p = 0.25, frameskip 4, "
                               "last two frames rendered + obs, eager steps", "num_envs": n,
                   "launch": launch, "launch_from": launch_from},
        "roofline": dict(interp_roofline(kern, instr_last, n, w.frameskip), traffic=None),
        "kernels_ms": {k: v["mean_ms"] for k, v in kern.items()},
        "emulated_instr_per_step": instr_last,
        "uniform_mode_fraction": instr_uniform / instr_last if instr_last else 0.0,
        "errors": bits, "cpu_baseline": cpu,
    }


def bench_stack(args):
    """Frame stack of the last four observations for 16384 envs (the paper's
    memory-wall point), 8-bit and 4-bit storage: push throughput against HBM."""
    import torch
    from paper_1907_08467_amd.env import FrameStack
    from paper_1907_08467_amd.inputs.workloads import config
    w = config(2)
    w.n_envs = 16384
    env, roms, env_rom = gpu_env(w)
    dev = torch.device("cuda", 0)
    n, K = w.n_envs, args.steps
    acts = torch.from_numpy(w.actions(steps=8)).to(dev)
    obs_steps = []
    for s in range(8):                         # real observations and done flags to push
        o, _, d, _ = env.step(acts[s])
        obs_steps.append((o.clone(), d.clone()))
    res = {}
    for bits in (8, 4):
        fs = FrameStack(env, depth=4, bits=bits)
        out = torch.empty((n, 4, 84, 84), dtype=torch.uint8, device=dev)
        fs.push(obs_steps[0][0], torch.ones_like(obs_steps[0][1]), out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(K):
            o, d = obs_steps[k % 8]
            fs.push(o, d, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        slot = 84 * 84 * bits // 8
        # per env: obs read, one slot written, four slots read, four obs written
        nbytes = n * (84 * 84 + slot + 4 * slot + 4 * 84 * 84)
        res[f"{bits}bit"] = {"ms_per_push": ms, "achieved_GBs": nbytes / (ms * 1e-3) / 1e9,
                             "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "ring_bytes": n * 4 * slot, "algorithmic_bytes_per_push": nbytes}
        fs.close()
    b = res["8bit"]
    return {
        "metric": "frame-stack pushes/s (envs x pushes / s) on 1 MI355X", "value": n / (b["ms_per_push"] * 1e-3),
        "unit": "env-pushes/s", "n_gpus": 1, "steps": K, "warmup": 1, "ms_per_step": b["ms_per_push"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"frame stack: last 4 84x84 observations of {n} envs, pushed after each step",
                   "num_envs": n, "depth": 4},
        "roofline": {"bound": "hbm", "kernel": "k_stack", "achieved": b["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": b["frac"], "traffic": None},
        "forms": res, "cpu_baseline": None,
    }


def cpu_baseline_inference(w, roms, env_rom, layers, steps, n):
    """The oracle's inference loop: oracle policy -> oracle step -> oracle stack."""
    import oracle
    from oracle.policy import forward, greedy
    from oracle.stack import FrameStack as OracleStack
    from paper_1907_08467_amd.inputs.palette import GRAY
    o = oracle.Oracle(n, GRAY, frameskip=w.frameskip, seed=w.rng_seed, render_mode=w.render_mode)
    o.load_roms(roms)
    o.assign(env_rom[:n])
    fs = OracleStack(n, depth=4, bits=8)
    st = fs.push(o.reset(), np.ones(n, np.uint8))
    t0 = time.perf_counter()
    for _ in range(steps):
        a = greedy(forward(st, layers))
        ob, _, d, _ = o.step(a)
        st = fs.push(ob, d)
    dt = time.perf_counter() - t0
    frames = n * w.frameskip * steps
    return {"value": frames / dt, "unit": "raw frames/s", "cores": oracle.get_threads(), "kind": "oracle",
            "sample": f"{n} envs x {steps} steps x frameskip {w.frameskip}: float64 policy forward (numpy), "
                      "oracle step with obs, oracle frame stack", "seconds": dt}


def bench_inference(args):
    """Inference path with a policy in the loop (the paper's 'inference only'
    load condition, Section 4): per step the policy CNN reads every env's
    frame stack and picks its action, the envs step with those actions and
    the stack takes the new observations; nothing leaves the device."""
    import torch
    from paper_1907_08467_amd.env import FrameStack, Policy
    from paper_1907_08467_amd.inputs.policy_weights import policy_weights
    from paper_1907_08467_amd.inputs.workloads import config
    w = config(2)
    env, roms, env_rom = gpu_env(w)
    dev = torch.device("cuda", 0)
    n, K, W = w.n_envs, args.steps, args.warmup
    layers = policy_weights(7)
    pol = Policy(env, [l[0] for l in layers], [l[2] for l in layers])
    fs = FrameStack(env, depth=4, bits=8)
    obs = env.reset()
    rew = torch.empty(n, dtype=torch.int32, device=dev)
    done = torch.empty(n, dtype=torch.uint8, device=dev)
    st = torch.empty((n, 4, 84, 84), dtype=torch.uint8, device=dev)
    act = torch.empty(n, dtype=torch.uint8, device=dev)
    fs.push(obs, torch.ones(n, dtype=torch.uint8, device=dev), out=st)

    def one_step():
        pol.act(st, actions=act)
        env.step(act, out=(obs, rew, done, None))
        fs.push(obs, done, out=st)

    for _ in range(W):
        one_step()
    torch.cuda.synchronize()
    env.timing(True)
    t0 = time.perf_counter()
    for _ in range(K):
        one_step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    env.timing(False)
    kern = kernel_table(env)
    value = n * w.frameskip * K / dt
    print(f"timed {K} inference steps in {dt:.3f}s", file=sys.stderr, flush=True)
    # the policy alone on the last stacks, HIP events on the stream it runs on
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        pol.act(st, actions=act)
    e1.record()
    torch.cuda.synchronize()
    pol_ms = e0.elapsed_time(e1) / K
    flops = POLICY_FLOPS_PER_ENV * n
    tflops = flops / (pol_ms * 1e-3) / 1e12
    hist = torch.bincount(act.long(), minlength=18).cpu().tolist()
    bits = env.poll_errors()[1]
    cpu = None
    if not args.no_cpu_baseline:
        print("cpu baseline: oracle inference loop", file=sys.stderr, flush=True)
        cpu = cpu_baseline_inference(w, roms, env_rom, layers, steps=8, n=256)
    pol.close()
    fs.close()
    return {
        "metric": "raw emulated frames/s on 1 MI355X, actions from a policy CNN on the device (inference only)",
        "value": value, "unit": "raw frames/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8 emulation, bf16 policy (fp32 accumulate)", "data": "synthetic",
        "config": {"workload": f"inference only: {n} envs x 1 seeded 4 KB synthetic cartridge, frameskip "
                               f"{w.frameskip}; per step a conv 8x8/4-4x4/2-3x3/1 + 512 + 19 policy (random "
                               "He-uniform weights, seed 7) on each env's 4-frame 8-bit stack, greedy actions",
                   "num_envs": n, "frameskip": w.frameskip, "stack": "4 x 84x84, 8-bit"},
        "roofline": {"bound": "mfma", "kernel": "k_conv (5 layers, one act call)", "achieved": tflops,
                     "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / BF16_MFMA_PEAK_TFLOPS,
                     "traffic": None, "work_per_launch": f"{POLICY_FLOPS_PER_ENV} flop/env x {n} envs"},
        "policy_ms": pol_ms,
        "kernels_ms": {k: v["mean_ms"] for k, v in kern.items()},
        "action_histogram_last_step": hist, "errors": bits,
        "cpu_baseline": cpu,
    }


def bench_serve(args):
    """131072 resident envs, 64 closed-loop actors, continuous batching."""
    import torch
    from paper_1907_08467_amd.inputs.workloads import config
    from paper_1907_08467_amd.serve import ActorPool, EnvServer, GpuBackend, run_served, slots_for_budget
    w = config(5)
    n = w.n_envs
    budget = 16 << 30
    pipes = args.serve_pipelines
    cap = slots_for_budget(budget - (512 << 20), n, 16, 2, pipes)   # 512 MiB kept for tile tables and tuning
    env, roms, env_rom = gpu_env(w, max_batch=cap, pipelines=pipes, hbm_budget_bytes=budget)
    dev = torch.device("cuda", 0)
    launch, launch_from = select_launch(env, args, min(cap, 16384), False, True)
    # the fixed-batch reference: 65536 listed envs per step, eager
    m = min(65536, cap)
    ids = torch.arange(m, dtype=torch.int32, device=dev)
    acts = torch.from_numpy(w.actions(steps=12, n=m)).to(dev)
    out = (torch.empty((m, 84, 84), dtype=torch.uint8, device=dev), torch.empty(m, dtype=torch.int32, device=dev),
           torch.empty(m, dtype=torch.uint8, device=dev), None)
    for s in range(2):
        env.step(acts[s], env_ids=ids, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(2, 12):
        env.step(acts[s], env_ids=ids, out=out)
    torch.cuda.synchronize()
    fixed_dt = (time.perf_counter() - t0) / 10
    fixed = {"envs_per_step": m, "ms_per_step": fixed_dt * 1e3, "value": m * w.frameskip / fixed_dt}
    print(f"fixed batch: {fixed}", file=sys.stderr, flush=True)

    backend = GpuBackend(env, cap)
    server = EnvServer(backend, cap, n)
    actors = ActorPool(64, n, mean_wait_s=2e-3, size_lo=64, size_hi=4096, seed0=5000)
    st = run_served(server, actors, seconds=args.serve_seconds)
    value = st["env_steps"] * w.frameskip / st["seconds"]
    print(f"served: {st}", file=sys.stderr, flush=True)
    # open loop: Poisson arrivals that do not wait for answers, from about the
    # served capacity to four times it; the backlog left at the end is dropped
    curve = []
    for wait_ms in args.serve_open_waits:
        op = ActorPool(64, n, mean_wait_s=wait_ms * 1e-3, size_lo=64, size_hi=4096, seed0=6000, open_loop=True)
        so = run_served(EnvServer(backend, cap, n), op, seconds=args.serve_open_seconds)
        offered = 64 / (wait_ms * 1e-3) * op.mean_size() * w.frameskip
        curve.append({"mean_gap_ms": wait_ms, "offered_frames_s": offered,
                      "served_frames_s": so["env_steps"] * w.frameskip / so["seconds"],
                      "p50_ms": so["p50_ms"], "p99_ms": so["p99_ms"], "requests": so["requests"],
                      "backlog_env_steps": so["backlog_env_steps"], "seconds": so["seconds"]})
        print(f"open loop {wait_ms} ms: {curve[-1]}", file=sys.stderr, flush=True)
    bits = env.poll_errors()[1]
    return {
        "metric": "raw emulated frames/s on 1 MI355X + p50/p99 step latency (served mode)",
        "value": value, "unit": "raw frames/s", "n_gpus": 1, "steps": st["batches"], "warmup": 0,
        "ms_per_step": st["seconds"] / max(1, st["batches"]) * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "latency_ms": {"p50": st["p50_ms"], "p99": st["p99_ms"]},
        "config": {"workload": f"serving form: {n} resident envs over 16 synthetic ROMs (Zipf 1.2), 64 closed-loop "
                               "actors, exponential think time (mean 2 ms), requests of floor(exp U(ln 64, ln 4096)) "
                               f"distinct env ids, continuous batching on {pipes} pipelines, 16 GiB budget",
                   "num_envs": n, "frameskip": w.frameskip, "render": "last two", "pipelines": pipes,
                   "max_batch": cap, "launch": launch, "launch_from": launch_from, "seconds": st["seconds"]},
        "served": st, "fixed_batch": fixed, "open_loop_curve": curve, "errors": bits, "roofline": None,
        "cpu_baseline": None,
    }


def cpu_legs(args):
    """The oracle on the host cores: configuration 1 in full, and bounded
    samples of the plain 4096-env step and of the 65,536-env batching
    workload (the same cartridges, seeds, actions and render modes)."""
    import oracle
    from paper_1907_08467_amd.inputs.palette import GRAY
    from paper_1907_08467_amd.inputs.workloads import config
    legs = {}
    for key, c, steps, with_frames in (("c1_full", 1, None, True), ("plain_4096", 2, args.cpu_steps, True),
                                       ("batching_65536", 4, args.cpu_c4_steps, False)):
        w = config(c)
        steps = w.steps if steps is None else steps
        roms = [(r.data, r.scheme) for r in w.roms()]
        env_rom = w.env_rom()
        print(f"cpu baseline {key}: oracle, {w.n_envs} envs x {steps} steps", file=sys.stderr, flush=True)
        o = oracle.Oracle(w.n_envs, GRAY, frameskip=w.frameskip, seed=w.rng_seed, render_mode=w.render_mode,
                          sticky_threshold=w.sticky_threshold, collisions=w.collisions)
        o.load_roms(roms)
        o.assign(env_rom)
        acts = w.actions(steps=steps)
        t0 = time.perf_counter()
        for s in range(steps):
            o.step(acts[s], want_frames=with_frames)
        dt = time.perf_counter() - t0
        frames = w.n_envs * w.frameskip * steps
        o.close()
        legs[key] = {"value": frames / dt, "unit": "raw frames/s", "cores": oracle.get_threads(), "kind": "oracle",
                     "sample": f"{w.name}: {w.n_envs} envs x {steps} steps x frameskip {w.frameskip} "
                               f"({frames} raw frames){', frames copied out' if with_frames else ''}",
                     "seconds": dt}
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    head = dict(legs["batching_65536"])
    head["legs"] = legs
    head["cpu_model"] = cpu_model
    head["host_cpus"] = os.cpu_count()
    return head


def bench_metric(args):
    """The metric's own configurations on one GPU: the batching form of
    65,536 envs (the value; the plain kernel on the same inputs beside it),
    the served form of 131,072 resident envs with p50/p99 step latency, and
    the plain 4096-env step as the baseline, each over exactly the steps
    named; the oracle's rates on the host cores."""
    import copy
    import torch
    t_start = time.perf_counter()
    res = bench_batching(args)
    torch.cuda.empty_cache()
    print(f"batching done at {time.perf_counter() - t_start:.0f}s", file=sys.stderr, flush=True)
    a2 = copy.copy(args)
    a2.serve_seconds = args.metric_serve_seconds
    a2.serve_open_waits = args.metric_open_waits
    served = bench_serve(a2)
    torch.cuda.empty_cache()
    print(f"serving done at {time.perf_counter() - t_start:.0f}s", file=sys.stderr, flush=True)
    a3 = copy.copy(args)
    a3.steps, a3.envs, a3.no_cpu_baseline, a3.count_episodes = args.c2_steps, 4096, True, True
    plain = bench_plain(a3, 2)
    torch.cuda.empty_cache()
    print(f"plain step done at {time.perf_counter() - t_start:.0f}s", file=sys.stderr, flush=True)
    res["metric"] = "raw emulated frames/s on 1 MI355X + p50/p99 step latency (served mode)"
    res["config"]["workload"] = "batching form (the largest fixed batch): " + res["config"]["workload"]
    res["served"] = {"value": served["value"], "unit": "raw frames/s", "p50_ms": served["latency_ms"]["p50"],
                     "p99_ms": served["latency_ms"]["p99"], "workload": served["config"]["workload"],
                     "seconds": served["served"]["seconds"], "requests": served["served"]["requests"],
                     "batches": served["served"]["batches"], "stats": served["served"],
                     "fixed_batch": served["fixed_batch"], "open_loop_curve": served["open_loop_curve"],
                     "errors": served["errors"], "launch": served["config"]["launch"],
                     "max_batch": served["config"]["max_batch"]}
    res["plain_batch_4096"] = {k: plain[k] for k in ("value", "steps", "warmup", "ms_per_step", "config", "eager",
                                                     "graph", "roofline", "render_roofline", "kernels_ms",
                                                     "emulated_instr_per_step", "uniform_mode_fraction",
                                                     "lane_utilisation", "wave_passes", "errors")}
    res["errors"] |= served["errors"] | plain["errors"]
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_legs(args)
    res["bench_seconds"] = time.perf_counter() - t_start
    return res


def main():
    args = parse()
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the envs are independent and "
              "shard by env id, but this benchmark measures the single-GPU path.", file=sys.stderr)
        sys.exit(2)
    fn = {"metric": bench_metric, "plain": bench_plain, "batching": bench_batching, "serve": bench_serve,
          "divergent": bench_divergent, "stack": bench_stack, "inference": bench_inference,
          "schemes": bench_schemes, "objects": lambda a: bench_plain(a, 7), "noops": bench_noops}[args.workload]
    print(json.dumps(fn(args)))


if __name__ == "__main__":
    main()
