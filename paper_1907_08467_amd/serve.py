"""Serving form: an env server with continuous batching over resident envs.

Many actors send step requests (a set of env ids and one action each) at
their own pace.  The request loop merges waiting requests into batches, runs
each batch as one step call on one of the library's pipelines, and admits new
requests into the next batch of any pipeline whose previous batch finished,
while batches on other pipelines are still on the device.  All machine state
stays on the device; a request's observations, rewards and done flags are
handed to its callback as device views.

Ordering rule (what makes served results equal to solo results): a request
is admitted only if none of its envs is in a batch on the device or in an
earlier request still waiting.  So every env takes its steps in the order its
requests arrived, and since envs are independent and every random draw is
keyed by the env's own id and counters, each result equals the one the same
request gets when run alone in that per-env order.

Admission by memory: each pipeline's scratch holds `max_batch` env-steps;
`slots_for_budget` sizes max_batch from a fixed device-memory budget.
"""

from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

# device bytes one in-flight env-step needs on a pipeline: row logs, obs,
# reward, done, step info, id validity, its share of a tile
LOG_BYTES = 210 * 112
OBS_BYTES = 84 * 84


def slot_bytes(n_slots):
    return n_slots * LOG_BYTES + OBS_BYTES + 4 + 1 + 4 + 1 + 2 * 4 + 8


def resident_bytes(num_envs, n_roms, cache_k=30):
    return num_envs * (256 + 2 + 4) + n_roms * cache_k * (256 + OBS_BYTES) + n_roms * 8192 * 9


def slots_for_budget(budget_bytes, num_envs, n_roms, n_slots, pipelines):
    """Largest batch per pipeline that fits the budget next to the resident state."""
    free = budget_bytes - resident_bytes(num_envs, n_roms)
    if free <= 0:
        raise ValueError("the budget does not hold the resident envs")
    per_pipe = free // pipelines
    return int(min(num_envs, per_pipe // slot_bytes(n_slots)))


@dataclasses.dataclass
class Request:
    client: int
    ids: np.ndarray          # int32 [k], distinct
    actions: np.ndarray      # uint8 [k]
    t_arrival: float
    seq: int = 0
    t_done: float = 0.0


class GpuBackend:
    """Runs merged batches on the library's pipelines, one HIP stream each."""

    def __init__(self, env, max_batch):
        import torch
        self.torch = torch
        self.env = env
        self.pipelines = env.pipelines
        dev = env.device
        self.streams = [torch.cuda.Stream(dev) for _ in range(self.pipelines)]
        pin = dict(dtype=torch.int32, pin_memory=True)
        self.h_ids = [torch.empty(max_batch, **pin) for _ in range(self.pipelines)]
        self.h_act = [torch.empty(max_batch, dtype=torch.uint8, pin_memory=True) for _ in range(self.pipelines)]
        self.d_ids = [torch.empty(max_batch, dtype=torch.int32, device=dev) for _ in range(self.pipelines)]
        self.d_act = [torch.empty(max_batch, dtype=torch.uint8, device=dev) for _ in range(self.pipelines)]
        self.obs = [torch.empty((max_batch, 84, 84), dtype=torch.uint8, device=dev) for _ in range(self.pipelines)]
        self.rew = [torch.empty(max_batch, dtype=torch.int32, device=dev) for _ in range(self.pipelines)]
        self.done = [torch.empty(max_batch, dtype=torch.uint8, device=dev) for _ in range(self.pipelines)]
        self.events = [None] * self.pipelines

    def launch(self, p, ids, actions):
        torch = self.torch
        n = ids.size
        st = self.streams[p]
        # the host staging buffers of pipeline p are free: its previous batch finished
        self.h_ids[p][:n].numpy()[:] = ids
        self.h_act[p][:n].numpy()[:] = actions
        with torch.cuda.stream(st):
            self.d_ids[p][:n].copy_(self.h_ids[p][:n], non_blocking=True)
            self.d_act[p][:n].copy_(self.h_act[p][:n], non_blocking=True)
            out = (self.obs[p][:n], self.rew[p][:n], self.done[p][:n], None)
            self.env.step(self.d_act[p][:n], env_ids=self.d_ids[p][:n], out=out, pipe=p)
            ev = torch.cuda.Event()
            ev.record(st)
        self.events[p] = ev

    def finished(self, p):
        return self.events[p] is not None and self.events[p].query()

    def results(self, p, lo, hi):
        return self.obs[p][lo:hi], self.rew[p][lo:hi], self.done[p][lo:hi]

    def release(self, p):
        self.events[p] = None


class EnvServer:
    """The request loop.  `on_result(req, obs, reward, done)` runs when a
    request's batch has finished; the views are valid during the call only."""

    def __init__(self, backend, max_batch, on_result=None, clock=time.perf_counter):
        self.backend = backend
        self.max_batch = max_batch
        self.on_result = on_result
        self.clock = clock
        self.pending = collections.deque()
        self.inflight = [None] * backend.pipelines     # (batch requests, offsets)
        self.busy = set()                               # envs in batches on the device
        self.seq = 0
        self.completed = 0
        self.env_steps = 0
        self.batches = 0
        self.batch_sizes = []
        self.deferred = 0          # times a waiting request was passed over by a batch

    def submit(self, req: Request):
        if req.ids.size > self.max_batch:
            raise ValueError(f"request of {req.ids.size} envs exceeds the batch capacity {self.max_batch}")
        if np.unique(req.ids).size != req.ids.size:
            raise ValueError("a request lists an env twice")
        req.seq = self.seq
        self.seq += 1
        self.pending.append(req)

    def _merge(self):
        """Admit waiting requests in arrival order under the ordering rule."""
        taken, blocked = [], set()
        size = 0
        keep = collections.deque()
        while self.pending:
            r = self.pending.popleft()
            ids = r.ids.tolist()
            fits = size + len(ids) <= self.max_batch
            free = fits and not any((e in self.busy) or (e in blocked) for e in ids)
            if free:
                taken.append(r)
                size += len(ids)
                self.busy.update(ids)
            else:
                keep.append(r)
                blocked.update(ids)
                self.deferred += 1
            if size == self.max_batch:
                break
        keep.extend(self.pending)
        self.pending = keep
        return taken, size

    def poll(self):
        """Finish batches that are done and start new ones; returns requests finished."""
        finished = 0
        for p in range(self.backend.pipelines):
            cur = self.inflight[p]
            if cur is not None and self.backend.finished(p):
                reqs, offs = cur
                now = self.clock()
                for r, lo in zip(reqs, offs):
                    r.t_done = now
                    if self.on_result is not None:
                        self.on_result(r, *self.backend.results(p, lo, lo + r.ids.size))
                    self.busy.difference_update(r.ids.tolist())
                self.backend.release(p)
                self.inflight[p] = None
                self.completed += len(reqs)
                finished += len(reqs)
        for p in range(self.backend.pipelines):
            if self.inflight[p] is None and self.pending:
                reqs, size = self._merge()
                if not reqs:
                    break
                ids = np.concatenate([r.ids for r in reqs]).astype(np.int32)
                act = np.concatenate([r.actions for r in reqs]).astype(np.uint8)
                offs = np.concatenate([[0], np.cumsum([r.ids.size for r in reqs])[:-1]]).tolist()
                self.backend.launch(p, ids, act)
                self.inflight[p] = (reqs, offs)
                self.env_steps += size
                self.batches += 1
                self.batch_sizes.append(size)
        return finished

    def idle(self):
        return not self.pending and all(x is None for x in self.inflight)

    def drain(self):
        while not self.idle():
            self.poll()


class ActorPool:
    """Closed-loop simulated actors: after its response each actor waits an
    exponential think time, then sends a request of floor(exp(U(ln lo, ln hi)))
    distinct env ids drawn uniformly from all envs, with uniform actions."""

    def __init__(self, n_clients, num_envs, mean_wait_s=2e-3, size_lo=64, size_hi=4096, seed0=5000,
                 n_actions=18):
        self.n, self.num_envs = n_clients, num_envs
        self.mean_wait = mean_wait_s
        self.lo, self.hi = size_lo, size_hi
        self.n_actions = n_actions
        self.rngs = [np.random.Generator(np.random.PCG64(seed0 + c)) for c in range(n_clients)]
        self.next_send = [0.0] * n_clients
        self.outstanding = [False] * n_clients

    def size(self, c):
        g = self.rngs[c]
        k = int(np.floor(np.exp(g.uniform(np.log(self.lo), np.log(self.hi)))))
        return max(1, min(k, self.num_envs))

    def start(self, t0):
        for c in range(self.n):
            self.next_send[c] = t0 + self.rngs[c].exponential(self.mean_wait)

    def due(self, now):
        out = []
        for c in range(self.n):
            if not self.outstanding[c] and self.next_send[c] <= now:
                g = self.rngs[c]
                k = self.size(c)
                ids = g.choice(self.num_envs, size=k, replace=False).astype(np.int32)
                act = g.integers(0, self.n_actions, k, dtype=np.uint8)
                out.append(Request(c, ids, act, self.next_send[c]))
                self.outstanding[c] = True
        return out

    def responded(self, c, now):
        self.outstanding[c] = False
        self.next_send[c] = now + self.rngs[c].exponential(self.mean_wait)


def run_served(server, actors, seconds, clock=time.perf_counter, record=None):
    """Drive the server with the actors for `seconds`; returns latency stats."""
    lat = []
    user_cb = server.on_result

    def on_result(req, obs, rew, done):
        lat.append(req.t_done - req.t_arrival)
        actors.responded(req.client, req.t_done)
        if user_cb is not None:
            user_cb(req, obs, rew, done)

    server.on_result = on_result
    t0 = clock()
    actors.start(t0)
    t_end = t0 + seconds
    steps0 = server.env_steps
    while True:
        now = clock()
        if now >= t_end:
            break
        for r in actors.due(now):
            server.submit(r)
        server.poll()
    server.drain()
    t1 = clock()
    server.on_result = user_cb
    lat = np.array(lat)
    return {
        "seconds": t1 - t0,
        "requests": int(lat.size),
        "env_steps": int(server.env_steps - steps0),
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
        "mean_batch": float(np.mean(server.batch_sizes)) if server.batch_sizes else 0.0,
        "batches": server.batches,
    }
