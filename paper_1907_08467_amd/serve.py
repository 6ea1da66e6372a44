"""Serving form: an env server with continuous batching over resident envs.

Many actors send step requests (a set of env ids and one action each) at
their own pace.  The request loop keeps a queue of pending env-steps and
merges them into batches: whenever one of the library's step pipelines is
free, every pending env-step that may run now goes into its next batch, while
batches on other pipelines are still on the device.  A request completes when
all of its env-steps have; its observations, rewards and done flags are
gathered on the device into the request's own buffers.  All machine state
stays on the device.

Ordering rule (what makes served results equal to solo results): an env-step
may run only when its env is in no batch on the device and no earlier request
still holds an unrun step of that env.  Every env therefore takes its steps
in the order its requests arrived, and since envs are independent and every
random draw is keyed by the env's own id and counters, each result equals the
one the same request gets when run alone, one request at a time in arrival
order.  Requests are split at env granularity, so two requests that share a
few envs still run their other envs in the same batch.

Admission by memory: each pipeline's scratch holds `max_batch` env-steps;
`slots_for_budget` sizes max_batch from a fixed device-memory budget.
"""

from __future__ import annotations

import collections
import dataclasses
import itertools
import time

import numpy as np

# device bytes one in-flight env-step needs on a pipeline: row logs, obs,
# reward, done, step info, id validity, its share of a tile
LOG_BYTES = 210 * 128
OBS_BYTES = 84 * 84


def slot_bytes(n_slots):
    return n_slots * LOG_BYTES + OBS_BYTES + 4 + 1 + 4 + 1 + 2 * 4 + 8


def resident_bytes(num_envs, n_roms, cache_k=30):
    # env records, ROM ids and tile entries; reset caches; 32 KB ROM slots and
    # the predecoded words of up to 8 banks of 4 KB (E0 cartridges take 8 MB)
    return num_envs * (384 + 2 + 4) + n_roms * cache_k * (384 + OBS_BYTES) + n_roms * (32768 + 8 * 4096 * 4)


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
    sched: np.ndarray | None = None   # env-steps already put into a batch
    unsched: int = 0                  # env-steps not put into a batch yet
    left: int = 0                     # env-steps not finished yet
    out: tuple | None = None          # (obs, reward, done) buffers of the request


class GpuBackend:
    """Runs merged batches on the library's pipelines, one HIP stream each.

    Request buffers live on the caller's current stream: gathers into them
    are enqueued there after the batch's event, and a pipeline's next batch
    waits for the gathers from its previous one."""

    def __init__(self, env, max_batch):
        import torch
        self.torch = torch
        self.env = env
        self.pipelines = env.pipelines
        dev = self.dev = env.device
        P = self.pipelines
        self.streams = [torch.cuda.Stream(dev) for _ in range(P)]
        self.h_ids = [torch.empty(max_batch, dtype=torch.int32, pin_memory=True) for _ in range(P)]
        self.h_act = [torch.empty(max_batch, dtype=torch.uint8, pin_memory=True) for _ in range(P)]
        self.d_ids = [torch.empty(max_batch, dtype=torch.int32, device=dev) for _ in range(P)]
        self.d_act = [torch.empty(max_batch, dtype=torch.uint8, device=dev) for _ in range(P)]
        self.obs = [torch.empty((max_batch, 84, 84), dtype=torch.uint8, device=dev) for _ in range(P)]
        self.rew = [torch.empty(max_batch, dtype=torch.int32, device=dev) for _ in range(P)]
        self.done = [torch.empty(max_batch, dtype=torch.uint8, device=dev) for _ in range(P)]
        self.events = [None] * P
        self.gathered = [None] * P

    def launch(self, p, ids, actions):
        torch = self.torch
        n = ids.size
        st = self.streams[p]
        # pipeline p's previous batch has finished, so its host staging buffers are free
        self.h_ids[p][:n].numpy()[:] = ids
        self.h_act[p][:n].numpy()[:] = actions
        with torch.cuda.stream(st):
            if self.gathered[p] is not None:
                st.wait_event(self.gathered[p])
            self.d_ids[p][:n].copy_(self.h_ids[p][:n], non_blocking=True)
            self.d_act[p][:n].copy_(self.h_act[p][:n], non_blocking=True)
            out = (self.obs[p][:n], self.rew[p][:n], self.done[p][:n], None)
            self.env.step(self.d_act[p][:n], env_ids=self.d_ids[p][:n], out=out, pipe=p)
            ev = torch.cuda.Event()
            ev.record(st)
        self.events[p] = ev

    def finished(self, p):
        return self.events[p] is not None and self.events[p].query()

    def alloc(self, k):
        t = self.torch
        return (t.empty((k, 84, 84), dtype=t.uint8, device=self.dev), t.empty(k, dtype=t.int32, device=self.dev),
                t.empty(k, dtype=t.uint8, device=self.dev))

    def scatter(self, out, pos, p, lo, hi):
        torch = self.torch
        cur = torch.cuda.current_stream(self.dev)
        cur.wait_event(self.events[p])
        if hi - lo == out[1].numel():                 # the whole request ran in this batch, in order
            out[0].copy_(self.obs[p][lo:hi])
            out[1].copy_(self.rew[p][lo:hi])
            out[2].copy_(self.done[p][lo:hi])
        else:
            idx = torch.from_numpy(pos.astype(np.int64)).to(self.dev, non_blocking=True)
            out[0].index_copy_(0, idx, self.obs[p][lo:hi])
            out[1].index_copy_(0, idx, self.rew[p][lo:hi])
            out[2].index_copy_(0, idx, self.done[p][lo:hi])

    def release(self, p):
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(self.dev))
        self.gathered[p] = ev
        self.events[p] = None


class EnvServer:
    """The request loop.  `on_result(req, obs, reward, done)` runs when the
    last env-step of a request has finished, with the request's buffers."""

    def __init__(self, backend, max_batch, num_envs, on_result=None, clock=time.perf_counter):
        self.backend = backend
        self.max_batch = max_batch
        self.num_envs = num_envs
        self.on_result = on_result
        self.clock = clock
        self.pending = collections.deque()              # requests with unscheduled env-steps, in arrival order
        self.inflight = [None] * backend.pipelines      # parts (request, positions, lo, hi)
        self.busy = np.zeros(num_envs, dtype=bool)      # env in a batch on the device
        self.stamp = np.zeros(num_envs, dtype=np.int64) # merge pass that last claimed the env
        self.passes = 0
        self.seq = 0
        self.completed = 0
        self.env_steps = 0
        self.batches = 0
        self.batch_sizes = []
        self.deferred = 0          # env-steps held back by an earlier step of their env

    def submit(self, req: Request):
        k = req.ids.size
        if k == 0:
            raise ValueError("empty request")
        if req.ids.min() < 0 or req.ids.max() >= self.num_envs:
            raise ValueError("env id out of range")
        if np.unique(req.ids).size != k:
            raise ValueError("a request lists an env twice")
        req.seq = self.seq
        self.seq += 1
        req.sched = np.zeros(k, dtype=bool)
        req.unsched = k
        req.left = k
        req.out = self.backend.alloc(k)
        self.pending.append(req)

    # a merge looks at most this many pending requests from the head of the
    # queue, so its cost stays bounded when requests pile up (overload)
    SCAN_REQUESTS = 256

    def _merge(self):
        """One batch of env-steps that may run now, in arrival order."""
        self.passes += 1
        stamp = self.passes
        parts, ids, acts = [], [], []
        size = 0
        for r in itertools.islice(self.pending, self.SCAN_REQUESTS):
            if size == self.max_batch:
                break
            if r.unsched == 0:
                continue
            un = np.flatnonzero(~r.sched)
            e = r.ids[un]
            ok = ~self.busy[e] & (self.stamp[e] != stamp)
            pos = un[ok][:self.max_batch - size]
            self.deferred += int(un.size - pos.size)
            self.stamp[e] = stamp                      # later requests may not pass these envs
            if pos.size:
                r.sched[pos] = True
                r.unsched -= pos.size
                self.busy[r.ids[pos]] = True
                parts.append((r, pos, size, size + pos.size))
                ids.append(r.ids[pos])
                acts.append(r.actions[pos])
                size += pos.size
        while self.pending and self.pending[0].unsched == 0:
            self.pending.popleft()
        if not parts:
            return None
        return parts, np.concatenate(ids).astype(np.int32), np.concatenate(acts).astype(np.uint8)

    def poll(self):
        """Finish batches that are done and start new ones; returns requests completed."""
        finished = 0
        for p in range(self.backend.pipelines):
            parts = self.inflight[p]
            if parts is None or not self.backend.finished(p):
                continue
            now = self.clock()
            for r, pos, lo, hi in parts:
                self.backend.scatter(r.out, pos, p, lo, hi)
                self.busy[r.ids[pos]] = False
                r.left -= pos.size
                if r.left == 0:
                    r.t_done = now
                    self.completed += 1
                    finished += 1
                    if self.on_result is not None:
                        self.on_result(r, *r.out)
            self.backend.release(p)
            self.inflight[p] = None
        for p in range(self.backend.pipelines):
            if self.inflight[p] is None and self.pending:
                m = self._merge()
                if m is None:
                    break
                parts, ids, acts = m
                self.backend.launch(p, ids, acts)
                self.inflight[p] = parts
                self.env_steps += ids.size
                self.batches += 1
                self.batch_sizes.append(ids.size)
        return finished

    def idle(self):
        return not self.pending and all(x is None for x in self.inflight)

    def drain(self):
        while not self.idle():
            self.poll()


class ActorPool:
    """Simulated actors.  Closed loop (the default): after its response each
    actor waits an exponential think time, then sends a request of
    floor(exp(U(ln lo, ln hi))) distinct env ids drawn uniformly from all
    envs, with uniform actions.  Open loop: each actor sends at the times of
    a Poisson process of that mean gap whether or not its earlier requests
    were answered (the offered load then does not adapt to the server)."""

    def __init__(self, n_clients, num_envs, mean_wait_s=2e-3, size_lo=64, size_hi=4096, seed0=5000,
                 n_actions=18, open_loop=False):
        self.n, self.num_envs = n_clients, num_envs
        self.open_loop = open_loop
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

    def mean_size(self):
        """Expected request size: E floor(exp U(ln lo, ln hi))."""
        ks = np.arange(self.lo, self.hi + 1, dtype=np.float64)
        p = (np.log(np.minimum(ks + 1, self.hi)) - np.log(ks)) / (np.log(self.hi) - np.log(self.lo))
        return float((ks * p).sum())

    def due(self, now):
        out = []
        for c in range(self.n):
            while (self.open_loop or not self.outstanding[c]) and self.next_send[c] <= now:
                g = self.rngs[c]
                k = self.size(c)
                ids = g.choice(self.num_envs, size=k, replace=False).astype(np.int32)
                act = g.integers(0, self.n_actions, k, dtype=np.uint8)
                out.append(Request(c, ids, act, self.next_send[c]))
                self.outstanding[c] = True
                if not self.open_loop:
                    break
                self.next_send[c] += g.exponential(self.mean_wait)
        return out

    def responded(self, c, now):
        self.outstanding[c] = False
        if not self.open_loop:
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
    backlog = 0
    if actors.open_loop:
        # an overloaded open loop never catches up: finish what is on the
        # device, count the rest as backlog and drop it
        backlog = int(sum(r.unsched for r in server.pending))
        server.pending = collections.deque()
    server.drain()
    t1 = clock()
    server.on_result = user_cb
    lat = np.array(lat)
    return {
        "seconds": t1 - t0,
        "requests": int(lat.size),
        "backlog_env_steps": backlog,
        "env_steps": int(server.env_steps - steps0),
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
        "mean_batch": float(np.mean(server.batch_sizes)) if server.batch_sizes else 0.0,
        "batches": server.batches,
    }
