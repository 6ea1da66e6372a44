"""Request loop of the env server, on the CPU with the oracle as its backend.

The loop logic (merging, the per-env ordering rule, capacity, several
pipelines in flight) does not depend on the device, so it is checked here
against solo runs of every request: each served result equals the result of
the same request run alone, one request at a time in arrival order.
"""
import numpy as np
import pytest

import oracle
from paper_1907_08467_amd.inputs.palette import GRAY
from paper_1907_08467_amd.inputs.romgen import RomSpec, generate
from paper_1907_08467_amd.serve import ActorPool, EnvServer, Request, slots_for_budget


class OracleBackend:
    """Batches run on the oracle when launched; a batch reports finished
    only after `latency` polls, so several pipelines are in flight at once."""

    def __init__(self, o, pipelines, latency):
        self.o, self.pipelines, self.latency = o, pipelines, latency
        self.res = [None] * pipelines
        self.age = [0] * pipelines
        self.max_inflight = 0

    def launch(self, p, ids, actions):
        obs, rew, done, _ = self.o.step(actions, env_ids=ids)
        self.res[p] = (obs, rew, done)
        self.age[p] = 0
        self.max_inflight = max(self.max_inflight, sum(r is not None for r in self.res))

    def finished(self, p):
        if self.res[p] is None:
            return False
        self.age[p] += 1
        return self.age[p] > self.latency

    def alloc(self, k):
        return np.zeros((k, 84, 84), np.uint8), np.zeros(k, np.int32), np.zeros(k, np.uint8)

    def scatter(self, out, pos, p, lo, hi):
        for dst, src in zip(out, self.res[p]):
            dst[pos] = src[lo:hi]

    def release(self, p):
        self.res[p] = None


def roms():
    return [(r.data, r.scheme) for r in (generate(RomSpec(4000, "4k", True)), generate(RomSpec(4001, "f8", True)))]


def make_oracle(n, seed=9):
    o = oracle.Oracle(n, GRAY, frameskip=4, render_mode=1, seed=seed, sticky_threshold=0x40000000)
    o.load_roms(roms())
    o.assign(np.arange(n, dtype=np.uint16) % 2)
    return o


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4
        return self.t


@pytest.mark.parametrize("pipelines,latency,cap", [(1, 0, 64), (3, 2, 40), (2, 5, 17)])
def test_served_equals_solo(pipelines, latency, cap):
    n_envs = 48
    backend = OracleBackend(make_oracle(n_envs), pipelines, latency)
    clock = FakeClock()
    actors = ActorPool(6, n_envs, mean_wait_s=2e-4, size_lo=2, size_hi=16, seed0=77)
    served = {}

    def keep(req, obs, rew, done):
        served[req.seq] = (req, obs.copy(), rew.copy(), done.copy())
        actors.responded(req.client, req.t_done)

    server = EnvServer(backend, max_batch=cap, num_envs=n_envs, on_result=keep, clock=clock)
    actors.start(clock())
    while server.completed < 120:
        for r in actors.due(clock()):
            server.submit(r)
        server.poll()
    server.drain()
    assert server.deferred > 0, "no env-step ever waited for an earlier step of its env"
    if pipelines > 1 and latency > 0:
        assert backend.max_inflight > 1
    assert max(server.batch_sizes) <= cap
    # solo: every request alone, in arrival order, on a fresh oracle
    solo = make_oracle(n_envs)
    for seq in sorted(served):
        req, obs, rew, done = served[seq]
        o_obs, o_rew, o_done, _ = solo.step(req.actions, env_ids=req.ids)
        assert np.array_equal(o_done, done), f"request {seq}: done"
        assert np.array_equal(o_rew, rew), f"request {seq}: reward"
        assert np.array_equal(o_obs, obs), f"request {seq}: obs"
    for e in range(n_envs):
        assert np.array_equal(solo.get_state(e), backend.o.get_state(e)), f"env {e}"


def test_submit_checks():
    backend = OracleBackend(make_oracle(8), 1, 0)
    server = EnvServer(backend, max_batch=4, num_envs=8)
    with pytest.raises(ValueError):
        server.submit(Request(0, np.array([1, 8], np.int32), np.zeros(2, np.uint8), 0.0))
    with pytest.raises(ValueError):
        server.submit(Request(0, np.array([1, 1], np.int32), np.zeros(2, np.uint8), 0.0))
    with pytest.raises(ValueError):
        server.submit(Request(0, np.zeros(0, np.int32), np.zeros(0, np.uint8), 0.0))


def test_requests_larger_than_a_batch_are_split():
    """A request of more envs than one batch holds runs over several batches."""
    backend = OracleBackend(make_oracle(16), 2, 1)
    got = {}
    server = EnvServer(backend, max_batch=5, num_envs=16, on_result=lambda r, o, rw, d: got.update({r.seq: rw}))
    rng = np.random.default_rng(3)
    reqs = [Request(0, rng.permutation(16)[:12].astype(np.int32), rng.integers(0, 18, 12).astype(np.uint8), 0.0)
            for _ in range(3)]
    for r in reqs:
        server.submit(r)
    server.drain()
    assert max(server.batch_sizes) <= 5 and len(got) == 3
    solo = make_oracle(16)
    for r in reqs:
        _, rew, _, _ = solo.step(r.actions, env_ids=r.ids)
        assert np.array_equal(rew, got[r.seq])


def test_budget_sizing():
    # 16 GiB, 131072 resident envs, 16 ROMs, last-two render, 2 pipelines
    m = slots_for_budget(16 << 30, 131072, 16, 2, 2)
    assert 100_000 < m <= 131072
    with pytest.raises(ValueError):
        slots_for_budget(1 << 20, 131072, 16, 2, 1)


def test_open_loop_actors_send_without_waiting():
    """Open loop: an actor's Poisson send times do not wait for its answers,
    so a client can have several requests outstanding; the arrival times are
    the Poisson times themselves."""
    a = ActorPool(3, 100, mean_wait_s=1e-3, size_lo=2, size_hi=8, seed0=9, open_loop=True)
    a.start(0.0)
    reqs = a.due(0.05)                       # 50 ms: about 50 requests per actor, none answered
    per = np.bincount([r.client for r in reqs], minlength=3)
    assert (per > 20).all() and (per < 100).all()
    for c in range(3):
        t = [r.t_arrival for r in reqs if r.client == c]
        assert all(x < y for x, y in zip(t, t[1:])) and t[-1] <= 0.05
    closed = ActorPool(3, 100, mean_wait_s=1e-3, size_lo=2, size_hi=8, seed0=9)
    closed.start(0.0)
    assert len(closed.due(0.05)) == 3        # closed loop: one outstanding request per actor
    assert abs(a.mean_size() - np.mean([np.floor(np.exp(u)) for u in
                                        np.random.default_rng(1).uniform(np.log(2), np.log(8), 100000)])) < 0.05


def test_open_loop_overload_reports_backlog():
    """Offered load far above what the backend serves: the run ends with a
    backlog, which is dropped (not drained) and reported; the requests before
    the first dropped one (all of them completed) equal their solo runs in
    arrival order."""
    from paper_1907_08467_amd.serve import run_served
    n_envs = 32
    backend = OracleBackend(make_oracle(n_envs), 2, 3)
    clock = FakeClock()
    actors = ActorPool(8, n_envs, mean_wait_s=1e-4, size_lo=4, size_hi=16, seed0=21, open_loop=True)
    served = {}
    server = EnvServer(backend, max_batch=8, num_envs=n_envs, clock=clock,
                       on_result=lambda r, o, rw, d: served.update({r.seq: (r, o.copy(), rw.copy(), d.copy())}))
    st = run_served(server, actors, seconds=0.02, clock=clock)
    assert st["backlog_env_steps"] > 0 and st["requests"] == len(served) > 0
    assert server.idle()
    first_dropped = min(set(range(server.seq)) - set(served))
    assert first_dropped > 0
    solo = make_oracle(n_envs)
    for seq in range(first_dropped):
        req, obs, rew, done = served[seq]
        o_obs, o_rew, o_done, _ = solo.step(req.actions, env_ids=req.ids)
        assert np.array_equal(o_rew, rew) and np.array_equal(o_obs, obs), f"request {seq}"
