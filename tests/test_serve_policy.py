"""The serving form's admission policy (csrc/serve_policy.h, what
rlu_serve.cpp's scheduler thread runs under its lock) as a pure host state
machine, driven on the CPU through tests/serve_policy_driver.cpp: fixed
scenarios for each rule, then an event simulation with a simulated clock
(seeded arrivals, two streams, service times, releases) that checks the
invariants at every event."""
import heapq
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver_bin(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp("policy") / "serve_policy_driver")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1310_7202_amd", "csrc"),
                    os.path.join(ROOT, "tests", "serve_policy_driver.cpp"), "-o", out],
                   check=True, capture_output=True, text=True)
    return out


class Policy:
    def __init__(self, exe, budget, max_inflight=0, max_queue=0):
        self.p = subprocess.Popen([exe], stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)
        assert self._cmd(f"new {budget} {max_inflight} {max_queue}") == "ok"

    def _cmd(self, line):
        self.p.stdin.write(line + "\n")
        self.p.stdin.flush()
        return self.p.stdout.readline().strip()

    def offer(self, ws, out):
        return self._cmd(f"offer {ws} {out}")

    def push(self, ticket, ws, out, key=1, solo=False):
        assert self._cmd(f"push {ticket} {ws} {out} {key} {int(solo)}") == "ok"

    def admit(self, max_batch=256):
        r = self._cmd(f"admit {max_batch}").split()
        assert r[0] == "batch"
        return [int(t) for t in r[1:]]

    def complete(self, ws):
        assert self._cmd(f"complete {ws}") == "ok"

    def release(self, out):
        assert self._cmd(f"release {out}") == "ok"

    def stats(self):
        r = self._cmd("stats").split()
        return int(r[1]), int(r[2]), int(r[3])

    def close(self):
        self.p.stdin.close()
        self.p.wait(timeout=10)


@pytest.fixture
def policy(driver_bin):
    made = []

    def make(budget, max_inflight=0, max_queue=0):
        p = Policy(driver_bin, budget, max_inflight, max_queue)
        made.append(p)
        return p
    yield make
    for p in made:
        p.close()


def test_offer_refuses_too_large_and_a_full_queue(policy):
    p = policy(100, 0, 2)
    assert p.offer(90, 10) == "accept"
    assert p.offer(91, 10) == "too_large"
    p.push(1, 10, 1)
    p.push(2, 10, 1)
    assert p.offer(1, 1) == "queue_full"
    assert p.admit() == [1, 2]
    assert p.offer(1, 1) == "accept"


def test_strict_fifo_nothing_overtakes_a_head_that_does_not_fit(policy):
    p = policy(100)
    p.push(1, 50, 10)
    p.push(2, 50, 10)
    p.push(3, 5, 1)          # would fit, but stays behind 2
    assert p.admit() == [1]
    assert p.admit() == []
    assert p.stats() == (60, 1, 2)
    p.complete(50)           # 1's workspace returns; its outputs stay charged
    assert p.stats() == (10, 0, 2)
    assert p.admit() == [2, 3]
    assert p.stats() == (10 + 60 + 6, 2, 0)


def test_a_batch_has_one_key(policy):
    p = policy(1000)
    for t, key in ((1, 1), (2, 1), (3, 2), (4, 1)):
        p.push(t, 10, 1, key=key)
    assert p.admit() == [1, 2]
    assert p.admit() == [3]
    assert p.admit() == [4]


def test_solo_requests_run_alone(policy):
    p = policy(1000)
    p.push(1, 10, 1)
    p.push(2, 10, 1, solo=True)
    p.push(3, 10, 1)
    p.push(4, 10, 1)
    assert p.admit() == [1]
    assert p.admit() == [2]
    assert p.admit() == [3, 4]


def test_in_flight_limit_and_batch_size(policy):
    p = policy(1000, max_inflight=3)
    for t in range(1, 7):
        p.push(t, 10, 1)
    assert p.admit(max_batch=2) == [1, 2]
    assert p.admit(max_batch=2) == [3]
    assert p.admit(max_batch=2) == []
    p.complete(10)
    p.complete(10)
    assert p.admit(max_batch=8) == [4, 5]


def test_release_returns_the_output_share(policy):
    p = policy(100)
    p.push(1, 40, 31)
    p.push(2, 40, 31)
    assert p.admit() == [1]
    p.complete(40)
    assert p.admit() == []   # 31 of 1's outputs + 71 of 2's would exceed 100
    p.release(31)
    assert p.admit() == [2]
    p.complete(40)
    p.release(31)
    assert p.stats() == (0, 0, 0)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_simulated_stream_keeps_every_invariant(policy, seed):
    """Seeded arrivals on a simulated clock, two streams, service time
    growing with the batch, outputs released a little after completion;
    at every event: the charged total within the budget, admission in
    ticket order, one key per batch and solo requests alone, and at the end
    every request done and every byte returned."""
    rng = np.random.default_rng(seed)
    budget, n, streams = 10_000, 300, 2
    p = policy(budget, max_inflight=40, max_queue=64)
    reqs = {}
    t, ticket = 0.0, 0
    events = []   # (time, order, kind, payload)
    order = 0
    for _ in range(n):
        t += rng.exponential(1.0)
        ws = int(rng.integers(50, 600))
        out = int(rng.integers(10, 200))
        key = int(rng.integers(1, 3))
        solo = bool(rng.random() < 0.05)
        heapq.heappush(events, (t, order, "arrive", (ws, out, key, solo)))
        order += 1
    free = list(range(streams))
    admitted, refused, done, released = [], 0, 0, 0
    while events:
        now, _, kind, pl = heapq.heappop(events)
        if kind == "arrive":
            ws, out, key, solo = pl
            v = p.offer(ws, out)
            if v == "accept":
                ticket += 1
                reqs[ticket] = (ws, out, key, solo)
                p.push(ticket, ws, out, key, solo)
            else:
                assert v == "queue_full"   # nothing here exceeds the budget alone
                refused += 1
        elif kind == "done":
            s, batch = pl
            for tk in batch:
                p.complete(reqs[tk][0])
                heapq.heappush(events, (now + 0.5, order, "release", tk))
                order += 1
                done += 1
            free.append(s)
        else:
            p.release(reqs[pl][1])
            released += 1
        while free:
            batch = p.admit(256)
            if not batch:
                break
            keys = {reqs[tk][2] for tk in batch}
            assert len(keys) == 1
            if any(reqs[tk][3] for tk in batch):
                assert len(batch) == 1
            admitted.extend(batch)
            s = free.pop()
            heapq.heappush(events, (now + 0.2 + 0.02 * len(batch), order, "done", (s, batch)))
            order += 1
        used, inflight, queued = p.stats()
        assert 0 <= used <= budget
        assert 0 <= inflight <= 40 and queued <= 64
    assert admitted == sorted(admitted) == list(range(1, ticket + 1))
    assert done == released == ticket and ticket + refused == n
    assert p.stats() == (0, 0, 0)
