"""Serving scheduler and batch planning on the CPU (fake executor, simulated
clock): admission by memory budget, arrival order, iteration-level batching,
latency accounting, and the split of a batch's amplicons by request."""
import numpy as np
import pytest

from paper_2511_00170_amd import serve, synth
from paper_2511_00170_amd.synth import PairSpec, Request


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


def _fake_executor(clock, log, per_req_s=0.01, fixed_s=0.005):
    def run(batch):
        log.append([r.rid for r in batch])
        clock.t += fixed_s + per_req_s * len(batch)
        return {r.rid: serve.RequestResult(r.rid, np.zeros(0), np.zeros(0), np.zeros((0, 2)), np.zeros(0, np.uint8),
                                           b"", np.zeros(1, np.uint64)) for r in batch}
    return run


def _reqs(arrivals, cost=1):
    return [Request(i, t, [0], np.arange(3, dtype=np.uint32), 0, 50.0) for i, t in enumerate(arrivals)]


def test_all_requests_complete_once_in_arrival_order():
    clock, log = SimClock(), []
    sch = serve.Scheduler(_fake_executor(clock, log), cost=lambda r: 1, budget_bytes=4, max_requests=64,
                          clock=clock, sleep_until=clock.sleep_until)
    reqs = _reqs(np.cumsum(np.full(20, 0.003)))
    out = sch.run(reqs, t0=0.0)
    assert sorted(out) == list(range(20))
    flat = [rid for b in log for rid in b]
    assert flat == list(range(20))                 # FIFO, each once
    assert all(len(b) <= 4 for b in log)           # budget of 4 units
    for r in reqs:
        res = out[r.rid]
        assert res.arrival_s == pytest.approx(r.arrival_s)
        assert res.done_s >= res.arrival_s


def test_requests_arriving_during_a_pass_join_the_next_batch():
    clock, log = SimClock(), []
    sch = serve.Scheduler(_fake_executor(clock, log, per_req_s=0.0, fixed_s=0.1), cost=lambda r: 1,
                          budget_bytes=100, clock=clock, sleep_until=clock.sleep_until)
    # r0 at 0; r1, r2 arrive while r0's pass (0.1 s) runs; r3 after an idle gap
    out = sch.run(_reqs([0.0, 0.05, 0.06, 0.5]), t0=0.0)
    assert log == [[0], [1, 2], [3]]
    assert out[0].latency_s == pytest.approx(0.1)
    assert out[1].latency_s == pytest.approx(0.2 - 0.05)
    assert out[3].latency_s == pytest.approx(0.1)


def test_oversized_request_runs_alone_and_max_requests_caps_batches():
    clock, log = SimClock(), []
    costs = {0: 1, 1: 50, 2: 1, 3: 1, 4: 1}
    sch = serve.Scheduler(_fake_executor(clock, log), cost=lambda r: costs[r.rid], budget_bytes=10, max_requests=2,
                          clock=clock, sleep_until=clock.sleep_until)
    sch.run(_reqs([0.0] * 5), t0=0.0)
    assert log == [[0], [1], [2, 3], [4]]


def test_plan_batch_masks_and_slots():
    pool = [PairSpec("ACGTACGTAC", "GGGCCCAAAT", k=3, clamp=3) for _ in range(5)]
    reqs = [Request(10, 0.0, [1, 3], np.array([0, 2, 4], np.uint32), 1, 45.0),
            Request(11, 0.0, [3], np.array([2, 5], np.uint32), 0, 55.0)]
    p = serve.plan_batch(reqs, pool, n_seqs=8)
    assert p.seq_list.tolist() == [0, 2, 4, 5]
    assert p.pair_mask.tolist() == [0b01010, 0b01010, 0b01010, 0b01000]
    assert p.seq_req.tolist() == [1, 0, 3, 0, 1, 2, 0, 0]
    assert p.vpair[0, 1] == 0 and p.vpair[0, 3] == 1 and p.vpair[1, 3] == 2
    assert (p.vpair[0, [0, 2, 4]] == 0xFFFF).all() and (p.vpair[1, [0, 1, 2, 4]] == 0xFFFF).all()
    assert p.kmax.tolist() == [1, 0]
    assert [s.k for s in p.slots] == [1, 1, 0]
    assert p.slot_req.tolist() == [0, 0, 1] and p.slot_thr.tolist() == [45.0, 45.0, 55.0]


def test_request_above_the_pool_k_is_refused():
    """The pool is scanned once at its k; a request asking for more would lose
    hits silently, so planning refuses it (a request at the pool's k plans)."""
    pool = [PairSpec("ACGTACGTAC", "GGGCCCAAAT", k=3, clamp=3) for _ in range(2)]
    ok = Request(1, 0.0, [0], np.array([0], np.uint32), 3, 45.0)
    over = Request(2, 0.0, [1], np.array([1], np.uint32), 4, 45.0)
    assert serve.plan_batch([ok], pool, n_seqs=2, pool_k=3).kmax.tolist() == [3]
    with pytest.raises(ValueError, match="k=4"):
        serve.plan_batch([ok, over], pool, n_seqs=2, pool_k=3)
    with pytest.raises(ValueError):
        serve.check_request_k(over, 3)


def test_split_results_by_request():
    from paper_2511_00170_amd import ah
    pool = [PairSpec("ACGTACGTAC", "GGGCCCAAAT", k=3, clamp=3) for _ in range(3)]
    reqs = [Request(7, 0.0, [0, 2], np.array([0, 1], np.uint32), 1, 45.0),
            Request(8, 0.0, [2], np.array([1], np.uint32), 0, 55.0)]
    p = serve.plan_batch(reqs, pool, n_seqs=2)
    a = np.zeros(4, ah.AMP_DTYPE)
    a["seq"] = [0, 1, 1, 1]
    a["pair"] = [1, 0, 1, 2]          # slots: (r0,q0)=0, (r0,q2)=1, (r1,q2)=2
    a["start"] = [5, 6, 7, 8]
    tm = np.array([50.0, 51.0, 52.0, 53.0])
    site = np.stack([tm, tm + 1], 1)
    pas = np.array([1, 0, 1, 1], np.uint8)
    seq = b"AAACCGGGG"
    off = np.array([0, 3, 3, 5, 9], np.uint64)
    out = serve.split_results(p, a, tm, site, pas, seq, off, [0, 1, 0])
    r7, r8 = out[7], out[8]
    assert r7.amps["pair"].tolist() == [1, 0, 1] and r7.amps["start"].tolist() == [5, 6, 7]
    assert r7.seq == b"AAACC" and r7.seq_off.tolist() == [0, 3, 3, 5]
    assert r8.amps["pair"].tolist() == [0] and r8.seq == b"GGGG" and r8.tm.tolist() == [53.0]


@pytest.mark.parametrize("n", [0, 1, 5, (8 << 20) - 1, 8 << 20, (8 << 20) + 1, 3 * (8 << 20) + 12345])
def test_parallel_copy_is_a_copy(n):
    src = np.random.default_rng(n).integers(0, 256, n, dtype=np.uint8)
    dst = serve.parallel_copy(src)
    assert dst.dtype == np.uint8 and dst.shape == src.shape and np.array_equal(dst, src)
    if n:
        assert not np.shares_memory(dst, src)


def test_request_cost_grows_with_subset_and_pairs():
    wl = synth.gen_config(5, n_seqs=50, len_scale=0.01)
    lens = wl.lengths.astype(np.int64)
    small = Request(0, 0.0, [0], np.arange(5, dtype=np.uint32), 0, 50.0)
    big = Request(1, 0.0, [0, 1, 2], np.arange(50, dtype=np.uint32), 0, 50.0)
    assert serve.request_bytes(small, wl.pairs, lens, 3) < serve.request_bytes(big, wl.pairs, lens, 3)


class FakeAsyncExecutor:
    """A GPU that runs launched batches one after another (FIFO), each taking
    fixed_s + per_req_s x requests, with n_slots batches in flight at most."""

    def __init__(self, clock, n_slots=2, per_req_s=0.01, fixed_s=0.02):
        self.clock, self.n_slots, self.per, self.fixed = clock, n_slots, per_req_s, fixed_s
        self.busy_until = 0.0
        self.inflight = 0
        self.log = []

    def free_slots(self):
        return self.n_slots - self.inflight

    def launch(self, batch):
        assert self.inflight < self.n_slots
        self.inflight += 1
        start = max(self.clock.t, self.busy_until)
        self.busy_until = start + self.fixed + self.per * len(batch)
        self.log.append(([r.rid for r in batch], self.clock.t, start, self.busy_until))
        return (batch, self.busy_until)

    def ready(self, tk):
        return self.clock.t >= tk[1]

    def eta(self, tk):
        return tk[1]

    def collect(self, tk):
        batch, done = tk
        self.clock.t = max(self.clock.t, done)
        self.inflight -= 1
        return {r.rid: serve.RequestResult(r.rid, np.zeros(0), np.zeros(0), np.zeros((0, 2)), np.zeros(0, np.uint8),
                                           b"", np.zeros(1, np.uint64)) for r in batch}


def test_async_batches_overlap_and_new_arrivals_launch_while_others_run():
    clock = SimClock()
    exe = FakeAsyncExecutor(clock, n_slots=2, per_req_s=0.0, fixed_s=0.1)
    sch = serve.Scheduler(exe, cost=lambda r: 1, budget_bytes=100, clock=clock, sleep_until=clock.sleep_until)
    # r0 at 0 starts batch A; r1 arrives during A and is launched at once in the
    # second slot (it queues on the device behind A); r2 and r3 arrive while
    # both slots are busy and are launched together when A's slot frees up
    out = sch.run(_reqs([0.0, 0.03, 0.05, 0.06]), t0=0.0)
    launches = [(ids, round(t, 3)) for ids, t, _, _ in exe.log]
    assert launches == [([0], 0.0), ([1], 0.03), ([2, 3], 0.1)]
    assert out[0].done_s == pytest.approx(0.1)
    assert out[1].done_s == pytest.approx(0.2)
    assert out[2].done_s == pytest.approx(0.3) and out[3].done_s == pytest.approx(0.3)
    assert sorted(out) == [0, 1, 2, 3]


def test_async_scheduler_serves_everything_once_under_load():
    clock = SimClock()
    exe = FakeAsyncExecutor(clock, n_slots=3, per_req_s=0.002, fixed_s=0.01)
    sch = serve.Scheduler(exe, cost=lambda r: 1, budget_bytes=8, clock=clock, sleep_until=clock.sleep_until)
    rng = np.random.default_rng(0)
    reqs = _reqs(np.cumsum(rng.exponential(0.004, 300)))
    out = sch.run(reqs, t0=0.0)
    assert sorted(out) == list(range(300))
    flat = [rid for ids, _, _, _ in exe.log for rid in ids]
    assert flat == list(range(300))                       # arrival order, each once
    assert all(len(ids) <= 8 for ids, _, _, _ in exe.log)  # budget
    assert exe.inflight == 0
    for r in reqs:
        assert out[r.rid].done_s >= r.arrival_s
