"""Continuous-batching primer search over a device-resident genome store.

A request names pool pairs, a subset of the stored sequences, its own
mismatch bound k and its own Tm threshold.  The engine runs one GPU pass per
batch of requests:

  scan (masked)  every pool pair that some request of the batch asks for on a
                 sequence, scanned once per (sequence, pair) at the pool's
                 largest k -- a tile is loaded once for all requests;
  route          each hit copied to every request that asked for its
                 (sequence, pair) and whose k admits its mismatch count, with
                 the request's own slot in a per-batch "virtual" primer set;
  pair, Tm, extract  over all routed hits at once, with per-slot windows and
                 per-slot Tm thresholds;

then splits the amplicons by slot.  Up to ``n_slots`` batches are in flight
at once, each with its own device buffers and stream: whenever a slot is
free, the requests that have arrived are admitted in arrival order while the
batch's estimated device memory stays within the budget, and that batch runs
alongside the ones already on the GPU (its scan starts as the earlier scan's
workgroups retire; copies and host work of one batch overlap another's
kernels).  A request's result does not depend on what it was batched with:
routing applies exactly its (sequence, pair, k) selection to hits that do not
depend on the batch, and pairing, Tm and extraction are per (sequence, slot).

The scheduler is separate from the GPU executor so that its policy can be
tested without a GPU.
"""
from __future__ import annotations

import os
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from .synth import PairSpec, Request, TmSpec

MAX_REQ_PER_BATCH = 64      # request bitmap of the routing kernel
MAX_POOL = 64               # pair bitmap of the masked scan


# --------------------------------------------------------------------------
# Results
# --------------------------------------------------------------------------
class RequestResult:
    """One request's amplicons (pair = index into the request's pair list),
    their Tm, pass flags and sequences.  ``seq`` may be given as bytes or as
    (batch buffer, per-amplicon start offsets): the per-request byte string is
    then cut out of the batch's host buffer when first read."""

    def __init__(self, rid: int, amps: np.ndarray, tm: np.ndarray, tm_site: np.ndarray, passed: np.ndarray, seq,
                 seq_off: np.ndarray):
        self.rid, self.amps, self.tm, self.tm_site, self.passed = rid, amps, tm, tm_site, passed
        self._seq = seq
        self.seq_off = seq_off
        self.arrival_s = 0.0
        self.done_s = 0.0
        self.batch = -1

    @property
    def seq(self) -> bytes:
        if isinstance(self._seq, tuple):
            buf, starts = self._seq
            lens = np.diff(self.seq_off.astype(np.int64))
            tot = int(lens.sum())
            if tot:
                pos = np.repeat(starts - (np.cumsum(lens) - lens), lens) + np.arange(tot, dtype=np.int64)
                self._seq = buf[pos].tobytes()
            else:
                self._seq = b""
        return self._seq

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def results_equal(a: RequestResult, b: RequestResult) -> bool:
    return (np.array_equal(a.amps, b.amps) and np.array_equal(a.tm, b.tm) and np.array_equal(a.tm_site, b.tm_site)
            and np.array_equal(a.passed, b.passed) and a.seq == b.seq and np.array_equal(a.seq_off, b.seq_off))


# --------------------------------------------------------------------------
# Cost model (host): expected device bytes of a request
# --------------------------------------------------------------------------
def request_bytes(req: Request, pool: Sequence[PairSpec], seq_lens: np.ndarray, pool_k: int) -> int:
    """Expected device bytes a request adds to a batch: its hits at the pool's
    k (12 B, twice: scanned and routed), sort keys (16 B per hit), amplicons
    (16 + 8 + 16 + 1 B) and amplicon sequences (about one window each)."""
    from .batch import expected_hits_per_base
    bases = float(seq_lens[req.seqs].sum())
    rate = sum(expected_hits_per_base(_with_k(pool[q], pool_k)) for q in req.pairs)
    hits = rate * bases + 64 * len(req.pairs)
    amps = 0.1 * hits + 64
    return int(hits * (24 + 16) + amps * (41 + 1200))


def _with_k(p: PairSpec, k: int) -> PairSpec:
    return PairSpec(p.fwd, p.rev, k=k, clamp=p.clamp, min_len=p.min_len, max_len=p.max_len)


# --------------------------------------------------------------------------
# Scheduler (no GPU)
# --------------------------------------------------------------------------
@dataclass
class SchedStats:
    batches: int = 0
    batch_sizes: List[int] = field(default_factory=list)
    busy_s: float = 0.0


class Scheduler:
    """Iteration-level batching with batches in flight concurrently.

    The executor either runs a batch synchronously (``executor(batch) ->
    {rid: RequestResult}``) or, when it has ``launch/ready/collect`` and
    ``free_slots``, asynchronously: a batch is launched whenever a slot (a
    set of device buffers and a stream) is free and requests are waiting, so
    a batch formed from requests that arrived while others were on the GPU
    runs alongside them.  ``clock()`` gives the current time and
    ``sleep_until(t)`` waits (both replaceable for simulated time)."""

    def __init__(self, executor, cost: Callable[[Request], int], budget_bytes: int,
                 max_requests: int = MAX_REQ_PER_BATCH, clock: Callable[[], float] = time.perf_counter,
                 sleep_until: Optional[Callable[[float], None]] = None, poll_s: float = 2e-4):
        self.executor = executor
        self.cost = cost
        self.budget = budget_bytes
        self.max_requests = max_requests
        self.clock = clock
        self.sleep_until = sleep_until or (lambda t: time.sleep(max(0.0, t - self.clock())))
        self.poll_s = poll_s
        self.stats = SchedStats()

    def admit(self, queue: List[Request]) -> List[Request]:
        """Take requests in arrival order while the batch fits the budget; the
        first request is always taken (a request larger than the budget runs
        alone)."""
        batch, used = [], 0
        while queue and len(batch) < self.max_requests:
            c = self.cost(queue[0])
            if batch and used + c > self.budget:
                break
            batch.append(queue.pop(0))
            used += c
        return batch

    def _finish(self, batch, res, t0, ts, te, out):
        self.stats.batches += 1
        self.stats.batch_sizes.append(len(batch))
        self.stats.busy_s += te - ts
        for r in batch:
            rr = res[r.rid]
            rr.arrival_s = t0 + r.arrival_s
            rr.done_s = te
            rr.batch = self.stats.batches - 1
            out[r.rid] = rr

    def run(self, requests: Sequence[Request], t0: Optional[float] = None) -> Dict[int, RequestResult]:
        """Serve ``requests`` (arrival_s relative to t0) to completion."""
        pending = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        t0 = self.clock() if t0 is None else t0
        queue: List[Request] = []
        out: Dict[int, RequestResult] = {}
        inflight = []  # (ticket, batch, launch time), oldest first
        asyn = hasattr(self.executor, "launch")
        i = 0
        while i < len(pending) or queue or inflight:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival_s <= now:
                queue.append(pending[i])
                i += 1
            # completed batches first (their slots free up)
            if inflight and self.executor.ready(inflight[0][0]):
                tk, batch, ts = inflight.pop(0)
                res = self.executor.collect(tk)
                self._finish(batch, res, t0, ts, self.clock(), out)
                continue
            if queue and (not asyn or self.executor.free_slots() > 0):
                batch = self.admit(queue)
                ts = self.clock()
                if asyn:
                    inflight.append((self.executor.launch(batch), batch, ts))
                else:
                    res = self.executor(batch)
                    self._finish(batch, res, t0, ts, self.clock(), out)
                continue
            if inflight:
                if queue or i >= len(pending):
                    # no slot for the waiting requests, or nothing more will
                    # arrive: wait for the oldest batch
                    tk, batch, ts = inflight.pop(0)
                    res = self.executor.collect(tk)
                    self._finish(batch, res, t0, ts, self.clock(), out)
                else:
                    # a slot is free: wake up for the next arrival or a completion
                    nxt = t0 + pending[i].arrival_s
                    eta = self.executor.eta(inflight[0][0]) if hasattr(self.executor, "eta") else None
                    wake = min(nxt, self.clock() + self.poll_s) if eta is None else min(nxt, eta)
                    self.sleep_until(wake)
                continue
            self.sleep_until(t0 + pending[i].arrival_s)
        return out


def latency_summary(results: Dict[int, RequestResult], skip: int = 0) -> dict:
    rs = sorted(results.values(), key=lambda r: r.rid)[skip:]
    lat = np.array([r.latency_s for r in rs]) * 1e3
    if not len(lat):
        return {"n": 0}
    return {"n": len(lat), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
            "max_ms": round(float(lat.max()), 3)}


# --------------------------------------------------------------------------
# Batch plan (host)
# --------------------------------------------------------------------------
@dataclass
class BatchPlan:
    reqs: List[Request]
    seq_list: np.ndarray        # sorted union of the requests' sequences (uint32)
    pair_mask: np.ndarray       # per listed sequence: pool pairs to scan (uint64)
    seq_req: np.ndarray         # per store sequence: requests that want it (uint64)
    vpair: np.ndarray           # [n_req, n_pool] slot of (request, pool pair) or 0xFFFF
    kmax: np.ndarray            # [n_req] uint8
    slots: List[PairSpec]       # the virtual primer set
    slot_req: np.ndarray        # slot -> request index
    slot_thr: np.ndarray        # slot -> Tm threshold


def check_request_k(req: Request, pool_k: int) -> None:
    """The pool is scanned once at pool_k; routing keeps a hit for a request
    when its mismatch count is at most the request's k.  A request asking for
    more than pool_k would silently lose the hits with pool_k < mm <= k, so it
    is refused."""
    if req.k > pool_k:
        raise ValueError("request %d asks for k=%d, but the pool is scanned at k=%d" % (req.rid, req.k, pool_k))


def plan_batch(reqs: Sequence[Request], pool: Sequence[PairSpec], n_seqs: int,
               pool_k: Optional[int] = None) -> BatchPlan:
    n_pool = len(pool)
    assert len(reqs) <= MAX_REQ_PER_BATCH and n_pool <= MAX_POOL
    if pool_k is not None:
        for rq in reqs:
            check_request_k(rq, pool_k)
    seq_req = np.zeros(n_seqs, np.uint64)
    seq_pairs = np.zeros(n_seqs, np.uint64)
    vpair = np.full((len(reqs), n_pool), 0xFFFF, np.uint16)
    kmax = np.zeros(len(reqs), np.uint8)
    slots, slot_req, slot_thr = [], [], []
    for r, rq in enumerate(reqs):
        bit = np.uint64(1) << np.uint64(r)
        pm = np.uint64(0)
        for q in rq.pairs:
            pm |= np.uint64(1) << np.uint64(q)
            vpair[r, q] = len(slots)
            slots.append(_with_k(pool[q], rq.k))
            slot_req.append(r)
            slot_thr.append(rq.threshold_C)
        kmax[r] = rq.k
        seq_req[rq.seqs] |= bit
        seq_pairs[rq.seqs] |= pm
    seq_list = np.nonzero(seq_req)[0].astype(np.uint32)
    return BatchPlan(list(reqs), seq_list, seq_pairs[seq_list], seq_req, vpair, kmax, slots,
                     np.array(slot_req, np.int64), np.array(slot_thr, np.float64))


_COPY_LOCK = threading.Lock()
_COPY_POOL: Optional[ThreadPoolExecutor] = None
_COPY_CHUNK = 8 << 20


def _copy_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(8, n))


def parallel_copy(src: np.ndarray) -> np.ndarray:
    """A copy of a byte buffer, made by up to 8 host threads in 8 MB chunks.
    A batch at saturation returns 100-200 MB of amplicon bytes; one thread's
    copy of that out of the pinned staging buffer takes tens of
    milliseconds, and numpy releases the GIL while it copies."""
    global _COPY_POOL
    src = np.asarray(src, np.uint8).reshape(-1)
    dst = np.empty_like(src)
    n = len(src)
    parts = -(-n // _COPY_CHUNK)
    if parts <= 1:
        dst[:] = src
        return dst
    with _COPY_LOCK:
        if _COPY_POOL is None:
            _COPY_POOL = ThreadPoolExecutor(_copy_threads(), thread_name_prefix="ah-copy")
        pool = _COPY_POOL

    def one(i):
        a, b = i * _COPY_CHUNK, min(n, (i + 1) * _COPY_CHUNK)
        np.copyto(dst[a:b], src[a:b])

    for f in [pool.submit(one, i) for i in range(parts)]:
        f.result()
    return dst


def split_results(plan: BatchPlan, amps, tm, tm_site, passed, seq: bytes, seq_off: np.ndarray,
                  slot_pair_index: List[int]) -> Dict[int, RequestResult]:
    """Split a batch's amplicons (ordered by sequence, slot, site) by request.
    The batch's arrays are permuted once into request order (a stable radix
    sort on the 8-bit request index keeps each request's own order); every
    request's result holds slices of them and its byte ranges of one shared
    copy of the batch's amplicon bytes."""
    out = {}
    n_req = len(plan.reqs)
    assert n_req <= 256
    req_of = (plan.slot_req[amps["pair"].astype(np.int64)] if len(amps) else np.zeros(0, np.int64)).astype(np.uint8)
    spi = np.asarray(slot_pair_index, np.uint16)
    sb = np.frombuffer(seq, np.uint8) if isinstance(seq, (bytes, bytearray)) else np.asarray(seq, np.uint8)
    off = seq_off.astype(np.int64)
    buf = parallel_copy(sb)                             # the batch's bytes, shared by its requests
    order = np.argsort(req_of, kind="stable")          # amplicons grouped by request, order kept
    bounds = np.zeros(n_req + 1, np.int64)
    bounds[1:] = np.cumsum(np.bincount(req_of, minlength=n_req)[:n_req])
    a_all = amps[order]
    if len(a_all):
        a_all["pair"] = spi[a_all["pair"].astype(np.int64)]
    tms = np.ascontiguousarray(tm_site, np.float64).reshape(-1, 2)
    tm_all, pas_all = tm[order], passed[order]
    tms_all = tms.view(np.complex128).reshape(-1)[order].view(np.float64).reshape(-1, 2)   # row gather
    start_all = off[:-1][order]
    len_all = off[1:][order] - start_all
    for r, rq in enumerate(plan.reqs):
        lo, hi = int(bounds[r]), int(bounds[r + 1])
        so = np.zeros(hi - lo + 1, np.uint64)
        np.cumsum(len_all[lo:hi], out=so[1:])
        out[rq.rid] = RequestResult(rq.rid, a_all[lo:hi], tm_all[lo:hi], tms_all[lo:hi], pas_all[lo:hi],
                                    (buf, start_all[lo:hi]), so)
    return out


# --------------------------------------------------------------------------
# GPU executor
# --------------------------------------------------------------------------
class _Slot:
    """Device buffers, pinned staging and a stream for one batch in flight."""

    def __init__(self, torch, dev, n_seqs):
        self.torch, self.dev = torch, dev
        self.stream = torch.cuda.Stream()
        self.caps = dict(hits=1 << 20, routed=1 << 20, amps=1 << 16, seq=1 << 24)
        self.bufs = {}
        pin = dict(dtype=torch.uint8, pin_memory=True)
        self.h_tables = torch.empty(max(n_seqs, 1) * 20 + (MAX_REQ_PER_BATCH * (2 * MAX_POOL + 1)) +
                                    8 * MAX_REQ_PER_BATCH * MAX_POOL + 64, **pin)
        self.h_cnt = torch.zeros(8, dtype=torch.int64, pin_memory=True)
        self.h_out = None  # pinned landing buffer for a batch's results
        self.event = torch.cuda.Event()

    def buf(self, name, n, dtype):
        t = self.bufs.get(name)
        if t is None or t.numel() < n or t.dtype != dtype:
            t = self.torch.empty(max(n, 1), dtype=dtype, device=self.dev)
            self.bufs[name] = t
        return t


@dataclass
class Ticket:
    slot: "_Slot"
    plan: BatchPlan
    vps: object
    tables: dict


class GpuExecutor:
    """Runs batches on one GPU against a resident store and a pool primer set
    compiled once (hipRTC-specialised scan at the pool's largest k).  Up to
    ``n_slots`` batches are in flight at once, each on its own stream with its
    own buffers, so one batch's stages and copies overlap another's scan."""

    def __init__(self, store, pool: Sequence[PairSpec], tm: TmSpec, ex=None, orient_mask: int = 0xF,
                 pool_k: int = 3, jit: bool = True, n_slots: int = 2):
        import torch

        from . import ah
        self.ah, self.torch = ah, torch
        self.store = store
        self.pool = list(pool)
        self.pool_k = pool_k
        assert len(self.pool) <= MAX_POOL
        self.pool_ps = ah.PrimerSet([_with_k(p, pool_k) for p in self.pool], jit=jit)
        self.tm = tm
        self.ex = ex
        self.orient_mask = orient_mask
        self.dev = store.blocks.device
        self.slots = [_Slot(torch, self.dev, store.n_seqs) for _ in range(n_slots)]
        self.free = list(range(n_slots))[::-1]
        self.last_counts = None
        self.host_s = dict(launch=0.0, wait=0.0, collect=0.0, batches=0)  # host time by phase

    # -- compatibility: the first slot's capacities --------------------------
    @property
    def caps(self):
        return self.slots[0].caps

    @caps.setter
    def caps(self, c):
        for sl in self.slots:
            sl.caps = dict(c)

    def free_slots(self) -> int:
        return len(self.free)

    def __call__(self, batch: List[Request]) -> Dict[int, RequestResult]:
        return self.collect(self.launch(batch))

    def execute(self, plan: BatchPlan) -> Dict[int, RequestResult]:
        return self.collect(self._launch_plan(plan))

    def launch(self, batch: List[Request]) -> Ticket:
        return self._launch_plan(plan_batch(batch, self.pool, self.store.n_seqs, self.pool_k))

    def ready(self, tk: Ticket) -> bool:
        return tk.slot.event.query()

    def _launch_plan(self, plan: BatchPlan) -> Ticket:
        t_in = time.perf_counter()
        tk = self._launch_plan_timed(plan)
        self.host_s["launch"] += time.perf_counter() - t_in
        return tk

    def _launch_plan_timed(self, plan: BatchPlan) -> Ticket:
        ah, T = self.ah, self.torch
        assert self.free, "no free slot"
        sl = self.slots[self.free.pop()]
        # the batch's own primer set (pair / Tm / extract), its tables copied
        # into the slot's buffer on the slot's stream: no allocation, no sync
        tbl = sl.buf("ptable", ah.table_bytes(len(plan.slots)), T.uint8)
        vps = ah.PrimerSet(plan.slots, table=tbl, stream=sl.stream)
        # stage the routing tables in pinned memory and copy them asynchronously
        arrs = [("list", plan.seq_list.view(np.int32), T.int32), ("pmask", plan.pair_mask.view(np.int64), T.int64),
                ("seq_req", plan.seq_req.view(np.int64), T.int64),
                ("vpair", plan.vpair.reshape(-1).view(np.int16), T.int16),
                ("kmax", plan.kmax.view(np.uint8), T.uint8), ("thr", plan.slot_thr, T.float64)]
        host = sl.h_tables.numpy()
        tables, at = {}, 0
        with T.cuda.stream(sl.stream):
            for name, arr, dt in arrs:
                raw = np.ascontiguousarray(arr).view(np.uint8).reshape(-1)
                at = (at + 7) & ~7
                host[at:at + raw.size] = raw
                d = sl.buf(name, max(arr.size, 1), dt)
                if raw.size:
                    d.view(T.uint8)[:raw.size].copy_(sl.h_tables[at:at + raw.size], non_blocking=True)
                tables[name] = d
                at += raw.size
        tk = Ticket(sl, plan, vps, tables)
        self._enqueue(tk)
        return tk

    def _enqueue(self, tk: Ticket):
        ah, T = self.ah, self.torch
        st, sl, plan, vps, tb = self.store, tk.slot, tk.plan, tk.vps, tk.tables
        n_list = len(plan.seq_list)
        params = ah.tm_params(self.tm)
        params.filter = 1
        params.d_pair_threshold = tb["thr"].data_ptr()
        opts = ah.extract_opts(self.ex) if self.ex is not None else ah.extract_opts(_NoExtract())
        c = sl.caps
        with T.cuda.stream(sl.stream):
            s = sl.stream
            cnt = sl.buf("cnt", 8, T.int64)
            hits = sl.buf("hits", 3 * c["hits"], T.int32)
            rh = sl.buf("routed", 3 * c["routed"], T.int32)
            amps = sl.buf("amps", 4 * c["amps"], T.int32)
            tmv = sl.buf("tm", c["amps"], T.float64)
            tms = sl.buf("tm_site", 2 * c["amps"], T.float64)
            pas = sl.buf("pass", c["amps"], T.uint8)
            seqb = sl.buf("seq", c["seq"], T.uint8)
            soff = sl.buf("seq_off", c["amps"] + 1, T.int64)
            fb = sl.buf("fb", c["amps"] * max(opts.fb_len, 1), T.uint8)
            rb = sl.buf("rb", c["amps"] * max(opts.rb_len, 1), T.uint8)
            bcl = sl.buf("bcl", 2 * c["amps"], T.uint8)
            fpr = sl.buf("fpr", 32 * c["amps"], T.uint8)
            rpr = sl.buf("rpr", 32 * c["amps"], T.uint8)
            wsz = max(ah.ws_scan(st, n_list), ah.ws_pair(st, vps, c["routed"]), ah.ws_extract(c["amps"]))
            ws = sl.buf("ws", wsz // 8 + 1, T.int64)
            ah.scan_primers_masked(st, self.pool_ps, tb["list"][:n_list], tb["pmask"], hits, c["hits"], cnt[0:1],
                                   ws, s)
            ah.route_hits(hits, cnt[0:1], c["hits"], st.n_seqs, tb["seq_req"], tb["vpair"], tb["kmax"],
                          len(plan.reqs), len(self.pool), rh, c["routed"], cnt[1:2], s)
            ah.pair_amplicons(st, vps, rh, cnt[1:2], c["routed"], self.orient_mask, amps, c["amps"], cnt[2:3], ws, s)
            ah.tm_nn(st, vps, amps, cnt[2:3], c["amps"], params, tmv, tms, pas, s)
            ah.extract(st, vps, amps, cnt[2:3], c["amps"], pas, opts, seqb, c["seq"], soff, fb, rb, bcl, fpr, rpr,
                       cnt[3:4], ws, s)
            sl.h_cnt.copy_(cnt, non_blocking=True)
            sl.event.record(s)

    def collect(self, tk: Ticket) -> Dict[int, RequestResult]:
        ah = self.ah
        sl = tk.slot
        t_in = time.perf_counter()
        while True:
            sl.event.synchronize()
            nh, nr, na, nb = (int(x) for x in sl.h_cnt.numpy()[:4])
            c = sl.caps
            if nh <= c["hits"] and nr <= c["routed"] and na <= c["amps"] and nb <= c["seq"]:
                break
            # a buffer overflowed: grow and run the batch again (exact)
            sl.caps = dict(hits=max(c["hits"], int(nh * 1.25) + 1024), routed=max(c["routed"], int(nr * 1.25) + 1024),
                           amps=max(c["amps"], int(na * 1.25) + 1024), seq=max(c["seq"], int(nb * 1.25) + 4096))
            self._enqueue(tk)
        self.last_counts = (nh, nr, na, nb)
        t_got = time.perf_counter()
        self.host_s["wait"] += t_got - t_in
        # results to pinned host buffers (asynchronous copies on the slot's stream)
        T = self.torch
        b = sl.bufs
        parts = [("amps", b["amps"], 16 * na), ("tm", b["tm"], 8 * na), ("tm_site", b["tm_site"], 16 * na),
                 ("pass", b["pass"], na), ("seq_off", b["seq_off"], 8 * (na + 1)), ("seq", b["seq"], nb)]
        need = sum((n + 255) & ~255 for _, _, n in parts)
        if sl.h_out is None or sl.h_out.numel() < need:
            sl.h_out = T.empty(int(need * 1.25) + 4096, dtype=T.uint8, pin_memory=True)
        host, at, views = sl.h_out.numpy(), 0, {}
        with T.cuda.stream(sl.stream):
            for name, d, n in parts:
                if n:
                    sl.h_out[at:at + n].copy_(d.view(T.uint8)[:n], non_blocking=True)
                views[name] = host[at:at + n]
                at += (n + 255) & ~255
            sl.event.record(sl.stream)
        sl.event.synchronize()
        t_d2h = time.perf_counter()
        self.host_s["d2h"] = self.host_s.get("d2h", 0.0) + t_d2h - t_got
        self.host_s["bytes"] = self.host_s.get("bytes", 0) + need
        a_host = views["amps"].view(ah.AMP_DTYPE)
        tm_h = views["tm"].view(np.float64)
        tms_h = views["tm_site"].view(np.float64).reshape(-1, 2)
        pas_h = views["pass"]
        soff_h = views["seq_off"].view(np.int64).astype(np.uint64)
        slot_pair_index = []
        for rq in tk.plan.reqs:
            slot_pair_index += list(range(len(rq.pairs)))
        # split copies everything out of the pinned buffer, which the slot reuses
        res = split_results(tk.plan, a_host, tm_h, tms_h, pas_h, views["seq"], soff_h, slot_pair_index)
        tk.vps.close()
        self.free.append(self.slots.index(sl))
        self.host_s["collect"] += time.perf_counter() - t_got
        self.host_s["batches"] += 1
        return res

    def alone_reference(self, req: Request) -> RequestResult:
        """The request through the plain single-request path (its own primer
        set at its own k, scanned with ah_scan_primers over its subset)."""
        ah, torch = self.ah, self.torch
        pairs = [_with_k(self.pool[q], req.k) for q in req.pairs]
        tm = TmSpec(**{**self.tm.__dict__, "threshold_C": req.threshold_C, "filter": True})
        sub = torch.from_numpy(np.asarray(req.seqs, np.uint32).view(np.int32)).to(self.dev)
        pipe = ah.Pipeline(self.store, ah.PrimerSet(pairs), self.orient_mask, tm, self.ex or _NoExtractSpec(),
                           subset=sub).run()
        r = pipe.results()
        return RequestResult(req.rid, r["amps"], r["tm"], r["tm_site"], r["pass"], r["seq"], r["seq_off"])


class _NoExtract:
    trim = False
    fb_len = 0
    rb_len = 0


def _NoExtractSpec():
    from .synth import ExtractSpec
    return ExtractSpec()


class ServeEngine:
    """Scheduler + GPU executor over one resident store."""

    def __init__(self, store, pool, tm: TmSpec, ex=None, orient_mask: int = 0xF, pool_k: int = 3,
                 budget_bytes: int = 2 << 30, max_requests: int = MAX_REQ_PER_BATCH, jit: bool = True,
                 n_slots: int = 2):
        self.exe = GpuExecutor(store, pool, tm, ex, orient_mask, pool_k, jit, n_slots)
        lens = store.lengths.astype(np.int64)
        self.sched = Scheduler(self.exe, lambda r: request_bytes(r, self.exe.pool, lens, pool_k), budget_bytes,
                               max_requests)

    def serve(self, requests: Sequence[Request]) -> Dict[int, RequestResult]:
        for rq in requests:  # refused before any of them runs
            check_request_k(rq, self.exe.pool_k)
        return self.sched.run(requests)
