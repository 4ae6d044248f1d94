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

then splits the amplicons by slot.  Requests join the batch formed at the
next pass (iteration-level batching): whatever has arrived when the GPU frees
up is admitted in arrival order while the batch's estimated device memory
stays within the budget.  A request's result does not depend on what it was
batched with: routing applies exactly its (sequence, pair, k) selection to
hits that do not depend on the batch, and pairing, Tm and extraction are per
(sequence, slot).

The scheduler is separate from the GPU executor so that its policy can be
tested without a GPU.
"""
from __future__ import annotations

import heapq
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from .synth import PairSpec, Request, TmSpec

MAX_REQ_PER_BATCH = 64      # request bitmap of the routing kernel
MAX_POOL = 64               # pair bitmap of the masked scan


# --------------------------------------------------------------------------
# Results
# --------------------------------------------------------------------------
@dataclass
class RequestResult:
    rid: int
    amps: np.ndarray            # AMP_DTYPE, pair = index into the request's pair list
    tm: np.ndarray
    tm_site: np.ndarray
    passed: np.ndarray
    seq: bytes                  # amplicon sequences (passing amplicons only)
    seq_off: np.ndarray
    arrival_s: float = 0.0
    done_s: float = 0.0
    batch: int = -1

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
    """Iteration-level batching.  ``executor(batch) -> {rid: RequestResult}``
    runs one pass; ``clock()`` gives the current time and ``sleep_until(t)``
    waits (both replaceable for simulated time)."""

    def __init__(self, executor: Callable[[List[Request]], Dict[int, RequestResult]],
                 cost: Callable[[Request], int], budget_bytes: int, max_requests: int = MAX_REQ_PER_BATCH,
                 clock: Callable[[], float] = time.perf_counter, sleep_until: Optional[Callable[[float], None]] = None):
        self.executor = executor
        self.cost = cost
        self.budget = budget_bytes
        self.max_requests = max_requests
        self.clock = clock
        self.sleep_until = sleep_until or (lambda t: time.sleep(max(0.0, t - self.clock())))
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

    def run(self, requests: Sequence[Request], t0: Optional[float] = None) -> Dict[int, RequestResult]:
        """Serve ``requests`` (arrival_s relative to t0) to completion."""
        pending = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        t0 = self.clock() if t0 is None else t0
        queue: List[Request] = []
        out: Dict[int, RequestResult] = {}
        i = 0
        while i < len(pending) or queue:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival_s <= now:
                queue.append(pending[i])
                i += 1
            if not queue:
                self.sleep_until(t0 + pending[i].arrival_s)
                continue
            batch = self.admit(queue)
            ts = self.clock()
            res = self.executor(batch)
            te = self.clock()
            self.stats.batches += 1
            self.stats.batch_sizes.append(len(batch))
            self.stats.busy_s += te - ts
            for r in batch:
                rr = res[r.rid]
                rr.arrival_s = t0 + r.arrival_s
                rr.done_s = te
                rr.batch = self.stats.batches - 1
                out[r.rid] = rr
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


def plan_batch(reqs: Sequence[Request], pool: Sequence[PairSpec], n_seqs: int) -> BatchPlan:
    n_pool = len(pool)
    assert len(reqs) <= MAX_REQ_PER_BATCH and n_pool <= MAX_POOL
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


def split_results(plan: BatchPlan, amps, tm, tm_site, passed, seq: bytes, seq_off: np.ndarray,
                  slot_pair_index: List[int]) -> Dict[int, RequestResult]:
    """Split a batch's amplicons (ordered by sequence, slot, site) by request."""
    out = {}
    req_of = plan.slot_req[amps["pair"].astype(np.int64)] if len(amps) else np.zeros(0, np.int64)
    spi = np.asarray(slot_pair_index, np.uint16)
    for r, rq in enumerate(plan.reqs):
        idx = np.nonzero(req_of == r)[0]
        a = amps[idx].copy()
        if len(a):
            a["pair"] = spi[a["pair"].astype(np.int64)]
        lens = (seq_off[idx + 1] - seq_off[idx]).astype(np.int64)
        so = np.zeros(len(idx) + 1, np.uint64)
        so[1:] = np.cumsum(lens)
        s = b"".join(seq[int(seq_off[i]):int(seq_off[i + 1])] for i in idx)
        out[rq.rid] = RequestResult(rq.rid, a, tm[idx], tm_site[idx], passed[idx], s, so)
    return out


# --------------------------------------------------------------------------
# GPU executor
# --------------------------------------------------------------------------
class GpuExecutor:
    """Runs batches on one GPU against a resident store and a pool primer set
    compiled once (hipRTC-specialised scan at the pool's largest k)."""

    def __init__(self, store, pool: Sequence[PairSpec], tm: TmSpec, ex=None, orient_mask: int = 0xF,
                 pool_k: int = 3, jit: bool = True):
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
        self.stream = torch.cuda.Stream()
        self.caps = dict(hits=1 << 20, routed=1 << 20, amps=1 << 16, seq=1 << 24)
        self._bufs = {}
        self.last_counts = None

    def _buf(self, name, n, dtype):
        t = self._bufs.get(name)
        if t is None or t.numel() < n or t.dtype != dtype:
            t = self.torch.empty(max(n, 1), dtype=dtype, device=self.dev)
            self._bufs[name] = t
        return t

    def _h2d(self, name, arr: np.ndarray, dtype):
        host = self.torch.from_numpy(np.ascontiguousarray(arr))
        t = self._buf(name, host.numel(), dtype)
        t[:host.numel()].copy_(host.view(dtype) if host.dtype != dtype else host, non_blocking=False)
        return t

    def __call__(self, batch: List[Request]) -> Dict[int, RequestResult]:
        plan = plan_batch(batch, self.pool, self.store.n_seqs)
        return self.execute(plan)

    def execute(self, plan: BatchPlan) -> Dict[int, RequestResult]:
        ah, torch = self.ah, self.torch
        st = self.store
        T = torch
        n_list = len(plan.seq_list)
        vps = ah.PrimerSet(plan.slots)  # pair / Tm / extract of this batch (host compile only)
        with torch.cuda.stream(self.stream):
            s = self.stream
            lst = self._h2d("list", plan.seq_list.view(np.int32), T.int32)
            pmask = self._h2d("pmask", plan.pair_mask.view(np.int64), T.int64)
            seq_req = self._h2d("seq_req", plan.seq_req.view(np.int64), T.int64)
            vpair = self._h2d("vpair", plan.vpair.reshape(-1).view(np.int16), T.int16)
            kmax = self._h2d("kmax", plan.kmax.view(np.uint8), T.uint8)
            thr = self._h2d("thr", plan.slot_thr, T.float64)
            params = ah.tm_params(self.tm)
            params.filter = 1
            params.d_pair_threshold = thr.data_ptr()
            opts = ah.extract_opts(self.ex) if self.ex is not None else ah.extract_opts(_NoExtract())
            cnt = self._buf("cnt", 8, T.int64)
            while True:
                c = self.caps
                hits = self._buf("hits", 3 * c["hits"], T.int32)
                rh = self._buf("routed", 3 * c["routed"], T.int32)
                amps = self._buf("amps", 4 * c["amps"], T.int32)
                tmv = self._buf("tm", c["amps"], T.float64)
                tms = self._buf("tm_site", 2 * c["amps"], T.float64)
                pas = self._buf("pass", c["amps"], T.uint8)
                seqb = self._buf("seq", c["seq"], T.uint8)
                soff = self._buf("seq_off", c["amps"] + 1, T.int64)
                fb = self._buf("fb", c["amps"] * max(opts.fb_len, 1), T.uint8)
                rb = self._buf("rb", c["amps"] * max(opts.rb_len, 1), T.uint8)
                bcl = self._buf("bcl", 2 * c["amps"], T.uint8)
                fpr = self._buf("fpr", 32 * c["amps"], T.uint8)
                rpr = self._buf("rpr", 32 * c["amps"], T.uint8)
                wsz = max(ah.ws_scan(st, n_list), ah.ws_pair(st, vps, c["routed"]), ah.ws_extract(c["amps"]))
                ws = self._buf("ws", wsz // 8 + 1, T.int64)
                ah.scan_primers_masked(st, self.pool_ps, lst[:n_list], pmask, hits, c["hits"], cnt[0:1], ws, s)
                ah.route_hits(hits, cnt[0:1], c["hits"], st.n_seqs, seq_req, vpair, kmax, len(plan.reqs),
                              len(self.pool), rh, c["routed"], cnt[1:2], s)
                ah.pair_amplicons(st, vps, rh, cnt[1:2], c["routed"], self.orient_mask, amps, c["amps"], cnt[2:3],
                                  ws, s)
                ah.tm_nn(st, vps, amps, cnt[2:3], c["amps"], params, tmv, tms, pas, s)
                ah.extract(st, vps, amps, cnt[2:3], c["amps"], pas, opts, seqb, c["seq"], soff, fb, rb, bcl, fpr, rpr,
                           cnt[3:4], ws, s)
                v = cnt[:4].cpu().numpy()  # synchronises the stream
                nh, nr, na, nb = (int(x) for x in v)
                if nh <= c["hits"] and nr <= c["routed"] and na <= c["amps"] and nb <= c["seq"]:
                    break
                self.caps = dict(hits=max(c["hits"], int(nh * 1.25) + 1024),
                                 routed=max(c["routed"], int(nr * 1.25) + 1024),
                                 amps=max(c["amps"], int(na * 1.25) + 1024), seq=max(c["seq"], int(nb * 1.25) + 4096))
            self.last_counts = (nh, nr, na, nb)
            a_host = amps[:4 * na].cpu().numpy().view(np.uint8).reshape(-1).view(ah.AMP_DTYPE)
            tm_h = tmv[:na].cpu().numpy()
            tms_h = tms[:2 * na].cpu().numpy().reshape(-1, 2)
            pas_h = pas[:na].cpu().numpy()
            seq_h = seqb[:nb].cpu().numpy().tobytes()
            soff_h = soff[:na + 1].cpu().numpy().astype(np.uint64)
        slot_pair_index = []
        for r, rq in enumerate(plan.reqs):
            slot_pair_index += list(range(len(rq.pairs)))
        vps.close()
        return split_results(plan, a_host, tm_h, tms_h, pas_h, seq_h, soff_h, slot_pair_index)

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
                 budget_bytes: int = 2 << 30, max_requests: int = MAX_REQ_PER_BATCH, jit: bool = True):
        self.exe = GpuExecutor(store, pool, tm, ex, orient_mask, pool_k, jit)
        lens = store.lengths.astype(np.int64)
        self.sched = Scheduler(self.exe, lambda r: request_bytes(r, self.exe.pool, lens, pool_k), budget_bytes,
                               max_requests)

    def serve(self, requests: Sequence[Request]) -> Dict[int, RequestResult]:
        return self.sched.run(requests)
