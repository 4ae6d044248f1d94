"""Batched execution of many primer pairs over a device-resident store.

All pairs go through ONE persistent scan launch (every tile is loaded once and
tested against every pair's patterns), then one pair / Tm / extract pass over
the combined hits; the four stages are captured into one HIP graph and
replayed.  Capacities are sized from the closed-form expected hit count of
each oriented pattern; a run that overflows is re-captured with the counted
sizes, so results are always exact.  An autotuner times kernel variants (the
primer-set specialised kernel against the generic one, and the persistent grid
size) on a sample of the store and keeps the fastest; every variant produces
the same hits.

The plain per-pair loop (one single-pair pipeline per pair, each re-reading
the store) is provided for comparison; its merged output is identical.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import ah

_IUPAC_SIZE = {c: n for c, n in zip("ACGTURYSWKMBDHVN", [1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 4])}


def _poisson_binomial_le(ps, k):
    dist = np.zeros(len(ps) + 1)
    dist[0] = 1.0
    for p in ps:
        dist[1:] = dist[1:] * (1 - p) + dist[:-1] * p
        dist[0] *= (1 - p)
    return float(dist[:k + 1].sum())


def expected_hits_per_base(pair) -> float:
    """Closed-form expected hits per genome position of a pair's four oriented
    patterns on iid sequence with equal base frequencies: for each pattern,
    prod over clamp positions of p_j times P(sum of Bernoulli(1 - p_j) over
    the other positions <= k), p_j = |IUPAC set_j| / 4."""
    tot = 0.0
    for prim in (pair.fwd, pair.rev):
        ps = [_IUPAC_SIZE[c.upper()] / 4.0 for c in prim]
        L = len(ps)
        c = min(pair.clamp, L)
        clamp, rest = ps[L - c:], ps[:L - c]
        p = math.prod(clamp) * _poisson_binomial_le([1 - x for x in rest], pair.k)
        tot += 2 * p  # plus and minus strand (same probability by symmetry)
    return tot


def hit_capacity(pairs, total_bases: int, margin: float = 2.0) -> int:
    e = sum(expected_hits_per_base(p) for p in pairs) * total_bases
    return int(margin * e + 8 * math.sqrt(e + 1) + (1 << 16))


@dataclass
class TuneResult:
    jit: bool
    wg_per_cu: int
    ms: float
    table: list = field(default_factory=list)
    variant: Optional[tuple] = None   # (blocks per lane, LDS hit buffer) of the specialised kernel


def tune_scan(store: ah.Store, ps: ah.PrimerSet, pairs, orient_mask: int, tm, stream, sample_bases: float = 1e9,
              wg_options=None, reps: int = 3, variants=None, tolerance: float = 0.02,
              prewarm_s: float = 0.3) -> TuneResult:
    """Time the scan of a leading sample of the store (about sample_bases)
    under each kernel variant -- the specialised kernel at every (tile size =
    blocks per lane, LDS hit buffer) of `variants`, the generic kernel -- and
    each persistent grid (workgroups per CU: the resident maximum, one less,
    half).  Keep the first candidate (default variant first, larger grids
    first) within `tolerance` of the fastest, so timing noise does not flip
    the choice between runs, and select it in `ps`.  Every variant must give
    the same hit set.  The GPU's clocks settle under sustained load (a scan
    right after idle time runs up to ~20% slower than in steady state), so
    the first candidate runs back to back for prewarm_s before any timing,
    and each candidate's reps run back to back, each between its own pair of
    events."""
    lens = store.lengths.astype(np.int64)
    m = int(np.searchsorted(np.cumsum(lens), sample_bases, side="left")) + 1
    m = max(1, min(m, store.n_seqs))
    sub = torch.arange(m, dtype=torch.int32, device=store.blocks.device)
    cap = hit_capacity(pairs, int(lens[:m].sum()))
    probe = ah.Pipeline(store, ps, orient_mask, tm, None, caps=ah.Caps(cap, 1, 1), subset=sub)
    kinds = [("jit", v) for v in (variants or ah.JIT_VARIANTS)] if ps.has_jit else []
    kinds.append(("generic", None))
    ref, table, cands = None, [], []
    for kind, v in kinds:
        if kind == "jit":
            ps.jit_variant(*v)
        elif ps.has_jit:
            ps.use_jit(False)
        max_wg = ps.launch_shape(0)
        opts = wg_options or sorted({max_wg, max(1, max_wg - 1), max(1, max_wg // 2)}, reverse=True)
        for wg in opts:
            if wg > max_wg:
                continue
            ps.launch_shape(wg)
            while True:  # warm-up launch, sized exactly
                probe.launch(stream, ("scan",))
                h = probe.counts()[0]
                if h <= probe.caps.hits:
                    break
                probe._alloc(ah.Caps(int(h * 1.25) + 1024, 1, 1))
            if not cands and prewarm_s > 0:
                t_w = time.perf_counter()
                while time.perf_counter() - t_w < prewarm_s:
                    for _ in range(8):
                        probe.launch(stream, ("scan",))
                    stream.synchronize()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for e0, e1 in evs:
                e0.record(stream)
                probe.launch(stream, ("scan",))
                e1.record(stream)
            stream.synchronize()
            ts = [e0.elapsed_time(e1) for e0, e1 in evs]
            h = probe.counts()[0]
            hits = ah.hits_canonical(probe.hits[:h].cpu().numpy().view(np.uint8).reshape(-1).view(ah.HIT_DTYPE))
            if ref is None:
                ref = hits
            elif not np.array_equal(ref, hits):
                raise RuntimeError("scan variant %s %s wg_per_cu=%d changed the hits" % (kind, v, wg))
            ms = float(np.median(ts))
            bpl, hb = v if v else (1, 48)
            table.append({"kernel": kind, "tile_bases": 4096 * bpl, "blocks_per_lane": bpl, "hit_buffer": hb,
                          "wg_per_cu": wg, "ms": round(ms, 4)})
            cands.append(TuneResult(kind == "jit", wg, ms, variant=v))
    fastest = min(c.ms for c in cands)
    best = next(c for c in cands if c.ms <= fastest * (1.0 + tolerance))
    best.table = table
    if best.jit:
        ps.jit_variant(*best.variant)
    elif ps.has_jit:
        ps.use_jit(False)
    ps.launch_shape(best.wg_per_cu)
    return best


class BatchRunner:
    """One graph = scan (all pairs, persistent) -> pair -> Tm -> extract."""

    def __init__(self, store: ah.Store, pairs, orient_mask: int, tm, ex=None, jit: bool = True,
                 caps: Optional[ah.Caps] = None):
        self.store = store
        self.pairs = list(pairs)
        self.orient_mask = orient_mask
        self.tm = tm
        self.ex = ex
        t0 = time.perf_counter()
        self.ps = ah.PrimerSet(self.pairs, jit=jit)
        self.setup_s = time.perf_counter() - t0
        if caps is None:
            h = hit_capacity(self.pairs, store.total_bases)
            caps = ah.Caps(hits=h, amps=max(1 << 15, h // 2), seq_bytes=1 << 24)
        self.pipe = ah.Pipeline(store, self.ps, orient_mask, tm, ex, caps=caps)
        self.stream = torch.cuda.Stream()
        self.graph = None
        self.tuned: Optional[TuneResult] = None

    # ------------------------------------------------------------- autotune
    def tune(self, sample_bases: float = 1e9, wg_options=None, reps: int = 3, variants=None,
             tolerance: float = 0.02) -> TuneResult:
        """Pick the scan kernel variant and launch shape (tune_scan) for this
        runner's pairs; the graph is captured again afterwards."""
        best = tune_scan(self.store, self.ps, self.pairs, self.orient_mask, self.tm, self.stream,
                         sample_bases, wg_options, reps, variants, tolerance)
        self.tuned = best
        self.graph = None
        return best

    # ------------------------------------------------------------- graph
    def capture(self):
        """Run once eagerly (sizing the buffers exactly), then capture."""
        with torch.cuda.stream(self.stream):
            self.pipe.run(self.stream)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.stream):
                self.pipe.launch()
        torch.cuda.synchronize()
        self.graph = g
        return self

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def run(self):
        """Replay the graph; on overflow re-size, re-capture and replay."""
        self.replay()
        if self.pipe.overflowed():
            self.graph = None
            self.capture()
            self.replay()
        return self.pipe.results()


def plain_loop(store: ah.Store, pairs, orient_mask: int, tm, ex=None, jit: bool = True, reps: int = 3):
    """The plain per-pair loop: one single-pair pipeline per pair, launched
    back to back on one stream (each re-reads the whole store).  Returns the
    merged results in batch order and the median time of one whole loop (ms)."""
    pipes = []
    for p in pairs:
        ps = ah.PrimerSet([p], jit=jit)
        h = hit_capacity([p], store.total_bases)
        pipes.append(ah.Pipeline(store, ps, orient_mask, tm, ex, caps=ah.Caps(h, max(1 << 14, h // 2), 1 << 22)))
    stream = torch.cuda.Stream()
    ts = []
    with torch.cuda.stream(stream):
        for pp in pipes:  # sizes every buffer exactly
            pp.run(stream)
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for pp in pipes:
                pp.launch(stream)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    return merge_results([pp.results() for pp in pipes], ex is not None), float(np.median(ts)) if ts else 0.0


def merge_results(per_pair: List[dict], with_extract: bool) -> dict:
    """Merge single-pair results (pair index = list position) into the batch
    order (sequence, pair, downstream site): a stable sort on (seq, pair)."""
    hits, amps, tm, site, pas = [], [], [], [], []
    seqs, fb, rb, bcl, fp, rp = [], [], [], [], [], []
    for q, r in enumerate(per_pair):
        h = r["hits"].copy()
        h["pair"] = q
        hits.append(h)
        a = r["amps"].copy()
        a["pair"] = q
        amps.append(a)
        tm.append(r["tm"])
        site.append(r["tm_site"])
        pas.append(r["pass"])
        if with_extract:
            off = r["seq_off"].astype(np.int64)
            seqs += [r["seq"][off[i]:off[i + 1]] for i in range(len(a))]
            fb.append(r["fb"])
            rb.append(r["rb"])
            bcl.append(r["bc_len"])
            fp.append(r["fprimer"])
            rp.append(r["rprimer"])
    amps_all = np.concatenate(amps) if amps else np.zeros(0, ah.AMP_DTYPE)
    order = np.lexsort((np.arange(len(amps_all)), amps_all["pair"], amps_all["seq"]))
    out = {"hits": np.concatenate(hits) if hits else np.zeros(0, ah.HIT_DTYPE),
           "amps": amps_all[order], "tm": np.concatenate(tm)[order], "tm_site": np.concatenate(site)[order],
           "pass": np.concatenate(pas)[order]}
    if with_extract:
        s_sorted = [seqs[i] for i in order]
        out["seq"] = b"".join(s_sorted)
        off = np.zeros(len(s_sorted) + 1, np.uint64)
        off[1:] = np.cumsum([len(x) for x in s_sorted])
        out["seq_off"] = off
        out["fb"] = np.concatenate(fb)[order]
        out["rb"] = np.concatenate(rb)[order]
        out["bc_len"] = np.concatenate(bcl)[order]
        out["fprimer"] = np.concatenate(fp)[order]
        out["rprimer"] = np.concatenate(rp)[order]
    return out
