"""Parity at the full workload sizes, in the launch configuration the
benchmark times: the 9 Gb genome store with the specialised scan, the 9 Gb
64-pair batch through the autotuned graph, the 2 Gb dense store with trimming
and barcodes, and the 20 Gb serving store.  Sites never cross sequences, so
the oracle computes any group of whole sequences alone: the genome and dense
outputs are compared with the oracle element by element in full (the oracle
runs over groups of about 1 Gb), the 64-pair batch on random sequences
holding at least 5% of its bases, and serving on 10 requests of mixed sizes;
the whole output is also checked against properties that hold at any size."""
import numpy as np
import pytest

import oracle
from paper_2511_00170_amd import synth
from tests import _parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ah():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00170_amd import ah
    return ah


def _say(*a):
    print(*a, flush=True)


def _sample(wl, n, seed):
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(wl.n_seqs, n, replace=False).tolist()) | {0, wl.n_seqs - 1}
    return np.array(sorted(idx), np.int64)


def _restrict(ah, r, idx):
    """The results of the sequences idx (sorted), renumbered 0..len(idx)-1."""
    pos = np.full(int(idx.max()) + 1, -1, np.int64)
    pos[idx] = np.arange(len(idx))
    hs = r["hits"]["seq"].astype(np.int64)
    hsel = (hs <= idx.max()) & (pos[np.minimum(hs, idx.max())] >= 0)
    hits = r["hits"][hsel].copy()
    hits["seq"] = pos[hits["seq"].astype(np.int64)]
    as_ = r["amps"]["seq"].astype(np.int64)
    sel = np.nonzero((as_ <= idx.max()) & (pos[np.minimum(as_, idx.max())] >= 0))[0]
    amps = r["amps"][sel].copy()
    amps["seq"] = pos[amps["seq"].astype(np.int64)]
    out = {"hits": hits, "amps": amps, "tm": r["tm"][sel], "tm_site": r["tm_site"][sel], "pass": r["pass"][sel]}
    if "seq" in r:
        so = r["seq_off"].astype(np.int64)
        parts = [r["seq"][so[i]:so[i + 1]] for i in sel]
        off = np.zeros(len(sel) + 1, np.uint64)
        off[1:] = np.cumsum([len(p) for p in parts])
        out.update(seq=b"".join(parts), seq_off=off, fb=r["fb"][sel], rb=r["rb"][sel], bc_len=r["bc_len"][sel],
                   fprimer=r["fprimer"][sel], rprimer=r["rprimer"][sel])
    return out


def _compare_sample(ah, wl, r, idx, pairs, ex, tm=None):
    tm = tm or wl.tm
    buf, off = wl.concat(idx.tolist())
    o = oracle.run(buf, off, pairs, wl.orient_mask, tm, ex)
    g = _restrict(ah, r, idx)
    P.compare_hits(g["hits"], o.hits, o.mm)
    P.compare_amps(g["amps"], o.amps)
    P.compare_tm(g["tm"], g["tm_site"], g["pass"], o.tm)
    if ex is not None:
        P.compare_extract(g, o.ext)
    return o


def _compare_all(ah, wl, r, pairs, ex, group_bases=1 << 30):
    """Every sequence against the oracle, a group of whole sequences at a time."""
    n_amps = 0
    for first, buf, off in wl.chunks(group_bases):
        idx = np.arange(first, first + len(off) - 1, dtype=np.int64)
        _say("oracle group", int(idx[0]), int(idx[-1]), int(off[-1]))
        o = oracle.run(buf, off, pairs, wl.orient_mask, wl.tm, ex)
        g = _restrict(ah, r, idx)
        P.compare_hits(g["hits"], o.hits, o.mm)
        P.compare_amps(g["amps"], o.amps)
        P.compare_tm(g["tm"], g["tm_site"], g["pass"], o.tm)
        if ex is not None:
            P.compare_extract(g, o.ext)
        n_amps += len(o.amps)
        del buf, off, o, g
    assert n_amps == len(r["amps"])
    return n_amps


def _sample_bases(wl, frac, seed):
    """Random sequences holding at least frac of the bases, plus the first and the last."""
    rng = np.random.default_rng(seed)
    lens = wl.lengths.astype(np.int64)
    order = rng.permutation(wl.n_seqs)
    take = np.searchsorted(np.cumsum(lens[order]), frac * lens.sum()) + 1
    return np.array(sorted(set(order[:take].tolist()) | {0, wl.n_seqs - 1}), np.int64)


def _properties(ah, wl, r, pairs, ex):
    """What holds for every record at any size."""
    lens = wl.lengths.astype(np.int64)
    L = np.array([[len(p.fwd), len(p.rev)] for p in pairs], np.int64)
    ks = np.array([p.k for p in pairs], np.int64)
    h = ah.hits_canonical(r["hits"])                     # [seq, pos, pair, kind, mm]
    assert len(np.unique(h, axis=0)) == len(h)           # no duplicate hits
    hl = L[h[:, 2], h[:, 3] & 1]
    assert (h[:, 1] + hl <= lens[h[:, 0]]).all() and (h[:, 4] <= ks[h[:, 2]]).all()
    a = ah.amps_array(r["amps"])                         # [seq, start, end, pair, orient]
    span = a[:, 2] - a[:, 1]
    mn = np.array([p.min_len for p in pairs])[a[:, 3]]
    mx = np.array([p.max_len for p in pairs])[a[:, 3]]
    assert ((span >= mn) & (span <= mx)).all() and (a[:, 2] <= lens[a[:, 0]]).all()
    assert (((wl.orient_mask >> a[:, 4]) & 1) == 1).all()
    key = a[:, 0] * (1 << 16) + a[:, 3]
    assert (np.diff(key) >= 0).all()                     # canonical order by (seq, pair)
    fin = np.isfinite(r["tm"])
    if wl.tm.filter:
        assert (r["pass"].astype(bool) == (fin & (r["tm"] >= wl.tm.threshold_C))).all()
    assert np.allclose(r["tm"][fin], np.minimum(r["tm_site"][fin, 0], r["tm_site"][fin, 1]), rtol=0, atol=0)
    if ex is not None:
        so = r["seq_off"].astype(np.int64)
        assert (np.diff(so) >= 0).all() and so[-1] == len(r["seq"])
        size = np.maximum(span - _trim_len(a, L), 0) if ex.trim else span
        written = r["pass"].astype(bool) if wl.tm.filter else np.ones(len(a), bool)
        assert (np.diff(so) == np.where(written, size, 0)).all()


def _trim_len(a, L):
    """Primer bases trimmed from each amplicon: upstream + downstream site lengths."""
    up = np.where((a[:, 4] == 0) | (a[:, 4] == 2), L[a[:, 3], 0], L[a[:, 3], 1])
    dn = np.where((a[:, 4] == 0) | (a[:, 4] == 3), L[a[:, 3], 1], L[a[:, 3], 0])
    return up + dn


@pytest.mark.timeout(900)
def test_genome_full_size(ah):
    wl = synth.gen_config(2)
    _say("full genome", wl.total_bases)
    st = ah.Store.from_workload(wl)
    ex = synth.ExtractSpec(trim=wl.extract.trim, fb_len=wl.extract.fb_len, rb_len=wl.extract.rb_len)
    r = ah.Pipeline(st, ah.PrimerSet(wl.pairs, jit=True), wl.orient_mask, wl.tm, ex).run().results()
    del st
    assert len(r["amps"]) > 10000
    _properties(ah, wl, r, wl.pairs, ex)
    assert _compare_all(ah, wl, r, wl.pairs, ex) > 10000


@pytest.mark.timeout(900)
def test_batch_full_size_tuned_graph(ah):
    from paper_2511_00170_amd import batch
    wl = synth.gen_config(3)
    _say("full batch", wl.total_bases, len(wl.pairs))
    st = ah.Store.from_workload(wl)
    ex = synth.ExtractSpec(trim=wl.extract.trim, fb_len=wl.extract.fb_len, rb_len=wl.extract.rb_len)
    br = batch.BatchRunner(st, wl.pairs, wl.orient_mask, wl.tm, ex, jit=True)
    br.tune(sample_bases=1e9)
    br.run()
    br.replay()
    r = br.pipe.results()
    del br, st
    _properties(ah, wl, r, wl.pairs, ex)
    idx = _sample_bases(wl, 0.05, 2)
    _say("full batch sample", len(idx), int(wl.lengths[idx].sum()))
    assert wl.lengths[idx].sum() >= 0.05 * wl.total_bases
    o = _compare_sample(ah, wl, r, idx, wl.pairs, ex)
    assert len(o.hits) > 0


@pytest.mark.timeout(600)
def test_dense_full_size(ah):
    wl = synth.gen_config(4)
    _say("full dense", wl.total_bases)
    st = ah.Store.from_workload(wl)
    ex = synth.ExtractSpec(trim=wl.extract.trim, fb_len=wl.extract.fb_len, rb_len=wl.extract.rb_len)
    r = ah.Pipeline(st, ah.PrimerSet(wl.pairs, jit=True), wl.orient_mask, wl.tm, ex).run().results()
    del st
    _properties(ah, wl, r, wl.pairs, ex)
    assert _compare_all(ah, wl, r, wl.pairs, ex) > 5000


@pytest.mark.timeout(900)
def test_serve_full_store(ah):
    from paper_2511_00170_amd import serve
    wl = synth.gen_config(5)
    _say("full serve store", wl.total_bases)
    st = ah.Store.from_workload(wl)
    reqs = synth.gen_requests(wl, 12, qps=0, seed=31)
    # ten requests of mixed sizes (1-8 pairs, 20-200 sequences, k 0-3) for the oracle
    small = synth.gen_requests(wl, 10, qps=0, seed=32, max_subset=200, min_subset=20)
    for i, r in enumerate(small):
        r.rid = 1000 + i
    ex = synth.ExtractSpec()
    exe = serve.GpuExecutor(st, wl.pairs, wl.tm, ex, wl.orient_mask, pool_k=3, jit=True)
    res = exe(reqs + small)
    for r in reqs[:4] + small:
        assert serve.results_equal(res[r.rid], exe.alone_reference(r)), r.rid
    for r in small:
        _say("full serve oracle request", r.rid, len(r.pairs), len(r.seqs), r.k)
        seqs = [wl.make_seq(int(i)) for i in r.seqs]
        off = np.zeros(len(seqs) + 1, np.uint64)
        off[1:] = np.cumsum([len(s) for s in seqs])
        pairs = [synth.PairSpec(wl.pairs[q].fwd, wl.pairs[q].rev, k=r.k, clamp=wl.pairs[q].clamp,
                                min_len=wl.pairs[q].min_len, max_len=wl.pairs[q].max_len) for q in r.pairs]
        tm = synth.TmSpec(**{**wl.tm.__dict__, "threshold_C": r.threshold_C, "filter": True})
        o = oracle.run(np.concatenate(seqs), off, pairs, wl.orient_mask, tm, ex)
        g = res[r.rid]
        a = g.amps.copy()
        local = {int(s): i for i, s in enumerate(r.seqs)}
        a["seq"] = [local[int(s)] for s in a["seq"]]
        P.compare_amps(a, o.amps)
        P.compare_tm(g.tm, g.tm_site, g.passed, o.tm)
