"""Serving on the GPU: the masked scan and the hit routing against plain
definitions, and every request's result identical whether served alone, in a
mix, or through the plain single-request pipeline -- and equal to the oracle."""
import numpy as np
import pytest

import oracle
from paper_2511_00170_amd import synth
from paper_2511_00170_amd.synth import ExtractSpec, TmSpec
from tests import _parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00170_amd import ah, serve
    wl = synth.gen_config(5, n_seqs=48, len_scale=0.01)   # 48 x 30-50 kb, 32-pair pool
    st = ah.Store.from_workload(wl)
    return ah, serve, wl, st


def _say(*a):
    print(*a, flush=True)


def _rows(a):
    r = np.ascontiguousarray(a).view(np.uint8).reshape(-1, 12).view(np.uint32).reshape(-1, 3)
    return r[np.lexsort(r.T[::-1])]


def _reqs(wl, n, seed):
    return synth.gen_requests(wl, n, qps=0, seed=seed, max_subset=40, min_subset=3)


def test_masked_scan_is_the_full_scan_restricted(env):
    ah, serve, wl, st = env
    _say("masked scan")
    rng = np.random.default_rng(5)
    ps = ah.PrimerSet(wl.pairs, jit=True)
    sub = np.sort(rng.choice(wl.n_seqs, 30, replace=False)).astype(np.uint32)
    mask = rng.integers(0, 1 << 32, size=len(sub), dtype=np.int64)
    mask[3] = 0
    d_sub = torch.from_numpy(sub.view(np.int32)).cuda()
    d_mask = torch.from_numpy(mask).cuda()
    full = ah.Pipeline(st, ps, wl.orient_mask, wl.tm, None, subset=d_sub).run().results()["hits"]
    cap = 1 << 20
    hits = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
    n = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(ah.ws_scan(st, len(sub)) // 8 + 1, dtype=torch.int64, device="cuda")
    for jit in (True, False):
        ps.use_jit(jit)
        ah.scan_primers_masked(st, ps, d_sub, d_mask, hits, cap, n, ws)
        torch.cuda.synchronize()
        got = hits[:int(n.item())].cpu().numpy().view(np.uint8).reshape(-1).view(ah.HIT_DTYPE)
        pos_of = {int(s): i for i, s in enumerate(sub)}
        keep = np.array([(int(mask[pos_of[int(h["seq"])]]) >> int(h["pair"])) & 1 for h in full], bool)
        assert np.array_equal(ah.hits_canonical(got), ah.hits_canonical(full[keep]))


def test_route_hits_matches_definition(env):
    ah, serve, wl, st = env
    _say("route")
    rng = np.random.default_rng(9)
    n_pool, n_req, n = 32, 37, 50000
    h = np.zeros(n, ah.HIT_DTYPE)
    h["seq"] = rng.integers(0, wl.n_seqs + 2, n)       # a few out-of-range sequence ids
    h["pos"] = rng.integers(0, 1 << 20, n)
    h["pair"] = rng.integers(0, n_pool + 1, n)         # and out-of-range pairs
    h["kind"] = rng.integers(0, 4, n)
    h["mm"] = rng.integers(0, 4, n)
    seq_req = rng.integers(0, 1 << 62, wl.n_seqs, dtype=np.int64) & rng.integers(0, 1 << 62, wl.n_seqs, dtype=np.int64)
    vpair = np.where(rng.random((n_req, n_pool)) < 0.3, rng.integers(0, 4000, (n_req, n_pool)), 0xFFFF).astype(np.uint16)
    kmax = rng.integers(0, 4, n_req).astype(np.uint8)
    want = []
    for x in h:
        s, q = int(x["seq"]), int(x["pair"])
        if s >= wl.n_seqs or q >= n_pool:
            continue
        for r in range(n_req):
            if (int(seq_req[s]) >> r) & 1 and vpair[r, q] != 0xFFFF and x["mm"] <= kmax[r]:
                y = x.copy()
                y["pair"] = vpair[r, q]
                want.append(y)
    want = np.array(want, ah.HIT_DTYPE)
    d_h = torch.from_numpy(h.view(np.uint8).reshape(-1).view(np.int32).reshape(-1, 3).copy()).cuda()
    d_n = torch.tensor([n], dtype=torch.int64, device="cuda")
    for cap in (len(want) + 100, len(want) // 3):
        out = torch.zeros((max(cap, 1), 3), dtype=torch.int32, device="cuda")
        n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
        ah.route_hits(d_h, d_n, n, wl.n_seqs, torch.from_numpy(seq_req).cuda(),
                      torch.from_numpy(vpair.view(np.int16)).cuda(), torch.from_numpy(kmax).cuda(), n_req, n_pool,
                      out, cap, n_out)
        torch.cuda.synchronize()
        assert int(n_out.item()) == len(want)
        got = out[:min(cap, len(want))].cpu().numpy().view(np.uint8).reshape(-1).view(ah.HIT_DTYPE)
        if cap >= len(want):
            assert np.array_equal(_rows(got), _rows(want))
        else:  # a subset of the true copies
            w = set(map(tuple, _rows(want).tolist()))
            assert all(tuple(x) in w for x in _rows(got).tolist())


def test_mix_equals_alone_equals_plain_pipeline(env):
    ah, serve, wl, st = env
    reqs = _reqs(wl, 10, seed=3)
    _say("serve mix", [(len(r.pairs), len(r.seqs), r.k) for r in reqs])
    exe = serve.GpuExecutor(st, wl.pairs, wl.tm, ExtractSpec(), wl.orient_mask, pool_k=3, jit=True)
    mix = exe(reqs)
    assert exe.last_counts[2] > 0
    total = 0
    for r in reqs:
        alone = exe([r])[r.rid]
        ref = exe.alone_reference(r)
        assert serve.results_equal(mix[r.rid], alone), r.rid
        assert serve.results_equal(alone, ref), r.rid
        total += len(ref.amps)
    assert total > 0
    # small capacities: the engine must grow them and rerun exactly
    exe.caps = dict(hits=16, routed=16, amps=8, seq=64)
    mix2 = exe(reqs)
    for r in reqs:
        assert serve.results_equal(mix[r.rid], mix2[r.rid])


def test_request_result_matches_oracle(env):
    ah, serve, wl, st = env
    reqs = [r for r in _reqs(wl, 12, seed=11) if len(r.pairs) <= 3][:2]
    exe = serve.GpuExecutor(st, wl.pairs, wl.tm, ExtractSpec(), wl.orient_mask, pool_k=3, jit=True)
    res = exe(reqs)
    for r in reqs:
        _say("oracle request", r.rid, len(r.pairs), len(r.seqs), r.k)
        seqs = [wl.make_seq(int(i)) for i in r.seqs]
        off = np.zeros(len(seqs) + 1, np.uint64)
        off[1:] = np.cumsum([len(s) for s in seqs])
        buf = np.concatenate(seqs)
        pairs = [synth.PairSpec(wl.pairs[q].fwd, wl.pairs[q].rev, k=r.k, clamp=wl.pairs[q].clamp,
                                min_len=wl.pairs[q].min_len, max_len=wl.pairs[q].max_len) for q in r.pairs]
        tm = TmSpec(**{**wl.tm.__dict__, "threshold_C": r.threshold_C, "filter": True})
        o = oracle.run(buf, off, pairs, wl.orient_mask, tm, ExtractSpec())
        g = res[r.rid]
        a = g.amps.copy()
        local = {int(s): i for i, s in enumerate(r.seqs)}
        a["seq"] = [local[int(s)] for s in a["seq"]]
        P.compare_amps(a, o.amps)
        P.compare_tm(g.tm, g.tm_site, g.passed, o.tm)
        assert g.seq == o.ext.seq
        assert np.array_equal(g.seq_off, o.ext.seq_off)


def test_engine_serves_poisson_stream(env):
    ah, serve, wl, st = env
    reqs = synth.gen_requests(wl, 30, qps=200.0, seed=4, max_subset=40, min_subset=3)
    _say("engine stream")
    eng = serve.ServeEngine(st, wl.pairs, wl.tm, ExtractSpec(), wl.orient_mask, budget_bytes=64 << 20)
    out = eng.serve(reqs)
    assert sorted(out) == [r.rid for r in reqs]
    lat = serve.latency_summary(out)
    assert lat["n"] == 30 and lat["p99_ms"] >= lat["p50_ms"] > 0
    # every result equals the request served alone
    for r in reqs[:6]:
        assert serve.results_equal(out[r.rid], eng.exe([r])[r.rid])


def test_two_batches_in_flight_match_alone(env):
    ah, serve, wl, st = env
    reqs = _reqs(wl, 8, seed=21)
    _say("two in flight")
    exe = serve.GpuExecutor(st, wl.pairs, wl.tm, ExtractSpec(), wl.orient_mask, pool_k=3, jit=True, n_slots=2)
    t1 = exe.launch(reqs[:5])
    t2 = exe.launch(reqs[5:])
    assert exe.free_slots() == 0
    r2 = exe.collect(t2)      # collected out of order
    r1 = exe.collect(t1)
    assert exe.free_slots() == 2
    both = {**r1, **r2}
    for r in reqs:
        assert serve.results_equal(both[r.rid], exe.alone_reference(r)), r.rid
