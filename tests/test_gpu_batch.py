"""Batched execution: one graph over all pairs against the plain per-pair loop
and the oracle; graph replays; the autotuner; overflow inside a graph."""
import numpy as np
import pytest

import oracle
from paper_2511_00170_amd import synth
from paper_2511_00170_amd.synth import ExtractSpec
from tests import _parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00170_amd import ah, batch
    return ah, batch


@pytest.fixture(scope="module")
def batch_wl():
    return synth.gen_config(3, len_scale=1e-4)  # ~0.9 Mb, 64 pairs, 256 oriented patterns


def _say(*a):
    print(*a, flush=True)


def _same(a, b, with_extract):
    from paper_2511_00170_amd import ah
    assert np.array_equal(ah.hits_canonical(a["hits"]), ah.hits_canonical(b["hits"]))
    assert np.array_equal(ah.amps_array(a["amps"]), ah.amps_array(b["amps"]))
    assert np.array_equal(a["amps"]["flags"], b["amps"]["flags"])
    # same kernel on the same inputs: Tm values are bitwise equal (-inf included)
    assert np.array_equal(a["tm"], b["tm"])
    assert np.array_equal(a["tm_site"], b["tm_site"])
    assert np.array_equal(a["pass"], b["pass"])
    if with_extract:
        for k in ("seq", "seq_off", "fb", "rb", "bc_len", "fprimer", "rprimer"):
            assert np.array_equal(np.asarray(a[k]) if k != "seq" else np.frombuffer(a[k], np.uint8),
                                  np.asarray(b[k]) if k != "seq" else np.frombuffer(b[k], np.uint8)), k


def test_batch_graph_matches_plain_loop_and_oracle(mods, batch_wl):
    ah, batch = mods
    wl = batch_wl
    ex = ExtractSpec(trim=True, fb_len=8, rb_len=8)
    _say("batch graph vs plain loop", wl.total_bases, len(wl.pairs))
    st = ah.Store.from_workload(wl)
    br = batch.BatchRunner(st, wl.pairs, wl.orient_mask, wl.tm, ex, jit=True)
    res = br.run()
    plain, _ = batch.plain_loop(st, wl.pairs, wl.orient_mask, wl.tm, ex, jit=False, reps=1)
    _same(res, plain, True)
    buf, off = wl.concat()
    o = oracle.run(buf, off, wl.pairs, wl.orient_mask, wl.tm, ex)
    P.compare_hits(res["hits"], o.hits, o.mm)
    P.compare_amps(res["amps"], o.amps)
    P.compare_tm(res["tm"], res["tm_site"], res["pass"], o.tm)
    P.compare_extract(res, o.ext)
    assert len(o.amps) > 0


def test_graph_replays_with_eager_work_between(mods, batch_wl):
    ah, batch = mods
    wl = batch_wl
    st = ah.Store.from_workload(wl)
    _say("graph replays")
    eager = ah.Pipeline(st, ah.PrimerSet(wl.pairs), wl.orient_mask, wl.tm, wl.extract).run().results()
    br = batch.BatchRunner(st, wl.pairs, wl.orient_mask, wl.tm, wl.extract, jit=True)
    br.capture()
    # unrelated eager work between the replays: another pipeline and torch ops
    other_wl = synth.gen_config(1, n_seqs=20)
    other_st = ah.Store.from_workload(other_wl)
    other = ah.Pipeline(other_st, ah.PrimerSet(other_wl.pairs), other_wl.orient_mask, other_wl.tm, other_wl.extract)
    junk = torch.randn(1 << 20, device="cuda")
    for i in range(3):
        br.replay()
        torch.cuda.synchronize()
        assert not br.pipe.overflowed()
        _same(br.pipe.results(), eager, True)
        other.run()
        junk = (junk * 1.0001).sin()
        br.pipe.hits.fill_(-1)  # stale outputs must not survive a replay
        br.pipe.counters.fill_(123)
        torch.cuda.synchronize()
        _say("replay", i, "ok")


def test_graph_overflow_recaptures_exactly(mods, batch_wl):
    ah, batch = mods
    wl = batch_wl
    st = ah.Store.from_workload(wl)
    _say("graph overflow")
    br = batch.BatchRunner(st, wl.pairs, wl.orient_mask, wl.tm, wl.extract, jit=False,
                           caps=ah.Caps(hits=8, amps=4, seq_bytes=16))
    small_caps = br.pipe.caps
    res = br.run()
    assert br.pipe.caps.hits > small_caps.hits
    ref = ah.Pipeline(st, ah.PrimerSet(wl.pairs), wl.orient_mask, wl.tm, wl.extract).run().results()
    _same(res, ref, True)


def test_autotuner_variants_agree_and_choice_is_applied(mods, batch_wl):
    ah, batch = mods
    wl = batch_wl
    st = ah.Store.from_workload(wl)
    _say("autotune")
    br = batch.BatchRunner(st, wl.pairs, wl.orient_mask, wl.tm, wl.extract, jit=True)
    best = br.tune(sample_bases=3e5, wg_options=[1, 2, 4], reps=2)  # raises if any variant differs
    kinds = {r["kernel"] for r in best.table}
    assert kinds == {"jit", "generic"}
    tried = {(r["blocks_per_lane"], r["hit_buffer"]) for r in best.table if r["kernel"] == "jit"}
    assert tried == set(ah.JIT_VARIANTS)              # tile sizes 4096 and 8192, two hit buffers
    assert best.ms <= 1.02 * min(r["ms"] for r in best.table) + 1e-4
    assert br.ps.jit == best.jit
    if best.jit:
        assert br.ps.variant == best.variant
    res = br.run()
    ref = ah.Pipeline(st, ah.PrimerSet(wl.pairs), wl.orient_mask, wl.tm, wl.extract).run().results()
    _same(res, ref, True)


def test_launch_shape_does_not_change_hits(mods):
    ah, batch = mods
    wl = synth.gen_config(2, n_seqs=12, len_scale=0.01)
    st = ah.Store.from_workload(wl)
    ps = ah.PrimerSet(wl.pairs, jit=True)
    _say("launch shapes")
    ref = None
    for jit in (True, False):
        ps.use_jit(jit)
        mx = ps.launch_shape(0)
        assert mx >= 1
        for wg in sorted({1, mx, mx + 5}):
            ps.launch_shape(wg)
            r = ah.Pipeline(st, ps, wl.orient_mask, wl.tm, None).run().results()
            h = ah.hits_canonical(r["hits"])
            if ref is None:
                ref = h
            assert np.array_equal(h, ref)
