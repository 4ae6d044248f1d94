"""Host logic of the batch layer (no GPU): the closed-form hit-rate estimate
that sizes the buffers, checked against exhaustive enumeration of windows,
and the merge of per-pair results into batch order."""
import itertools

import numpy as np
import pytest

from paper_2511_00170_amd.synth import PairSpec

batch = pytest.importorskip("paper_2511_00170_amd.batch")

CODES = {"A": "A", "C": "C", "G": "G", "T": "T", "R": "AG", "Y": "CT", "S": "CG", "W": "AT", "K": "GT", "M": "AC",
         "B": "CGT", "D": "AGT", "H": "ACT", "V": "ACG", "N": "ACGT"}
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def _rc_sets(p):
    return [set(COMP[b] for b in CODES[c]) for c in reversed(p)]


def _count_matching_windows(sets, clamp_idx, k):
    n = 0
    for w in itertools.product("ACGT", repeat=len(sets)):
        if any(w[j] not in sets[j] for j in clamp_idx):
            continue
        if sum(w[j] not in sets[j] for j in range(len(sets))) <= k:
            n += 1
    return n


@pytest.mark.parametrize("fwd,rev,k,c", [("ARNGTC", "CYTAKG", 1, 2), ("GGHAT", "WWCAN", 2, 3), ("ACGTA", "TTTGC", 0, 0),
                                         ("NNRNN", "SCYWG", 3, 5)])
def test_expected_hits_equals_enumeration(fwd, rev, k, c):
    pair = PairSpec(fwd, rev, k=k, clamp=c)
    total = 0.0
    for p in (fwd, rev):
        L = len(p)
        plus = [set(CODES[x]) for x in p]
        minus = _rc_sets(p)
        total += _count_matching_windows(plus, range(L - c, L), k) / 4.0 ** L
        total += _count_matching_windows(minus, range(0, c), k) / 4.0 ** L
    assert abs(batch.expected_hits_per_base(pair) - total) < 1e-12


def test_capacity_grows_with_rate_and_size():
    lo = PairSpec("ACGTACGTACGTACGTAC", "GTACGTACGTACGTACGT", k=0, clamp=5)
    hi = PairSpec("NNNNNNNNNNNNNNNNNN", "GTACGTACGTACGTACGT", k=3, clamp=3)
    assert batch.hit_capacity([lo], 10 ** 9) < batch.hit_capacity([hi], 10 ** 9)
    assert batch.hit_capacity([hi], 10 ** 6) < batch.hit_capacity([hi], 10 ** 9)
    # a fully degenerate primer hits every position on both strands
    assert batch.hit_capacity([hi], 10 ** 6) >= 2 * 2 * 10 ** 6


def test_merge_results_orders_by_sequence_then_pair():
    from paper_2511_00170_amd import ah
    def mk(rows):
        a = np.zeros(len(rows), ah.AMP_DTYPE)
        for i, (s, st) in enumerate(rows):
            a[i]["seq"], a[i]["start"], a[i]["end"] = s, st, st + 10
        return {"hits": np.zeros(0, ah.HIT_DTYPE), "amps": a, "tm": np.arange(len(rows), dtype=float),
                "tm_site": np.zeros((len(rows), 2)), "pass": np.ones(len(rows), np.uint8)}
    r0 = mk([(0, 5), (0, 50), (2, 1)])
    r1 = mk([(0, 1), (1, 7)])
    m = batch.merge_results([r0, r1], with_extract=False)
    got = [(int(x["seq"]), int(x["pair"]), int(x["start"])) for x in m["amps"]]
    assert got == [(0, 0, 5), (0, 0, 50), (0, 1, 1), (1, 1, 7), (2, 0, 1)]
    assert list(m["tm"]) == [0.0, 1.0, 0.0, 1.0, 2.0]


def test_sweep_pair_constructions():
    from paper_2511_00170_amd import synth
    base = synth.PairSpec("ACGTRYACGT", "TTGGCCAANN", k=3, clamp=4, min_len=100, max_len=900)
    deg = synth.sweep_pairs(base, "degeneracy")
    assert [n for n, _ in deg] == [0, 2, 4, 6]
    for n, p in deg:
        assert p.fwd == "N" * (n // 2) + base.fwd and p.rev == "N" * (n // 2) + base.rev
        assert p.fwd.endswith(base.fwd) and (p.k, p.clamp, p.min_len, p.max_len) == (3, 4, 100, 900)
    mm = synth.sweep_pairs(base, "mismatch")
    assert [k for k, _ in mm] == list(range(7)) and all(p.k == k and p.fwd == base.fwd for k, p in mm)
