"""GPU parity of the nearest-neighbour Tm for every Watson-Crick parameter set
of the Tm_NN model and for explicit duplexes with dangling ends and unequal
lengths (Implementations, "AHv2": any parameter combination), through
ah_tm_duplex and ah_tm_nn, against the oracle: |dTm| <= 1e-9 C with the same
untabulated (NaN) duplexes and the same pass/fail."""
import os

import numpy as np
import pytest

import oracle
from paper_2511_00170_amd import synth
from paper_2511_00170_amd.synth import TmSpec
from tests import _parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


@pytest.fixture(scope="module")
def ah():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00170_amd import ah
    return ah


def _say(*a):
    print("case:", *a, flush=True)


def _oracle_tm(s, c, cond, shift=0):
    try:
        return oracle.tm_duplex(s, c, cond, shift=shift)
    except ValueError:       # fewer than two facing positions: the GPU reports NaN
        return float("nan")


def _random_duplexes(rng, n, max_mm=4, dangling=False):
    seqs, cseqs, shifts = [], [], []
    for _ in range(n):
        L = int(rng.integers(2, 33))
        s = "".join(rng.choice(list("ACGT"), size=L))
        c = [COMP[x] for x in s]
        for j in rng.choice(L, size=int(rng.integers(0, min(L, max_mm) + 1)), replace=False):
            c[j] = rng.choice([b for b in "ACGT" if b != c[j]])
        sh = 0
        if dangling:
            # overhangs of 0-3 bases of either strand on either side
            left, right = int(rng.integers(-3, 4)), int(rng.integers(-3, 4))
            if left > 0:
                c = list(rng.choice(list("ACGT"), size=left)) + c
                sh = left
            elif left < 0:
                c = c[-left:]
                sh = left
            if right > 0:
                c = c + list(rng.choice(list("ACGT"), size=right))
            elif right < 0:
                c = c[:len(c) + right] if len(c) + right > 0 else c[:1]
        seqs.append(s)
        cseqs.append("".join(c))
        shifts.append(sh)
    return seqs, cseqs, shifts


def _compare(ah, seqs, cseqs, shifts, cond, min_finite):
    g = ah.tm_duplex(seqs, cseqs, cond, shifts)
    o = np.array([_oracle_tm(s, c, cond, sh) for s, c, sh in zip(seqs, cseqs, shifts)])
    bad = np.nonzero(np.isnan(g) != np.isnan(o))[0]
    assert len(bad) == 0, [(seqs[i], cseqs[i], shifts[i], g[i], o[i]) for i in bad[:8]]
    fin = ~np.isnan(o)
    assert fin.sum() >= min_finite, fin.sum()
    assert np.abs(g[fin] - o[fin]).max() <= P.TM_TOL


def test_documented_values_on_the_gpu(ah):
    rows = []
    with open(os.path.join(GOLDEN, "tm_nn_documented.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    seqs, cseqs, shifts, conds, want = [], [], [], [], []
    for seq, cseq, shift, table, na, k, tris, mg, dntps, d1, d2, sc, tm2 in rows:
        cond = TmSpec(na_mM=float(na), k_mM=float(k), tris_mM=float(tris), mg_mM=float(mg),
                      dntps_mM=float(dntps), dnac1_nM=float(d1), dnac2_nM=float(d2), saltcorr=int(sc),
                      nn_table=int(table))
        c = "".join(COMP[x] for x in seq) if cseq == "-" else cseq
        g = ah.tm_duplex([seq], [c], cond, [int(shift)])
        _say("documented", table, sc, shift)
        assert "%.2f" % g[0] == tm2


@pytest.mark.parametrize("table", [1, 2, 3, 4])
def test_random_duplexes_every_table(ah, table):
    rng = np.random.default_rng(300 + table)
    seqs, cseqs, shifts = _random_duplexes(rng, 6000)
    _say("table", table)
    for cond in (TmSpec(nn_table=table),
                 TmSpec(nn_table=table, na_mM=10, k_mM=40, tris_mM=10, mg_mM=1.5, dntps_mM=0.2, dnac1_nM=500,
                        dnac2_nM=50, saltcorr=7)):
        _compare(ah, seqs, cseqs, shifts, cond, 1500)


@pytest.mark.parametrize("table", [3, 1])
def test_random_duplexes_with_dangling_ends(ah, table):
    rng = np.random.default_rng(400 + table)
    seqs, cseqs, shifts = _random_duplexes(rng, 8000, max_mm=2, dangling=True)
    _say("dangling", table)
    _compare(ah, seqs, cseqs, shifts, TmSpec(nn_table=table), 2000)
    # dangling-end cases are among them
    assert sum(1 for s, c, sh in zip(seqs, cseqs, shifts) if sh != 0 or len(s) != len(c)) > 4000


def test_hand_worked_duplexes_on_the_gpu(ah):
    with open(os.path.join(GOLDEN, "tm_nn_hand_worked.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    seqs = [r[1] for r in rows]
    cseqs = [r[2] for r in rows]
    shifts = [int(r[3]) for r in rows]
    _compare(ah, seqs, cseqs, shifts, TmSpec(), len(rows) - 1)


@pytest.mark.parametrize("table", [1, 2, 4])
def test_amplicon_tm_every_table(ah, table):
    wl = synth.gen_config(1, n_seqs=60)
    buf, off = wl.concat()
    st = ah.Store.from_workload(wl)
    tm = TmSpec(nn_table=table, threshold_C=50.0)
    _say("amplicon Tm table", table)
    r = P.gpu_run(st, wl.pairs, wl.orient_mask, tm, None)
    o = oracle.run(buf, off, wl.pairs, wl.orient_mask, tm, None)
    P.compare_amps(r["amps"], o.amps)
    P.compare_tm(r["tm"], r["tm_site"], r["pass"], o.tm)
    assert len(o.amps) > 0


def test_invalid_table_is_rejected(ah):
    with pytest.raises(ah.AhError):
        ah.tm_duplex(["ACGTACGT"], ["TGCATGCA"], TmSpec(nn_table=5))
    with pytest.raises(ah.AhError):
        ah.tm_duplex(["ACGTACGT"], ["TGCATGCA"], TmSpec(nn_table=-1))
