"""Seeded random cases of the whole GPU path against the oracle: random
stores (empty, short and ~20 kb sequences, N runs), 1-3 random degenerate
primer pairs with planted variants (and substitutions) in every orientation,
random k, clamp, window, orientation mask, Tm threshold and filter, trimming
and barcodes -- compared element by element for the generic and the
specialised scan kernel; and 8-24 random pairs at once through the batch
runner (tuned variant, captured graph, replay).  The cases are fixed by
their seeds."""
import numpy as np
import pytest

from paper_2511_00170_amd import synth
from paper_2511_00170_amd.synth import ExtractSpec, PairSpec, TmSpec
from tests import _parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ah():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00170_amd import ah
    return ah


def _mutate(rng, site: bytearray, n: int) -> None:
    for p in rng.choice(len(site), size=min(n, len(site)), replace=False):
        site[p] = b"ACGT"[(b"ACGT".index(site[p]) + int(rng.integers(1, 4))) % 4]


def _case(seed):
    rng = np.random.default_rng(5000 + seed)
    pairs = []
    for _ in range(int(rng.integers(1, 4))):
        Lf, Lr = int(rng.integers(12, 27)), int(rng.integers(12, 27))
        fwd = synth.make_primer(rng, Lf, int(rng.integers(0, 5)), folds=(2, 3))
        rev = synth.make_primer(rng, Lr, int(rng.integers(0, 5)), folds=(2, 3))
        lo = int(rng.integers(30, 300))
        pairs.append(PairSpec(fwd, rev, k=int(rng.integers(0, 5)), clamp=int(rng.integers(0, min(Lf, Lr) + 1)),
                              min_len=lo, max_len=lo + int(rng.integers(100, 3000))))
    seqs = []
    for _ in range(int(rng.integers(20, 41))):
        kind = rng.random()
        L = 0 if kind < 0.05 else int(rng.integers(1, 40)) if kind < 0.15 else int(rng.integers(2000, 20000))
        s = bytearray(synth.random_ascii(rng, L, gc=float(rng.uniform(0.3, 0.7))).tobytes())
        if L > 100 and rng.random() < 0.3:  # an N run
            a, n = int(rng.integers(0, L - 50)), int(rng.integers(1, 50))
            s[a:a + n] = b"N" * n
        for pr in pairs:  # planted sites: a plus site and, downstream, a minus site, in random roles
            for _ in range(int(rng.integers(0, 4))):
                if L < 400:
                    break
                up = bytearray(synth.random_variant(rng, pr.fwd if rng.random() < 0.7 else pr.rev).tobytes())
                dn = bytearray(synth.random_variant(rng, pr.rev if rng.random() < 0.7 else pr.fwd).tobytes())
                _mutate(rng, up, int(rng.integers(0, pr.k + 2)))
                _mutate(rng, dn, int(rng.integers(0, pr.k + 2)))
                dn = bytearray(synth.revcomp_str(dn.decode()).encode())
                a = int(rng.integers(0, max(1, L - 3500)))
                b = a + len(up) + int(rng.integers(0, pr.max_len + 50))
                if b + len(dn) <= L:
                    s[a:a + len(up)] = up
                    s[b:b + len(dn)] = dn
        seqs.append(s.decode())
    tm = TmSpec(threshold_C=float(rng.uniform(20, 60)), filter=bool(rng.random() < 0.7),
                saltcorr=int(rng.choice([0, 1, 2, 3, 4, 5, 6])))
    ex = ExtractSpec(trim=bool(rng.random() < 0.5), fb_len=int(rng.integers(0, 13)), rb_len=int(rng.integers(0, 13)))
    return seqs, pairs, int(rng.integers(1, 16)), tm, ex


@pytest.mark.parametrize("kernel", ["generic", "jit"])
@pytest.mark.parametrize("seed", range(30))
def test_random_case_matches_oracle(ah, seed, kernel):
    seqs, pairs, orient, tm, ex = _case(seed)
    print("random case", seed, kernel, len(seqs), [(p.fwd, p.rev, p.k, p.clamp, p.min_len, p.max_len) for p in pairs],
          orient, tm, ex, flush=True)
    arrs = [np.frombuffer(s.encode(), np.uint8) for s in seqs]
    off = np.zeros(len(arrs) + 1, np.uint64)
    off[1:] = np.cumsum([len(a) for a in arrs])
    buf = np.concatenate(arrs)
    st = ah.Store.from_ascii(seqs)
    jit, variant = P.KERNELS[kernel]
    r, o = P.full_parity(st, buf, off, pairs, orient, tm, ex, jit=jit, variant=variant)
    assert len(o.hits) > 0


def _many_pair_case(seed):
    """8-24 random pairs over a random store: the many-group kernels (group
    loop, empty-group skip, per-pattern filter plans) with every pair's sites
    planted."""
    rng = np.random.default_rng(9000 + seed)
    n_pairs = int(rng.integers(8, 25))
    pairs = []
    for _ in range(n_pairs):
        Lf, Lr = int(rng.integers(12, 27)), int(rng.integers(12, 27))
        fwd = synth.make_primer(rng, Lf, int(rng.integers(0, 5)), folds=(2, 3))
        rev = synth.make_primer(rng, Lr, int(rng.integers(0, 5)), folds=(2, 3))
        lo = int(rng.integers(30, 300))
        pairs.append(PairSpec(fwd, rev, k=int(rng.integers(0, 4)), clamp=int(rng.integers(0, min(Lf, Lr) + 1)),
                              min_len=lo, max_len=lo + int(rng.integers(100, 2000))))
    seqs = []
    for _ in range(int(rng.integers(10, 21))):
        L = int(rng.integers(3000, 15000))
        s = bytearray(synth.random_ascii(rng, L).tobytes())
        for pr in pairs:
            if rng.random() < 0.5:
                continue
            up = bytearray(synth.random_variant(rng, pr.fwd).tobytes())
            dn = bytearray(synth.revcomp_str(synth.random_variant(rng, pr.rev).tobytes().decode()).encode())
            _mutate(rng, up, int(rng.integers(0, pr.k + 1)))
            a = int(rng.integers(0, max(1, L - 2500)))
            b = a + len(up) + int(rng.integers(0, pr.max_len))
            if b + len(dn) <= L:
                s[a:a + len(up)] = up
                s[b:b + len(dn)] = dn
        seqs.append(s.decode())
    tm = TmSpec(threshold_C=float(rng.uniform(20, 55)), filter=bool(rng.random() < 0.7))
    ex = ExtractSpec(trim=bool(rng.random() < 0.5), fb_len=int(rng.integers(0, 9)), rb_len=int(rng.integers(0, 9)))
    return seqs, pairs, int(rng.integers(1, 16)) | 1, tm, ex  # FR always: the planted orientation


@pytest.mark.parametrize("seed", range(6))
def test_random_many_pairs_batched_graph_matches_oracle(ah, seed):
    """Through the batch runner: tuned variant, captured graph, replay."""
    import oracle
    from paper_2511_00170_amd import batch
    seqs, pairs, orient, tm, ex = _many_pair_case(seed)
    print("random many-pair case", seed, len(seqs), len(pairs), orient, tm, ex, flush=True)
    arrs = [np.frombuffer(s.encode(), np.uint8) for s in seqs]
    off = np.zeros(len(arrs) + 1, np.uint64)
    off[1:] = np.cumsum([len(a) for a in arrs])
    buf = np.concatenate(arrs)
    st = ah.Store.from_ascii(seqs)
    br = batch.BatchRunner(st, pairs, orient, tm, ex, jit=True)
    br.tune(sample_bases=1e5, wg_options=[2, 4], reps=1)
    br.run()
    br.replay()
    res = br.pipe.results()
    o = oracle.run(buf, off, pairs, orient, tm, ex)
    P.compare_hits(res["hits"], o.hits, o.mm)
    P.compare_amps(res["amps"], o.amps)
    P.compare_tm(res["tm"], res["tm_site"], res["pass"], o.tm)
    P.compare_extract(res, o.ext)
    assert len(o.hits) > 0
