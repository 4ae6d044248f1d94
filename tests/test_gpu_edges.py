"""Degenerate inputs through the whole GPU path, against the oracle: an empty
store, a store of empty sequences, a pair that never hits, k at least the
primer length (every window whose clamp matches is a hit), a clamp spanning
the whole primer, no orientation asked for, an empty sequence subset, and
amplicons longer than one staging pass of the extraction kernel."""
import numpy as np
import pytest

from paper_2511_00170_amd import synth
from paper_2511_00170_amd.synth import ExtractSpec, PairSpec, TmSpec
from tests import _parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KERNELS = ["generic", "jit"]


@pytest.fixture(scope="module")
def ah():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00170_amd import ah
    return ah


def _concat(seqs):
    arrs = [np.frombuffer(s.encode(), np.uint8) for s in seqs]
    off = np.zeros(len(arrs) + 1, np.uint64)
    off[1:] = np.cumsum([len(a) for a in arrs])
    return (np.concatenate(arrs) if arrs else np.zeros(0, np.uint8)), off


def _run(ah, seqs, pairs, kernel, orient=0xF, tm=None):
    print("edge case", len(seqs), [(p.fwd, p.rev, p.k, p.clamp) for p in pairs], kernel, flush=True)
    buf, off = _concat(seqs)
    st = ah.Store.from_ascii(seqs)
    return P.full_parity(st, buf, off, pairs, orient, tm or TmSpec(threshold_C=30.0),
                         ExtractSpec(trim=True, fb_len=4, rb_len=4), jit=kernel == "jit")


@pytest.mark.parametrize("kernel", KERNELS)
def test_empty_store_and_empty_sequences(ah, kernel):
    pair = PairSpec("ACGTACGTAC", "TTGCATTGCA", k=2, clamp=3, min_len=20, max_len=500)
    for seqs in ([], ["", "", ""]):
        r, o = _run(ah, seqs, [pair], kernel)
        assert len(o.hits) == 0 and len(r["hits"]) == 0 and len(r["amps"]) == 0 and r["seq"] == b""


@pytest.mark.parametrize("kernel", KERNELS)
def test_pair_that_never_hits(ah, kernel):
    seqs = ["A" * 5000, "AT" * 3000, "A" * 70]
    r, o = _run(ah, seqs, [PairSpec("GGGGGGGGGG", "CCCCCCGGGG", k=0, clamp=4, min_len=20, max_len=500)], kernel)
    assert len(o.hits) == 0 and len(r["amps"]) == 0


@pytest.mark.parametrize("kernel", KERNELS)
def test_k_at_least_primer_length(ah, kernel):
    rng = np.random.default_rng(4)
    seqs = [synth.random_ascii(rng, L).tobytes().decode() for L in (300, 5000, 4097)]
    r, o = _run(ah, seqs, [PairSpec("ACGTACGT", "GATTACAG", k=8, clamp=2, min_len=10, max_len=40)], kernel)
    assert len(o.hits) > 1000 and len(o.amps) > 100


@pytest.mark.parametrize("kernel", KERNELS)
def test_clamp_spans_the_whole_primer(ah, kernel):
    rng = np.random.default_rng(5)
    F, R = "ACGTRYAC", "GGTTKMCA"
    s = list(synth.random_ascii(rng, 9000).tobytes().decode())
    s[100:108] = "ACGTACAC"                                # an exact variant of F
    s[400:408] = synth.revcomp_str("GGTTGACA")             # an exact variant of R, minus strand
    s[5000:5008] = "ACGTACAA"                              # one substitution at the 3' end: no hit
    r, o = _run(ah, ["".join(s)], [PairSpec(F, R, k=3, clamp=8, min_len=50, max_len=1000)], kernel)
    assert (o.mm == 0).all() and len(o.amps) >= 1


@pytest.mark.parametrize("kernel", KERNELS)
def test_no_orientation_asked_for(ah, kernel):
    wl = synth.gen_config(1, n_seqs=30)
    buf, off = wl.concat()
    seqs = [bytes(buf[int(off[i]):int(off[i + 1])]).decode() for i in range(wl.n_seqs)]
    r, o = _run(ah, seqs, wl.pairs, kernel, orient=0)
    assert len(o.hits) > 0 and len(o.amps) == 0 and len(r["amps"]) == 0


def test_empty_subset(ah):
    wl = synth.gen_config(1, n_seqs=10)
    st = ah.Store.from_workload(wl)
    print("edge case empty subset", flush=True)
    r = P.gpu_run(st, wl.pairs, wl.orient_mask, wl.tm, ExtractSpec(), subset=np.zeros(0, np.uint32), jit=True)
    assert len(r["hits"]) == 0 and len(r["amps"]) == 0


@pytest.mark.parametrize("kernel", KERNELS)
def test_long_amplicons_span_many_blocks(ah, kernel):
    """Amplicons of 4-12 kb (FR, and RF from swapped sites) with barcodes and
    an N run inside: their windows exceed one 64-block staging pass of the
    extraction kernel, so the chunked path writes them."""
    rng = np.random.default_rng(6)
    F, R = "ACGGTCAGTRCAGTACGT", "TTGACYGATCGGATCA"
    Fv, Rv = "ACGGTCAGTACAGTACGT", "TTGACTGATCGGATCA"      # exact variants
    s = list(synth.random_ascii(rng, 40000).tobytes().decode())
    for at in (100, 12000):
        s[at:at + len(Fv)] = Fv                            # F on the plus strand
    for at in (5000, 21000):
        s[at:at + len(Rv)] = synth.revcomp_str(Rv)         # R on the minus strand
    s[26000:26000 + len(Rv)] = Rv                          # R on the plus strand ...
    s[33000:33000 + len(Fv)] = synth.revcomp_str(Fv)       # ... F on the minus strand: RF
    s[15000:15040] = "N" * 40                               # inside the second FR amplicon
    tm = TmSpec(threshold_C=30.0, filter=False)
    r, o = _run(ah, ["".join(s)], [PairSpec(F, R, k=1, clamp=3, min_len=3000, max_len=12000)], kernel, tm=tm)
    a = o.amps.astype(np.int64)                            # [seq, start, end, pair, orient]
    assert len(a) >= 3 and (a[:, 2] - a[:, 1]).max() > 64 * 64 and (a[:, 4] == 1).any()
    assert len(r["seq"]) > 3 * 4096


@pytest.mark.parametrize("kernel", KERNELS)
def test_subset_index_outside_the_store_is_skipped(ah, kernel):
    """A listed index >= n_seqs contributes nothing (and is never read as a
    sequence): the hits equal those of the valid entries alone."""
    wl = synth.gen_config(1, n_seqs=24)
    buf, off = wl.concat()
    st = ah.Store.from_workload(wl)
    valid = [0, 3, 7, 11, 19, 23]
    listed = [0, 3, 1 << 20, 7, 11, wl.n_seqs, 19, 0xFFFFFFFF, 23]
    print("subset with out-of-range ids", kernel, listed, flush=True)
    r = P.gpu_run(st, wl.pairs, wl.orient_mask, wl.tm, subset=listed, jit=kernel == "jit")
    sel = np.concatenate([np.arange(int(off[i]), int(off[i + 1])) for i in valid])
    sub_off = np.zeros(len(valid) + 1, np.uint64)
    sub_off[1:] = np.cumsum([int(off[i + 1] - off[i]) for i in valid])
    o = P.oracle.run(buf[sel], sub_off, wl.pairs, wl.orient_mask, wl.tm)
    oh = o.hits.copy()
    oh[:, 0] = np.asarray(valid, np.uint32)[oh[:, 0]]
    P.compare_hits(r["hits"], oh, o.mm)
    assert len(o.hits) > 0
