"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs -- element by element, bit-exact for hits, amplicons,
sequences and barcodes, |dTm| <= 1e-9 C with identical pass/fail."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_2511_00170_amd import synth
from paper_2511_00170_amd.synth import ExtractSpec, PairSpec, TmSpec
from tests import _parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ah():
    _need_gpu()
    from paper_2511_00170_amd import ah as mod
    return mod


def _concat(seqs):
    arrs = [np.frombuffer(s.encode() if isinstance(s, str) else s, np.uint8) for s in seqs]
    off = np.zeros(len(arrs) + 1, np.uint64)
    off[1:] = np.cumsum([len(a) for a in arrs])
    buf = np.concatenate(arrs) if arrs else np.zeros(0, np.uint8)
    return buf, off


def _say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ pack
def test_pack_roundtrip_with_n_and_case(ah):
    rng = np.random.default_rng(1)
    seqs = []
    for L in [0, 1, 31, 32, 33, 63, 64, 65, 127, 4095, 4096, 4097, 10000, 70000]:
        s = rng.choice(list("ACGTacgtNnRY-"), size=L, p=[.2, .2, .2, .2, .03, .03, .03, .03, .02, .02, .01, .01,
                                                       .02]).tolist()
        seqs.append("".join(s))
    _say("pack roundtrip", len(seqs))
    st = ah.Store.from_ascii(seqs)
    for i, s in enumerate(seqs):
        want = "".join(c.upper() if c.upper() in "ACGT" else "N" for c in s).encode()
        assert st.unpack(i) == want, i


# ------------------------------------------------------------------ scan
ADVERSARIAL_PAIRS = [
    PairSpec("ACGTRYACGTNNACG", "TTGCAKCCAGTMA", k=2, clamp=3, min_len=20, max_len=600),
    PairSpec("AAAAAAAAAA", "TTTTTTTTTT", k=1, clamp=2, min_len=10, max_len=300),   # homopolymer storms
    # no clamp: every window is a candidate; F matches half of all positions
    PairSpec("NNRNN", "ACGTACGTACGTACGTACGTACGTACGTACGT", k=0, clamp=0, min_len=20, max_len=100),
    PairSpec("GATTACAGATTACAGATTACAGATTACAGATT", "CC", k=3, clamp=2, min_len=5, max_len=5000),
]


KERNELS = list(P.KERNELS)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("pi", range(len(ADVERSARIAL_PAIRS)))
def test_scan_pair_tm_adversarial(ah, pi, kernel):
    rng = np.random.default_rng(100 + pi)
    pair = ADVERSARIAL_PAIRS[pi]
    seqs = []
    # lengths around tile (4096) and block (64) boundaries, sequences shorter than the primers
    for L in [0, 5, 31, 64, 65, 100, 4095, 4096, 4097, 4160, 8191, 8192, 12000, 20000]:
        s = synth.random_ascii(rng, L, gc=0.5).tobytes().decode()
        seqs.append(s)
    seqs.append("A" * 9000)                      # poly-A
    seqs.append("T" * 5000 + "A" * 5000)         # poly-T then poly-A
    s = list(synth.random_ascii(rng, 6000).tobytes().decode())
    for j in rng.choice(6000, 60, replace=False):
        s[j] = "N"                                # scattered N
    seqs.append("".join(s))
    # planted sites across a tile boundary
    s = list(synth.random_ascii(rng, 9000).tobytes().decode())
    F = "".join(synth._IUPAC_SETS[c][0] for c in pair.fwd)
    R = synth.revcomp_str("".join(synth._IUPAC_SETS[c][-1] for c in pair.rev))
    for at in [0, 4096 - len(F) // 2, 4096 - 3, 8191 - len(F) + 1]:
        s[at:at + len(F)] = F
    for at in [300, 4096 - 2, 8000]:
        s[at:at + len(R)] = R
    seqs.append("".join(s)[:9000])
    buf, off = _concat(seqs)
    _say("adversarial pair", pi, kernel)
    st = ah.Store.from_ascii(seqs)
    tm = TmSpec(threshold_C=40.0)
    jit, variant = P.KERNELS[kernel]
    r, o = P.full_parity(st, buf, off, [pair], 0xF, tm, ExtractSpec(trim=True, fb_len=7, rb_len=9),
                         jit=jit, variant=variant)
    assert len(o.hits) > 0


@pytest.mark.parametrize("kernel", ["generic", "jit"])
def test_all_n_primers(ah, kernel):
    """Primers of N only, no clamp, k = 0: every window without an N is a hit of
    all four patterns; each plus site pairs with the minus sites at its own
    position (the next plus site stops the walk); every site's Tm is the
    maximum over 4^6 variants (more than the per-primer variant table holds)."""
    rng = np.random.default_rng(77)
    seqs = [synth.random_ascii(rng, L).tobytes().decode() for L in (0, 5, 6, 7, 64, 65, 300)]
    s = list(synth.random_ascii(rng, 400).tobytes().decode())
    for j in (10, 11, 200, 399):
        s[j] = "N"
    seqs.append("".join(s))
    buf, off = _concat(seqs)
    pair = PairSpec("NNNNNN", "NNNNNN", k=0, clamp=0, min_len=1, max_len=50)
    _say("all-N primers", kernel)
    st = ah.Store.from_ascii(seqs)
    r, o = P.full_parity(st, buf, off, [pair], 0xF, TmSpec(threshold_C=0.0),
                         ExtractSpec(trim=True, fb_len=3, rb_len=3), jit=kernel == "jit")
    windows = sum(1 for x in seqs for p in range(len(x) - 5) if "N" not in x[p:p + 6])
    assert len(o.hits) == 4 * windows and len(o.amps) == 2 * windows


def test_tiny_config_full_path(ah):
    wl = synth.gen_config(1)
    buf, off = wl.concat()
    _say("config tiny")
    st = ah.Store.from_ascii([buf[int(off[i]):int(off[i + 1])] for i in range(wl.n_seqs)])
    r, o = P.full_parity(st, buf, off, wl.pairs, wl.orient_mask, wl.tm, ExtractSpec(trim=False, fb_len=16, rb_len=16))
    assert len(o.amps) >= len(wl.truth["amplicons"])


@pytest.mark.parametrize("kernel", KERNELS)
def test_genome_config_reduced_full_path(ah, kernel):
    wl = synth.gen_config(2, n_seqs=60, len_scale=0.02)   # 60 x 60-120 kb
    buf, off = wl.concat()
    _say("config genome reduced", wl.total_bases, kernel)
    st = ah.Store.from_workload(wl)
    r, o = P.full_parity(st, buf, off, wl.pairs, wl.orient_mask, wl.tm, ExtractSpec(trim=True, fb_len=16, rb_len=16),
                         jit=P.KERNELS[kernel][0], variant=P.KERNELS[kernel][1])
    assert len(o.amps) > 20


def test_dense_config_reduced_full_path(ah):
    wl = synth.gen_config(4, n_seqs=8, len_scale=0.05)
    buf, off = wl.concat()
    _say("config dense reduced", wl.total_bases)
    st = ah.Store.from_workload(wl)
    r, o = P.full_parity(st, buf, off, wl.pairs, wl.orient_mask, wl.tm, wl.extract)
    n_units = sum(len(t["units"]) for t in wl.truth["operons"])
    assert len(o.amps) == n_units


@pytest.mark.parametrize("kernel", KERNELS)
def test_many_pairs_batch_reduced(ah, kernel):
    wl = synth.gen_config(3, len_scale=1e-4)   # ~0.9 Mb, 64 pairs
    buf, off = wl.concat()
    _say("config batch reduced", wl.total_bases, wl.n_seqs, kernel)
    st = ah.Store.from_workload(wl)
    jit, variant = P.KERNELS[kernel]
    P.full_parity(st, buf, off, wl.pairs, wl.orient_mask, wl.tm, ExtractSpec(), jit=jit, variant=variant)


def test_overflow_rerun_is_exact(ah):
    wl = synth.gen_config(1)
    buf, off = wl.concat()
    st = ah.Store.from_workload(wl)
    _say("overflow rerun")
    small = ah.Caps(hits=3, amps=2, seq_bytes=10)
    r = P.gpu_run(st, wl.pairs, wl.orient_mask, wl.tm, ExtractSpec(fb_len=4, rb_len=4), caps=small)
    o = oracle.run(buf, off, wl.pairs, wl.orient_mask, wl.tm, ExtractSpec(fb_len=4, rb_len=4))
    P.compare_hits(r["hits"], o.hits, o.mm)
    P.compare_amps(r["amps"], o.amps)
    P.compare_extract(r, o.ext)


def test_subset_scan_matches_full(ah):
    wl = synth.gen_config(1)
    buf, off = wl.concat()
    st = ah.Store.from_workload(wl)
    sub = np.array(sorted(np.random.default_rng(3).choice(wl.n_seqs, 37, replace=False)), np.uint32)
    _say("subset scan")
    r_sub = P.gpu_run(st, wl.pairs, wl.orient_mask, wl.tm, subset=sub)
    r_all = P.gpu_run(st, wl.pairs, wl.orient_mask, wl.tm)
    g_all = ah.hits_canonical(r_all["hits"])
    g_all = g_all[np.isin(g_all[:, 0], sub)]
    assert (ah.hits_canonical(r_sub["hits"]) == g_all).all()
    a_all = ah.amps_array(r_all["amps"])
    assert (ah.amps_array(r_sub["amps"]) == a_all[np.isin(a_all[:, 0], sub)]).all()


# ------------------------------------------------------------------ Tm
def test_tm_duplex_documented_value(ah):
    comp = {"A": "T", "C": "G", "G": "C", "T": "A"}
    seq = "CGTTCCAAAGATGTGGGCATGAGCTTAC"
    t = ah.tm_duplex([seq], ["".join(comp[c] for c in seq)], TmSpec(dnac1_nM=25, dnac2_nM=25))
    assert "%.2f" % t[0] == "60.32"


def test_tm_duplex_random_mismatches_match_oracle(ah):
    """Every tabulated stack (Watson-Crick, internal and terminal mismatch)
    is exercised; the GPU's own copy of the tables must agree with the oracle's."""
    rng = np.random.default_rng(7)
    seqs, cseqs = [], []
    comp = {"A": "T", "C": "G", "G": "C", "T": "A"}
    for _ in range(20000):
        L = int(rng.integers(2, 33))
        s = "".join(rng.choice(list("ACGT"), size=L))
        c = [comp[x] for x in s]
        for j in rng.choice(L, size=int(rng.integers(0, min(L, 4) + 1)), replace=False):
            c[j] = rng.choice([b for b in "ACGT" if b != c[j]])
        seqs.append(s)
        cseqs.append("".join(c))
    for cond in [TmSpec(), TmSpec(na_mM=10, k_mM=40, tris_mM=10, mg_mM=1.5, dntps_mM=0.2, dnac1_nM=500, dnac2_nM=50),
                 TmSpec(saltcorr=0)]:
        g = ah.tm_duplex(seqs, cseqs, cond)
        o = np.array([oracle.tm_duplex(s, c, cond) for s, c in zip(seqs, cseqs)])
        assert (np.isnan(g) == np.isnan(o)).all()
        fin = ~np.isnan(o)
        assert fin.sum() > 5000
        assert np.abs(g[fin] - o[fin]).max() <= P.TM_TOL


SALT_CONDITIONS = [
    dict(na_mM=50),
    dict(na_mM=10, k_mM=40, tris_mM=10, mg_mM=1.5, dntps_mM=0.2),
    dict(na_mM=20, mg_mM=3.0),                 # method 7: Mg2+ model, 0.22 <= R < 6
    dict(na_mM=1, mg_mM=10.0),                 # method 7: R >= 6
    dict(na_mM=0, mg_mM=2.0, dntps_mM=0.5),    # method 7: no monovalent ions
    dict(na_mM=200, mg_mM=0.1),                # method 7: R < 0.22, the 2004 formula
]


@pytest.mark.parametrize("method", [1, 2, 3, 4, 5, 6, 7])
def test_tm_duplex_every_salt_correction_matches_oracle(ah, method):
    rng = np.random.default_rng(70 + method)
    comp = {"A": "T", "C": "G", "G": "C", "T": "A"}
    seqs, cseqs = [], []
    for _ in range(3000):
        L = int(rng.integers(2, 33))
        s = "".join(rng.choice(list("ACGT"), size=L))
        c = [comp[x] for x in s]
        for j in rng.choice(L, size=int(rng.integers(0, min(L, 3) + 1)), replace=False):
            c[j] = rng.choice([b for b in "ACGT" if b != c[j]])
        seqs.append(s)
        cseqs.append("".join(c))
    _say("salt method", method)
    for kw in SALT_CONDITIONS:
        cond = TmSpec(saltcorr=method, **kw)
        try:
            oracle.salt_correction(cond, "ACGT")
        except ValueError:
            # undefined for these concentrations: the library refuses as well
            with pytest.raises(ah.AhError):
                ah.tm_duplex(seqs[:4], cseqs[:4], cond)
            continue
        g = ah.tm_duplex(seqs, cseqs, cond)
        o = np.array([oracle.tm_duplex(s, c, cond) for s, c in zip(seqs, cseqs)])
        assert (np.isnan(g) == np.isnan(o)).all(), kw
        fin = ~np.isnan(o)
        assert fin.sum() > 1000
        assert np.abs(g[fin] - o[fin]).max() <= P.TM_TOL, kw


@pytest.mark.parametrize("method", [2, 6, 7])
def test_amplicon_tm_with_other_salt_corrections(ah, method):
    wl = synth.gen_config(1, n_seqs=60)
    buf, off = wl.concat()
    st = ah.Store.from_workload(wl)
    tm = TmSpec(na_mM=30, mg_mM=2.0, dntps_mM=0.4, saltcorr=method, threshold_C=50.0)
    _say("amplicon Tm salt", method)
    r = P.gpu_run(st, wl.pairs, wl.orient_mask, tm, None)
    o = oracle.run(buf, off, wl.pairs, wl.orient_mask, tm, None)
    P.compare_amps(r["amps"], o.amps)
    P.compare_tm(r["tm"], r["tm_site"], r["pass"], o.tm)
    assert len(o.amps) > 0


def test_invalid_salt_method_is_rejected(ah):
    with pytest.raises(ah.AhError):
        ah.tm_duplex(["ACGTACGT"], ["TGCATGCA"], TmSpec(saltcorr=8))
    with pytest.raises(ah.AhError):
        ah.tm_duplex(["ACGTACGT"], ["TGCATGCA"], TmSpec(na_mM=0, saltcorr=1))


def test_read_probe_reads_every_word(ah):
    """The bandwidth probe touches every 16-byte word once: the XOR of its
    per-workgroup folds equals the XOR of the buffer (also with a ragged tail)."""
    rng = np.random.default_rng(12)
    for n in (1 << 22, (1 << 22) + 36):
        x = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
        d = torch.from_numpy(x.view(np.int32)).cuda()
        out = torch.zeros(8192, dtype=torch.int32, device="cuda")
        ah.read_probe(d, out)
        torch.cuda.synchronize()
        got = np.bitwise_xor.reduce(out.cpu().numpy().view(np.uint32))
        assert got == np.bitwise_xor.reduce(x[:n // 4 * 4])
