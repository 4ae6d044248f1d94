"""FASTQ input with quality propagation on the GPU: reads shaped like
amplicon sequencing (300-700 bases, a primer-pair amplicon in either
orientation, sometimes none, N bases, random qualities) go through
ah_fastq_read -> ah_pack -> scan, pair, Tm, extract -> ah_extract_qual ->
ah_fastq_format; the store equals the one ah_pack builds from the same bases,
and the amplicons, their qualities and the FASTQ text equal the oracle's."""
import numpy as np
import pytest

import oracle
from oracle import fasta as of
from oracle import fastq as oq
from paper_2511_00170_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD, REV = "GATCMTGGCTAGTCAGKAC", "TTCGAYGTACCAGGTTCAG"  # a made-up degenerate pair
PAIR = synth.PairSpec(FWD, REV, k=2, clamp=3, min_len=60, max_len=700)
_COMP = bytes.maketrans(b"ACGT", b"TGCA")


@pytest.fixture(scope="module")
def ah():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00170_amd import ah
    return ah


def _say(*a):
    print(*a, flush=True)


def _concrete(rng, primer):
    sets = {"A": "A", "C": "C", "G": "G", "T": "T", "M": "AC", "Y": "CT", "R": "AG", "K": "GT", "S": "CG",
            "W": "AT"}
    return "".join(rng.choice(list(sets[c])) for c in primer).encode()


def _reads(rng, n):
    """(id, description, bases, qualities) of n reads."""
    out = []
    for i in range(n):
        L = int(rng.integers(300, 701))
        seq = bytearray(rng.choice(np.frombuffer(b"ACGT", np.uint8), L).tobytes())
        if rng.random() < 0.85:  # one amplicon: forward primer ... rc(reverse primer)
            f, r = _concrete(rng, FWD), _concrete(rng, REV).translate(_COMP)[::-1]
            span = int(rng.integers(len(f) + len(r) + 40, min(L, 600)))
            a = int(rng.integers(0, L - span + 1))
            amp = f + bytes(seq[a + len(f):a + span - len(r)]) + r
            if rng.random() < 0.5:  # the read runs the other way
                amp = amp.translate(_COMP)[::-1]
            seq[a:a + span] = amp
            for _ in range(int(rng.integers(0, 3))):  # substitutions, some inside primer sites
                j = int(rng.integers(a, a + span))
                seq[j] = int(rng.choice(np.frombuffer(b"ACGT", np.uint8)))
        if rng.random() < 0.1:
            seq[int(rng.integers(0, L))] = ord("N")
        qual = rng.integers(0x21, 0x4B, L, dtype=np.uint8).tobytes()
        out.append((b"m%d" % i, b"bc=%d" % (i % 7), bytes(seq), qual))
    return out


def _files(tmp_path, rng, n_files, n_reads):
    paths = []
    for k in range(n_files):
        p = str(tmp_path / ("reads%d.fq" % k))
        oq.write_fastq(p, _reads(rng, n_reads), crlf=bool(k % 2), plus_id=bool(k % 3 == 2))
        paths.append(p)
    return paths


def _oracle_run(paths, ex, tm, orient=0b1111):
    recs = oq.read_fastq(paths)
    buf, off = oq.concat(recs)
    o = oracle.run(buf, off, [PAIR], orient, tm, ex)
    quals = oq.amplicon_qualities([r[3] for r in recs], [PAIR], o.amps, ex.trim,
                                  o.tm.passed if tm.filter else None)
    return recs, o, quals


@pytest.mark.parametrize("trim,filt", [(False, False), (True, True), (True, False)])
def test_fastq_in_fastq_out_matches_oracle(ah, tmp_path, trim, filt):
    rng = np.random.default_rng(11 + 2 * trim + filt)
    paths = _files(tmp_path, rng, 3, 400)
    _say("fastq", trim, filt)
    st = ah.Store.from_fastq(paths)
    recs = oq.read_fastq(paths)
    ref = ah.Store.from_ascii([r[2] for r in recs])
    nb = st.n_blocks
    assert st.n_blocks == ref.n_blocks and torch.equal(st.blocks[:nb], ref.blocks[:nb])
    assert torch.equal(st.nbits[:(nb + 31) // 32], ref.nbits[:(nb + 31) // 32])
    ex = synth.ExtractSpec(trim=trim, fb_len=6, rb_len=6)
    tm = synth.TmSpec(threshold_C=52.0, filter=filt)
    res = ah.Pipeline(st, ah.PrimerSet([PAIR], jit=True), 0b1111, tm, ex).run().results()
    recs, o, quals = _oracle_run(paths, ex, tm)
    assert (ah.amps_array(res["amps"]) == o.amps).all() and len(o.amps) > 500
    assert {int(x) for x in o.amps[:, 4]} >= {0, 1}  # FR and RF both present
    assert res["seq"] == o.ext.seq
    assert res["qual"] == b"".join(quals)
    assert len(res["qual"]) == len(res["seq"])
    sources = [of.source_names(paths)[r[1]] for r in recs]
    want = oq.format_fastq([r[0] for r in recs], sources, o.amps, o.tm.tm, o.tm.passed if filt else None, o.ext,
                           quals, 6, 6)
    assert ah.format_fastq(st.fasta, res, 6, 6, tm_filter=filt) == want


def test_cli_writes_the_oracle_fastq(ah, tmp_path):
    from paper_2511_00170_amd import cli
    rng = np.random.default_rng(29)
    paths = _files(tmp_path, rng, 2, 300)
    out = str(tmp_path / "amplicons.fq")
    _say("cli fastq")
    rc = cli.main(["--input", *paths, "--input-fq", "--forward", FWD, "--reverse", REV, "--mismatches", "2",
                   "--clamp", "3", "--min-length", "60", "--max-length", "700", "--include-offtarget",
                   "--trim-primers", "--fb-len", "5", "--rb-len", "5", "--tm-threshold", "50", "--output", out,
                   "--quiet"])
    assert rc == 0
    ex = synth.ExtractSpec(trim=True, fb_len=5, rb_len=5)
    tm = synth.TmSpec(threshold_C=50.0, filter=True)
    recs, o, quals = _oracle_run(paths, ex, tm)
    sources = [of.source_names(paths)[r[1]] for r in recs]
    want = oq.format_fastq([r[0] for r in recs], sources, o.amps, o.tm.tm, o.tm.passed, o.ext, quals, 5, 5)
    assert int(o.tm.passed.sum()) > 100
    assert open(out, "rb").read() == want


def test_quality_extraction_respects_capacity_and_arguments(ah, tmp_path):
    rng = np.random.default_rng(3)
    paths = _files(tmp_path, rng, 1, 50)
    st = ah.Store.from_fastq(paths)
    ex = synth.ExtractSpec(trim=False)
    pipe = ah.Pipeline(st, ah.PrimerSet([PAIR], jit=True), 0b0011, synth.TmSpec(filter=False), ex).run()
    full = pipe.results()["qual"]
    n_amps = pipe.counters[1:2]
    # a short output buffer: the bytes below the capacity, nothing past it
    cap = max(len(full) // 2, 1)
    out = torch.full((len(full) + 64,), 7, dtype=torch.uint8, device=st.blocks.device)
    ah.extract_qual(st, pipe.ps, pipe.amps, n_amps, pipe.caps.amps, None, pipe.opts, pipe.seq_off, out, cap)
    torch.cuda.synchronize()
    got = out.cpu().numpy().tobytes()
    assert got[:cap] == full[:cap] and set(got[cap:]) == {7}
    # a quality array shorter than the store is refused before any work
    short = st.qual[:max(st.qual.numel() - 64, 1)]
    saved = st.qual
    st.qual = short
    with pytest.raises(ah.AhError):
        ah.extract_qual(st, pipe.ps, pipe.amps, n_amps, pipe.caps.amps, None, pipe.opts, pipe.seq_off, out, cap)
    st.qual = saved
