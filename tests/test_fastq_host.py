"""FASTQ input with quality propagation, on the CPU: the oracle's reader,
quality propagation and writer pinned by hand-worked cases; libah.so's host
reader (ah_fastq_read, no GPU) and FASTQ writer (ah_fastq_format) against
the oracle on random and messy files."""
import os

import numpy as np
import pytest

from oracle import fasta as of
from oracle import fastq as oq
from paper_2511_00170_amd import ah
from paper_2511_00170_amd.synth import PairSpec

HAND = (b"@read1 sample=A run=7\n"
        b"ACGTNacgt\n"
        b"+\n"
        b"!#%')+-/1\n"
        b"\n"
        b"@read2\r\n"
        b"GGCC\r\n"
        b"+read2\r\n"
        b"~}|{\r\n"
        b"@ read3\tdesc\n"
        b"\n"
        b"+\n"
        b"\n")


def _write(tmp_path, name, data):
    p = os.path.join(str(tmp_path), name)
    with open(p, "wb") as fh:
        fh.write(data)
    return p


def test_oracle_reads_a_hand_written_file(tmp_path):
    p = _write(tmp_path, "hand.fq", HAND)
    assert oq.read_fastq([p]) == [
        (b"read1", 0, b"ACGTNacgt", b"!#%')+-/1"),
        (b"read2", 0, b"GGCC", b"~}|{"),
        (b"read3", 0, b"", b""),
    ]


@pytest.mark.parametrize("bad", [
    b"ACGT\n+\nIIII\n",                      # no '@' line
    b"@r\nACGT\n-\nIIII\n",                  # third line not '+'
    b"@r\nACGT\n+\nIII\n",                   # fewer qualities than bases
    b"@r\nACGT\n+\nIII \n",                  # a quality byte below '!'
    b"@r\nAC GT\n+\nIIIII\n",                # white space inside the bases
    b"@r\nACGT\n+\n",                        # record cut short
    b"@r\nACGT\nACGT\n+\nIIIIIIII\n",        # bases wrapped over two lines
])
def test_malformed_files_are_rejected_by_both_readers(tmp_path, bad):
    p = _write(tmp_path, "bad.fq", bad)
    with pytest.raises(ValueError):
        oq.read_fastq([p])
    with pytest.raises(ah.AhError) as e:
        ah.read_fastq([p])
    assert e.value.status == ah.AH_E_FORMAT


def test_oracle_quality_propagation_by_hand():
    # one read; forward primer ACGT, reverse primer TTGA (rc = TCAA)
    pairs = [PairSpec("ACGT", "TTGA", k=0, clamp=2, min_len=1, max_len=100)]
    q = [b"ABCDEFGHIJKLMNOPQRST"]
    amps = np.array([[0, 2, 14, 0, 0],     # FR: span [2, 14)
                     [0, 3, 15, 0, 1]])    # RF: span [3, 15), written reverse-complemented
    full = oq.amplicon_qualities(q, pairs, amps, trim=False)
    assert full == [b"CDEFGHIJKLMN", b"ONMLKJIHGFED"]
    # trimmed: FR drops 4 (ACGT) at the start and 4 (TTGA) at the end; RF
    # drops the reverse primer's 4 upstream and the forward primer's 4 downstream
    trimmed = oq.amplicon_qualities(q, pairs, amps, trim=True)
    assert trimmed == [b"GHIJ", b"KJIH"]
    # a site pair closer than both primers leaves nothing; a failed amplicon is empty
    near = oq.amplicon_qualities(q, pairs, np.array([[0, 0, 6, 0, 0]]), trim=True)
    assert near == [b""]
    assert oq.amplicon_qualities(q, pairs, amps, trim=False, passed=np.array([1, 0])) == [b"CDEFGHIJKLMN", b""]


class _Ext:
    """The parts of the oracle's extract the writers read, built by hand."""

    def __init__(self, seqs, fb, rb, fprimer, rprimer):
        self.seq = b"".join(seqs)
        self.seq_off = np.concatenate([[0], np.cumsum([len(s) for s in seqs])]).astype(np.uint64)
        w = max([len(x) for x in fb + rb] + [1])
        self.fb = np.zeros((len(seqs), w), np.uint8)
        self.rb = np.zeros((len(seqs), w), np.uint8)
        self.bc_len = np.zeros((len(seqs), 2), np.uint8)
        self.fprimer = np.zeros((len(seqs), 32), np.uint8)
        self.rprimer = np.zeros((len(seqs), 32), np.uint8)
        for i in range(len(seqs)):
            self.fb[i, :len(fb[i])] = np.frombuffer(fb[i], np.uint8)
            self.rb[i, :len(rb[i])] = np.frombuffer(rb[i], np.uint8)
            self.bc_len[i] = (len(fb[i]), len(rb[i]))
            self.fprimer[i, :len(fprimer[i])] = np.frombuffer(fprimer[i], np.uint8)
            self.rprimer[i, :len(rprimer[i])] = np.frombuffer(rprimer[i], np.uint8)

    def amplicon(self, i):
        return self.seq[int(self.seq_off[i]):int(self.seq_off[i + 1])]


def test_oracle_writer_by_hand():
    amps = np.array([[0, 2, 14, 0, 0], [1, 3, 15, 0, 1]])
    ext = _Ext([b"ACGTAC", b"TTGG"], [b"AA", b"C"], [b"GG", b""], [b"ACGT", b"ACGA"], [b"TTGA", b"TCGA"])
    text = oq.format_fastq([b"r0", b"r1"], [b"x.fq", b"y.fq"], amps, np.array([51.234, float("nan")]), None, ext,
                           [b"IIIIII", b"#$%&"], 2, 2)
    assert text == (b"@r0.source=x.fq.coordinates=3-14.Tm=51.23.orientation=FR.fprimer=ACGT.rprimer=TTGA"
                    b".fb=AA.rb=GG\nACGTAC\n+\nIIIIII\n"
                    b"@r1.source=y.fq.coordinates=4-15.Tm=NA.orientation=RF.fprimer=ACGA.rprimer=TCGA"
                    b".fb=C.rb=\nTTGG\n+\n#$%&\n")
    # the FASTA writer's records with '@', then '+' and the qualities
    fa = of.format_fasta([b"r0", b"r1"], [b"x.fq", b"y.fq"], amps, np.array([51.234, float("nan")]), None, ext, 2, 2)
    assert fa.replace(b">", b"@").split(b"\n")[0::2][:2] == text.split(b"\n")[0::4][:2]


_ALPHA = np.frombuffer(b"ACGTACGTACGTNacgtnRYKM", np.uint8)


def _random_reads(rng, n, max_len):
    recs = []
    for i in range(n):
        L = int(rng.integers(0, max_len + 1))
        bases = bytes(rng.choice(_ALPHA, L))
        qual = bytes(rng.integers(0x21, 0x7F, L, dtype=np.uint8))
        desc = b"len=%d x" % L if rng.random() < 0.5 else b""
        recs.append((b"q%d" % i, desc, bases, qual))
    return recs


def _write_messy(path, recs, rng):
    out = [b"\n"] if rng.random() < 0.5 else []
    for rid, desc, bases, qual in recs:
        nl = b"\r\n" if rng.random() < 0.3 else b"\n"
        lead = b" " if rng.random() < 0.1 else b""
        plus = b"+" + (rid if rng.random() < 0.3 else b"")
        out.append(b"@" + lead + rid + ((b"\t" + desc) if desc else b"") + nl + bases + nl + plus + nl + qual + nl)
        if rng.random() < 0.05:
            out.append(nl)
    data = b"".join(out)
    if rng.random() < 0.3:
        data = data.rstrip(b"\r\n")
    with open(path, "wb") as fh:
        fh.write(data)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_library_reader_equals_the_oracle(tmp_path, seed):
    rng = np.random.default_rng(seed)
    paths = []
    for f in range(3):
        p = os.path.join(str(tmp_path), "f%d.fq" % f)
        _write_messy(p, _random_reads(rng, int(rng.integers(0, 60)), 300), rng)
        paths.append(p)
    want = oq.read_fastq(paths)
    tab, bases, off, qual = ah.read_fastq(paths)
    assert tab.n_records == len(want)
    assert tab.ids == [r[0] for r in want]
    assert tab.seq_file.tolist() == [r[1] for r in want]
    assert tab.lengths.tolist() == [len(r[2]) for r in want]
    assert tab.files == of.source_names(paths)
    blocks = [(len(r[2]) + 63) // 64 for r in want]
    assert tab.block0.tolist() == np.concatenate([[0], np.cumsum(blocks)[:-1]]).astype(int).tolist()[:len(want)]
    assert tab.n_blocks == sum(blocks)
    b, o = oq.concat(want)
    assert np.array_equal(off, o) and bases.tobytes() == b.tobytes()
    # qualities at the store positions of their bases, zero elsewhere
    expect = np.zeros(max(64 * sum(blocks), 1), np.uint8)
    for r, b0 in zip(want, tab.block0.tolist()):
        expect[64 * b0:64 * b0 + len(r[3])] = np.frombuffer(r[3], np.uint8)
    assert np.array_equal(qual, expect)


def test_library_writer_equals_the_oracle(tmp_path):
    rng = np.random.default_rng(5)
    p = os.path.join(str(tmp_path), "names.fq")
    _write_messy(p, _random_reads(rng, 20, 50), rng)
    tab = ah.read_fastq([p])[0]
    n = 40
    seqs = [bytes(rng.choice(_ALPHA[:4], int(rng.integers(0, 30)))) for _ in range(n)]
    quals = [bytes(rng.integers(0x21, 0x7F, len(s), dtype=np.uint8)) for s in seqs]
    fb = [bytes(rng.choice(_ALPHA[:4], int(rng.integers(0, 5)))) for _ in range(n)]
    rb = [bytes(rng.choice(_ALPHA[:4], int(rng.integers(0, 5)))) for _ in range(n)]
    fp = [bytes(rng.choice(_ALPHA[:4], int(rng.integers(1, 32)))) for _ in range(n)]
    rp = [bytes(rng.choice(_ALPHA[:4], int(rng.integers(1, 32)))) for _ in range(n)]
    ext = _Ext(seqs, fb, rb, fp, rp)
    amps = np.zeros(n, ah.AMP_DTYPE)
    amps["seq"] = rng.integers(0, tab.n_records, n)
    amps["start"] = rng.integers(0, 1000, n)
    amps["end"] = amps["start"] + rng.integers(1, 500, n)
    amps["orient"] = rng.integers(0, 4, n)
    tm = rng.normal(50, 10, n)
    tm[::7] = float("nan")
    passed = (rng.random(n) < 0.7).astype(np.uint8)
    res = {"amps": amps, "tm": tm, "pass": passed, "seq": ext.seq, "seq_off": ext.seq_off, "qual": b"".join(quals),
           "fb": ext.fb[:, :4], "rb": ext.rb[:, :4], "bc_len": ext.bc_len, "fprimer": ext.fprimer,
           "rprimer": ext.rprimer}
    got = ah.format_fastq(tab, res, 4, 4, tm_filter=True)
    arr = ah.amps_array(amps)
    sources = [tab.files[f] for f in tab.seq_file.tolist()]  # per sequence
    want = oq.format_fastq(tab.ids, sources, arr, tm, passed, ext, quals, 4, 4)
    assert got == want
