"""FASTA ingest on the GPU: the store built by ah_fasta_ingest (one pass,
pinned double-buffered chunks, pieces cut on block boundaries) is identical
to the store ah_pack builds from the same sequences and decodes to the
oracle's reading of the files; FASTA in -> amplicons -> FASTA out equals the
oracle end to end."""
import numpy as np
import pytest

import oracle
from oracle import fasta as of
from paper_2511_00170_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_ALPHA = np.frombuffer(b"ACGTACGTACGTACGTacgtNnRY", np.uint8)


@pytest.fixture(scope="module")
def ah():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00170_amd import ah
    return ah


def _say(*a):
    print(*a, flush=True)


def _norm(seq: bytes) -> bytes:
    u = np.frombuffer(seq.upper(), np.uint8).copy()
    u[~np.isin(u, np.frombuffer(b"ACGT", np.uint8))] = ord("N")
    return u.tobytes()


def _files(tmp_path, rng, n_files, n_recs, max_len, tiny=False):
    paths = []
    for k in range(n_files):
        recs = []
        for i in range(n_recs):
            L = int(rng.integers(0, 20)) if tiny else int(rng.integers(0, max_len + 1))
            seq = rng.choice(_ALPHA, L)
            if L > 500 and rng.random() < 0.3:                 # an N run
                a = int(rng.integers(0, L - 200))
                seq[a:a + int(rng.integers(1, 200))] = ord("N")
            recs.append((b"f%dr%d" % (k, i), b"x" if i % 2 else b"", seq.tobytes()))
        p = str(tmp_path / ("in%d.fa" % k))
        of.write_fasta(p, recs, width=int(rng.choice([60, 61, 80])), crlf=bool(k % 2))
        paths.append(p)
    return paths


def _same_store(a, b):
    assert a.n_seqs == b.n_seqs and a.n_blocks == b.n_blocks
    nb, nw = a.n_blocks, (a.n_blocks + 31) // 32
    assert torch.equal(a.blocks[:nb], b.blocks[:nb])
    assert torch.equal(a.nbits[:nw], b.nbits[:nw])
    assert torch.equal(a.nrank[:nw], b.nrank[:nw])
    assert a.n_nblocks == b.n_nblocks
    assert torch.equal(a.nmask[:a.n_nblocks], b.nmask[:b.n_nblocks])
    assert torch.equal(a.seq_len[:a.n_seqs], b.seq_len[:b.n_seqs])
    assert torch.equal(a.seq_block0[:a.n_seqs], b.seq_block0[:b.n_seqs])


@pytest.mark.parametrize("n_threads", [1, 4])
@pytest.mark.parametrize("chunk,tiny", [(4096, False), (4096, True), (64 << 20, False)])
def test_ingest_equals_pack_and_oracle(ah, tmp_path, chunk, tiny, n_threads):
    rng = np.random.default_rng(chunk % 1000 + tiny)
    paths = _files(tmp_path, rng, 5, 300 if tiny else 20, 20000, tiny)
    _say("fasta ingest chunk", chunk, "tiny", tiny, "threads", n_threads)
    st = ah.Store.from_fasta(paths, chunk_bytes=chunk, n_threads=n_threads)
    recs = of.read_fasta(paths)
    ref = ah.Store.from_ascii([s for _, _, s in recs])
    _same_store(st, ref)
    assert st.fasta.ids == [r for r, _, _ in recs]
    for i in rng.choice(len(recs), min(len(recs), 40), replace=False):
        assert st.unpack(int(i)) == _norm(recs[i][2]), i


def test_ingest_grows_small_arrays(ah, tmp_path):
    rng = np.random.default_rng(4)
    paths = _files(tmp_path, rng, 2, 30, 5000)
    _say("fasta ingest regrow")
    recs = of.read_fasta(paths)
    ref = ah.Store.from_ascii([s for _, _, s in recs])
    for n_threads in (1, 2):
        st = ah.Store.from_fasta(paths, chunk_bytes=8192, blocks_cap=10, nmask_cap=2, n_threads=n_threads)
        _same_store(st, ref)


def test_ingest_large_file(ah, tmp_path):
    """~60 Mb in few long records and many short ones, default chunks."""
    rng = np.random.default_rng(5)
    recs = []
    for i in range(12):
        L = int(rng.integers(1, 8_000_000)) if i % 3 == 0 else int(rng.integers(0, 5000))
        recs.append((b"c%d" % i, b"", rng.choice(_ALPHA, L).tobytes()))
    p = str(tmp_path / "big.fa")
    of.write_fasta(p, recs, width=80)
    _say("fasta ingest large", sum(len(s) for _, _, s in recs))
    st = ah.Store.from_fasta([p], chunk_bytes=1 << 20)
    ref = ah.Store.from_ascii([s for _, _, s in recs], nmask_cap=1 << 19)   # most blocks hold an N
    _same_store(st, ref)


@pytest.mark.parametrize("ex", [synth.ExtractSpec(), synth.ExtractSpec(trim=True, fb_len=8, rb_len=5)])
def test_fasta_in_fasta_out_matches_oracle(ah, tmp_path, ex):
    wl = synth.gen_config(1, n_seqs=60)
    buf, off = wl.concat()
    recs = [(b"g%d" % i, b"sample", bytes(buf[int(off[i]):int(off[i + 1])])) for i in range(wl.n_seqs)]
    paths = [str(tmp_path / "a.fa"), str(tmp_path / "b.fna")]
    of.write_fasta(paths[0], recs[:25], width=60)
    of.write_fasta(paths[1], recs[25:], width=77, crlf=True)
    _say("fasta end to end", ex)
    st = ah.Store.from_fasta(paths, chunk_bytes=1 << 16)
    r = ah.Pipeline(st, ah.PrimerSet(wl.pairs, jit=True), wl.orient_mask, wl.tm, ex).run().results()
    got = ah.format_fasta(st.fasta, r, ex.fb_len, ex.rb_len, tm_filter=wl.tm.filter)
    orecs = of.read_fasta(paths)
    obuf, ooff = of.concat(orecs)
    o = oracle.run(obuf, ooff, wl.pairs, wl.orient_mask, wl.tm, ex)
    srcs = of.source_names(paths)
    want = of.format_fasta([x for x, _, _ in orecs], [srcs[fi] for _, fi, _ in orecs], o.amps, o.tm.tm,
                           o.tm.passed if wl.tm.filter else None, o.ext, ex.fb_len, ex.rb_len)
    assert len(o.amps) > 0 and want.count(b">") > 0
    assert got == want


def test_cli_writes_the_oracle_fasta(ah, tmp_path):
    from paper_2511_00170_amd import cli
    wl = synth.gen_config(1, n_seqs=40)
    buf, off = wl.concat()
    recs = [(b"s%d" % i, b"", bytes(buf[int(off[i]):int(off[i + 1])])) for i in range(wl.n_seqs)]
    p = str(tmp_path / "genomes.fa")
    of.write_fasta(p, recs, width=60)
    q = wl.pairs[0]
    out = str(tmp_path / "amplicons.fa")
    _say("cli")
    rc = cli.main(["--input", p, "--forward", q.fwd, "--reverse", q.rev, "--mismatches", str(q.k), "--clamp",
                   str(q.clamp), "--min-length", str(q.min_len), "--max-length", str(q.max_len),
                   "--include-offtarget", "--trim-primers", "--fb-len", "6", "--rb-len", "6", "--tm-threshold",
                   "50", "--output", out, "--chunk-mb", "1", "--quiet"])
    assert rc == 0
    tm = synth.TmSpec(threshold_C=50.0, filter=True)
    ex = synth.ExtractSpec(trim=True, fb_len=6, rb_len=6)
    orecs = of.read_fasta([p])
    obuf, ooff = of.concat(orecs)
    o = oracle.run(obuf, ooff, [q], 0b1111, tm, ex)
    want = of.format_fasta([r for r, _, _ in orecs], [b"genomes.fa"] * len(orecs), o.amps, o.tm.tm, o.tm.passed,
                           o.ext, 6, 6)
    assert int(o.tm.passed.sum()) > 0
    assert open(out, "rb").read() == want
