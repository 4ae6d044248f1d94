"""FASTA record tables and the AHv2 FASTA writer of libah.so against the
oracle's plain reader and formatter, on the CPU (the record table of
ah_fasta_ingest without a store needs no GPU; the writer is host code)."""
import os

import numpy as np
import pytest

import oracle
from oracle import fasta as of
from paper_2511_00170_amd import ah

_ALPHA = np.frombuffer(b"ACGTACGTACGTNacgtnRYKM", np.uint8)


def _random_records(rng, n, max_len, prefix=b"r"):
    recs = []
    for i in range(n):
        L = int(rng.integers(0, max_len + 1)) if rng.random() < 0.9 else 0
        seq = bytes(rng.choice(_ALPHA, L))
        desc = b"len=%d some words" % L if rng.random() < 0.5 else b""
        recs.append((prefix + b"%d" % i, desc, seq))
    return recs


def _write_messy(path, recs, rng):
    """FASTA with mixed line widths, CRLF, blank lines, stray white space."""
    out = [b"\n \t\n"] if rng.random() < 0.5 else []
    for rid, desc, seq in recs:
        nl = b"\r\n" if rng.random() < 0.3 else b"\n"
        lead = b" " if rng.random() < 0.1 else b""
        out.append(b">" + lead + rid + ((b"\t" + desc) if desc else b"") + nl)
        w = int(rng.choice([1, 7, 60, 61, 80, 1000]))
        for j in range(0, len(seq), w):
            line = seq[j:j + w]
            if rng.random() < 0.05 and len(line) > 2:
                line = line[:1] + b" " + line[1:]
            out.append(line + nl)
            if rng.random() < 0.02:
                out.append(nl)
    data = b"".join(out)
    if data.endswith(b"\n") and rng.random() < 0.3:
        data = data.rstrip(b"\r\n")
    with open(path, "wb") as fh:
        fh.write(data)


def _check_table(tab, paths):
    want = of.read_fasta(paths)
    assert tab.n_records == len(want)
    assert tab.ids == [r for r, _, _ in want]
    assert tab.seq_file.tolist() == [fi for _, fi, _ in want]
    assert tab.lengths.tolist() == [len(s) for _, _, s in want]
    assert tab.files == of.source_names(paths)
    blocks = [(len(s) + 63) // 64 for _, _, s in want]
    assert tab.block0.tolist() == np.concatenate([[0], np.cumsum(blocks)[:-1]]).astype(int).tolist()[:len(want)]
    assert tab.n_blocks == sum(blocks) and tab.n_bases == sum(len(s) for _, _, s in want)
    assert tab.max_len == max([len(s) for _, _, s in want], default=0)


@pytest.mark.parametrize("n_threads", [1, 4])
def test_record_table_matches_oracle(tmp_path, n_threads):
    rng = np.random.default_rng(7)
    paths = []
    for k in range(4):
        p = str(tmp_path / ("g%d.fa" % k))
        _write_messy(p, _random_records(rng, int(rng.integers(0, 60)), 3000, prefix=b"f%d_" % k), rng)
        paths.append(p)
    empty = str(tmp_path / "empty.fa")
    open(empty, "wb").close()
    paths.insert(2, empty)
    _check_table(ah.fasta_index(paths, n_threads=n_threads), paths)


def test_record_table_across_read_buffers(tmp_path):
    """Lines and headers that cross the reader's 16 MiB buffers."""
    rng = np.random.default_rng(8)
    p = str(tmp_path / "big.fa")
    long_id = b"x" * ((16 << 20) - 3)
    seq1 = bytes(rng.choice(_ALPHA, (16 << 20) + 4097))
    with open(p, "wb") as fh:
        fh.write(b">" + long_id + b" desc\n" + seq1 + b"\n>b\n" + seq1[:100] + b"\r\n")
    _check_table(ah.fasta_index([p]), [p])


def test_record_table_errors(tmp_path):
    bad = tmp_path / "bad.fa"
    bad.write_bytes(b"\n  ACGT\n>x\nA\n")
    with pytest.raises(ah.AhError) as e:
        ah.fasta_index([str(bad)])
    assert e.value.status == ah.AH_E_FORMAT
    with pytest.raises(ah.AhError) as e:
        ah.fasta_index([str(tmp_path / "missing.fa")])
    assert e.value.status == ah.AH_E_IO
    good = tmp_path / "good.fa"
    good.write_bytes(b">a\nACGT\n")
    for n_threads in (1, 3):                     # an error in any file, any worker
        with pytest.raises(ah.AhError) as e:
            ah.fasta_index([str(good), str(tmp_path / "missing.fa"), str(good)], n_threads=n_threads)
        assert e.value.status == ah.AH_E_IO
        with pytest.raises(ah.AhError) as e:
            ah.fasta_index([str(good), str(good), str(bad)], n_threads=n_threads)
        assert e.value.status == ah.AH_E_FORMAT
    assert ah.fasta_index([]).n_records == 0


def _random_run(rng, n, n_seqs, fb_len, rb_len):
    """Host results of a run (the fields ah_extract produces), random."""
    amps = np.zeros(n, ah.AMP_DTYPE)
    amps["seq"] = rng.integers(0, n_seqs, n)
    amps["start"] = rng.integers(0, 1 << 31, n)
    amps["end"] = amps["start"] + rng.integers(0, 5000, n)
    amps["pair"] = rng.integers(0, 3, n)
    amps["orient"] = rng.integers(0, 4, n)
    tm = rng.uniform(-10, 100, n)
    tm[rng.random(n) < 0.05] = -np.inf
    tm[rng.random(n) < 0.02] = np.nan
    tm[:4] = [60.425, 0.125, -0.004, 45.0][:min(4, n)]
    lens = rng.integers(0, 300, n)
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum(lens)
    seq = bytes(rng.choice(np.frombuffer(b"ACGTN", np.uint8), int(off[-1])))
    fb = rng.choice(np.frombuffer(b"ACGT", np.uint8), (n, max(fb_len, 0)))
    rb = rng.choice(np.frombuffer(b"ACGT", np.uint8), (n, max(rb_len, 0)))
    bc = np.stack([rng.integers(0, fb_len + 1, n), rng.integers(0, rb_len + 1, n)], 1).astype(np.uint8)
    fp = np.zeros((n, 32), np.uint8)
    rp = np.zeros((n, 32), np.uint8)
    for i in range(n):
        a, b = int(rng.integers(0, 33)), int(rng.integers(1, 33))
        fp[i, :a] = rng.choice(np.frombuffer(b"ACGT", np.uint8), a)
        rp[i, :b] = rng.choice(np.frombuffer(b"ACGT", np.uint8), b)
    passed = (rng.random(n) < 0.7).astype(np.uint8)
    res = {"amps": amps, "tm": tm, "pass": passed, "seq": seq, "seq_off": off, "fb": fb, "rb": rb, "bc_len": bc,
           "fprimer": fp, "rprimer": rp}
    ext = oracle.Extracted(seq, off, fb, rb, bc, fp, rp, np.zeros(n, np.uint8))
    return res, ext


@pytest.mark.parametrize("fb_len,rb_len", [(0, 0), (8, 0), (5, 12)])
def test_writer_matches_oracle(fb_len, rb_len):
    rng = np.random.default_rng(100 + fb_len + rb_len)
    n_seqs = 23
    ids = [b"seq%d" % i if i % 5 else b"" for i in range(n_seqs)]
    files = [b"GCF_000001.fa", b"b.fasta", b"c"]
    seq_file = rng.integers(0, len(files), n_seqs)
    names = ah.FastaNames(ids, seq_file, files)
    res, ext = _random_run(rng, 400, n_seqs, fb_len, rb_len)
    srcs = [files[int(f)] for f in seq_file]
    amps5 = ah.amps_array(res["amps"])
    for filt in (True, False):
        got = ah.format_fasta(names, res, fb_len, rb_len, tm_filter=filt)
        want = of.format_fasta(ids, srcs, amps5, res["tm"], res["pass"] if filt else None, ext, fb_len, rb_len)
        assert got == want
    # an empty run writes nothing
    empty = {k: v[:0] for k, v in res.items() if k != "seq"}
    empty["seq"], empty["seq_off"] = b"", np.zeros(1, np.uint64)
    assert ah.format_fasta(names, empty, fb_len, rb_len) == b""


def test_writer_with_oracle_run_and_fasta_names(tmp_path):
    """Records of a real (oracle) run named from an ingested record table."""
    from paper_2511_00170_amd import synth
    wl = synth.gen_config(1, n_seqs=30)
    buf, off = wl.concat()
    recs = [(b"chr%d" % i, b"", bytes(buf[int(off[i]):int(off[i + 1])])) for i in range(wl.n_seqs)]
    p1, p2 = str(tmp_path / "one.fa"), str(tmp_path / "two.fa")
    of.write_fasta(p1, recs[:12], width=70)
    of.write_fasta(p2, recs[12:], width=61, crlf=True)
    tab = ah.fasta_index([p1, p2])
    ex = synth.ExtractSpec(trim=True, fb_len=6, rb_len=4)
    o = oracle.run(buf, off, wl.pairs, wl.orient_mask, wl.tm, ex)
    assert len(o.amps) > 0
    res = {"amps": np.zeros(len(o.amps), ah.AMP_DTYPE), "tm": o.tm.tm, "pass": o.tm.passed, "seq": o.ext.seq,
           "seq_off": o.ext.seq_off, "fb": o.ext.fb, "rb": o.ext.rb, "bc_len": o.ext.bc_len,
           "fprimer": o.ext.fprimer, "rprimer": o.ext.rprimer}
    for j, name in enumerate(["seq", "start", "end", "pair", "orient"]):
        res["amps"][name] = o.amps[:, j]
    got = ah.format_fasta(tab, res, 6, 4, tm_filter=wl.tm.filter)
    want = of.format_fasta(tab.ids, [tab.files[int(f)] for f in tab.seq_file], o.amps, o.tm.tm,
                           o.tm.passed if wl.tm.filter else None, o.ext, 6, 4)
    assert got == want and got.count(b"\n>") + 1 == int(o.tm.passed.sum() if wl.tm.filter else len(o.amps))


def test_writer_rejects_bad_records():
    names = ah.FastaNames([b"a"], [0], [b"f.fa"])
    rng = np.random.default_rng(5)
    res, _ = _random_run(rng, 3, 1, 0, 0)
    res["amps"]["seq"][1] = 1
    with pytest.raises(ah.AhError):
        ah.format_fasta(names, res, 0, 0)
    res["amps"]["seq"][1] = 0
    res["amps"]["orient"][2] = 4
    with pytest.raises(ah.AhError):
        ah.format_fasta(names, res, 0, 0)


def test_cli_flags(tmp_path):
    from paper_2511_00170_amd import cli
    lst = tmp_path / "inputs.txt"
    lst.write_text("a.fa\n\nb.fa\n")
    a = cli.parse_args(["--input", "x.fa", "--input-list", str(lst), "--forward", "ACGT", "--reverse", "TTGG",
                        "--include-offtarget", "--trim-primers", "--fb-len", "4"])
    assert a.input == ["x.fa", "a.fa", "b.fa"] and a.include_offtarget and a.trim_primers and a.fb_len == 4
    assert a.tm_threshold is None and a.mismatches == 0
    with pytest.raises(SystemExit):
        cli.parse_args(["--forward", "ACGT", "--reverse", "TTGG"])
