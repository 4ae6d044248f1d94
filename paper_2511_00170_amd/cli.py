"""Command line: FASTA genomes in, AHv2-format amplicon FASTA out (or FASTQ
reads in, amplicon FASTQ with their qualities out).

    python -m paper_2511_00170_amd.cli --input g1.fa g2.fa --forward F --reverse R \\
        --mismatches 3 --clamp 5 --min-length 200 --max-length 2000 \\
        [--include-offtarget] [--trim-primers] [--fb-len N] [--rb-len N] \\
        [--tm-threshold 45] [--input-fq] [--output amplicons.fa]

The flags follow the tool's own (Supplementary, "Amplicon calling and
orientation" and "Primer trimming and barcode extraction"): FR and RF
amplicons by default, FF/RR too with --include-offtarget; --trim-primers
removes the primer sites from the written sequence; --fb-len/--rb-len cut
barcodes; --input-fq reads FASTQ and writes each amplicon with the
qualities of its bases.  Every sequence and primer pair runs through the GPU
path (ah_fasta_ingest or ah_fastq_read, scan, pair, Tm, extract, and
ah_extract_qual for FASTQ); the records are written by ah_fasta_format or
ah_fastq_format.
"""
from __future__ import annotations

import argparse
import sys
import time

from . import synth


def parse_args(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2511_00170_amd.cli", description=__doc__.split("\n\n")[0])
    ap.add_argument("--input", nargs="+", default=[], help="FASTA files (genomes)")
    ap.add_argument("--input-list", help="text file with one FASTA path per line (added to --input)")
    ap.add_argument("--forward", required=True, help="forward primer, 5'->3', IUPAC codes")
    ap.add_argument("--reverse", required=True, help="reverse primer, 5'->3', IUPAC codes")
    ap.add_argument("--mismatches", type=int, default=0, help="substitutions allowed per primer site (k)")
    ap.add_argument("--clamp", type=int, default=5, help="3'-terminal primer positions that must match exactly")
    ap.add_argument("--min-length", type=int, default=50, help="shortest amplicon, primers included")
    ap.add_argument("--max-length", type=int, default=5000, help="longest amplicon, primers included")
    ap.add_argument("--include-offtarget", action="store_true", help="also write FF and RR amplicons")
    ap.add_argument("--trim-primers", action="store_true", help="remove the primer sites from the sequence")
    ap.add_argument("--fb-len", type=int, default=0, help="forward barcode length (bases upstream)")
    ap.add_argument("--rb-len", type=int, default=0, help="reverse barcode length (bases downstream)")
    ap.add_argument("--tm-threshold", type=float, default=None,
                    help="write only amplicons whose Tm (the lower of the two sites) is at least this, in C")
    ap.add_argument("--na-mM", type=float, default=50.0)
    ap.add_argument("--k-mM", type=float, default=0.0)
    ap.add_argument("--tris-mM", type=float, default=0.0)
    ap.add_argument("--mg-mM", type=float, default=0.0)
    ap.add_argument("--dntps-mM", type=float, default=0.0)
    ap.add_argument("--dnac1-nM", type=float, default=250.0, help="primer strand concentration")
    ap.add_argument("--dnac2-nM", type=float, default=0.0, help="template strand concentration")
    ap.add_argument("--saltcorr", type=int, default=5, help="salt correction method 0-7 (Tm_NN's numbering)")
    ap.add_argument("--input-fq", action="store_true",
                    help="the inputs are FASTQ; write FASTQ with each amplicon's qualities")
    ap.add_argument("--output", default="-", help="output FASTA or FASTQ ('-' = standard output)")
    ap.add_argument("--chunk-mb", type=int, default=64, help="staging chunk for FASTA ingest, MiB")
    ap.add_argument("--quiet", action="store_true")
    a = ap.parse_args(argv)
    if a.input_list:
        with open(a.input_list) as fh:
            a.input += [ln.strip() for ln in fh if ln.strip()]
    if not a.input:
        ap.error("no input files")
    return a


def main(argv=None) -> int:
    a = parse_args(argv)
    import torch

    from . import ah
    if not torch.cuda.is_available():
        print("error: no GPU visible (the path runs only on the GPU)", file=sys.stderr)
        return 2
    t0 = time.perf_counter()
    pair = synth.PairSpec(a.forward, a.reverse, k=a.mismatches, clamp=a.clamp, min_len=a.min_length,
                          max_len=a.max_length)
    tm = synth.TmSpec(na_mM=a.na_mM, k_mM=a.k_mM, tris_mM=a.tris_mM, mg_mM=a.mg_mM, dntps_mM=a.dntps_mM,
                      dnac1_nM=a.dnac1_nM, dnac2_nM=a.dnac2_nM, saltcorr=a.saltcorr,
                      threshold_C=a.tm_threshold if a.tm_threshold is not None else 0.0,
                      filter=a.tm_threshold is not None)
    ex = synth.ExtractSpec(trim=a.trim_primers, fb_len=a.fb_len, rb_len=a.rb_len)
    orient = 0b1111 if a.include_offtarget else 0b0011
    if a.input_fq:
        store = ah.Store.from_fastq(a.input)
    else:
        store = ah.Store.from_fasta(a.input, chunk_bytes=a.chunk_mb << 20)
    t1 = time.perf_counter()
    res = ah.Pipeline(store, ah.PrimerSet([pair], jit=True), orient, tm, ex).run().results()
    t2 = time.perf_counter()
    fmt = ah.format_fastq if a.input_fq else ah.format_fasta
    text = fmt(store.fasta, res, ex.fb_len, ex.rb_len, tm_filter=tm.filter)
    if a.output == "-":
        sys.stdout.buffer.write(text)
        sys.stdout.buffer.flush()
    else:
        with open(a.output, "wb") as fh:
            fh.write(text)
    t3 = time.perf_counter()
    if not a.quiet:
        n_out = res["pass"].astype(bool).sum() if tm.filter else len(res["amps"])
        print("%d files, %d sequences, %.3f Gbases; %d amplicons, %d written; ingest %.2f s, path %.2f s, "
              "write %.2f s" % (len(a.input), store.n_seqs, store.total_bases / 1e9, len(res["amps"]), n_out,
                                t1 - t0, t2 - t1, t3 - t2), file=sys.stderr)
    return 0


if __name__ == "__main__":
    sys.exit(main())
