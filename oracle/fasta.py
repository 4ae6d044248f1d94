"""FASTA input and AHv2-format FASTA output, written plainly (test
infrastructure: only the test suite, the smoke check and the benchmark's CPU
baseline leg use it; the product path never does).

What is followed:
* Implementations (AHv2 reads FASTA; its 2-bit batches keep headers, lengths
  and bases) and Discussion (headers kept apart from the bases);
* Supplementary, "Headers and outputs": FASTA output whose header carries
  the record identifier, source file, coordinates, Tm, orientation, the
  matched primer snippets and, when asked for, the barcodes, in the order of
  the paper's example header.

Readings where the paper is silent:
* a record is a line starting with '>' plus the lines up to the next such
  line or the end of the file; records never span files; a file may hold
  only white space before its first header, anything else is not FASTA;
* the identifier is the first white-space-separated word of the header text
  (empty when there is none);
* the sequence is the bytes of the record's other lines with ASCII white
  space (space, tab, LF, CR, VT, FF) removed; bytes other than A/C/G/T in
  either case read as N (the genome store's rule);
* coordinates are 1-based inclusive, start + 1 to end, of the whole amplicon
  (primer sites included) on the plus strand, also when primers are trimmed;
* Tm is printed with two decimals, rounded from the exact binary value, and
  as NA when it is not finite; the amplicon's sequence is one line;
* only amplicons that pass the Tm filter are written when the filter is on,
  in the library's amplicon order.
"""
from __future__ import annotations

import math
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

WHITESPACE = b" \t\n\r\x0b\x0c"
ORIENT = (b"FR", b"RF", b"FF", b"RR")


def read_fasta(paths: Sequence[str]) -> List[Tuple[bytes, int, bytes]]:
    """Records of the files in order: (identifier, file index, raw sequence bytes)."""
    out = []
    for fi, path in enumerate(paths):
        with open(path, "rb") as fh:
            data = fh.read()
        cur = None
        for line in data.split(b"\n"):
            if line.startswith(b">"):
                if cur is not None:
                    out.append(cur)
                words = line[1:].split()
                cur = (words[0] if words else b"", fi, [])
            elif cur is None:
                if line.strip():
                    raise ValueError("%s: data before the first header" % path)
            else:
                cur[2].append(line)
        if cur is not None:
            out.append(cur)
    return [(rid, fi, b"".join(lines).translate(None, WHITESPACE)) for rid, fi, lines in out]


def concat(records) -> Tuple[np.ndarray, np.ndarray]:
    """The records' sequences as one byte buffer plus offsets (n + 1)."""
    seqs = [s for _, _, s in records]
    off = np.zeros(len(seqs) + 1, np.uint64)
    off[1:] = np.cumsum([len(s) for s in seqs])
    buf = np.frombuffer(b"".join(seqs), np.uint8) if off[-1] else np.zeros(0, np.uint8)
    return buf, off


def write_fasta(path: str, records, width: int = 60, crlf: bool = False) -> None:
    """Write (identifier, description, sequence) records with lines of `width` bases."""
    nl = b"\r\n" if crlf else b"\n"
    with open(path, "wb") as fh:
        for rid, desc, seq in records:
            fh.write(b">" + rid + ((b" " + desc) if desc else b"") + nl)
            for i in range(0, len(seq), width):
                fh.write(seq[i:i + width] + nl)


def _cstr(row) -> bytes:
    b = bytes(np.asarray(row, np.uint8))
    return b.split(b"\0", 1)[0]


def tm_text(t: float) -> bytes:
    return b"NA" if not math.isfinite(t) else ("%.2f" % t).encode()


def header(rid: bytes, source: bytes, start: int, end: int, tm: float, orient: int, fprimer: bytes,
           rprimer: bytes, fb: Optional[bytes] = None, rb: Optional[bytes] = None) -> bytes:
    """One header line (without the newline), fields in the paper's order."""
    h = b">%s.source=%s.coordinates=%d-%d.Tm=%s.orientation=%s.fprimer=%s.rprimer=%s" % (
        rid, source, start + 1, end, tm_text(tm), ORIENT[orient], fprimer, rprimer)
    if fb is not None:
        h += b".fb=" + fb
    if rb is not None:
        h += b".rb=" + rb
    return h


def format_fasta(ids: Sequence[bytes], sources: Sequence[bytes], amps: np.ndarray, tm: np.ndarray,
                 passed: Optional[np.ndarray], ext, fb_len: int, rb_len: int) -> bytes:
    """AHv2 FASTA text of a run: amps (n, 5) [seq, start, end, pair, orient],
    tm (n,), passed (n,) or None (no filter), ext = the oracle's extract."""
    out = []
    for i in range(len(amps)):
        if passed is not None and not passed[i]:
            continue
        s, start, end, _, o = (int(x) for x in amps[i])
        fb = bytes(ext.fb[i, :int(ext.bc_len[i, 0])]) if fb_len else None
        rb = bytes(ext.rb[i, :int(ext.bc_len[i, 1])]) if rb_len else None
        out.append(header(ids[s], sources[s], start, end, float(tm[i]), o, _cstr(ext.fprimer[i]),
                          _cstr(ext.rprimer[i]), fb, rb))
        out.append(b"\n" + ext.amplicon(i) + b"\n")
    return b"".join(out)


def source_names(paths: Sequence[str]) -> List[bytes]:
    return [os.fsencode(os.path.basename(p)) for p in paths]
