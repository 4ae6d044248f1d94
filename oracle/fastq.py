"""FASTQ input with quality propagation and FASTQ output, written plainly
(test infrastructure: only the test suite uses it; the product path never
does).

What is followed:
* Discussion: FASTQ input with the qualities carried to the amplicons, for
  amplicon sequencing reads (the Python AHv1.1 reads FASTQ);
* Supplementary, "Headers and outputs": the header fields of FASTA output,
  here after "@".

Readings where the paper is silent:
* a record is four lines: "@" and a header, the bases, a line starting with
  "+" (the rest ignored), the qualities; lines end in LF or CR LF; empty
  lines between records are skipped; a record wrapped over several lines,
  a quality line of another length than its bases, a quality byte outside
  '!'..'~' or a base byte outside '!'..'~' is not FASTQ;
* the identifier is the first white-space-separated word of the header;
* bases other than A/C/G/T in either case read as N (the store's rule);
* an amplicon's qualities are those of the read bases it is made of, in the
  order of its written bases: forward, or reversed for RF, whose bases are
  reverse-complemented (a quality has no complement); trimming drops the
  primer sites' qualities with their bases;
* a record is written as its FASTA record with "@" for ">", then "+" and the
  qualities on one line.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import fasta as _fa


def _lines(data: bytes):
    for line in data.split(b"\n"):
        yield line[:-1] if line.endswith(b"\r") else line


def read_fastq(paths: Sequence[str]) -> List[Tuple[bytes, int, bytes, bytes]]:
    """Records of the files in order: (identifier, file index, bases, qualities)."""
    out = []
    for fi, path in enumerate(paths):
        with open(path, "rb") as fh:
            data = fh.read()
        if data.endswith(b"\n"):
            data = data[:-1]  # the final line end closes the last line
        it = iter(_lines(data)) if data else iter(())
        for head in it:
            if head == b"":
                continue
            if not head.startswith(b"@"):
                raise ValueError("%s: a record must start with '@'" % path)
            try:
                bases, plus, qual = next(it), next(it), next(it)
            except StopIteration:
                raise ValueError("%s: incomplete record" % path) from None
            if not plus.startswith(b"+") or len(qual) != len(bases):
                raise ValueError("%s: malformed record" % path)
            if any(c < 0x21 or c > 0x7E for c in qual) or any(c < 0x21 or c > 0x7E for c in bases):
                raise ValueError("%s: byte outside '!'..'~'" % path)
            words = head[1:].split()  # ASCII white space, as in the header rule
            out.append((words[0] if words else b"", fi, bases, qual))
    return out


def concat(records) -> Tuple[np.ndarray, np.ndarray]:
    """The records' bases as one byte buffer plus offsets (n + 1)."""
    return _fa.concat([(r[0], r[1], r[2]) for r in records])


def write_fastq(path: str, records, crlf: bool = False, plus_id: bool = False) -> None:
    """Write (identifier, description, bases, qualities) records, four lines each."""
    nl = b"\r\n" if crlf else b"\n"
    with open(path, "wb") as fh:
        for rid, desc, bases, qual in records:
            fh.write(b"@" + rid + ((b" " + desc) if desc else b"") + nl + bases + nl)
            fh.write(b"+" + (rid if plus_id else b"") + nl + qual + nl)


def amplicon_qualities(quals: Sequence[bytes], pairs, amps: np.ndarray, trim: bool,
                       passed: Optional[np.ndarray] = None) -> List[bytes]:
    """Per amplicon (seq, start, end, pair, orient) the qualities of its written
    bases; empty for one that did not pass."""
    out = []
    for i, (s, start, end, q, o) in enumerate(np.asarray(amps, np.int64).tolist()):
        if passed is not None and not passed[i]:
            out.append(b"")
            continue
        up = pairs[q].fwd if o in (0, 2) else pairs[q].rev      # upstream site: FR/FF forward, RF/RR reverse
        down = pairs[q].rev if o in (0, 3) else pairs[q].fwd    # downstream: FR/RR reverse, RF/FF forward
        a0, a1 = (start + len(up), max(end - len(down), start + len(up))) if trim else (start, end)
        qa = quals[s][a0:a1]
        out.append(qa[::-1] if o == 1 else qa)
    return out


def format_fastq(ids: Sequence[bytes], sources: Sequence[bytes], amps: np.ndarray, tm: np.ndarray,
                 passed: Optional[np.ndarray], ext, quals: Sequence[bytes], fb_len: int, rb_len: int) -> bytes:
    """FASTQ text of a run: the oracle's FASTA records with '@' headers, then
    '+' and each amplicon's qualities (amplicon_qualities)."""
    out = []
    for i in range(len(amps)):
        if passed is not None and not passed[i]:
            continue
        s, start, end, _, o = (int(x) for x in amps[i])
        fb = bytes(ext.fb[i, :int(ext.bc_len[i, 0])]) if fb_len else None
        rb = bytes(ext.rb[i, :int(ext.bc_len[i, 1])]) if rb_len else None
        h = _fa.header(ids[s], sources[s], start, end, float(tm[i]), o, _fa._cstr(ext.fprimer[i]),
                       _fa._cstr(ext.rprimer[i]), fb, rb)
        out.append(b"@" + h[1:] + b"\n" + ext.amplicon(i) + b"\n+\n" + quals[i] + b"\n")
    return b"".join(out)
