"""Plain CPU oracle (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline leg may import this package.  The GPU product path never touches
it; the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, compiled by ``build()`` or on
first import).  This module marshals numpy arrays into it and returns
records as numpy structured data:

* hits      (n, 4) uint32 ``[seq, pos, pair, kind]`` + ``mm`` (n,) -- order
            (seq, pair, pos, kind), kind bit0 = reverse primer, bit1 = minus;
* amplicons (n, 5) uint32 ``[seq, start, end, pair, orient]`` in the
            canonical order (seq, pair, downstream site start, end, primer).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

PARITY_UNPINNED = (
    "the numeric values of the terminal-mismatch stacks (only a physical range is checked: every "
    "entry but GG/CG is stabilising)",
    "the numeric values of the dangling-end parameters other than .C/TG and CG/.C (only a range is checked)",
    "the three tandem G.T stacks GG/TT, GT/TG, TG/GT (no printed free energy at hand)",
)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU, no HIP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        P = C.POINTER
        L.or_primer_masks.argtypes = [C.c_char_p, P(C.c_uint8)]
        L.or_primer_revcomp.argtypes = [C.c_char_p, C.c_char_p]
        L.or_scan.restype = C.c_int64
        L.or_scan.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_uint32, C.c_void_p, C.c_uint64, C.c_int]
        L.or_pair.restype = C.c_int64
        L.or_pair.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_uint32, C.c_uint32, C.c_void_p, C.c_uint64]
        L.or_nn_thermo.restype = C.c_int
        L.or_nn_thermo.argtypes = [C.c_char_p, C.c_char_p, C.c_int, C.c_int, P(C.c_double), P(C.c_double)]
        L.or_nn_table.restype = C.c_int
        L.or_nn_table.argtypes = [C.c_int, C.c_int, C.c_char_p, P(C.c_double), C.c_int]
        L.or_nn_init.restype = C.c_int
        L.or_nn_init.argtypes = [C.c_int, P(C.c_double)]
        L.or_salt_correction.restype = C.c_int
        L.or_salt_correction.argtypes = [C.c_void_p, C.c_char_p, P(C.c_double), P(C.c_int)]
        L.or_tm_duplex.restype = C.c_double
        L.or_tm_duplex.argtypes = [C.c_char_p, C.c_char_p, C.c_int, C.c_void_p, P(C.c_int)]
        L.or_tm_amps.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                 C.c_double, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.or_extract.restype = C.c_int64
        L.or_extract.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                 C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


class _TmCond(C.Structure):
    _fields_ = [("na", C.c_double), ("k", C.c_double), ("tris", C.c_double), ("mg", C.c_double),
                ("dntps", C.c_double), ("dnac1", C.c_double), ("dnac2", C.c_double), ("saltcorr", C.c_int),
                ("nn_table", C.c_int)]


def _cond(tm) -> _TmCond:
    return _TmCond(tm.na_mM, tm.k_mM, tm.tris_mM, tm.mg_mM, tm.dntps_mM, tm.dnac1_nM, tm.dnac2_nM, tm.saltcorr,
                   int(getattr(tm, "nn_table", 3)))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _primer_array(pairs) -> tuple:
    strs = []
    for p in pairs:
        strs += [p.fwd.encode(), p.rev.encode()]
    arr = (C.c_char_p * len(strs))(*strs)
    return arr, strs


def n_threads_default() -> int:
    """The CPUs this process may run on, capped by the OpenMP thread setting
    (the host's share of a shared machine)."""
    n = len(os.sched_getaffinity(0))
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS") or n))
    except ValueError:
        pass
    return max(1, n)


# ---------------------------------------------------------------- primers
def primer_masks(primer: str) -> np.ndarray:
    m = (C.c_uint8 * 32)()
    L = lib().or_primer_masks(primer.encode(), m)
    if L < 0:
        raise ValueError("bad primer %r (%d)" % (primer, L))
    return np.frombuffer(bytes(m), np.uint8)[:L].copy()


def primer_revcomp(primer: str) -> str:
    buf = C.create_string_buffer(len(primer) + 1)
    if lib().or_primer_revcomp(primer.encode(), buf) < 0:
        raise ValueError(primer)
    return buf.value.decode()


# ---------------------------------------------------------------- scan
def scan(ascii: np.ndarray, off: np.ndarray, pairs, n_threads: Optional[int] = None):
    """All hits (order seq, pair, pos, kind).  Returns (hits[n,4] u32, mm[n] u8)."""
    ascii = np.ascontiguousarray(ascii, np.uint8)
    off = np.ascontiguousarray(off, np.uint64)
    n_seqs = len(off) - 1
    arr, keep = _primer_array(pairs)
    k = np.array([p.k for p in pairs], np.int32)
    c = np.array([p.clamp for p in pairs], np.int32)
    nt = n_threads or n_threads_default()
    cap = 1 << 16
    while True:
        out = np.zeros((cap, 4), np.uint32)
        n = lib().or_scan(_ptr(ascii), _ptr(off), n_seqs, C.cast(arr, C.c_void_p), _ptr(k), _ptr(c),
                          len(pairs), _ptr(out), cap, nt)
        if n < 0:
            raise ValueError("oracle scan: bad primer or parameters (%d)" % n)
        if n <= cap:
            break
        cap = int(n)
    out = out[:n]
    mm = (out[:, 3] >> 8).astype(np.uint8)
    out[:, 3] &= 0xFF
    return out, mm


# ---------------------------------------------------------------- pair
def pair(hits: np.ndarray, pairs, orient_mask: int) -> np.ndarray:
    hits = np.ascontiguousarray(hits, np.uint32)
    Lf = np.array([len(p.fwd) for p in pairs], np.int32)
    Lr = np.array([len(p.rev) for p in pairs], np.int32)
    mn = np.array([p.min_len for p in pairs], np.uint32)
    mx = np.array([p.max_len for p in pairs], np.uint32)
    cap = max(1024, len(hits))
    while True:
        out = np.zeros((cap, 5), np.uint32)
        n = lib().or_pair(_ptr(hits), len(hits), _ptr(Lf), _ptr(Lr), _ptr(mn), _ptr(mx), len(pairs),
                          orient_mask, _ptr(out), cap)
        if n <= cap:
            return out[:n]
        cap = int(n)


# ---------------------------------------------------------------- Tm
def nn_thermo(seq: str, cseq: str, shift: int = 0, table: int = 3):
    """(dH kcal/mol, dS cal/K/mol) before salt correction, or None if untabulated.
    cseq is the partner strand written 3'->5'; cseq[i] faces seq[i - shift]."""
    dh, ds = C.c_double(0), C.c_double(0)
    st = lib().or_nn_thermo(seq.encode(), cseq.encode(), int(shift), int(table), C.byref(dh), C.byref(ds))
    if st == 2:
        raise ValueError("bad duplex")
    return None if st == 1 else (dh.value, ds.value)


def nn_table(which: str, table: int = 3):
    """Parameter table as {key: (dH, dS)}: which = "wc" (Watson-Crick set
    `table`), "imm" (internal mismatches), "tmm" (terminal mismatches), "de"
    (dangling ends)."""
    w = {"wc": 0, "imm": 1, "tmm": 2, "de": 3}[which]
    keys = C.create_string_buffer(6 * 64)
    vals = (C.c_double * 128)()
    n = lib().or_nn_table(w, int(table), keys, vals, 64)
    if n < 0:
        raise ValueError((which, table))
    raw = keys.raw
    return {raw[6 * i:6 * i + 5].decode(): (vals[2 * i], vals[2 * i + 1]) for i in range(n)}


def nn_init(table: int = 3) -> dict:
    """Initiation terms of a Watson-Crick set: {name: (dH, dS)}."""
    v = (C.c_double * 10)()
    if lib().or_nn_init(int(table), v) < 0:
        raise ValueError(table)
    names = ("init", "terminal_AT", "terminal_GC", "one_GC", "all_AT")
    return {n: (v[2 * i], v[2 * i + 1]) for i, n in enumerate(names)}


def salt_correction(tm, seq: str):
    """(correction, kind): kind 1 = added to Tm (C), 5 = added to dS,
    6 = added to 1/Tm (1/K), 0 = none.  ValueError for zero concentrations."""
    cond = _cond(tm)
    corr, kind = C.c_double(0), C.c_int(0)
    if lib().or_salt_correction(C.byref(cond), seq.encode(), C.byref(corr), C.byref(kind)):
        raise ValueError("salt correction %d undefined for these concentrations" % tm.saltcorr)
    return corr.value, kind.value


def tm_duplex(seq: str, cseq: str, tm, shift: int = 0) -> float:
    st = C.c_int(0)
    cond = _cond(tm)
    v = lib().or_tm_duplex(seq.encode(), cseq.encode(), int(shift), C.byref(cond), C.byref(st))
    if st.value == 2:
        raise ValueError("bad duplex")
    return float("nan") if st.value == 1 else v


@dataclass
class TmResult:
    tm: np.ndarray
    tm_site: np.ndarray
    passed: np.ndarray
    skipped: np.ndarray


def tm_amps(ascii, off, pairs, amps: np.ndarray, tm, n_threads: Optional[int] = None) -> TmResult:
    amps = np.ascontiguousarray(amps, np.uint32)
    n = len(amps)
    arr, keep = _primer_array(pairs)
    out_tm = np.zeros(n, np.float64)
    out_site = np.zeros((n, 2), np.float64)
    out_pass = np.zeros(n, np.uint8)
    skipped = np.zeros((n, 2), np.uint32)
    cond = _cond(tm)
    lib().or_tm_amps(_ptr(np.ascontiguousarray(ascii, np.uint8)), _ptr(np.ascontiguousarray(off, np.uint64)),
                     C.cast(arr, C.c_void_p), _ptr(amps), n, C.byref(cond), tm.threshold_C, int(tm.filter),
                     _ptr(out_tm), _ptr(out_site), _ptr(out_pass), _ptr(skipped), n_threads or n_threads_default())
    return TmResult(out_tm, out_site, out_pass, skipped)


# ---------------------------------------------------------------- extract
@dataclass
class Extracted:
    seq: bytes
    seq_off: np.ndarray
    fb: np.ndarray
    rb: np.ndarray
    bc_len: np.ndarray
    fprimer: np.ndarray
    rprimer: np.ndarray
    flags: np.ndarray       # 1 where a barcode was clipped at a sequence end

    def amplicon(self, i: int) -> bytes:
        return self.seq[int(self.seq_off[i]):int(self.seq_off[i + 1])]


def extract(ascii, off, pairs, amps: np.ndarray, ex, passed: Optional[np.ndarray] = None) -> Extracted:
    amps = np.ascontiguousarray(amps, np.uint32)
    n = len(amps)
    arr, keep = _primer_array(pairs)
    ascii = np.ascontiguousarray(ascii, np.uint8)
    off = np.ascontiguousarray(off, np.uint64)
    fb = np.zeros((n, max(ex.fb_len, 1)), np.uint8)
    rb = np.zeros((n, max(ex.rb_len, 1)), np.uint8)
    bc = np.zeros((n, 2), np.uint8)
    fp = np.zeros((n, 32), np.uint8)
    rp = np.zeros((n, 32), np.uint8)
    so = np.zeros(n + 1, np.uint64)
    fl = np.zeros(max(n, 1), np.uint8)
    pas = None if passed is None else np.ascontiguousarray(passed, np.uint8)
    cap = 1 << 20
    while True:
        buf = np.zeros(cap, np.uint8)
        tot = lib().or_extract(_ptr(ascii), _ptr(off), C.cast(arr, C.c_void_p), _ptr(amps), n,
                               None if pas is None else _ptr(pas), int(ex.trim), ex.fb_len, ex.rb_len,
                               _ptr(buf), cap, _ptr(so), _ptr(fb), _ptr(rb), _ptr(bc), _ptr(fp), _ptr(rp), _ptr(fl))
        if tot <= cap:
            break
        cap = int(tot)
    return Extracted(buf[:tot].tobytes(), so, fb[:, :ex.fb_len], rb[:, :ex.rb_len], bc, fp, rp, fl[:n])


# ---------------------------------------------------------------- pipeline
@dataclass
class Result:
    hits: np.ndarray
    mm: np.ndarray
    amps: np.ndarray
    tm: TmResult
    ext: Optional[Extracted]


def run(ascii, off, pairs, orient_mask, tm, ex=None, n_threads=None) -> Result:
    """The whole path: scan -> pair -> Tm -> extract."""
    hits, mm = scan(ascii, off, pairs, n_threads)
    amps = pair(hits, pairs, orient_mask)
    t = tm_amps(ascii, off, pairs, amps, tm, n_threads)
    e = extract(ascii, off, pairs, amps, ex, t.passed if tm.filter else None) if ex is not None else None
    return Result(hits, mm, amps, t, e)
