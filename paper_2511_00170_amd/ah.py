"""Thin Python binding of libah.so (ctypes).

Argument marshalling only: every step of the path runs in the HIP kernels of
libah.so.  PyTorch provides device memory and streams.  If the library has
not been built this module raises at import time -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libah.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libah.so is not built (run `python -m paper_2511_00170_amd.build`): %s" % LIB_PATH)

_lib = C.CDLL(LIB_PATH)

AH_OK, AH_E_ARG, AH_E_ALPHABET, AH_E_LIMIT, AH_E_HIP, AH_E_WORKSPACE, AH_E_IO, AH_E_FORMAT = 0, 1, 2, 3, 4, 5, 6, 7
AH_E_SCRATCH = 8
STATIC_SCAN_MAX_LIST = 65536
AH_STORE_SCRATCH = 2048
ORIENT_ALL = 0xF

VP = C.c_void_p
U32, U64, I32 = C.c_uint32, C.c_uint64, C.c_int32


class AhError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.ah_status_str(status).decode()
        super().__init__("%s: %s (status %d)" % (where, msg, status))
        self.status = status


class ah_store(C.Structure):
    _fields_ = [("n_seqs", U32), ("max_len", U32), ("n_blocks", U64),
                ("d_blocks", VP), ("d_seq_block0", VP), ("d_seq_len", VP),
                ("d_nbits", VP), ("d_nrank", VP), ("d_nmask", VP), ("nmask_cap", U64),
                ("d_counters", VP)]


class ah_pair_spec(C.Structure):
    _fields_ = [("fwd", C.c_char_p), ("rev", C.c_char_p), ("k", U32), ("clamp", U32),
                ("min_len", U32), ("max_len", U32)]


class ah_tm_params(C.Structure):
    _fields_ = [("na_mM", C.c_double), ("k_mM", C.c_double), ("tris_mM", C.c_double), ("mg_mM", C.c_double),
                ("dntps_mM", C.c_double), ("dnac1_nM", C.c_double), ("dnac2_nM", C.c_double),
                ("threshold_C", C.c_double), ("saltcorr", I32), ("filter", I32), ("d_pair_threshold", VP),
                ("nn_table", I32), ("reserved", I32)]


class ah_extract_opts(C.Structure):
    _fields_ = [("trim", U32), ("fb_len", U32), ("rb_len", U32)]


class ah_pack_piece(C.Structure):
    _fields_ = [("src", U64), ("block", U64), ("n", U32), ("reserved", U32)]


class ah_fasta_names(C.Structure):
    _fields_ = [("ids", VP), ("id_off", VP), ("seq_file", VP), ("files", VP), ("n_seqs", U32), ("n_files", U32)]


def _sig(name, restype, *args):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(args)
    return f


_lib.ah_status_str.restype = C.c_char_p
_lib.ah_status_str.argtypes = [I32]
_sig("ah_version", C.c_int)
_sig("ah_pack_layout", I32, VP, U32, VP, C.POINTER(U64))
_sig("ah_pack_begin", I32, C.POINTER(ah_store), VP)
_sig("ah_pack", I32, C.POINTER(ah_store), VP, VP, U32, U32, VP, U64, VP)
_sig("ah_pack_finish", I32, C.POINTER(ah_store), VP, U64, VP)
_sig("ah_unpack", I32, C.POINTER(ah_store), U32, U64, U64, VP, VP)
_sig("ah_pack_pieces", I32, VP, U64, VP, VP, VP, VP, U32, VP, U64, VP)
_sig("ah_read_probe", I32, VP, U64, VP, U32, VP)
_sig("ah_fasta_ws_size", I32, U64, C.POINTER(U64))
_sig("ah_fasta_ingest", I32, C.POINTER(C.c_char_p), U32, VP, U64, VP, VP, VP, U64, U64, U32, VP, U64, VP,
     C.POINTER(VP))
_sig("ah_fasta_info", I32, VP, C.POINTER(U32), C.POINTER(U64), C.POINTER(U64), C.POINTER(U32))
_sig("ah_fasta_table", I32, VP, VP, VP)
_sig("ah_fasta_names_of", I32, VP, C.POINTER(ah_fasta_names))
_sig("ah_fasta_free", None, VP)
_sig("ah_fasta_format", I32, C.POINTER(ah_fasta_names), U32, U32, VP, U64, VP, VP, VP, VP, VP, VP, VP, VP, VP, VP,
     U64, C.POINTER(U64))
_sig("ah_fastq_read", I32, C.POINTER(C.c_char_p), U32, C.POINTER(VP))
_sig("ah_fastq_bases", I32, VP, C.POINTER(VP), C.POINTER(VP))
_sig("ah_fastq_qual_layout", I32, VP, VP, U64)
_sig("ah_fastq_format", I32, C.POINTER(ah_fasta_names), U32, U32, VP, U64, VP, VP, VP, VP, VP, VP, VP, VP, VP, VP,
     VP, U64, C.POINTER(U64))
_sig("ah_primers_compile", I32, C.POINTER(ah_pair_spec), U32, C.POINTER(VP))
_sig("ah_primers_free", None, VP)
_sig("ah_primers_compile_into", I32, C.POINTER(ah_pair_spec), U32, VP, U64, VP, C.POINTER(VP))
_sig("ah_primers_table_bytes", U64, U32)
_sig("ah_primers_count", U32, VP)
_sig("ah_primers_jit", I32, VP)
_sig("ah_primers_jit_check", I32, C.POINTER(ah_pair_spec), U32, C.c_char_p, U32, U32)
_sig("ah_primers_jit_variant", I32, VP, U32, U32)
_sig("ah_primers_use_jit", I32, VP, I32)
_sig("ah_primers_launch_shape", I32, VP, I32, C.POINTER(I32))
_sig("ah_scan_ws_size", I32, C.POINTER(ah_store), U32, C.POINTER(U64))
_sig("ah_scan_primers", I32, C.POINTER(ah_store), VP, VP, U32, VP, U64, VP, VP, U64, VP)
_sig("ah_scan_primers_static", I32, C.POINTER(ah_store), VP, VP, U32, VP, U64, VP, VP)
_sig("ah_scan_primers_masked", I32, C.POINTER(ah_store), VP, VP, U32, VP, VP, U64, VP, VP, U64, VP)
_sig("ah_route_hits", I32, VP, VP, U64, U32, VP, VP, VP, U32, U32, VP, U64, VP, VP)
_sig("ah_pair_ws_size", I32, C.POINTER(ah_store), VP, U64, C.POINTER(U64))
_sig("ah_pair_amplicons", I32, C.POINTER(ah_store), VP, VP, VP, U64, U32, VP, U64, VP, VP, U64, VP)
_sig("ah_tm_nn", I32, C.POINTER(ah_store), VP, VP, VP, U64, C.POINTER(ah_tm_params), VP, VP, VP, VP)
_sig("ah_tm_duplex", I32, VP, VP, VP, VP, VP, U32, U32, C.POINTER(ah_tm_params), VP, VP)
_sig("ah_extract_ws_size", I32, U64, C.POINTER(U64))
_sig("ah_extract", I32, C.POINTER(ah_store), VP, VP, VP, U64, VP, C.POINTER(ah_extract_opts), VP, U64, VP, VP, VP,
     VP, VP, VP, VP, VP, U64, VP)
_sig("ah_extract_qual", I32, C.POINTER(ah_store), VP, U64, VP, VP, VP, U64, VP, C.POINTER(ah_extract_opts), VP, VP,
     U64, VP)

EXPORTED = ["ah_status_str", "ah_version", "ah_pack_layout", "ah_pack_begin", "ah_pack", "ah_pack_finish",
            "ah_unpack", "ah_primers_compile", "ah_primers_compile_into", "ah_primers_table_bytes", "ah_primers_free", "ah_primers_count", "ah_primers_jit", "ah_primers_jit_check", "ah_primers_jit_variant", "ah_primers_use_jit",
            "ah_primers_launch_shape", "ah_scan_ws_size",
            "ah_scan_primers", "ah_scan_primers_static", "ah_scan_primers_masked", "ah_route_hits", "ah_pair_ws_size", "ah_pair_amplicons", "ah_tm_nn", "ah_tm_duplex",
            "ah_extract_ws_size", "ah_extract", "ah_pack_pieces", "ah_fasta_ws_size", "ah_fasta_ingest",
            "ah_fasta_info", "ah_fasta_table", "ah_fasta_names_of", "ah_fasta_free", "ah_fasta_format",
            "ah_fastq_read", "ah_fastq_bases", "ah_fastq_qual_layout", "ah_extract_qual", "ah_fastq_format",
            "ah_read_probe"]

HIT_DTYPE = np.dtype([("seq", "<u4"), ("pos", "<u4"), ("pair", "<u2"), ("kind", "u1"), ("mm", "u1")])
AMP_DTYPE = np.dtype([("seq", "<u4"), ("start", "<u4"), ("end", "<u4"), ("pair", "<u2"), ("orient", "u1"),
                      ("flags", "u1")])
assert HIT_DTYPE.itemsize == 12 and AMP_DTYPE.itemsize == 16


def check(st: int, where: str) -> None:
    if st != AH_OK:
        raise AhError(st, where)


def _p(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev():
    return torch.device("cuda", torch.cuda.current_device())


# ---------------------------------------------------------------------------
# Store
# ---------------------------------------------------------------------------
class Store:
    """Device-resident 2-bit genome store (all arrays are torch tensors)."""

    def __init__(self, lengths: Sequence[int], nmask_cap: int = 1 << 16, device=None):
        dev = device or _dev()
        lens = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint64))
        n = len(lens)
        b0 = np.zeros(max(n, 1), np.uint64)
        nb = U64(0)
        check(_lib.ah_pack_layout(lens.ctypes.data_as(VP), n, b0.ctypes.data_as(VP), C.byref(nb)), "ah_pack_layout")
        n_blocks = int(nb.value)
        nw = (n_blocks + 31) // 32
        blocks = torch.empty((max(n_blocks, 1), 4), dtype=torch.int32, device=dev)
        nbits = torch.zeros(max(nw, 1), dtype=torch.int32, device=dev)
        counters = torch.zeros(AH_STORE_SCRATCH, dtype=torch.int64, device=dev)
        self._bind(lens, b0[:n].copy(), n_blocks, blocks, nbits, counters, nmask_cap, dev)

    def _bind(self, lens, b0, n_blocks, blocks, nbits, counters, nmask_cap, dev):
        """Per-sequence tables, the N side table and the C struct over the
        given block, N-bit and counter arrays (which may be larger than
        needed)."""
        n = len(lens)
        self.n_seqs = n
        self.n_blocks = int(n_blocks)
        self.lengths = np.asarray(lens, np.uint64)
        self.seq_block0_host = np.asarray(b0, np.uint64)
        self.blocks = blocks
        self.seq_block0 = torch.from_numpy(self.seq_block0_host.astype(np.int64)).to(dev) if n else torch.zeros(
            1, dtype=torch.int64, device=dev)
        self.seq_len = torch.from_numpy(self.lengths.astype(np.uint32).view(np.int32)).to(dev) if n else \
            torch.zeros(1, dtype=torch.int32, device=dev)
        self.nbits = nbits
        self.nrank = torch.zeros(nbits.numel(), dtype=torch.int32, device=dev)
        self.nmask = torch.zeros(max(nmask_cap, 1), dtype=torch.int64, device=dev)
        self.nmask_cap = nmask_cap
        self.counters = counters
        self.c = ah_store(n, int(self.lengths.max()) if n else 0, self.n_blocks, self.blocks.data_ptr(),
                          self.seq_block0.data_ptr(), self.seq_len.data_ptr(), self.nbits.data_ptr(),
                          self.nrank.data_ptr(), self.nmask.data_ptr(), nmask_cap, self.counters.data_ptr())

    @property
    def total_bases(self) -> int:
        return int(self.lengths.sum())

    @property
    def hbm_bytes(self) -> int:
        return 16 * self.n_blocks

    # -- ingest -------------------------------------------------------------
    def pack_chunks(self, chunks, stream=None, nlist_cap: Optional[int] = None):
        """chunks: iterable of (first_seq, ascii uint8 array, offsets uint64[n+1])."""
        s = _stream(stream)
        cap = nlist_cap or self.nmask_cap
        nlist = torch.zeros((max(cap, 1), 2), dtype=torch.int64, device=self.blocks.device)
        check(_lib.ah_pack_begin(C.byref(self.c), s), "ah_pack_begin")
        for first, buf, off in chunks:
            n = len(off) - 1
            d_buf = torch.from_numpy(np.ascontiguousarray(buf)).to(self.blocks.device, non_blocking=False)
            d_off = torch.from_numpy(np.ascontiguousarray(off, dtype=np.uint64).view(np.int64)).to(
                self.blocks.device)
            check(_lib.ah_pack(C.byref(self.c), _p(d_buf), _p(d_off), first, n, _p(nlist), cap, s), "ah_pack")
            torch.cuda.current_stream().synchronize()
            del d_buf, d_off
        check(_lib.ah_pack_finish(C.byref(self.c), _p(nlist), cap, s), "ah_pack_finish")
        torch.cuda.synchronize()
        n_flag = int(self.counters[0].item())
        if n_flag > cap or n_flag > self.nmask_cap:
            raise AhError(AH_E_LIMIT, "store: %d blocks hold N, capacity %d" % (n_flag, min(cap, self.nmask_cap)))
        self.n_nblocks = n_flag
        return self

    @classmethod
    def from_workload(cls, wl, chunk_bases: int = 1 << 30, nmask_cap: int = 1 << 16):
        st = cls(wl.lengths, nmask_cap=nmask_cap)
        return st.pack_chunks(wl.chunks(chunk_bases))

    @classmethod
    def from_ascii(cls, seqs: Sequence[bytes], nmask_cap: int = 1 << 16):
        arrs = [np.frombuffer(s if isinstance(s, (bytes, bytearray)) else s.encode(), np.uint8) if not isinstance(
            s, np.ndarray) else s for s in seqs]
        lens = [len(a) for a in arrs]
        st = cls(lens, nmask_cap=nmask_cap)
        off = np.zeros(len(arrs) + 1, np.uint64)
        off[1:] = np.cumsum(lens)
        buf = np.concatenate(arrs) if arrs else np.zeros(0, np.uint8)
        if len(buf) == 0:
            buf = np.zeros(1, np.uint8)
        return st.pack_chunks([(0, buf, off)])

    @classmethod
    def from_fasta(cls, paths: Sequence[str], chunk_bytes: Optional[int] = None, nmask_cap: int = 1 << 16,
                   blocks_cap: Optional[int] = None, n_threads: Optional[int] = None, stream=None):
        """Read FASTA files into a new store (ah_fasta_ingest): one file in one
        pass, many files by up to n_threads host threads (default: the CPUs
        this process may use, at most 8); the record table (identifiers,
        sources, lengths) is ``store.fasta``.  Arrays too small for the files
        are grown and the files read again."""
        paths = [os.fspath(p) for p in paths]
        size = sum(os.path.getsize(p) for p in paths)
        cap = int(blocks_cap) if blocks_cap is not None else size // 64 + size // 4096 + 64 * len(paths) + 64
        if n_threads is None:
            n_threads = min(8, len(os.sched_getaffinity(0)))
        workers = max(1, min(int(n_threads), len(paths)))
        if chunk_bytes is None:
            chunk_bytes = (64 << 20) if workers == 1 else (16 << 20)
        dev = _dev()
        ws_n = U64(0)
        check(_lib.ah_fasta_ws_size(chunk_bytes, C.byref(ws_n)), "ah_fasta_ws_size")
        ws = torch.empty(int(ws_n.value) * workers, dtype=torch.uint8, device=dev)
        arr = (C.c_char_p * max(1, len(paths)))(*[os.fsencode(p) for p in paths])
        s = _stream(stream)
        while True:
            blocks = torch.empty((max(cap, 1), 4), dtype=torch.int32, device=dev)
            nbits = torch.empty(max((cap + 31) // 32, 1), dtype=torch.int32, device=dev)
            counters = torch.empty(AH_STORE_SCRATCH, dtype=torch.int64, device=dev)
            nlist = torch.empty((max(nmask_cap, 1), 2), dtype=torch.int64, device=dev)
            h = VP()
            check(_lib.ah_fasta_ingest(arr, len(paths), _p(blocks), cap, _p(nbits), _p(counters), _p(nlist),
                                       nmask_cap, chunk_bytes, workers, _p(ws), ws.numel(), s, C.byref(h)),
                  "ah_fasta_ingest")
            tab = FastaTable(h)
            n_flag = int(counters[0].item())
            if tab.n_blocks > cap:
                cap = tab.n_blocks
            elif n_flag > nmask_cap:
                nmask_cap = n_flag
            else:
                break
        del ws
        lens = tab.lengths.astype(np.uint64)
        b0 = np.zeros(max(len(lens), 1), np.uint64)
        nb = U64(0)
        check(_lib.ah_pack_layout(lens.ctypes.data_as(VP), len(lens), b0.ctypes.data_as(VP), C.byref(nb)),
              "ah_pack_layout")
        if int(nb.value) != tab.n_blocks or not np.array_equal(b0[:len(lens)], tab.block0):
            raise AhError(AH_E_ARG, "ah_fasta_ingest: record layout differs from ah_pack_layout")
        st = cls.__new__(cls)
        st._bind(lens, tab.block0, tab.n_blocks, blocks, nbits, counters, nmask_cap, dev)
        check(_lib.ah_pack_finish(C.byref(st.c), _p(nlist), nmask_cap, s), "ah_pack_finish")
        torch.cuda.synchronize()
        st.n_nblocks = n_flag
        st.fasta = tab
        return st

    @classmethod
    def from_fastq(cls, paths: Sequence[str], nmask_cap: int = 1 << 16):
        """Read FASTQ files into a new store (ah_fastq_read, then ah_pack):
        the record table is ``store.fasta`` and the qualities, laid out like
        the bases (record r's base j at byte 64 * block0[r] + j), are the
        device array ``store.qual``."""
        tab, bases, off, qual = read_fastq(paths)
        st = cls(tab.lengths.astype(np.uint64), nmask_cap=nmask_cap)
        if st.n_blocks != tab.n_blocks or not np.array_equal(st.seq_block0_host, tab.block0):
            raise AhError(AH_E_ARG, "ah_fastq_read: record layout differs from ah_pack_layout")
        if tab.n_records:
            st.pack_chunks([(0, bases if len(bases) else np.zeros(1, np.uint8), off)])
        st.qual = torch.from_numpy(qual).to(st.blocks.device)
        st.fasta = tab
        return st

    def unpack(self, seq: int, start: int = 0, n: Optional[int] = None) -> bytes:
        n = int(self.lengths[seq]) - start if n is None else n
        out = torch.zeros(max(n, 1), dtype=torch.uint8, device=self.blocks.device)
        check(_lib.ah_unpack(C.byref(self.c), seq, start, n, _p(out), _stream()), "ah_unpack")
        torch.cuda.synchronize()
        return out[:n].cpu().numpy().tobytes()


# ---------------------------------------------------------------------------
# FASTA record tables and output
# ---------------------------------------------------------------------------
class FastaTable:
    """Record table of ingested FASTA files (host memory owned by libah.so)."""

    def __init__(self, handle: VP):
        self._h = handle
        n, nbase, nblk, ml = U32(0), U64(0), U64(0), U32(0)
        check(_lib.ah_fasta_info(handle, C.byref(n), C.byref(nbase), C.byref(nblk), C.byref(ml)), "ah_fasta_info")
        self.n_records, self.n_bases, self.n_blocks, self.max_len = int(n.value), int(nbase.value), \
            int(nblk.value), int(ml.value)
        self.lengths = np.zeros(max(self.n_records, 1), np.uint32)
        self.block0 = np.zeros(max(self.n_records, 1), np.uint64)
        check(_lib.ah_fasta_table(handle, self.lengths.ctypes.data_as(VP), self.block0.ctypes.data_as(VP)),
              "ah_fasta_table")
        self.lengths = self.lengths[:self.n_records]
        self.block0 = self.block0[:self.n_records]
        self.names = ah_fasta_names()
        check(_lib.ah_fasta_names_of(handle, C.byref(self.names)), "ah_fasta_names_of")

    @property
    def ids(self) -> List[bytes]:
        nm = self.names
        if not self.n_records:
            return []
        off = np.ctypeslib.as_array(C.cast(nm.id_off, C.POINTER(U64)), (self.n_records,))
        end = int(off[-1])
        blob = C.string_at(nm.ids, end + len(C.string_at(nm.ids + end)) + 1)
        return [blob[o:blob.index(b"\0", o)] for o in off.tolist()]

    @property
    def seq_file(self) -> np.ndarray:
        if not self.n_records:
            return np.zeros(0, np.uint32)
        return np.ctypeslib.as_array(C.cast(self.names.seq_file, C.POINTER(U32)), (self.n_records,)).copy()

    @property
    def files(self) -> List[bytes]:
        arr = C.cast(self.names.files, C.POINTER(C.c_char_p))
        return [arr[i] for i in range(self.names.n_files)]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:  # (module globals are gone at interpreter exit)
            _lib.ah_fasta_free(self._h)
            self._h = None


def fasta_index(paths: Sequence[str], n_threads: int = 1) -> FastaTable:
    """Record table of FASTA files without reading them into a store (no GPU);
    many files are indexed by up to n_threads host threads."""
    paths = [os.fspath(p) for p in paths]
    arr = (C.c_char_p * max(1, len(paths)))(*[os.fsencode(p) for p in paths])
    h = VP()
    check(_lib.ah_fasta_ingest(arr, len(paths), None, 0, None, None, None, 0, 0, int(n_threads), None, 0, None,
                               C.byref(h)), "ah_fasta_ingest")
    return FastaTable(h)


class FastaNames:
    """Identifiers and source names of a store's sequences for ah_fasta_format,
    from Python lists (for stores not read from FASTA files)."""

    def __init__(self, ids: Sequence[bytes], seq_file: Sequence[int], files: Sequence[bytes]):
        ids = [bytes(x) for x in ids]
        self._blob = b"".join(x + b"\0" for x in ids) or b"\0"
        self._id_off = np.zeros(max(len(ids), 1), np.uint64)
        if ids:
            self._id_off[1:len(ids)] = np.cumsum([len(x) + 1 for x in ids])[:-1]
        self._seq_file = np.ascontiguousarray(np.asarray(seq_file, np.uint32).reshape(-1))
        if len(self._seq_file) == 0:
            self._seq_file = np.zeros(1, np.uint32)
        self._files = (C.c_char_p * max(1, len(files)))(*[bytes(f) for f in files])
        self._blob_buf = C.create_string_buffer(self._blob, len(self._blob))
        self.names = ah_fasta_names(C.cast(self._blob_buf, VP), self._id_off.ctypes.data, self._seq_file.ctypes.data,
                                    C.cast(self._files, VP), len(ids), len(files))


def format_fasta(names, res: dict, fb_len: int, rb_len: int, tm_filter: bool = True) -> bytes:
    """AHv2 FASTA text of a run's host results (``Pipeline.results()``):
    names = a FastaTable or FastaNames; with tm_filter only amplicons that
    passed the Tm threshold are written."""
    amps = np.ascontiguousarray(res["amps"])
    n = len(amps)
    tm = np.ascontiguousarray(res["tm"], np.float64)
    pas = np.ascontiguousarray(res["pass"], np.uint8) if tm_filter else None
    seq = res["seq"]
    seq_buf = np.frombuffer(seq, np.uint8) if len(seq) else np.zeros(1, np.uint8)
    so = np.ascontiguousarray(res["seq_off"], np.uint64)
    fb = np.ascontiguousarray(res["fb"], np.uint8) if fb_len else np.zeros(1, np.uint8)
    rb = np.ascontiguousarray(res["rb"], np.uint8) if rb_len else np.zeros(1, np.uint8)
    bc = np.ascontiguousarray(res["bc_len"], np.uint8)
    fp = np.ascontiguousarray(res["fprimer"], np.uint8)
    rp = np.ascontiguousarray(res["rprimer"], np.uint8)

    def ptr(a):
        return a.ctypes.data_as(VP)
    args = (C.byref(names.names), fb_len, rb_len, ptr(amps) if n else None, n, ptr(tm) if n else None,
            ptr(pas) if pas is not None and n else None, ptr(seq_buf), ptr(so), ptr(fb), ptr(rb),
            ptr(bc) if n else None, ptr(fp) if n else None, ptr(rp) if n else None)
    need = U64(0)
    check(_lib.ah_fasta_format(*args, None, 0, C.byref(need)), "ah_fasta_format")
    out = C.create_string_buffer(max(int(need.value), 1))
    check(_lib.ah_fasta_format(*args, out, int(need.value), C.byref(need)), "ah_fasta_format")
    return out.raw[:int(need.value)]


def read_fastq(paths: Sequence[str]):
    """Parse FASTQ files on the host (ah_fastq_read; no GPU): the record table,
    the bases back to back with their offsets, and the qualities laid out
    like the store's bases (64 * n_blocks bytes)."""
    paths = [os.fspath(p) for p in paths]
    arr = (C.c_char_p * max(1, len(paths)))(*[os.fsencode(p) for p in paths])
    h = VP()
    check(_lib.ah_fastq_read(arr, len(paths), C.byref(h)), "ah_fastq_read")
    tab = FastaTable(h)
    bp, op = VP(), VP()
    check(_lib.ah_fastq_bases(h, C.byref(bp), C.byref(op)), "ah_fastq_bases")
    off = np.ctypeslib.as_array(C.cast(op, C.POINTER(U64)), (tab.n_records + 1,)).copy()
    total = int(off[-1])
    bases = np.ctypeslib.as_array(C.cast(bp, C.POINTER(C.c_uint8)), (total,)).copy() if total else \
        np.zeros(0, np.uint8)
    qual = np.empty(max(64 * tab.n_blocks, 1), np.uint8)
    check(_lib.ah_fastq_qual_layout(h, qual.ctypes.data_as(VP), qual.size), "ah_fastq_qual_layout")
    return tab, bases, off, qual


def format_fastq(names, res: dict, fb_len: int, rb_len: int, tm_filter: bool = True) -> bytes:
    """FASTQ text of a run over a FASTQ store (``Pipeline.results()`` with
    ``qual``): the records of format_fasta with "@" headers, then "+" and the
    amplicon's qualities."""
    amps = np.ascontiguousarray(res["amps"])
    n = len(amps)
    tm = np.ascontiguousarray(res["tm"], np.float64)
    pas = np.ascontiguousarray(res["pass"], np.uint8) if tm_filter else None
    seq_buf = np.frombuffer(res["seq"], np.uint8) if len(res["seq"]) else np.zeros(1, np.uint8)
    qual_buf = np.frombuffer(res["qual"], np.uint8) if len(res["qual"]) else np.zeros(1, np.uint8)
    so = np.ascontiguousarray(res["seq_off"], np.uint64)
    fb = np.ascontiguousarray(res["fb"], np.uint8) if fb_len else np.zeros(1, np.uint8)
    rb = np.ascontiguousarray(res["rb"], np.uint8) if rb_len else np.zeros(1, np.uint8)
    bc = np.ascontiguousarray(res["bc_len"], np.uint8)
    fp = np.ascontiguousarray(res["fprimer"], np.uint8)
    rp = np.ascontiguousarray(res["rprimer"], np.uint8)

    def ptr(a):
        return a.ctypes.data_as(VP)
    args = (C.byref(names.names), fb_len, rb_len, ptr(amps) if n else None, n, ptr(tm) if n else None,
            ptr(pas) if pas is not None and n else None, ptr(seq_buf), ptr(so), ptr(qual_buf), ptr(fb), ptr(rb),
            ptr(bc) if n else None, ptr(fp) if n else None, ptr(rp) if n else None)
    need = U64(0)
    check(_lib.ah_fastq_format(*args, None, 0, C.byref(need)), "ah_fastq_format")
    out = C.create_string_buffer(max(int(need.value), 1))
    check(_lib.ah_fastq_format(*args, out, int(need.value), C.byref(need)), "ah_fastq_format")
    return out.raw[:int(need.value)]


# ---------------------------------------------------------------------------
# Primer sets
# ---------------------------------------------------------------------------
class PrimerSet:
    """Compiled primer pairs.  jit=True also compiles (hipRTC) a scan kernel
    specialised to these pairs; results are identical to the generic kernel."""

    def __init__(self, pairs, jit: bool = False, table: Optional[torch.Tensor] = None, stream=None):
        """table: optional device buffer (>= table_bytes(len(pairs)) bytes) that
        receives the device tables by an asynchronous copy on `stream`."""
        self.pairs = list(pairs)
        arr = (ah_pair_spec * len(self.pairs))()
        self._keep = []
        for i, p in enumerate(self.pairs):
            f, r = p.fwd.encode(), p.rev.encode()
            self._keep += [f, r]
            arr[i] = ah_pair_spec(f, r, int(p.k), int(p.clamp), int(p.min_len), int(p.max_len))
        h = VP()
        if table is None:
            check(_lib.ah_primers_compile(arr, len(self.pairs), C.byref(h)), "ah_primers_compile")
        else:
            check(_lib.ah_primers_compile_into(arr, len(self.pairs), _p(table), table.numel() * table.element_size(),
                                               _stream(stream), C.byref(h)), "ah_primers_compile_into")
            self._table = table
        self.h = h
        self.jit = False       # specialised kernel selected
        self.has_jit = False   # specialised kernel compiled
        self.variant = None    # (blocks per lane, LDS hit buffer) of the selected specialised kernel
        if jit:
            self.enable_jit()

    def enable_jit(self):
        check(_lib.ah_primers_jit(self.h), "ah_primers_jit")
        self.jit = self.has_jit = True
        if self.variant is None:
            self.variant = JIT_DEFAULT_VARIANT

    def jit_variant(self, blocks_per_lane: int, hit_buffer: int):
        """Select (compiling on first use) the specialised kernel with this
        tile size (blocks per lane: a wave scans 4096 x blocks_per_lane
        positions per step) and LDS hit buffer per wave."""
        check(_lib.ah_primers_jit_variant(self.h, int(blocks_per_lane), int(hit_buffer)), "ah_primers_jit_variant")
        self.jit = self.has_jit = True
        self.variant = (int(blocks_per_lane), int(hit_buffer))

    def use_jit(self, on: bool):
        check(_lib.ah_primers_use_jit(self.h, int(bool(on))), "ah_primers_use_jit")
        self.jit = bool(on)

    def launch_shape(self, wg_per_cu: int = 0) -> int:
        """Set the persistent scan's workgroups per CU (0 = resident maximum);
        returns the resident maximum of the selected kernel."""
        m = I32(0)
        check(_lib.ah_primers_launch_shape(self.h, int(wg_per_cu), C.byref(m)), "ah_primers_launch_shape")
        return int(m.value)

    def __len__(self):
        return len(self.pairs)

    def close(self):
        if self.h:
            _lib.ah_primers_free(self.h)
            self.h = VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def table_bytes(n_pairs: int) -> int:
    return int(_lib.ah_primers_table_bytes(n_pairs))


JIT_DEFAULT_VARIANT = (2, 48)
JIT_VARIANTS = ((2, 48), (2, 16), (1, 48), (1, 16))   # (blocks per lane, LDS hit buffer per wave), default first


def read_probe(buf: torch.Tensor, out: torch.Tensor, stream=None) -> None:
    """One read-only stream over buf (see ah_read_probe); out: int32 scratch."""
    check(_lib.ah_read_probe(_p(buf), buf.numel() * buf.element_size() // 16 * 16, _p(out), out.numel(),
                             _stream(stream)), "ah_read_probe")


def jit_check(pairs, arch: str = "gfx950", variant=JIT_DEFAULT_VARIANT) -> int:
    """Generate and compile the specialised scan kernel variant of `pairs` for
    `arch` without loading it (no GPU needed); returns the ah_status."""
    arr = (ah_pair_spec * max(len(pairs), 1))()
    keep = []
    for i, p in enumerate(pairs):
        f, r = p.fwd.encode(), p.rev.encode()
        keep += [f, r]
        arr[i] = ah_pair_spec(f, r, int(p.k), int(p.clamp), int(p.min_len), int(p.max_len))
    return int(_lib.ah_primers_jit_check(arr, len(pairs), arch.encode(), int(variant[0]), int(variant[1])))


def tm_params(tm) -> ah_tm_params:
    return ah_tm_params(tm.na_mM, tm.k_mM, tm.tris_mM, tm.mg_mM, tm.dntps_mM, tm.dnac1_nM, tm.dnac2_nM,
                        tm.threshold_C, int(tm.saltcorr), int(bool(tm.filter)), None,
                        int(getattr(tm, "nn_table", 3)), 0)


def extract_opts(ex) -> ah_extract_opts:
    return ah_extract_opts(int(bool(ex.trim)), int(ex.fb_len), int(ex.rb_len))


# ---------------------------------------------------------------------------
# Stage wrappers (device buffers in, device buffers out)
# ---------------------------------------------------------------------------
def ws_scan(store: Store, n_list: int) -> int:
    b = U64(0)
    check(_lib.ah_scan_ws_size(C.byref(store.c), n_list, C.byref(b)), "ah_scan_ws_size")
    return int(b.value)


def ws_pair(store: Store, ps: PrimerSet, hit_cap: int) -> int:
    b = U64(0)
    check(_lib.ah_pair_ws_size(C.byref(store.c), ps.h, hit_cap, C.byref(b)), "ah_pair_ws_size")
    return int(b.value)


def ws_extract(amp_cap: int) -> int:
    b = U64(0)
    check(_lib.ah_extract_ws_size(amp_cap, C.byref(b)), "ah_extract_ws_size")
    return int(b.value)


def _list_ptr(subset, stand_in):
    """Device pointer of a sequence list: None for "every sequence"; for an
    empty list a non-null stand-in (an empty tensor may have a null data
    pointer, which the library would read as every sequence; with zero
    entries the pointer is never read)."""
    if subset is None:
        return None
    return _p(subset) if subset.numel() else _p(stand_in)


def scan_primers(store, ps, hits, hit_cap, n_hits, ws, subset=None, stream=None):
    n_sub = 0 if subset is None else int(subset.numel())
    check(_lib.ah_scan_primers(C.byref(store.c), ps.h, _list_ptr(subset, n_hits), n_sub, _p(hits), hit_cap,
                               _p(n_hits), _p(ws), ws.numel() * ws.element_size(), _stream(stream)),
          "ah_scan_primers")


def scan_primers_static(store, ps, hits, hit_cap, n_hits, subset=None, stream=None):
    """ah_scan_primers with the library's fixed scratch array as its workspace
    (no allocation anywhere; at most STATIC_SCAN_MAX_LIST listed sequences)."""
    n_sub = 0 if subset is None else int(subset.numel())
    check(_lib.ah_scan_primers_static(C.byref(store.c), ps.h, _list_ptr(subset, n_hits), n_sub, _p(hits), hit_cap,
                                      _p(n_hits), _stream(stream)), "ah_scan_primers_static")


def scan_primers_masked(store, ps, subset, pair_mask, hits, hit_cap, n_hits, ws, stream=None):
    """Scan with the pairs chosen per listed sequence (pair_mask: int64 tensor,
    one word per subset entry)."""
    n_sub = int(subset.numel()) if subset is not None else store.n_seqs
    assert pair_mask.numel() >= n_sub and pair_mask.dtype == torch.int64
    check(_lib.ah_scan_primers_masked(C.byref(store.c), ps.h, _list_ptr(subset, n_hits),
                                      n_sub if subset is not None else 0,
                                      _p(pair_mask), _p(hits), hit_cap, _p(n_hits), _p(ws),
                                      ws.numel() * ws.element_size(), _stream(stream)), "ah_scan_primers_masked")


def route_hits(hits, n_hits, hit_cap, n_seqs, seq_req, vpair, kmax, n_req, n_pool, out, out_cap, n_out, stream=None):
    check(_lib.ah_route_hits(_p(hits), _p(n_hits), hit_cap, n_seqs, _p(seq_req), _p(vpair), _p(kmax), n_req, n_pool,
                             _p(out), out_cap, _p(n_out), _stream(stream)), "ah_route_hits")


def pair_amplicons(store, ps, hits, n_hits, hit_cap, orient_mask, amps, amp_cap, n_amps, ws, stream=None):
    check(_lib.ah_pair_amplicons(C.byref(store.c), ps.h, _p(hits), _p(n_hits), hit_cap, orient_mask, _p(amps),
                                 amp_cap, _p(n_amps), _p(ws), ws.numel() * ws.element_size(), _stream(stream)),
          "ah_pair_amplicons")


def tm_nn(store, ps, amps, n_amps, amp_cap, params: ah_tm_params, tm, tm_site, passed, stream=None):
    check(_lib.ah_tm_nn(C.byref(store.c), ps.h, _p(amps), _p(n_amps), amp_cap, C.byref(params), _p(tm),
                        _p(tm_site), _p(passed), _stream(stream)), "ah_tm_nn")


def extract(store, ps, amps, n_amps, amp_cap, passed, opts: ah_extract_opts, seq, seq_cap, seq_off, fb, rb, bc_len,
            fpr, rpr, n_bytes, ws, stream=None):
    check(_lib.ah_extract(C.byref(store.c), ps.h, _p(amps), _p(n_amps), amp_cap, _p(passed), C.byref(opts), _p(seq),
                          seq_cap, _p(seq_off), _p(fb), _p(rb), _p(bc_len), _p(fpr), _p(rpr), _p(n_bytes), _p(ws),
                          ws.numel() * ws.element_size(), _stream(stream)), "ah_extract")


def extract_qual(store, ps, amps, n_amps, amp_cap, passed, opts: ah_extract_opts, seq_off, out, out_cap,
                 stream=None):
    check(_lib.ah_extract_qual(C.byref(store.c), _p(store.qual), store.qual.numel(), ps.h, _p(amps), _p(n_amps),
                               amp_cap, _p(passed), C.byref(opts), _p(seq_off), _p(out), out_cap, _stream(stream)),
          "ah_extract_qual")


def tm_duplex(seqs: Sequence[str], cseqs: Sequence[str], tm, shifts: Optional[Sequence[int]] = None) -> np.ndarray:
    """Tm of explicit duplexes on the GPU (seq 5'->3', cseq its partner 3'->5',
    cseq[j] facing seq[j - shift]; lengths may differ)."""
    n = len(seqs)
    stride = 64
    a = np.zeros((max(n, 1), stride), np.uint8)
    b = np.zeros((max(n, 1), stride), np.uint8)
    ln = np.zeros(max(n, 1), np.uint32)
    lc = np.zeros(max(n, 1), np.uint32)
    sh = np.zeros(max(n, 1), np.int32)
    for i, (s, c) in enumerate(zip(seqs, cseqs)):
        a[i, :len(s)] = np.frombuffer(s.encode(), np.uint8)
        b[i, :len(c)] = np.frombuffer(c.encode(), np.uint8)
        ln[i], lc[i] = len(s), len(c)
        if shifts is not None:
            sh[i] = int(shifts[i])
    dev = _dev()
    da, db = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    dl = torch.from_numpy(ln.view(np.int32)).to(dev)
    dc = torch.from_numpy(lc.view(np.int32)).to(dev)
    ds = torch.from_numpy(sh).to(dev)
    out = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    prm = tm_params(tm)
    check(_lib.ah_tm_duplex(_p(da), _p(db), _p(dl), _p(dc), _p(ds), n, stride, C.byref(prm), _p(out), _stream()),
          "ah_tm_duplex")
    torch.cuda.synchronize()
    return out[:n].cpu().numpy()


# ---------------------------------------------------------------------------
# The whole path with preallocated buffers
# ---------------------------------------------------------------------------
@dataclass
class Caps:
    hits: int
    amps: int
    seq_bytes: int


class Pipeline:
    """scan -> pair -> Tm -> extract over a store with fixed capacities.

    All buffers are allocated once; ``launch()`` only enqueues kernels (so it
    can be captured into a HIP graph); ``counts()`` synchronises and reads the
    device counters; ``run()`` re-launches with larger capacities on overflow.
    """

    def __init__(self, store: Store, ps: PrimerSet, orient_mask: int, tm, ex=None, caps: Optional[Caps] = None,
                 subset: Optional[torch.Tensor] = None):
        self.store, self.ps = store, ps
        self.orient_mask = orient_mask
        self.tm_spec = tm
        self.params = tm_params(tm)
        self.ex = ex
        self.opts = extract_opts(ex) if ex is not None else None
        self.subset = subset
        self.dev = store.blocks.device
        self._alloc(caps or Caps(1 << 16, 1 << 15, 1 << 22))

    def _alloc(self, caps: Caps):
        d = self.dev
        self.caps = caps
        n_list = self.store.n_seqs if self.subset is None else int(self.subset.numel())
        self.counters = torch.zeros(4, dtype=torch.int64, device=d)  # hits, amps, bytes
        self.hits = torch.empty((caps.hits, 3), dtype=torch.int32, device=d)
        self.amps = torch.empty((caps.amps, 4), dtype=torch.int32, device=d)
        self.tm = torch.empty(caps.amps, dtype=torch.float64, device=d)
        self.tm_site = torch.empty((caps.amps, 2), dtype=torch.float64, device=d)
        self.passed = torch.empty(caps.amps, dtype=torch.uint8, device=d)
        ws = max(ws_scan(self.store, n_list), ws_pair(self.store, self.ps, caps.hits), ws_extract(caps.amps))
        self.ws = torch.empty(ws // 8 + 1, dtype=torch.int64, device=d)
        if self.opts is not None:
            fb, rb = max(self.opts.fb_len, 1), max(self.opts.rb_len, 1)
            self.seq = torch.empty(max(caps.seq_bytes, 1), dtype=torch.uint8, device=d)
            self.seq_off = torch.empty(caps.amps + 1, dtype=torch.int64, device=d)
            self.fb = torch.empty((caps.amps, fb), dtype=torch.uint8, device=d)
            self.rb = torch.empty((caps.amps, rb), dtype=torch.uint8, device=d)
            self.bc_len = torch.empty((caps.amps, 2), dtype=torch.uint8, device=d)
            self.fpr = torch.empty((caps.amps, 32), dtype=torch.uint8, device=d)
            self.rpr = torch.empty((caps.amps, 32), dtype=torch.uint8, device=d)
            if getattr(self.store, "qual", None) is not None:  # FASTQ input: qualities beside the bases
                self.qual = torch.empty(max(caps.seq_bytes, 1), dtype=torch.uint8, device=d)

    def launch(self, stream=None, stages=("scan", "pair", "tm", "extract")):
        c = self.counters
        n_hits, n_amps, n_bytes = c[0:1], c[1:2], c[2:3]
        if "scan" in stages:
            scan_primers(self.store, self.ps, self.hits, self.caps.hits, n_hits, self.ws, self.subset, stream)
        if "pair" in stages:
            pair_amplicons(self.store, self.ps, self.hits, n_hits, self.caps.hits, self.orient_mask, self.amps,
                           self.caps.amps, n_amps, self.ws, stream)
        if "tm" in stages:
            tm_nn(self.store, self.ps, self.amps, n_amps, self.caps.amps, self.params, self.tm, self.tm_site,
                  self.passed, stream)
        if "extract" in stages and self.opts is not None:
            extract(self.store, self.ps, self.amps, n_amps, self.caps.amps,
                    self.passed if self.tm_spec.filter else None, self.opts, self.seq, self.caps.seq_bytes,
                    self.seq_off, self.fb, self.rb, self.bc_len, self.fpr, self.rpr, n_bytes, self.ws, stream)
            if getattr(self.store, "qual", None) is not None:
                extract_qual(self.store, self.ps, self.amps, n_amps, self.caps.amps,
                             self.passed if self.tm_spec.filter else None, self.opts, self.seq_off, self.qual,
                             self.caps.seq_bytes, stream)

    def counts(self):
        torch.cuda.synchronize()
        v = self.counters.cpu().numpy()
        return int(v[0]), int(v[1]), int(v[2])

    def overflowed(self):
        h, a, b = self.counts()
        return h > self.caps.hits or a > self.caps.amps or (self.opts is not None and b > self.caps.seq_bytes)

    def run(self, stream=None):
        """Launch; on overflow grow the capacities and launch again (exact)."""
        while True:
            self.launch(stream)
            h, a, b = self.counts()
            if h <= self.caps.hits and a <= self.caps.amps and (self.opts is None or b <= self.caps.seq_bytes):
                return self
            self._alloc(Caps(max(self.caps.hits, int(h * 1.25) + 1024), max(self.caps.amps, int(a * 1.25) + 1024),
                             max(self.caps.seq_bytes, int(b * 1.25) + 4096)))

    # -- results to host ------------------------------------------------------
    def results(self):
        h, a, b = self.counts()
        out = {}
        out["hits"] = self.hits[:h].cpu().numpy().view(np.uint8).reshape(-1).view(HIT_DTYPE)
        out["amps"] = self.amps[:a].cpu().numpy().view(np.uint8).reshape(-1).view(AMP_DTYPE)
        out["tm"] = self.tm[:a].cpu().numpy()
        out["tm_site"] = self.tm_site[:a].cpu().numpy()
        out["pass"] = self.passed[:a].cpu().numpy()
        if self.opts is not None:
            out["seq"] = self.seq[:b].cpu().numpy().tobytes()
            out["seq_off"] = self.seq_off[:a + 1].cpu().numpy().astype(np.uint64)
            out["fb"] = self.fb[:a, :self.opts.fb_len].cpu().numpy()
            out["rb"] = self.rb[:a, :self.opts.rb_len].cpu().numpy()
            out["bc_len"] = self.bc_len[:a].cpu().numpy()
            out["fprimer"] = self.fpr[:a].cpu().numpy()
            out["rprimer"] = self.rpr[:a].cpu().numpy()
            if getattr(self.store, "qual", None) is not None:
                out["qual"] = self.qual[:b].cpu().numpy().tobytes()
        return out


def hits_canonical(h: np.ndarray) -> np.ndarray:
    """Hits as an (n, 5) array [seq, pos, pair, kind, mm] in the oracle's order (seq, pair, pos, kind)."""
    a = np.stack([h["seq"].astype(np.int64), h["pos"], h["pair"], h["kind"], h["mm"]], axis=1).astype(np.int64)
    order = np.lexsort((a[:, 3], a[:, 1], a[:, 2], a[:, 0]))
    return a[order]


def amps_array(a: np.ndarray) -> np.ndarray:
    """Amplicons as (n, 5) [seq, start, end, pair, orient] (library order kept)."""
    return np.stack([a["seq"], a["start"], a["end"], a["pair"], a["orient"]], axis=1).astype(np.int64)
