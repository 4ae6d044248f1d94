"""Seeded synthetic workloads shaped like the paper's benchmark inputs.

The paper benchmarks on AllTheBacteria assemblies with the V1V9, Titan and
V3V4 primer pairs (Results; Supplementary "Hardware and software
environment").  None of those are available here, so every workload is
generated: bacterial-chromosome-like iid sequences with a per-genome GC
content, degenerate synthetic primers, and planted primer sites whose
positions, strands, variants and barcodes are recorded as ground truth.

This module is shared by the oracle tests and by the GPU path's tests and
benchmark.  It holds none of the method's arithmetic (no matching, pairing,
melting temperature or extraction); it only draws random inputs.  Its small
IUPAC and complement tables exist to *build* inputs (pick a concrete primer
variant, plant a site on the minus strand).

Seeds: config ``c`` uses master seed ``170000 + c``.  A ``SeedSequence`` of
that seed is split into a layout stream (lengths, GC, primers, planting
plan) and one independent stream per sequence, so any single sequence can be
regenerated alone (``Workload.make_seq(i)``).
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Iterator, List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Input-construction tables (IUPAC nucleotide nomenclature).
# --------------------------------------------------------------------------
_IUPAC_SETS = {
    "A": "A", "C": "C", "G": "G", "T": "T",
    "R": "AG", "Y": "CT", "S": "CG", "W": "AT", "K": "GT", "M": "AC",
    "B": "CGT", "D": "AGT", "H": "ACT", "V": "ACG", "N": "ACGT",
}
# codes of each fold, indexed by the base they must contain
_CODES_BY_FOLD = {
    2: {b: [c for c, s in _IUPAC_SETS.items() if len(s) == 2 and b in s] for b in "ACGT"},
    3: {b: [c for c, s in _IUPAC_SETS.items() if len(s) == 3 and b in s] for b in "ACGT"},
}
_COMP = {ord("A"): ord("T"), ord("C"): ord("G"), ord("G"): ord("C"), ord("T"): ord("A")}
_COMP_LUT = np.arange(256, dtype=np.uint8)
for _a, _b in _COMP.items():
    _COMP_LUT[_a] = _b
_ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)

ORIENT_FR, ORIENT_RF, ORIENT_FF, ORIENT_RR = 0, 1, 2, 3
ORIENT_ALL = 0xF
ORIENT_NAMES = ("FR", "RF", "FF", "RR")

MASTER_SEED = 170000

# threads used to draw bases (numpy releases the GIL while filling arrays)
GEN_THREADS = max(1, min(16, os.cpu_count() or 1))


def revcomp_bytes(a: np.ndarray) -> np.ndarray:
    """Reverse complement of an ASCII ACGT array (input construction only)."""
    return _COMP_LUT[a[::-1]]


def revcomp_str(s: str) -> str:
    return revcomp_bytes(np.frombuffer(s.encode(), np.uint8)).tobytes().decode()


# --------------------------------------------------------------------------
# Specs
# --------------------------------------------------------------------------
@dataclasses.dataclass
class PairSpec:
    fwd: str
    rev: str
    k: int
    clamp: int
    min_len: int = 200
    max_len: int = 2000


@dataclasses.dataclass
class TmSpec:
    """Nearest-neighbour Tm conditions (concentrations as the paper's tool takes them)."""
    na_mM: float = 50.0
    k_mM: float = 0.0
    tris_mM: float = 0.0
    mg_mM: float = 0.0
    dntps_mM: float = 0.0
    dnac1_nM: float = 250.0   # primer strand
    dnac2_nM: float = 0.0     # template strand
    saltcorr: int = 5
    threshold_C: float = 45.0
    filter: bool = True
    nn_table: int = 3          # Watson-Crick parameter set, numbered as the Tm_NN model numbers them


@dataclasses.dataclass
class ExtractSpec:
    trim: bool = False
    fb_len: int = 0
    rb_len: int = 0


@dataclasses.dataclass
class SeqMeta:
    length: int
    gc_q: int                     # P(G) = P(C) = gc_q / 256
    plants: list                  # list of plant dicts (see _plant_*)


@dataclasses.dataclass
class Workload:
    name: str
    config: int
    pairs: List[PairSpec]
    tm: TmSpec
    extract: ExtractSpec
    orient_mask: int
    metas: List[SeqMeta]
    seq_seeds: list
    truth: dict = dataclasses.field(default_factory=dict)
    _cache: dict = dataclasses.field(default_factory=dict, repr=False)

    @property
    def n_seqs(self) -> int:
        return len(self.metas)

    @property
    def lengths(self) -> np.ndarray:
        return np.array([m.length for m in self.metas], dtype=np.uint64)

    @property
    def total_bases(self) -> int:
        return int(sum(m.length for m in self.metas))

    def make_seq(self, i: int) -> np.ndarray:
        """Regenerate sequence i (ASCII uint8) from its own stream."""
        return _make_seq(self.metas[i], self.seq_seeds[i], self.pairs)

    def seqs(self, idx: Optional[Sequence[int]] = None) -> List[np.ndarray]:
        idx = range(self.n_seqs) if idx is None else idx
        idx = list(idx)
        with ThreadPoolExecutor(GEN_THREADS) as ex:
            return list(ex.map(self.make_seq, idx))

    def concat(self, idx: Optional[Sequence[int]] = None) -> Tuple[np.ndarray, np.ndarray]:
        """ASCII of the chosen sequences concatenated, plus offsets (n+1, uint64)."""
        parts = self.seqs(idx)
        off = np.zeros(len(parts) + 1, dtype=np.uint64)
        off[1:] = np.cumsum([len(p) for p in parts], dtype=np.uint64)
        buf = np.empty(int(off[-1]), dtype=np.uint8)
        for p, o in zip(parts, off[:-1]):
            buf[int(o):int(o) + len(p)] = p
        return buf, off

    def chunks(self, max_bases: int) -> Iterator[Tuple[int, np.ndarray, np.ndarray]]:
        """Yield (first_seq, ascii, offsets) groups of whole sequences of at most
        ``max_bases`` bases each (a single longer sequence forms its own group)."""
        i = 0
        n = self.n_seqs
        while i < n:
            j = i
            tot = 0
            while j < n and (j == i or tot + self.metas[j].length <= max_bases):
                tot += self.metas[j].length
                j += 1
            buf, off = self.concat(range(i, j))
            yield i, buf, off
            i = j


# --------------------------------------------------------------------------
# Drawing helpers
# --------------------------------------------------------------------------
def _gc_lut(gc_q: int) -> np.ndarray:
    """Byte -> ASCII base table with P(G) = P(C) = gc_q/256, P(A) = P(T)."""
    assert 0 <= gc_q <= 128
    lut = np.empty(256, dtype=np.uint8)
    lut[0:gc_q] = ord("G")
    lut[gc_q:2 * gc_q] = ord("C")
    rest = 256 - 2 * gc_q
    lut[2 * gc_q:2 * gc_q + rest // 2] = ord("A")
    lut[2 * gc_q + rest // 2:] = ord("T")
    return lut


def _gc_to_q(g: float) -> int:
    return int(round(g * 128))


def _random_bases(rng: np.random.Generator, n: int, gc_q: int = 64) -> np.ndarray:
    b = rng.integers(0, 256, size=n, dtype=np.uint8)
    out = np.empty_like(b)
    np.take(_gc_lut(gc_q), b, out=out)
    return out


def make_primer(rng: np.random.Generator, L: int, n_deg: int, folds=(2,)) -> str:
    """Random concrete primer of length L with n_deg positions (uniform over all
    L positions) replaced by an IUPAC code of a fold drawn from ``folds`` that
    contains the original base."""
    base = _ACGT[rng.integers(0, 4, size=L)].tobytes().decode()
    s = list(base)
    pos = rng.choice(L, size=n_deg, replace=False) if n_deg else []
    for p in pos:
        f = int(folds[rng.integers(0, len(folds))])
        choices = _CODES_BY_FOLD[f][s[p]]
        s[p] = choices[rng.integers(0, len(choices))]
    return "".join(s)


def random_variant(rng: np.random.Generator, primer: str) -> np.ndarray:
    """A uniformly random concrete expansion of an IUPAC primer (ASCII)."""
    out = np.empty(len(primer), dtype=np.uint8)
    for j, c in enumerate(primer.upper().replace("U", "T")):
        s = _IUPAC_SETS[c]
        out[j] = ord(s[rng.integers(0, len(s))])
    return out


def _substitute(rng: np.random.Generator, a: np.ndarray, positions) -> None:
    """Change each listed position to a different base (uniform over the other 3)."""
    for p in positions:
        cur = a[p]
        others = [x for x in b"ACGT" if x != cur]
        a[p] = others[rng.integers(0, 3)]


def _mutate_rate(rng: np.random.Generator, a: np.ndarray, r: float) -> None:
    if r <= 0:
        return
    hit = np.nonzero(rng.random(len(a)) < r)[0]
    _substitute(rng, a, hit)


# --------------------------------------------------------------------------
# Per-sequence construction
# --------------------------------------------------------------------------
def _make_seq(meta: SeqMeta, seed, pairs: List[PairSpec]) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    s = _random_bases(rng, meta.length, meta.gc_q)
    for pl in meta.plants:
        kind = pl["kind"]
        if kind == "amplicon":          # tiny config: one primer pair site pair
            _plant_amplicon(rng, s, pl, pairs)
        elif kind == "segment":         # genome configs: conserved segment copy
            _plant_segment(rng, s, pl, pairs)
        elif kind == "operon":          # tandem operon units with barcodes
            _plant_operon(rng, s, pl, pairs)
        else:  # pragma: no cover
            raise ValueError(kind)
    return s


def _site_variant(rng, primer: str, n_subs: int, clamp: int) -> np.ndarray:
    v = random_variant(rng, primer)
    L = len(v)
    free = np.arange(0, L - clamp)
    if n_subs:
        _substitute(rng, v, rng.choice(free, size=min(n_subs, len(free)), replace=False))
    return v


def _plant_amplicon(rng, s: np.ndarray, pl: dict, pairs: List[PairSpec]) -> None:
    p = pairs[pl["pair"]]
    o = pl["orient"]
    first = p.fwd if o in (ORIENT_FR, ORIENT_FF) else p.rev
    second = p.rev if o in (ORIENT_FR, ORIENT_RR) else p.fwd
    v1 = _site_variant(rng, first, pl["subs"][0], p.clamp)
    v2 = _site_variant(rng, second, pl["subs"][1], p.clamp)
    n = pl["length"]
    mid = _random_bases(rng, n - len(v1) - len(v2))
    amp = np.concatenate([v1, mid, revcomp_bytes(v2)])
    st = pl["start"]
    s[st:st + n] = amp


def _segment(rng, p: PairSpec, rate: float) -> np.ndarray:
    """1.5 kb conserved-segment copy: forward-primer variant at offset 20, the
    reverse complement of a reverse-primer variant ending at offset 1480."""
    seg = _random_bases(rng, 1500)
    vf = random_variant(rng, p.fwd)
    vr = random_variant(rng, p.rev)
    seg[20:20 + len(vf)] = vf
    seg[1480 - len(vr):1480] = revcomp_bytes(vr)
    _mutate_rate(rng, seg, rate)
    return seg


def _plant_segment(rng, s, pl, pairs) -> None:
    seg = _segment(rng, pairs[pl["pair"]], pl["rate"])
    if pl["strand"] < 0:
        seg = revcomp_bytes(seg)
    st = pl["start"]
    s[st:st + len(seg)] = seg


def _plant_operon(rng, s, pl, pairs) -> None:
    p = pairs[pl["pair"]]
    pos = pl["start"]
    for u in pl["units"]:
        spacer = _random_bases(rng, u["spacer"])
        vf = random_variant(rng, p.fwd)
        vr = random_variant(rng, p.rev)
        mid = _random_bases(rng, u["amp_len"] - len(vf) - len(vr))
        bl = np.frombuffer(u["bc_l"].encode(), np.uint8)
        br = np.frombuffer(u["bc_r"].encode(), np.uint8)
        unit = np.concatenate([spacer, bl, vf, mid, revcomp_bytes(vr), br])
        if u["strand"] < 0:
            unit = revcomp_bytes(unit)
        s[pos:pos + len(unit)] = unit
        pos += len(unit)


def operon_unit_len(u: dict) -> int:
    return u["spacer"] + 16 + u["amp_len"] + 16


# --------------------------------------------------------------------------
# Configs
# --------------------------------------------------------------------------
def _spawn(cfg: int):
    ss = np.random.SeedSequence(MASTER_SEED + cfg)
    layout_ss, seq_ss = ss.spawn(2)
    return np.random.Generator(np.random.PCG64(layout_ss)), seq_ss


def _random_pool_pair(rng) -> PairSpec:
    """Pair drawn as in the batching workload: L ~ U{17..26}, degeneracy 2^u
    with u ~ U{0..9} two-fold codes, k ~ U{0..3}, clamp ~ U{3,4,5}."""
    c = int(rng.integers(3, 6))
    k = int(rng.integers(0, 4))
    prim = []
    for _ in range(2):
        L = int(rng.integers(17, 27))
        u = int(rng.integers(0, 10))
        prim.append(make_primer(rng, L, min(u, L), folds=(2,)))
    return PairSpec(prim[0], prim[1], k=k, clamp=c, min_len=200, max_len=2000)


def _segment_plants(rng, length: int, n_copies: int, pair_choices) -> list:
    n_copies = min(n_copies, max(0, length // 1600))
    plants = []
    if n_copies == 0:
        return plants
    region = length // n_copies
    for c in range(n_copies):
        st = c * region + int(rng.integers(0, region - 1500 + 1))
        plants.append(dict(kind="segment", pair=int(pair_choices[c]), start=st,
                           strand=int(rng.choice([1, -1])), rate=float(rng.uniform(0, 0.03))))
    return plants


# Sweeps shaped like the paper's (Results, "Primer degeneracy and mismatch
# tolerance"): N bases added two at a time, one per primer, at the 5' ends
# (the 3' clamp is untouched); and the substitutions allowed, 0 to 6.
SWEEP_N = (0, 2, 4, 6)
SWEEP_K = (0, 1, 2, 3, 4, 5, 6)


def sweep_pairs(base: PairSpec, kind: str) -> List[tuple]:
    """(x, PairSpec) for each point of a sweep: kind "degeneracy" (x = N bases
    added over both primers) or "mismatch" (x = k)."""
    if kind == "degeneracy":
        return [(n, dataclasses.replace(base, fwd="N" * (n // 2) + base.fwd, rev="N" * (n // 2) + base.rev))
                for n in SWEEP_N]
    if kind == "mismatch":
        return [(k, dataclasses.replace(base, k=k)) for k in SWEEP_K]
    raise ValueError(kind)


def gen_config(cfg: int, n_seqs: Optional[int] = None, len_scale: float = 1.0) -> Workload:
    """Build workload ``cfg`` (1..5).  ``n_seqs``/``len_scale`` shrink it for
    tests (same recipe, fewer/shorter sequences)."""
    rng, seq_ss = _spawn(cfg)
    if cfg == 1:
        return _cfg1(rng, seq_ss, n_seqs)
    if cfg == 2:
        return _cfg2(rng, seq_ss, n_seqs, len_scale)
    if cfg == 3:
        return _cfg3(rng, seq_ss, len_scale)
    if cfg == 4:
        return _cfg4(rng, seq_ss, n_seqs, len_scale)
    if cfg == 5:
        return _cfg5(rng, seq_ss, n_seqs, len_scale)
    raise ValueError(cfg)


def _finish(name, cfg, pairs, tm, ex, orient, metas, seq_ss, truth) -> Workload:
    seeds = seq_ss.spawn(len(metas))
    return Workload(name=name, config=cfg, pairs=pairs, tm=tm, extract=ex,
                    orient_mask=orient, metas=metas, seq_seeds=seeds, truth=truth)


def _cfg1(rng, seq_ss, n_seqs):
    n = n_seqs or 200
    F = make_primer(rng, 20, 3, folds=(2, 3))
    R = make_primer(rng, 20, 3, folds=(2, 3))
    pair = PairSpec(F, R, k=2, clamp=3, min_len=200, max_len=2000)
    lengths = rng.integers(1000, 5001, size=n)
    planted = rng.permutation(n)[: n // 2]
    metas = [SeqMeta(int(L), 64, []) for L in lengths]
    truth = []
    for i in sorted(planted.tolist()):
        L = metas[i].length
        alen = int(rng.integers(300, 501))
        orient = int(rng.integers(0, 4))
        subs = [int(rng.integers(0, 3)), int(rng.integers(0, 3))]
        st = int(rng.integers(0, L - alen + 1))
        pl = dict(kind="amplicon", pair=0, orient=orient, length=alen, start=st, subs=subs)
        metas[i].plants.append(pl)
        truth.append(dict(seq=i, **pl))
    return _finish("tiny", 1, [pair], TmSpec(threshold_C=45.0, filter=True), ExtractSpec(),
                   ORIENT_ALL, metas, seq_ss, {"amplicons": truth})


def _cfg2(rng, seq_ss, n_seqs, len_scale, lo=3e6, hi=6e6, n_default=2000, name="genome"):
    n = n_seqs or n_default
    F = make_primer(rng, 19, 4, folds=(2,))
    R = make_primer(rng, 21, 5, folds=(2,))
    pair = PairSpec(F, R, k=3, clamp=5, min_len=200, max_len=2000)
    metas = []
    for _ in range(n):
        L = int(rng.integers(int(lo * len_scale), int(hi * len_scale) + 1))
        g = float(rng.uniform(0.3, 0.7))
        nc = int(rng.integers(1, 16))
        plants = _segment_plants(rng, L, nc, [0] * nc)
        metas.append(SeqMeta(L, _gc_to_q(g), plants))
    return _finish(name, 2, [pair], TmSpec(threshold_C=45.0, filter=True), ExtractSpec(),
                   ORIENT_ALL, metas, seq_ss, {})


def _cfg3(rng, seq_ss, len_scale, target=9e9):
    pairs = [_random_pool_pair(rng) for _ in range(64)]
    metas = []
    tot = 0
    target = target * len_scale
    while tot < target:
        if rng.random() < 0.2:
            L = max(int(math.exp(rng.uniform(math.log(5e3), math.log(2e5))) * len_scale), 2000)
            g = float(rng.uniform(0.3, 0.7))
            nc = int(rng.integers(0, 3))
            pc = [int(rng.integers(0, 64))] * nc
        else:
            while True:
                L = math.exp(rng.normal(math.log(4e6), 0.6))
                if 0.5e6 <= L <= 12e6:
                    break
            L = max(int(L * len_scale), 4000)
            g = float(rng.uniform(0.3, 0.7))
            nc = int(rng.integers(1, 16))
            four = rng.choice(64, size=4, replace=False)
            pc = [int(four[rng.integers(0, 4)]) for _ in range(nc)]
        metas.append(SeqMeta(L, _gc_to_q(g), _segment_plants(rng, L, len(pc), pc)))
        tot += L
    return _finish("batch", 3, pairs, TmSpec(threshold_C=45.0, filter=True), ExtractSpec(),
                   ORIENT_ALL, metas, seq_ss, {})


def _cfg4(rng, seq_ss, n_seqs, len_scale):
    n = n_seqs or 500
    # the pair of the genome-scale config, drawn from config 2's layout stream
    rng2, _ = _spawn(2)
    F = make_primer(rng2, 19, 4, folds=(2,))
    R = make_primer(rng2, 21, 5, folds=(2,))
    pair = PairSpec(F, R, k=2, clamp=4, min_len=200, max_len=2000)
    L = int(4_000_000 * len_scale)
    metas = []
    truth = []
    for i in range(n):
        g = float(rng.uniform(0.3, 0.7))
        n_units = int(rng.integers(10, 41))
        units = []
        for _ in range(n_units):
            units.append(dict(spacer=int(rng.integers(100, 301)),
                              amp_len=int(rng.integers(1000, 1501)),
                              strand=int(rng.choice([1, -1])),
                              bc_l=_ACGT[rng.integers(0, 4, 16)].tobytes().decode(),
                              bc_r=_ACGT[rng.integers(0, 4, 16)].tobytes().decode()))
        tot = sum(operon_unit_len(u) for u in units)
        while tot > L - 100 and units:
            units.pop()
            tot = sum(operon_unit_len(u) for u in units)
        start = int(rng.integers(50, L - tot - 50 + 1)) if units else 0
        pl = dict(kind="operon", pair=0, start=start, units=units)
        metas.append(SeqMeta(L, _gc_to_q(g), [pl] if units else []))
        truth.append(dict(seq=i, start=start, units=units))
    return _finish("dense", 4, [pair], TmSpec(threshold_C=45.0, filter=False),
                   ExtractSpec(trim=True, fb_len=16, rb_len=16), ORIENT_ALL, metas, seq_ss,
                   {"operons": truth})


def _cfg5(rng, seq_ss, n_seqs, len_scale):
    n = n_seqs or 5000
    pool = [_random_pool_pair(rng) for _ in range(32)]
    metas = []
    for _ in range(n):
        L = int(rng.integers(int(3e6 * len_scale), int(5e6 * len_scale) + 1))
        g = float(rng.uniform(0.3, 0.7))
        m = int(rng.integers(2, 5))
        chosen = rng.choice(32, size=m, replace=False)
        pc = []
        for c in chosen:
            pc += [int(c)] * int(rng.integers(1, 5))
        metas.append(SeqMeta(L, _gc_to_q(g), _segment_plants(rng, L, len(pc), pc)))
    return _finish("serve", 5, pool, TmSpec(threshold_C=50.0, filter=True), ExtractSpec(),
                   ORIENT_ALL, metas, seq_ss, {})


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    pairs: List[int]          # indices into the pool
    seqs: np.ndarray          # sequence ids (sorted, unique)
    k: int
    threshold_C: float


def gen_requests(wl: Workload, n: int, qps: float, seed: int = 0,
                 max_subset: int = 5000, min_subset: int = 100) -> List[Request]:
    """Poisson request stream over a serving store: each request takes U{1..8}
    pool pairs, a random subset of U{min..max} sequence ids, k ~ U{0..3} and a
    Tm threshold ~ U[40, 60] C."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([MASTER_SEED + 5, 1, seed])))
    t = 0.0
    out = []
    hi = min(max_subset, wl.n_seqs)
    lo = min(min_subset, hi)
    for r in range(n):
        t += float(rng.exponential(1.0 / qps)) if qps > 0 else 0.0
        npairs = int(rng.integers(1, 9))
        pairs = sorted(rng.choice(len(wl.pairs), size=npairs, replace=False).tolist())
        m = int(rng.integers(lo, hi + 1))
        seqs = np.sort(rng.choice(wl.n_seqs, size=m, replace=False)).astype(np.uint32)
        out.append(Request(r, t, pairs, seqs, int(rng.integers(0, 4)), float(rng.uniform(40, 60))))
    return out


def random_ascii(rng: np.random.Generator, n: int, gc: float = 0.5) -> np.ndarray:
    """Plain iid ASCII bases (for unit tests)."""
    return _random_bases(rng, n, _gc_to_q(gc))
