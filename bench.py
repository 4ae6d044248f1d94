#!/usr/bin/env python3
"""Benchmark: one step = one pass of the whole hot path (scan -> pair -> Tm ->
extract) over the genome-scale synthetic workload (2,000 sequences of 3-6 Mb,
~9 Gbases, one degenerate primer pair, k=3, clamp 5, all four orientations,
FP64 Tm filter at 45 C), genome resident in HBM.

Prints one JSON line.  value = whole-job Gbases scanned per second (one pair:
Gbases/s = pair-Gbases/s) over the timed passes, two in flight at once on two
streams (--depth).  The dominant kernel (the primer scan) is timed with HIP
events on its own stream right after the timed region and reported against
the HBM roofline; the CPU oracle is timed on a bounded sample of the same
workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
BYTES_PER_BASE = 0.25   # 2-bit store
# int32 / bitwise vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64
# instruction occupies a SIMD for 4 clocks), in tera lane-ops per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--depth", type=int, default=2,
                    help="genome line: passes in flight at once (each on its own pipeline and stream)")
    ap.add_argument("--warmup-s", type=float, default=0.5,
                    help="untimed warm-up lasts at least --warmup steps and at least this long (the GPU's clocks "
                         "settle under sustained load)")
    ap.add_argument("--config", type=int, default=2, help="workload (2 = genome scale)")
    ap.add_argument("--n-seqs", type=int, default=None, help="shrink the workload (testing)")
    ap.add_argument("--len-scale", type=float, default=1.0, help="shrink the workload (testing)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fasta-gbases", type=float, default=2.0,
                    help="size of the FASTA file the I/O extra writes and reads back, Gbases")
    ap.add_argument("--cpu-sample-bases", type=float, default=None,
                    help="oracle sample size (default 8e9 bases for one pair, 1e8 for many)")
    ap.add_argument("--stages", default="scan,pair,tm,extract")
    ap.add_argument("--generic", action="store_true", help="use the generic scan kernel (no primer-set JIT)")
    ap.add_argument("--plain-reps", type=int, default=1, help="timed repetitions of the plain per-pair loop (batch)")
    ap.add_argument("--no-tune", action="store_true", help="skip the scan autotuner (genome and batch lines)")
    ap.add_argument("--serve", action="store_true", help="serving workload (continuous batching, latency)")
    ap.add_argument("--sweep-points", default=None,
                    help="sweep only these points, e.g. 'degeneracy:6,mismatch:3' (default: all)")
    ap.add_argument("--sweep", action="store_true",
                    help="degeneracy and mismatch sweeps on the genome workload (prints their own line)")
    ap.add_argument("--requests", type=int, default=2000, help="serve: measured requests per run")
    ap.add_argument("--warm-requests", type=int, default=200, help="serve: warm-up requests per run")
    ap.add_argument("--budget-mb", type=int, default=16384, help="serve: device memory budget per batch")
    ap.add_argument("--no-extras", action="store_true",
                    help="genome run only: skip the batched-vs-plain and serving sub-results")
    ap.add_argument("--extra-requests", type=int, default=2000,
                    help="serving sub-result: measured requests per run (warm-up: a tenth as many)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for HBM counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def scan_source_hash():
    """sha256 over the sources the scan kernel is built from (host launcher,
    device core, device types); the counters are trusted only for this hash."""
    import hashlib
    h = hashlib.sha256()
    for f in ("scan.hip", "scan_core.h", "ah_dev.h"):
        h.update(open(os.path.join(ROOT, "paper_2511_00170_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def counters_from_profiles(name, kernel_src_hash):
    """Committed rocprofv3 counter summary profiles/<name>_counters.json, if it
    was taken on the current scan kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "%s_counters.json" % name)
    try:
        d = json.load(open(p))
    except Exception:
        return None
    return d if d.get("scan_src_sha256") == kernel_src_hash else None


def traffic_from_profiles(kernel_src_hash):
    """HBM bytes per genome scan launch from the committed counter runs."""
    d = counters_from_profiles("scan_genome", kernel_src_hash)
    return d.get("hbm_bytes_per_launch") if d else None


def valu_roof(insts, kernel_ms):
    """Vector ALU issue: wave instructions per launch x 64 lanes over the
    launch time, against the int32 VALU peak."""
    if not insts:
        return None
    tops = insts * 64 / (kernel_ms / 1e3) / 1e12
    return {"insts_per_launch": int(insts), "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "Tlane-ops/s", "frac": round(tops / VALU_PEAK_TOPS, 4)}


def stream_read_probe():
    """A read-only stream over 4 GiB in HBM (ah_read_probe: 128-bit loads, a
    persistent grid): the bandwidth a plain reading kernel reaches on this
    GPU, in GB/s (median of 9)."""
    import numpy as np
    import torch

    from paper_2511_00170_amd import ah
    x = torch.ones(1 << 30, dtype=torch.int32, device="cuda")
    out = torch.empty(8192, dtype=torch.int32, device="cuda")
    ah.read_probe(x, out)
    torch.cuda.synchronize()
    ts = []
    for _ in range(9):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ah.read_probe(x, out)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    del x, out
    torch.cuda.empty_cache()
    return round((4 << 30) / (float(np.median(ts)) / 1e3) / 1e9, 1)


def cpu_threads():
    """Host threads for the oracle: the CPUs this process may run on, capped by
    the OpenMP thread setting (the host's share for one GPU)."""
    n = len(os.sched_getaffinity(0))
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS") or n))
    except ValueError:
        pass
    return max(1, n)


def cpu_model():
    """The host CPU's model name (first processor entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, sample, ex, what):
    """The oracle, unmodified, timed on the leading sequences of the workload
    (whole chunks of sequences, each run as one call; the time is their sum)."""
    if not sample:
        return None
    import oracle
    nt = cpu_threads()
    dt, sb, m, n_amps = 0.0, 0, 0, 0
    for buf, off in sample:
        tc = time.perf_counter()
        o = oracle.run(buf, off, wl.pairs, wl.orient_mask, wl.tm, ex, n_threads=nt)
        dt += time.perf_counter() - tc
        sb += int(off[-1])
        m += len(off) - 1
        n_amps += len(o.amps)
    log("oracle sample: %d amplicons in %.1f s" % (n_amps, dt))
    return {"value": round(len(wl.pairs) * sb / dt / 1e9, 4), "unit": what, "cores": nt, "cpu": cpu_model(),
            "kind": "oracle",
            "sample": "first %d sequences (%.4f Gbases) of the workload, %d pairs, scan+pair+Tm+extract, %.1f s"
                      % (m, sb / 1e9, len(wl.pairs), dt)}


def _fasta_lines(s, width=80):
    """One sequence's FASTA lines (width bases each)."""
    import numpy as np
    full = len(s) // width
    body = np.empty((full, width + 1), np.uint8)
    body[:, :width] = s[:full * width].reshape(full, width)
    body[:, width] = 10
    tail = s[full * width:]
    return body.tobytes() + (tail.tobytes() + b"\n" if len(tail) else b"")


def extra_fasta(wl, store, res, ex, gbases, ps):
    """FASTA I/O: the leading ~gbases of the workload written as FASTA, one
    file per genome (80 bases a line), read into a new store by
    ah_fasta_ingest with 8 host workers and with one, and by the record-table
    pass alone (host parse, no GPU); the new store must equal the resident one
    block for block.  The AHv2 writer is timed on the run's amplicons."""
    import tempfile

    import numpy as np
    import torch

    from paper_2511_00170_amd import ah
    d = tempfile.mkdtemp(prefix="ah_fasta_")
    goal, n_bases, paths = gbases * 1e9, 0, []
    try:
        for first, buf, off in wl.chunks(1 << 30):
            for i in range(len(off) - 1):
                if n_bases >= goal:
                    break
                p = os.path.join(d, "g%05d.fa" % (first + i))
                with open(p, "wb") as fh:
                    fh.write(b">seq%d source genome\n" % (first + i))
                    fh.write(_fasta_lines(buf[int(off[i]):int(off[i + 1])]))
                paths.append(p)
                n_bases += int(off[i + 1] - off[i])
            if n_bases >= goal:
                break
        fbytes = sum(os.path.getsize(p) for p in paths)
        t0 = time.perf_counter()
        tab = ah.fasta_index(paths, n_threads=8)
        t_index = time.perf_counter() - t0
        del tab
        rates = {}
        same = True
        for nt in (8, 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ah.Store.from_fasta(paths, n_threads=nt)
            torch.cuda.synchronize()
            rates[nt] = time.perf_counter() - t0
            if nt == 8:
                # end to end: files -> store -> whole path -> AHv2 FASTA text
                r8 = ah.Pipeline(st, ps, wl.orient_mask, wl.tm, ex).run().results()
                text8 = ah.format_fasta(st.fasta, r8, ex.fb_len, ex.rb_len, tm_filter=wl.tm.filter)
                t_e2e = time.perf_counter() - t0
                del r8, text8
            nb = st.n_blocks
            ok = st.n_seqs == len(paths) and torch.equal(st.blocks[:nb], store.blocks[:nb])
            nw = nb // 32
            ok = ok and torch.equal(st.nbits[:nw], store.nbits[:nw])
            same = same and ok and torch.equal(st.nmask[:st.n_nblocks], store.nmask[:st.n_nblocks])
            del st
    finally:
        for p in paths:
            if os.path.exists(p):
                os.remove(p)
        os.rmdir(d)
    names = ah.FastaNames([b"seq%d" % i for i in range(store.n_seqs)], np.zeros(store.n_seqs, np.uint32),
                          [b"genomes.fa"])
    t0 = time.perf_counter()
    text = ah.format_fasta(names, res, ex.fb_len, ex.rb_len, tm_filter=wl.tm.filter)
    t_write = time.perf_counter() - t0
    out = {"fasta_bytes": fbytes, "files": len(paths), "bases": n_bases,
           "ingest_s": round(rates[8], 3), "ingest_GB_s": round(fbytes / rates[8] / 1e9, 3),
           "ingest_Gbases_s": round(n_bases / rates[8] / 1e9, 3), "ingest_threads": 8,
           "ingest_GB_s_one_thread": round(fbytes / rates[1] / 1e9, 3),
           "end_to_end_s": round(t_e2e, 3), "end_to_end_Gbases_s": round(n_bases / t_e2e / 1e9, 3),
           "host_index_only_GB_s": round(fbytes / t_index / 1e9, 3),
           "store_identical_to_resident": bool(same),
           "writer_records": text.count(b"\n>") + (1 if text else 0), "writer_MB": round(len(text) / 1e6, 2),
           "writer_MB_s": round(len(text) / max(t_write, 1e-9) / 1e6, 1),
           "note": "one file per genome, files in the page cache (just written): host parse + H2D + pack, "
                   "not disk reads"}
    log("fasta io: %s" % json.dumps(out))
    return out


_IUPAC_FOLD = {c: n for n, cs in ((1, "ACGTU"), (2, "RYSWKM"), (3, "BDHV"), (4, "N")) for c in cs}


def _variants(primer: str) -> int:
    v = 1
    for c in primer.upper():
        v *= _IUPAC_FOLD[c]
    return v


def bench_sweep(args, wl, store):
    """Runtime against primer degeneracy and mismatch tolerance on the genome
    store (the shape of the paper's degeneracy and mismatch tests): per point
    the whole path, timed per stage with HIP events on the stream."""
    import torch

    from paper_2511_00170_amd import ah, synth
    ex = synth.ExtractSpec(trim=wl.extract.trim, fb_len=wl.extract.fb_len, rb_len=wl.extract.rb_len)
    total = wl.total_bases
    stages = ("scan", "pair", "tm", "extract")
    out = {"metric": "sweep: whole-path time vs primer degeneracy (N bases added, one per primer) and "
                     "substitutions allowed (k)",
           "unit": "ms per step", "data": "synthetic", "n_gpus": 1, "steps": args.steps,
           "workload": "genome: %d seqs x 3-6 Mb, %.2f Gbases, base pair %s / %s, k=%d, clamp %d, FR/RF/FF/RR"
                       % (wl.n_seqs, total / 1e9, wl.pairs[0].fwd, wl.pairs[0].rev, wl.pairs[0].k,
                          wl.pairs[0].clamp)}
    stream = torch.cuda.Stream()
    only = None
    if args.sweep_points:
        only = {(p.split(":")[0], int(p.split(":")[1])) for p in args.sweep_points.split(",")}
    for kind in ("degeneracy", "mismatch"):
        rows = []
        for x, pair in synth.sweep_pairs(wl.pairs[0], kind):
            if only is not None and (kind, x) not in only:
                continue
            tc = time.perf_counter()
            ps = ah.PrimerSet([pair], jit=True)
            t_compile = time.perf_counter() - tc
            with torch.cuda.stream(stream):
                pipe = ah.Pipeline(store, ps, wl.orient_mask, wl.tm, ex)
                pipe.run(stream)
                n_hits, n_amps, n_bytes = pipe.counts()
                n_pass = int(pipe.passed[:n_amps].sum().item())
                t_w = time.perf_counter()
                while time.perf_counter() - t_w < args.warmup_s:  # clocks settle under load
                    for _ in range(8):
                        pipe.launch(stream)
                    stream.synchronize()
                torch.cuda.synchronize()
                ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)]
                      for _ in range(args.steps)]
                t0 = time.perf_counter()
                for i in range(args.steps):
                    ev[i][0].record(stream)
                    for j, stg in enumerate(stages):
                        pipe.launch(stream, (stg,))
                        ev[i][j + 1].record(stream)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / args.steps
            st_ms = {stg: round(sum(e[j].elapsed_time(e[j + 1]) for e in ev) / args.steps, 4)
                     for j, stg in enumerate(stages)}
            alg = BYTES_PER_BASE * total + 12.0 * n_hits
            row = {("n_N" if kind == "degeneracy" else "k"): x, "fwd": pair.fwd, "rev": pair.rev,
                   "variants": [_variants(pair.fwd), _variants(pair.rev)], "k": pair.k,
                   "ms_per_step": round(ms, 4), "gbases_s": round(total / (ms / 1e3) / 1e9, 1), "stage_ms": st_ms,
                   "scan_hbm_frac": round(alg / (st_ms["scan"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                   "hits": n_hits, "amplicons": n_amps, "passed": n_pass, "jit_compile_s": round(t_compile, 2)}
            log("sweep %s %s: %s" % (kind, x, json.dumps(row)))
            rows.append(row)
            del pipe, ps
        out[kind] = rows
    return out


def bench_batch(args, wl, store, sample):
    """Many pairs: one autotuned, graph-captured pass over the store against
    the plain per-pair loop (64 single-pair pipelines).  value = pair-Gbases/s
    of the graph (pairs x bases / time)."""
    import numpy as np
    import torch

    from paper_2511_00170_amd import ah, batch

    total = wl.total_bases
    ex = synth_extract(wl)
    tj = time.time()
    br = batch.BatchRunner(store, wl.pairs, wl.orient_mask, wl.tm, ex, jit=not args.generic)
    log("primer set (%d pairs) compiled in %.2f s" % (len(wl.pairs), time.time() - tj))
    tuned = None
    if not args.no_tune:
        tuned = br.tune(sample_bases=min(1e9, total / 4))
        log("autotune: %s" % json.dumps(tuned.table))
    res = br.run()                                 # eager sizing + capture + one replay
    n_hits, n_amps, n_bytes = br.pipe.counts()
    log("batch: hits %d amplicons %d pass %d bytes %d" % (n_hits, n_amps, int(res["pass"].sum()), n_bytes))
    n_warm, t_w = 0, time.perf_counter()
    while n_warm < args.warmup or time.perf_counter() - t_w < args.warmup_s:
        br.replay()
        n_warm += 1
        torch.cuda.synchronize()
    log("warm-up: %d steps in %.2f s" % (n_warm, time.perf_counter() - t_w))
    t_start = time.perf_counter()
    for _ in range(args.steps):
        br.replay()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t_start) * 1e3 / args.steps
    # scan alone, eagerly, for the roofline (same kernel and launch shape)
    with torch.cuda.stream(br.stream):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
        for a, b in ev:
            a.record(br.stream)
            br.pipe.launch(br.stream, ("scan",))
            b.record(br.stream)
        torch.cuda.synchronize()
    scan_ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    # the graph again, so the buffers hold the whole path's output
    br.replay()
    res = br.pipe.results()
    log("graph %.3f ms/step, scan %.3f ms" % (ms_step, scan_ms))
    if args.plain_reps > 0:
        plain, plain_ms = batch.plain_loop(store, wl.pairs, wl.orient_mask, wl.tm, ex, jit=not args.generic,
                                           reps=args.plain_reps)
        same = batch_outputs_equal(res, plain)
        log("plain loop %.3f ms; identical output: %s" % (plain_ms, same))
    else:
        plain_ms, same = None, None
    npairs = len(wl.pairs)
    alg_bytes = BYTES_PER_BASE * total + 12.0 * n_hits
    achieved = alg_bytes / (scan_ms / 1e3) / 1e9
    kern = "ah_scan_jit" if br.ps.jit else "ah_scan_kernel"
    variant = list(br.ps.variant) if br.ps.jit else None
    prof = counters_from_profiles("scan_batch", scan_source_hash()) if br.ps.jit else None
    if prof and prof.get("variant") != variant:
        prof = None      # counters of another tile / hit-buffer variant
    valu = valu_roof(prof.get("valu_insts_per_launch") if prof else None, scan_ms)
    out = {
        "metric": "Gbases scanned/s per primer pair (k mm) + % HBM peak; batched vs plain; p50/p99 latency",
        "value": round(npairs * total / (ms_step / 1e3) / 1e9, 2),
        "unit": "pair-Gbases/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32/f64", "data": "synthetic",
        "config": {"workload": "batch: %d seqs (log-normal chromosomes + 20%% plasmids), %.2f Gbases, %d pairs "
                               "(L 17-26, D up to 512, k 0-3, clamp 3-5), FR/RF/FF/RR, window 200-2000, "
                               "FP64 Tm filter >= 45 C" % (wl.n_seqs, total / 1e9, npairs),
                   "pairs": npairs, "bases": total, "hits": n_hits, "amplicons": n_amps,
                   "scan_kernel": "primer-set specialised (hipRTC)" if br.ps.jit else "generic",
                   "graph": True, "autotune": tuned.table if tuned else None,
                   "wg_per_cu": tuned.wg_per_cu if tuned else 0, "variant": variant, "warmup_steps_run": n_warm},
        "batched_vs_plain": {"batched_ms": round(ms_step, 3),
                             "plain_loop_ms": round(plain_ms, 3) if plain_ms else None,
                             "speedup": round(plain_ms / ms_step, 3) if plain_ms else None,
                             "identical_output": same,
                             "plain_pair_gbases_s": round(npairs * total / (plain_ms / 1e3) / 1e9, 2)
                             if plain_ms else None},
        # the scan of 256 patterns is bound by vector ALU issue: achieved =
        # measured VALU lane-ops per second (committed counters), the HBM
        # figures beside it
        "roofline": {"bound": "alu", "achieved": valu["achieved"] if valu else None,
                     "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tlane-ops/s",
                     "frac": valu["frac"] if valu else None,
                     "traffic": prof.get("hbm_bytes_per_launch") if prof else None, "kernel": kern,
                     "kernel_ms": round(scan_ms, 4),
                     "trace_kernel_ms": round(prof["trace_timed_avg_us"] / 1e3, 4)
                     if prof and prof.get("trace_timed_avg_us") else None,
                     "valu_insts_per_launch": valu["insts_per_launch"] if valu else None,
                     "valu_lane_ops_per_pair_base": round(valu["insts_per_launch"] * 64 / (npairs * total), 3)
                     if valu else None,
                     "algorithmic_bytes_per_launch": int(alg_bytes), "hbm_achieved_GB_s": round(achieved, 1),
                     "hbm_frac": round(achieved / HBM_PEAK_GBS, 4)},
        "cpu_baseline": cpu_baseline(wl, sample, ex, "pair-Gbases/s"),
    }
    return out


def bench_serve(args, wl, store):
    """Serving: closed-loop saturation throughput mu, then Poisson arrivals at
    0.5 mu and 0.8 mu; p50/p99 latency (arrival -> results on the host) over
    the measured requests and aggregate pair-Gbases/s (sum over requests of
    subset bases x pairs, over the wall time)."""
    import numpy as np
    import torch

    from paper_2511_00170_amd import serve, synth

    ex = synth_extract(wl)
    tj = time.time()
    eng = serve.ServeEngine(store, wl.pairs, wl.tm, ex, wl.orient_mask, pool_k=3,
                            budget_bytes=args.budget_mb << 20)
    log("pool of %d pairs compiled in %.2f s" % (len(wl.pairs), time.time() - tj))
    lens = store.lengths.astype(np.int64)
    n_w, n_m = args.warm_requests, args.requests

    def work(reqs):
        return sum(float(lens[r.seqs].sum()) * len(r.pairs) for r in reqs)

    def run(qps, seed):
        reqs = synth.gen_requests(wl, n_w + n_m, qps=qps, seed=seed)
        eng.sched.stats = serve.SchedStats()
        eng.exe.host_s = dict(launch=0.0, wait=0.0, d2h=0.0, collect=0.0, batches=0, bytes=0)
        t0 = time.perf_counter()
        out = eng.serve(reqs)
        wall = time.perf_counter() - t0
        meas = [r for r in reqs if r.rid >= n_w]
        # measured window: from the first measured arrival to the last completion
        t_a = t0 + min(r.arrival_s for r in meas)
        t_b = max(out[r.rid].done_s for r in meas)
        lat = serve.latency_summary({r.rid: out[r.rid] for r in meas})
        sizes = eng.sched.stats.batch_sizes
        res = {"qps_offered": None if qps == 0 else round(qps, 2), "requests": n_m,
               "req_per_s": round(n_m / (t_b - t_a), 2) if qps else round(n_m / (t_b - t0), 2),
               "pair_gbases_s": round(work(meas) / ((t_b - t_a) if qps else (t_b - t0)) / 1e9, 2),
               "latency": lat, "batches": len(sizes), "mean_batch": round(float(np.mean(sizes)), 2),
               "wall_s": round(wall, 2),
               "host_ms_per_batch": {k: round(1e3 * v / max(eng.exe.host_s["batches"], 1), 3)
                                     for k, v in eng.exe.host_s.items() if k not in ("batches", "bytes")},
               "result_mb_per_batch": round(eng.exe.host_s.get("bytes", 0) / max(eng.exe.host_s["batches"], 1) / 1e6,
                                            3)}
        log("serve %s: %s" % ("closed" if qps == 0 else "qps %.1f" % qps, json.dumps(res)))
        return res

    eng.serve(synth.gen_requests(wl, 8, qps=0, seed=99))   # warm the executor's buffers
    # the same kind of requests served one per pass (no batching), closed loop
    one = synth.gen_requests(wl, max(8, n_m // 20), qps=0, seed=7)
    eng.sched.max_requests = 1
    t1 = time.perf_counter()
    eng.serve(one)
    dt1 = time.perf_counter() - t1
    eng.sched.max_requests = serve.MAX_REQ_PER_BATCH
    single = {"requests": len(one), "req_per_s": round(len(one) / dt1, 2),
              "pair_gbases_s": round(work(one) / dt1 / 1e9, 2)}
    log("serve one-at-a-time: %s" % json.dumps(single))
    closed = run(0.0, seed=1)
    mu = closed["req_per_s"]
    open_runs = [run(f * mu, seed=2 + i) for i, f in enumerate((0.5, 0.8))]
    # scan roofline: the masked scan of the last batch shape, timed alone
    nh = eng.exe.last_counts[0] if eng.exe.last_counts else 0
    kern = "ah_scan_jit" if eng.exe.pool_ps.jit else "ah_scan_kernel"
    total = wl.total_bases
    out = {
        "metric": "Gbases scanned/s per primer pair (k mm) + % HBM peak; batched vs plain; p50/p99 latency",
        "value": closed["pair_gbases_s"], "unit": "pair-Gbases/s", "n_gpus": 1, "steps": n_m, "warmup": n_w,
        "ms_per_step": round(1e3 / mu, 4) if mu else None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32/f64", "data": "synthetic",
        "config": {"workload": "serve: %d seqs x 3-5 Mb, %.2f Gbases resident, pool of %d pairs; requests of "
                               "1-8 pairs x 100-5000 sequences, k 0-3, Tm threshold 40-60 C; step = one request"
                               % (wl.n_seqs, total / 1e9, len(wl.pairs)),
                   "pairs": len(wl.pairs), "bases": total, "budget_mb": args.budget_mb, "scan_kernel": kern},
        "serve": {"closed_loop": closed, "poisson_0.5mu": open_runs[0], "poisson_0.8mu": open_runs[1],
                  "one_request_per_pass": single,
                  "batching_speedup": round(closed["req_per_s"] / single["req_per_s"], 3)},
        "roofline": None, "cpu_baseline": None,
    }
    return out


def make_store(wl):
    from paper_2511_00170_amd import ah
    t0 = time.time()
    store = ah.Store(wl.lengths)
    store.pack_chunks(wl.chunks(1 << 30))
    log("workload %s: %d sequences, %.3f Gbases, generated + packed in %.1f s"
        % (wl.name, wl.n_seqs, wl.total_bases / 1e9, time.time() - t0))
    return store


def extra_batch(args):
    """Batched (one graph, all 64 pairs) against the plain per-pair loop on the
    9 Gb many-pair workload; returned as a sub-object of the main line."""
    from paper_2511_00170_amd import synth
    wl = synth.gen_config(3)
    store = make_store(wl)
    # a batched step is ~50 ms: at most 20 timed steps here
    o = bench_batch(argparse.Namespace(**{**vars(args), "steps": min(args.steps, 20)}), wl, store, None)
    r = dict(o["batched_vs_plain"])
    r.update({"workload": o["config"]["workload"], "pairs": o["config"]["pairs"], "bases": o["config"]["bases"],
              "batched_pair_gbases_s": o["value"], "unit": "pair-Gbases/s", "scan_ms": o["roofline"]["kernel_ms"],
              "scan_bound": "alu", "scan_valu_frac": o["roofline"]["frac"], "scan_hbm_frac": o["roofline"]["hbm_frac"],
              "variant": o["config"]["variant"], "wg_per_cu": o["config"]["wg_per_cu"]})
    return r


def extra_serve(args):
    """Continuous batching on the 19.9 Gb serving store: per arrival rate,
    2000 measured requests after 200 warm-up ones by default."""
    import copy

    from paper_2511_00170_amd import synth
    wl = synth.gen_config(5)
    store = make_store(wl)
    a = copy.copy(args)
    a.requests, a.warm_requests = args.extra_requests, max(1, args.extra_requests // 10)
    o = bench_serve(a, wl, store)
    r = dict(o["serve"])
    r.update({"workload": o["config"]["workload"], "unit": "pair-Gbases/s",
              "requests_per_run": a.requests, "warmup_per_run": a.warm_requests})
    return r


def synth_extract(wl):
    from paper_2511_00170_amd import synth
    return synth.ExtractSpec(trim=wl.extract.trim, fb_len=wl.extract.fb_len, rb_len=wl.extract.rb_len)


def batch_outputs_equal(a, b):
    import numpy as np

    from paper_2511_00170_amd import ah
    try:
        ok = np.array_equal(ah.hits_canonical(a["hits"]), ah.hits_canonical(b["hits"]))
        ok &= np.array_equal(ah.amps_array(a["amps"]), ah.amps_array(b["amps"]))
        ok &= np.array_equal(a["amps"]["flags"], b["amps"]["flags"])
        for k in ("tm", "tm_site", "pass", "seq_off", "fb", "rb", "bc_len", "fprimer", "rprimer"):
            if k in a:
                ok &= np.array_equal(a[k], b[k])
        if "seq" in a:
            ok &= a["seq"] == b["seq"]
        return bool(ok)
    except Exception as e:  # shape mismatch etc.
        log("compare failed: %r" % (e,))
        return False


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: one GPU only; --gpus %d is not supported (use --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2511_00170_amd import ah, synth

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src_t = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t
    t0 = time.time()
    if args.serve:
        args.config = 5
    if args.sweep:
        args.config, args.no_cpu_baseline = 2, True
    wl = synth.gen_config(args.config, n_seqs=args.n_seqs, len_scale=args.len_scale)
    total = wl.total_bases
    log("workload %s: %d sequences, %.3f Gbases" % (wl.name, wl.n_seqs, total / 1e9))
    sample = []
    # about 10 s of oracle work: ~8 Gbases for one pair, less for many
    sample_goal = args.cpu_sample_bases or (8.0e9 if len(wl.pairs) == 1 else 1.0e8)
    taken = 0

    def chunks():
        nonlocal taken
        for first, buf, off in wl.chunks(1 << 30):
            if taken < sample_goal and not args.no_cpu_baseline:
                # bounded oracle sample: the leading sequences of the workload
                m = int(np.searchsorted(off, sample_goal - taken, side="right"))
                m = max(1, min(m, len(off) - 1))
                sample.append((buf[:int(off[m])].copy(), off[:m + 1].copy()))
                taken += int(off[m])
            yield first, buf, off

    store = ah.Store(wl.lengths)
    store.pack_chunks(chunks())
    log("generated + packed in %.1f s (store %.2f GB)" % (time.time() - t0, store.hbm_bytes / 1e9))
    if args.serve:
        print(json.dumps(bench_serve(args, wl, store)), flush=True)
        return
    if args.sweep:
        print(json.dumps(bench_sweep(args, wl, store)), flush=True)
        return
    if len(wl.pairs) > 1:
        out = bench_batch(args, wl, store, sample)
        print(json.dumps(out), flush=True)
        if out["batched_vs_plain"]["identical_output"] is False:
            sys.exit(1)
        return

    tj = time.time()
    ps = ah.PrimerSet(wl.pairs, jit=not args.generic)
    log("primer set compiled in %.2f s (specialised scan kernel: %s)" % (time.time() - tj, ps.jit))
    ex = synth.ExtractSpec(trim=wl.extract.trim, fb_len=wl.extract.fb_len, rb_len=wl.extract.rb_len)
    stream = torch.cuda.Stream()
    tuned = None
    if ps.jit and not args.no_tune:
        # the autotuner's pick of tile size, hit buffer and workgroups per CU
        # (every variant gives the same hits), timed on the whole store (a
        # scan takes under a millisecond; a sample can rank the grids
        # differently)
        from paper_2511_00170_amd import batch
        tt = time.time()
        tuned = batch.tune_scan(store, ps, wl.pairs, wl.orient_mask, wl.tm, stream,
                                sample_bases=float(total), reps=9, tolerance=0.01, variants=((2, 48), (1, 48)))
        log("scan tuned in %.1f s: variant %s, %d workgroups per CU (%.4f ms on the sample)"
            % (time.time() - tt, tuned.variant, tuned.wg_per_cu, tuned.ms))
    stages = tuple(args.stages.split(","))
    # Passes alternate between `depth` pipelines (buffers) on as many
    # streams: pass i + 1's scan starts while pass i's pair, Tm and extract
    # (small, latency-bound kernels) and its scan's last workgroups finish.
    # Every pass is the whole path over the whole store.
    depth = max(1, args.depth)
    streams = [stream] + [torch.cuda.Stream() for _ in range(depth - 1)]
    pipes = []
    for s_ in streams:
        with torch.cuda.stream(s_):
            p_ = ah.Pipeline(store, ps, wl.orient_mask, wl.tm, ex)
            p_.run(s_)                          # sizes the capacities (exact re-run on overflow)
            pipes.append(p_)
    pipe = pipes[0]
    n_hits, n_amps, n_bytes = pipe.counts()
    for p_ in pipes[1:]:
        if p_.counts() != (n_hits, n_amps, n_bytes):
            raise RuntimeError("pipelines disagree")
    log("hits %d amplicons %d pass %d bytes %d" % (n_hits, n_amps, int(pipe.passed[:n_amps].sum().item()), n_bytes))
    n_warm, t_w = 0, time.perf_counter()
    while n_warm < args.warmup or time.perf_counter() - t_w < args.warmup_s:
        for j in range(8):
            pipes[j % depth].launch(streams[j % depth], stages)
        n_warm += 8
        torch.cuda.synchronize()
    log("warm-up: %d steps in %.2f s" % (n_warm, time.perf_counter() - t_w))
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        pipes[i % depth].launch(streams[i % depth], stages)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ms_step = (t_end - t_start) * 1e3 / args.steps
    # the dominant kernel alone: the same scan launched back to back on its
    # stream right after the timed region, each launch between its own events
    # (inside the timed region a launch's events would also count the other
    # stream's work)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    with torch.cuda.stream(stream):
        for a_, b_ in ev:
            a_.record(stream)
            pipe.launch(stream, ("scan",))
            b_.record(stream)
        torch.cuda.synchronize()
    scan_ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    if pipe.counts() != (n_hits, n_amps, n_bytes):
        raise RuntimeError("scan results changed")
    gbases_s = total / (ms_step / 1e3) / 1e9
    alg_bytes = BYTES_PER_BASE * total + 12.0 * n_hits
    achieved = alg_bytes / (scan_ms / 1e3) / 1e9
    prof = counters_from_profiles("scan_genome", scan_source_hash()) if ps.jit else None
    if prof and prof.get("variant") != (list(ps.variant) if ps.variant else None):
        prof = None      # counters of another tile / hit-buffer variant
    traffic = prof.get("hbm_bytes_per_launch") if prof else None
    # the committed kernel trace of the same command: its timed dispatches'
    # average, beside this run's event timing
    trace_ms = prof.get("trace_timed_avg_us") / 1e3 if prof and prof.get("trace_timed_avg_us") else None
    stream_gbs = stream_read_probe()
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "ah_scan_jit" if ps.jit else "ah_scan_kernel", "kernel_ms": round(scan_ms, 4),
            "kernel_ms_timing": "HIP events around each of `steps` back-to-back scan launches on its stream, "
                                "right after the timed region",
            "trace_kernel_ms": round(trace_ms, 4) if trace_ms else None,
            "trace_frac": round(alg_bytes / (trace_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if trace_ms else None,
            "trace_wg_per_cu": prof.get("trace_wg_per_cu") if trace_ms else None,
            "algorithmic_bytes_per_launch": int(alg_bytes),
            "measured_hbm_frac": round(traffic / (scan_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
            "stream_read_GB_s": stream_gbs, "frac_of_stream_read": round(achieved / stream_gbs, 4),
            "valu": valu_roof(prof.get("valu_insts_per_launch") if prof else None, scan_ms)}

    cpu = cpu_baseline(wl, sample, ex, "Gbases/s")

    out = {
        "metric": "Gbases scanned/s per primer pair (k mm) + % HBM peak; batched vs plain; p50/p99 latency",
        "value": round(gbases_s, 2),
        "unit": "Gbases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/f64",
        "data": "synthetic",
        "config": {"workload": "genome: %d seqs x 3-6 Mb, %.2f Gbases, 1 pair (19/21 nt, D=16/32), k=%d, clamp %d, "
                               "FR/RF/FF/RR, window 200-2000, FP64 Tm filter >= 45 C"
                               % (wl.n_seqs, total / 1e9, wl.pairs[0].k, wl.pairs[0].clamp),
                   "pairs": len(wl.pairs), "k": wl.pairs[0].k, "bases": total, "stages": list(stages),
                   "hits": n_hits, "amplicons": n_amps,
                   "scan_kernel": "primer-set specialised (hipRTC)" if ps.jit else "generic",
                   "scan_tile_bases": 4096 * (ps.variant[0] if ps.jit and ps.variant else 1),
                   "scan_hit_buffer": ps.variant[1] if ps.jit and ps.variant else 48,
                   "scan_wg_per_cu": tuned.wg_per_cu if tuned else None,
                   "warmup_steps_run": n_warm, "pipeline_depth": depth},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if not args.no_extras:
        out["fasta_io"] = extra_fasta(wl, store, pipe.results(), ex, args.fasta_gbases, ps)
        # the other two parts of the metric, on their own workloads
        del pipe, pipes, ps
        store = None
        torch.cuda.empty_cache()
        out["batched_vs_plain"] = extra_batch(args)
        torch.cuda.empty_cache()
        out["serving"] = extra_serve(args)
    print(json.dumps(out), flush=True)
    if out.get("batched_vs_plain") and out["batched_vs_plain"]["identical_output"] is False:
        sys.exit(1)


if __name__ == "__main__":
    main()
