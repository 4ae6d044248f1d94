"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same seeded input and compare element by element."""
import math

import numpy as np

import oracle

TM_TOL = 1e-9  # degrees C, FP64 (same operation order on both sides)


def gpu_run(store, pairs, orient_mask, tm, ex=None, subset=None, caps=None, jit=False, variant=None):
    from paper_2511_00170_amd import ah
    import torch
    ps = ah.PrimerSet(pairs, jit=jit and variant is None)
    if variant is not None:
        ps.jit_variant(*variant)
    sub = None
    if subset is not None:
        sub = torch.from_numpy(np.asarray(subset, np.uint32).view(np.int32)).cuda()
    pipe = ah.Pipeline(store, ps, orient_mask, tm, ex, caps=caps, subset=sub)
    pipe.run()
    r = pipe.results()
    r["_pipe"] = pipe
    return r


def compare_hits(gpu_hits, o_hits, o_mm):
    from paper_2511_00170_amd import ah
    g = ah.hits_canonical(gpu_hits)
    o = np.concatenate([o_hits.astype(np.int64), o_mm.astype(np.int64)[:, None]], axis=1)
    assert g.shape == o.shape, (g.shape, o.shape)
    if len(o):
        bad = np.nonzero((g != o).any(axis=1))[0]
        assert len(bad) == 0, ("hit mismatch", g[bad[:5]], o[bad[:5]])


def compare_amps(gpu_amps, o_amps):
    from paper_2511_00170_amd import ah
    g = ah.amps_array(gpu_amps)
    o = o_amps.astype(np.int64)
    assert g.shape == o.shape, (g.shape, o.shape)
    if len(o):
        bad = np.nonzero((g != o).any(axis=1))[0]
        assert len(bad) == 0, ("amplicon mismatch", g[bad[:5]], o[bad[:5]])


def compare_tm(g_tm, g_site, g_pass, o):
    assert len(g_tm) == len(o.tm)
    for a, b in ((g_tm, o.tm), (g_site.reshape(-1), o.tm_site.reshape(-1))):
        fin = np.isfinite(b)
        assert (np.isfinite(a) == fin).all()
        assert (a[~fin] == b[~fin]).all()
        if fin.any():
            d = np.abs(a[fin] - b[fin]).max()
            assert d <= TM_TOL, d
    assert (g_pass == o.passed).all()


def compare_extract(r, e):
    assert r["seq"] == e.seq
    assert (r["amps"]["flags"] == e.flags).all()
    assert (r["seq_off"] == e.seq_off).all()
    assert (r["bc_len"] == e.bc_len).all()
    if r["fb"].shape[1]:
        assert (r["fb"] == e.fb).all()
    if r["rb"].shape[1]:
        assert (r["rb"] == e.rb).all()
    assert (r["fprimer"] == e.fprimer).all()
    assert (r["rprimer"] == e.rprimer).all()


# scan kernels: the generic one and the specialised one in every variant
# (blocks per lane, LDS hit buffer) the autotuner may pick
KERNELS = {"generic": (False, None), "jit": (True, None), "jit-1x48": (True, (1, 48)), "jit-1x16": (True, (1, 16)),
           "jit-2x16": (True, (2, 16))}


def full_parity(store, ascii_buf, off, pairs, orient_mask, tm, ex=None, n_threads=None, jit=False, variant=None):
    """Run both sides on the same input; assert every output agrees."""
    r = gpu_run(store, pairs, orient_mask, tm, ex, jit=jit, variant=variant)
    o = oracle.run(ascii_buf, off, pairs, orient_mask, tm, ex, n_threads=n_threads)
    compare_hits(r["hits"], o.hits, o.mm)
    compare_amps(r["amps"], o.amps)
    compare_tm(r["tm"], r["tm_site"], r["pass"], o.tm)
    if ex is not None:
        compare_extract(r, o.ext)
    return r, o
