"""ah_scan_primers_static (the scan with the library's fixed scratch array as
its workspace, for callers that cannot allocate) gives the same hits as
ah_scan_primers with a caller workspace: two calls in a row on one GPU, the
second over fewer sequences, for the generic and the specialised kernel; a
list longer than the scratch allows is refused before any work."""
import ctypes as C

import numpy as np
import pytest

from paper_2511_00170_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ah():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00170_amd import ah
    return ah


def _hits(ah, store, ps, subset, static):
    cap = 1 << 16
    hits = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
    n = torch.zeros(1, dtype=torch.int64, device="cuda")
    if static:
        ah.scan_primers_static(store, ps, hits, cap, n, subset)
    else:
        n_list = store.n_seqs if subset is None else int(subset.numel())
        ws = torch.empty(ah.ws_scan(store, n_list) // 8 + 1, dtype=torch.int64, device="cuda")
        ah.scan_primers(store, ps, hits, cap, n, ws, subset)
    torch.cuda.synchronize()
    k = int(n.item())
    assert k <= cap
    return k, ah.hits_canonical(hits[:k].cpu().numpy().view(np.uint8).reshape(-1).view(ah.HIT_DTYPE))


@pytest.mark.parametrize("kernel", ["generic", "jit"])
def test_static_scan_equals_workspace_scan(ah, kernel):
    wl = synth.gen_config(1, n_seqs=160)
    store = ah.Store.from_workload(wl)
    ps = ah.PrimerSet(wl.pairs, jit=kernel == "jit")
    rng = np.random.default_rng(11)
    small = np.sort(rng.choice(wl.n_seqs, 37, replace=False)).astype(np.uint32)
    # every sequence, then a smaller list (the array keeps the first call's
    # contents: the second must not depend on them)
    for subset in (None, torch.from_numpy(small.view(np.int32)).cuda()):
        print("static scan", kernel, "all" if subset is None else len(small), flush=True)
        n_ws, h_ws = _hits(ah, store, ps, subset, static=False)
        n_st, h_st = _hits(ah, store, ps, subset, static=True)
        assert n_ws == n_st and n_ws > 0
        assert np.array_equal(h_ws, h_st)


def test_static_scan_refuses_a_list_beyond_the_scratch(ah):
    wl = synth.gen_config(1, n_seqs=4)
    store = ah.Store.from_workload(wl)
    ps = ah.PrimerSet(wl.pairs)
    hits = torch.empty((16, 3), dtype=torch.int32, device="cuda")
    n = torch.zeros(1, dtype=torch.int64, device="cuda")
    lst = torch.zeros(4, dtype=torch.int32, device="cuda")
    # the length is checked on the host before anything is launched or read
    st = ah._lib.ah_scan_primers_static(C.byref(store.c), ps.h, C.c_void_p(lst.data_ptr()),
                                        ah.STATIC_SCAN_MAX_LIST + 1, C.c_void_p(hits.data_ptr()), 16,
                                        C.c_void_p(n.data_ptr()), ah._stream())
    assert st == ah.AH_E_SCRATCH
    torch.cuda.synchronize()
    assert int(n.item()) == 0
