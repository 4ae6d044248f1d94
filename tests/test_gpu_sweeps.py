"""GPU parity at every point of the degeneracy and mismatch sweeps (the
primer constructions the benchmark's sweep times): N bases appended to the 5'
ends of both primers (0-6 in all) and k = 0..6, on a reduced genome workload,
both scan kernels, every output against the oracle."""
import pytest

from paper_2511_00170_amd import synth
from paper_2511_00170_amd.synth import ExtractSpec
from tests import _parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00170_amd import ah
    wl = synth.gen_config(2, n_seqs=24, len_scale=0.02)   # 24 x 60-120 kb
    buf, off = wl.concat()
    return ah, wl, buf, off, ah.Store.from_workload(wl)


def _point(env, pair, jit):
    ah, wl, buf, off, st = env
    print("sweep point", pair.fwd, pair.rev, "k", pair.k, "jit", jit, flush=True)
    return P.full_parity(st, buf, off, [pair], wl.orient_mask, wl.tm, ExtractSpec(trim=True, fb_len=8, rb_len=8),
                         jit=jit)


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("i", range(len(synth.SWEEP_N)))
def test_degeneracy_point_matches_oracle(env, i, jit):
    n, pair = synth.sweep_pairs(env[1].pairs[0], "degeneracy")[i]
    r, o = _point(env, pair, jit)
    assert len(o.amps) > 0


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("k", synth.SWEEP_K)
def test_mismatch_point_matches_oracle(env, k, jit):
    _, pair = synth.sweep_pairs(env[1].pairs[0], "mismatch")[k]
    r, o = _point(env, pair, jit)
    assert len(o.hits) > 0
