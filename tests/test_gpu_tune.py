"""Automatic and measured choices of the FLASH parallelism never change a
result: P <= 0 and the tuner's pick decode exactly as the oracle."""
import numpy as np
import pytest

import oracle
from workloads import hmm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fv():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2510_19301_amd as m
    m.lib()
    return m


def _dev(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _bits(x):
    return np.asarray(x, np.float32).reshape(-1).view(np.uint32)


@pytest.mark.parametrize("K,T", [(20, 1), (50, 40), (64, 700), (130, 300)])
def test_auto_parallelism_is_exact(fv, K, T):
    lp, la, lb = hmm.random_dense(K, T, 70 + K + T)
    po, so, rc = oracle.vanilla(lp, la, lb)
    p, s, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="flash", P=0)
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == rc and (p.cpu().numpy() == po).all() and _bits(s.cpu().numpy()) == _bits(so)


def test_tuner_picks_a_candidate_and_keeps_results(fv):
    K = 96
    _, la, _ = hmm.random_dense(K, 1, 71)
    rng = np.random.default_rng(72)
    lens = [300, 700, 50, 1200, 999]
    lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in lens]
    batch = fv.Batch([_dev(x) for x in lbs])
    best, times = fv.best_parallelism(_dev(la), batch, None, candidates=(4, 16, 64))
    assert best in (4, 16, 64) and set(times) == {4, 16, 64}
    torch.cuda.synchronize()
    paths, scores = batch.paths.cpu().numpy(), batch.scores.cpu().numpy()
    for b, T in enumerate(lens):
        po, so, rc = oracle.vanilla(None, la, lbs[b])
        assert (paths[b, :T] == po).all() and _bits(scores[b]) == _bits(so)
