"""FLASH schedules: leaf subtasks (default for dense K <= 2048 with rows on
their XCD) and full bisection (FV_FLAG_NO_LEAVES) both reproduce vanilla
bit for bit, for lengths that make segments leaves, bisect them first, or
mix both, and for the placements where leaves are off (wide rows, K > 2048)."""
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


@pytest.mark.parametrize("K,T", [(37, 63), (37, 127), (37, 128), (37, 129), (64, 300), (100, 513), (256, 260)])
@pytest.mark.parametrize("P", [1, 2, 5])
@pytest.mark.parametrize("leaves", [True, False])
def test_flash_schedules_match_vanilla(fv, K, T, P, leaves):
    lp, la, lb = hmm.random_dense(K, T, 90 + K + T)
    po, so, rc = oracle.vanilla(lp, la, lb)
    p, s, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="flash", P=P, leaves=leaves)
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == rc and (p.cpu().numpy() == po).all() and _bits(s.cpu().numpy()) == _bits(so)


@pytest.mark.parametrize("K,T", [(12, 90), (30, 300)])
def test_flash_leaves_integer_ties(fv, K, T):
    lp, la, lb = hmm.random_dense(K, T, 7 * K + T, integer=True, lo=-2, hi=0)
    po, so, rc = oracle.vanilla(lp, la, lb)
    for P in (1, 3, 8):
        for leaves in (True, False):
            p, s, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="flash", P=P, leaves=leaves)
            torch.cuda.synchronize()
            assert (p.cpu().numpy() == po).all() and _bits(s.cpu().numpy()) == _bits(so), (P, leaves)


def test_flash_leaves_batch_and_placements(fv):
    rng = np.random.default_rng(91)
    for K, rows in ((64, "local"), (64, "wide"), (2100, "auto")):
        _, la, _ = hmm.random_dense(K, 1, 92 + K)
        lens = [1, 2, 128, 129, 260, 600] if K < 2000 else [1, 70, 140]
        lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in lens]
        batch = fv.Batch([_dev(x) for x in lbs])
        fv.decode_batch(_dev(la), batch, None, method="flash", P=3, rows=rows)
        torch.cuda.synchronize()
        paths, scores = batch.paths.cpu().numpy(), batch.scores.cpu().numpy()
        for b, T in enumerate(lens):
            po, so, rc = oracle.vanilla(None, la, lbs[b])
            assert (paths[b, :T] == po).all() and _bits(scores[b]) == _bits(so), (K, rows, b)


def test_flash_leaves_infeasible(fv):
    K, T = 20, 150
    lp, la, lb = hmm.random_dense(K, T, 93)
    la[:] = -np.inf
    p, s, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="flash", P=2)
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == fv.FV_E_INFEASIBLE and (p.cpu().numpy() == -1).all()
