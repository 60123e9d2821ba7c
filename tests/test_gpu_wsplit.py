"""GPU parity of w-way subtasks: FLASH on wide rows with K above the leaf
limit (K = 2112 here) splits each subtask [m, n] into up to 8 segments with
the root's division rule over its own span, resolves all division states at
its end from snapshots of delta and of the division chain, and spawns one
child per segment of two or more positions (Sec. V-A's P-way split applied
at every level; the bisection of Alg. 1 is the 2-way case).

FLASH equals vanilla for every schedule (anchored start, Sec. V-B Def. 3),
so every decode must equal the oracle's vanilla result: paths element by
element, scores bit for bit.  Lengths cover subtasks shorter than the split
width (every position a division) up to several split levels; P covers the
serial root (P = 1) to many segments.  FV_FLAG_NO_LEAVES and the relative
start keep the bisection and must stay exact too."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from workloads import hmm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K = 2112


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


@pytest.mark.parametrize("T", [2, 3, 9, 17, 65, 300, 1000])
@pytest.mark.parametrize("P", [1, 2, 5, 16])
def test_wsplit_single_matches_oracle(fv, T, P):
    lp, la, lb = hmm.random_dense(K, T, 17 * T + P)
    po, so, rc = oracle.vanilla(lp, la, lb)
    assert rc == oracle.OK
    print(f"w-way K={K} T={T} P={P}", flush=True)
    path, score, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="flash", P=P, rows="wide")
    torch.cuda.synchronize()
    assert int(st.item()) == fv.FV_OK
    assert (path.cpu().numpy() == po).all(), np.flatnonzero(path.cpu().numpy() != po)[:10]
    assert _bits(score.cpu().numpy()) == _bits(so)


@pytest.mark.parametrize("kind", ["integer", "neginf"])
def test_wsplit_ties_and_neginf(fv, kind):
    T = 129
    if kind == "integer":
        lp, la, lb = hmm.random_dense(K, T, 5, integer=True, lo=-2, hi=0)
    else:
        lp, la, lb = hmm.random_dense(K, T, 6, neg_inf_frac=0.6)
    po, so, rc = oracle.vanilla(lp, la, lb)
    for P in (1, 4):
        path, score, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="flash", P=P, rows="wide")
        torch.cuda.synchronize()
        assert int(st.item()) == (fv.FV_OK if rc == oracle.OK else fv.FV_E_INFEASIBLE)
        assert (path.cpu().numpy() == po).all()
        assert _bits(score.cpu().numpy()) == _bits(so)


def test_wsplit_batch_and_bisection_flags(fv):
    """A batch of three uneven sequences (one launch), then the same with
    FV_FLAG_NO_LEAVES (Alg. 1's bisection) and, on integer inputs where every
    sum is exact, with the relative start (bisection too)."""
    rng = np.random.default_rng(9)
    lp, la, _ = hmm.random_dense(K, 1, 9)
    lens = [250, 7, 611]
    lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in lens]
    with ThreadPoolExecutor(3) as ex:
        refs = list(ex.map(lambda x: oracle.vanilla(lp, la, x), lbs))
    for leaves in (True, False):
        batch = fv.Batch([_dev(x) for x in lbs])
        fv.decode_batch(_dev(la), batch, _dev(lp), method="flash", P=8, rows="wide", leaves=leaves)
        torch.cuda.synchronize()
        assert (batch.status.cpu().numpy() == fv.FV_OK).all()
        for b, (po, so, _) in enumerate(refs):
            assert (batch.paths[b, :lens[b]].cpu().numpy() == po).all(), (leaves, b)
            assert _bits(batch.scores[b].cpu().numpy()) == _bits(so)
    lpi, lai, lbi = hmm.random_dense(K, 140, 10, integer=True, lo=-2, hi=0)
    po, so, _ = oracle.vanilla(lpi, lai, lbi)
    path, score, st = fv.decode(_dev(lai), _dev(lbi), _dev(lpi), method="flash", P=4, rows="wide",
                                relative_init=True)
    torch.cuda.synchronize()
    assert (path.cpu().numpy() == po).all() and _bits(score.cpu().numpy()) == _bits(so)
