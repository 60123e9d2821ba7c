"""GPU parity of the column-slab step (dense model with K = 512 or 1024,
rows kept on their XCD, at most 160 rows per XCD): every block holds a slab
of log A in registers and takes an even share of (row, column pass) units.

Batches of uneven lengths (1 to 700 steps) decode in one launch with vanilla
and FLASH (several P, with and without leaf subtasks, and the relative
start), and every sequence must equal the oracle (FLASH = vanilla for every
P under the anchored start, Sec. V-B Def. 3): paths element by element,
scores bit for bit.  Inputs cover float scores, small integers (many exact
ties, so the lowest-index rule decides), -inf transitions (all--inf
columns) and signed zeros on both sides of a 64-column boundary."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from workloads import hmm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LENS = [1, 2, 3, 17, 64, 65, 129, 200, 257, 700, 5, 130]


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


def _instance(K, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "float":
        lp, la, _ = hmm.random_dense(K, 1, seed)
        lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in LENS]
    elif kind == "integer":
        la = rng.integers(-3, 1, size=(K, K)).astype(np.float32)
        lp = rng.integers(-3, 1, size=K).astype(np.float32)
        lbs = [rng.integers(-3, 1, size=(T, K)).astype(np.float32) for T in LENS]
    else:   # "neginf": half of log A is -inf, some whole columns too
        lp, la, _ = hmm.random_dense(K, 1, seed, neg_inf_frac=0.5)
        la[:, rng.choice(K, 5, replace=False)] = -np.inf
        lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in LENS]
    return lp, la, lbs


def _check(fv, lp, la, lbs, method, P, leaves=True, relative_init=False):
    batch = fv.Batch([_dev(x) for x in lbs])
    fv.decode_batch(_dev(la), batch, _dev(lp), method=method, P=P, rows="local", leaves=leaves,
                    relative_init=relative_init)
    torch.cuda.synchronize()
    st = batch.status.cpu().numpy()
    paths, scores = batch.paths.cpu().numpy(), batch.scores.cpu().numpy()
    with ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(lambda x: oracle.vanilla(lp, la, x), lbs))
    for b, (x, (po, so, rc)) in enumerate(zip(lbs, refs)):
        T = x.shape[0]
        assert st[b] == (fv.FV_OK if rc == oracle.OK else fv.FV_E_INFEASIBLE), (b, st[b], rc)
        assert (paths[b, :T] == po).all(), (b, T, np.flatnonzero(paths[b, :T] != po)[:8])
        assert _bits(scores[b]) == _bits(so), (b, scores[b], so)


@pytest.mark.parametrize("K", [512, 1024])
@pytest.mark.parametrize("kind", ["float", "integer", "neginf"])
@pytest.mark.parametrize("method,P,leaves", [("vanilla", 1, True), ("flash", 1, True), ("flash", 16, True),
                                             ("flash", 4, False), ("flash", 64, True)])
def test_slab_batch_matches_oracle(fv, K, kind, method, P, leaves):
    print(f"slab K={K} {kind} {method} P={P} leaves={leaves}", flush=True)
    lp, la, lbs = _instance(K, kind, 1000 + K + len(kind))
    _check(fv, lp, la, lbs, method, P, leaves)


@pytest.mark.parametrize("K", [512, 1024])
def test_slab_relative_init_on_integers(fv, K):
    """The paper's displayed subtask start (carried score dropped) is exact
    when every float32 sum is exact: integer inputs return vanilla's path."""
    lp, la, lbs = _instance(K, "integer", 77 + K)
    _check(fv, lp, la, lbs, "flash", 8, relative_init=True)


@pytest.mark.parametrize("K", [512, 1024])
@pytest.mark.parametrize("T", [1, 2, 40])
def test_slab_signed_zero_across_columns(fv, K, T):
    """Scores -0 (state 70) and +0 (state 90), other states far lower: the
    states sit in different 64-column units of the slab; -0 and +0 are equal,
    so the lower index wins and its score keeps its sign."""
    lp = np.full(K, -5.0, np.float32)
    lp[70], lp[90] = -0.0, 0.0
    la = np.full((K, K), -np.inf, np.float32)
    la[70, 70], la[90, 90] = -0.0, 0.0
    lbs = []
    for _ in range(3):
        lb = np.full((T, K), -1.0, np.float32)
        lb[:, 70], lb[:, 90] = -0.0, 0.0
        lbs.append(lb)
    po, so, _ = oracle.vanilla(lp, la, lbs[0])
    assert po[-1] == 70 and _bits(so)[0] == 0x80000000
    for method, P in (("vanilla", 1), ("flash", 4)):
        _check(fv, lp, la, lbs, method, P)


@pytest.mark.parametrize("seed,B,P", [(610, 2, 1), (610, 2, 2), (2428, 2, 2)])
def test_slab_beam_fallback_exact_redecode(fv, seed, B, P):
    """A narrow beam loses a subtask's known end state; the subtask is then
    re-decoded exactly as a dense subtask on column slabs.  A small sparse
    integer instance is embedded in K = 512 (the other states unreachable:
    -inf start, transitions into and out of them -inf), so the beams, and the
    fallback, are the small instance's."""
    lp0, la0, lb0 = hmm.sparse_integer_instance(seed)
    k0, T, K = la0.shape[0], lb0.shape[0], 512
    lp = np.full(K, -np.inf, np.float32)
    lp[:k0] = lp0
    la = np.full((K, K), -np.inf, np.float32)
    la[:k0, :k0] = la0
    lb = np.zeros((T, K), np.float32)
    lb[:, :k0] = lb0
    po, so, rc, st = oracle.beam(lp, la, lb, B, P)
    assert rc == oracle.BEAM_FALLBACK and st["fallbacks"] >= 1
    print(f"slab beam fallback seed={seed} B={B} P={P}", flush=True)
    path, score, status = fv.decode(_dev(la), _dev(lb), _dev(lp), method="beam", P=P, B=B, rows="local")
    torch.cuda.synchronize()
    assert int(status.item()) == fv.FV_W_BEAM_FALLBACK
    assert (path.cpu().numpy() == po).all()
    assert _bits(score.cpu().numpy()) == _bits(so)


def test_slab_many_rows_per_xcd(fv):
    """Row counts that move across the 160-rows-per-XCD line during one
    launch (1500 sequences of K = 512: the first steps run as lane tiles,
    later ones as slabs), every sequence checked."""
    K = 512
    rng = np.random.default_rng(41)
    lp, la, _ = hmm.random_dense(K, 1, 41)
    lens = [int(x) for x in rng.integers(2, 40, size=1500)]
    lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in lens]
    for method, P in (("flash", 4), ("vanilla", 1)):
        print(f"slab many rows {method}", flush=True)
        batch = fv.Batch([_dev(x) for x in lbs])
        fv.decode_batch(_dev(la), batch, _dev(lp), method=method, P=P, rows="local")
        torch.cuda.synchronize()
        paths, scores, st = batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()
        assert (st == fv.FV_OK).all()
        with ThreadPoolExecutor(8) as ex:
            refs = list(ex.map(lambda x: oracle.vanilla(lp, la, x), lbs))
        for b, (po, so, _) in enumerate(refs):
            assert (paths[b, :lens[b]] == po).all(), b
            assert _bits(scores[b]) == _bits(so), b
