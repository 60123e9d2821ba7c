"""GPU parity of the wide-row placement (every block takes a 64-column
slice of every dense row; log A streamed once per step for up to 16 rows)
against the CPU oracle.  The placement never changes results, so every
case must match the oracle bit for bit, as the local placement does."""
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


def _run(fv, lp, la, lb, method, P=16, B=0, rows="wide"):
    path, score, status = fv.decode(_dev(la), _dev(lb), _dev(lp), method=method, P=P, B=B, rows=rows)
    torch.cuda.synchronize()
    return path.cpu().numpy(), score.cpu().numpy(), int(status.cpu()[0])


SHAPES = [(1, 1), (2, 2), (5, 7), (17, 40), (63, 33), (64, 64), (65, 50), (130, 21), (200, 9), (300, 17)]


@pytest.mark.parametrize("K,T", SHAPES)
@pytest.mark.parametrize("method,P", [("vanilla", 1), ("flash", 1), ("flash", 3), ("flash", 16)])
def test_wide_matches_oracle(fv, K, T, method, P):
    lp, la, lb = hmm.random_dense(K, T, 19 * K + T)
    print(f"wide {method} K={K} T={T} P={P}", flush=True)
    p, s, st = _run(fv, lp, la, lb, method, P=P)
    po, so, _ = oracle.vanilla(lp, la, lb)
    assert st == fv.FV_OK
    assert (p == po).all(), np.flatnonzero(p != po)[:10]
    assert (_bits(s) == _bits(so)).all()


@pytest.mark.parametrize("seed", range(3))
def test_wide_integer_ties(fv, seed):
    lp, la, lb = hmm.random_dense(70, 37, seed, integer=True, lo=-2, hi=0)
    po, so, _ = oracle.vanilla(lp, la, lb)
    for method, P in (("vanilla", 1), ("flash", 5)):
        p, s, _ = _run(fv, lp, la, lb, method, P=P)
        assert (p == po).all() and s[0] == so


def test_wide_infeasible_and_signed_zero(fv):
    lp, la, lb = hmm.random_dense(20, 9, 3)
    la[:] = -np.inf
    for method in ("vanilla", "flash"):
        p, s, st = _run(fv, lp, la, lb, method, P=3)
        assert st == fv.FV_E_INFEASIBLE and (p == -1).all() and s[0] == -np.inf
    lp = np.array([-0.0, 0.0], np.float32)
    la = np.array([[-0.0, -0.0], [0.0, 0.0]], np.float32)
    lb = np.array([[-0.0, -0.0], [-0.0, -0.0]], np.float32)
    po, so, _ = oracle.vanilla(lp, la, lb)
    for method in ("vanilla", "flash"):
        p, s, _ = _run(fv, lp, la, lb, method, P=2)
        assert (p == po).all() and (_bits(s) == _bits(so)).all()


def test_wide_batch_many_rows(fv):
    """More than 16 rows per XCD list: several row groups per column chunk."""
    K = 160
    rng = np.random.default_rng(4)
    lengths = [0, 1, 2, 90, 3, 120, 64, 77] + [int(x) for x in rng.integers(20, 140, size=40)]
    _, la, _ = hmm.random_dense(K, 1, 21)
    lp = rng.normal(size=K).astype(np.float32)
    lbs = [rng.normal(size=(T, K)).astype(np.float32) for T in lengths]
    for method, P in (("vanilla", 1), ("flash", 4), ("flash", 64)):
        batch = fv.Batch([_dev(x) if len(x) else torch.empty((0, K), device="cuda") for x in lbs])
        fv.decode_batch(_dev(la), batch, _dev(lp), method=method, P=P, rows="wide")
        torch.cuda.synchronize()
        paths, scores, status = batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()
        for b, T in enumerate(lengths):
            if T == 0:
                continue
            po, so, _ = oracle.vanilla(lp, la, lbs[b])
            assert status[b] == 0 and (paths[b, :T] == po).all() and _bits(scores[b]) == _bits(so), (method, P, b)


@pytest.mark.parametrize("K,T", [(1024, 300), (4096, 60), (4100, 40)])
def test_wide_by_default_for_large_k(fv, K, T):
    """Large K picks wide rows on its own (K = 4100 also exercises the
    padded copy of log A)."""
    rng = np.random.default_rng(K)
    la = (rng.standard_normal((K, K), dtype=np.float32) * np.float32(2.0) - np.float32(8.0))
    lb = rng.standard_normal((T, K), dtype=np.float32) * np.float32(2.0)
    lp = hmm.uniform_log_pi(K)
    po, so, _ = oracle.vanilla(lp, la, lb)
    for method, P in (("vanilla", 1), ("flash", 16)):
        p, s, st = _run(fv, lp, la, lb, method, P=P, rows="auto")
        assert st == fv.FV_OK and (p == po).all() and (_bits(s) == _bits(so)).all(), method


@pytest.mark.parametrize("seed,B,P", [(610, 2, 1), (699, 2, 3), (2428, 2, 2)])
def test_wide_beam_fallback(fv, seed, B, P):
    """A beam subtask's exact re-decode runs as a dense row: here a wide one."""
    lp, la, lb = hmm.sparse_integer_instance(seed)
    po, so, rc, _ = oracle.beam(lp, la, lb, B, P)
    p, s, st = _run(fv, lp, la, lb, "beam", P=P, B=B)
    assert st == rc == oracle.BEAM_FALLBACK
    assert (p == po).all() and (_bits(s) == _bits(so)).all()


def test_local_flag_and_exclusive_flags(fv):
    lp, la, lb = hmm.random_dense(40, 30, 9)
    po, so, _ = oracle.vanilla(lp, la, lb)
    p, s, _ = _run(fv, lp, la, lb, "flash", P=4, rows="local")
    assert (p == po).all() and (_bits(s) == _bits(so)).all()
    import ctypes as C
    l = fv.lib()
    rc = l.fv_decode_flash(C.byref(fv.dense_model(_dev(la))), None, _dev(lb).data_ptr(), 40, 30, 4,
                           C.c_void_p(256), C.c_void_p(256), None, 3, C.c_void_p(4096), 1 << 30, None)
    assert rc == fv.FV_E_INVALID_ARG
