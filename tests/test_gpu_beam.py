"""GPU parity of FLASH-BS (beam decoding) against the CPU oracle.

For B < K the result is defined by the oracle's procedure (top B by score
then state, segments restarted from their anchored boundary state, end-only
last step, exact re-decode when the end state is lost), so the GPU must
return the same path, the same re-summed score bit for bit and the same
status.
"""
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


def _run(fv, lp, la, lb, B, P):
    path, score, status = fv.decode(_dev(la), _dev(lb), _dev(lp), method="beam", P=P, B=B)
    torch.cuda.synchronize()
    return path.cpu().numpy(), score.cpu().numpy(), int(status.cpu()[0])


def _check(fv, lp, la, lb, B, P, tag):
    print(tag, flush=True)
    p, s, st = _run(fv, lp, la, lb, B, P)
    po, so, rc, _ = oracle.beam(lp, la, lb, B, P)
    assert st == rc, (st, rc)
    assert (p == po).all(), np.flatnonzero(p != po)[:10]
    assert (_bits(s) == _bits(so)).all(), (s, so)


SHAPES = [(2, 1), (3, 3), (5, 7), (17, 40), (63, 33), (65, 50), (130, 21), (200, 9)]


@pytest.mark.parametrize("K,T", SHAPES)
@pytest.mark.parametrize("P", [1, 3, 16])
def test_beam_matches_oracle(fv, K, T, P):
    lp, la, lb = hmm.random_dense(K, T, 17 * K + T)
    for B in sorted({1, 2, 5, K // 2, K - 1}):
        if 1 <= B < K:
            _check(fv, lp, la, lb, B, P, f"beam K={K} T={T} B={B} P={P}")


@pytest.mark.parametrize("K,T", [(4, 9), (16, 30), (40, 25)])
@pytest.mark.parametrize("B", [2, 3])
def test_beam_integer_ties(fv, K, T, B):
    lp, la, lb = hmm.random_dense(K, T, 5 * K + T, integer=True, lo=-2, hi=0)
    for P in (1, 2, 5):
        _check(fv, lp, la, lb, B, P, f"beam ties K={K} T={T} B={B} P={P}")


def test_beam_without_pi(fv):
    lp, la, lb = hmm.random_dense(33, 41, 7, with_pi=False)
    _check(fv, None, la, lb, 4, 6, "beam no pi")


@pytest.mark.parametrize("K,T,P", [(6, 20, 3), (50, 37, 1), (64, 64, 16)])
def test_beam_full_width_is_flash(fv, K, T, P):
    lp, la, lb = hmm.random_dense(K, T, K + 2 * T)
    pv, sv, _ = oracle.vanilla(lp, la, lb)
    for B in (K, K + 5):
        p, s, st = _run(fv, lp, la, lb, B, P)
        assert st == fv.FV_OK and (p == pv).all() and (_bits(s) == _bits(sv)).all()


@pytest.mark.parametrize("seed,B,P", [(610, 2, 1), (610, 2, 2), (699, 2, 3), (2428, 2, 1), (2428, 2, 2)])
def test_beam_fallback(fv, seed, B, P):
    """Instances where a restarted segment's beam loses the known end state
    (sparse transitions): the task is re-decoded exactly and the call
    reports FV_W_BEAM_FALLBACK."""
    lp, la, lb = hmm.sparse_integer_instance(seed)
    _, _, rc, st = oracle.beam(lp, la, lb, B, P)
    assert rc == oracle.BEAM_FALLBACK and st["fallbacks"] >= 1
    _check(fv, lp, la, lb, B, P, f"beam fallback seed={seed} B={B} P={P}")


def test_beam_sparse_instances(fv):
    for seed in range(60):
        lp, la, lb = hmm.sparse_integer_instance(seed)
        K = la.shape[0]
        for B in (1, 2, 3):
            if B < K:
                _check(fv, lp, la, lb, B, 2, f"beam sparse seed={seed} B={B}")


def test_beam_infeasible(fv):
    K, T = 8, 12
    lp, la, lb = hmm.random_dense(K, T, 3)
    la[:] = -np.inf
    p, s, st = _run(fv, lp, la, lb, 3, 4)
    po, so, rc, _ = oracle.beam(lp, la, lb, 3, 4)
    assert rc == oracle.INFEASIBLE and st == fv.FV_E_INFEASIBLE
    assert (p == -1).all() and (po == -1).all() and s[0] == -np.inf


def test_beam_batch_uneven(fv):
    K, B, P = 96, 8, 4
    lens = [0, 1, 2, 3, 5, 64, 100, 257, 31]
    rng = np.random.default_rng(5)
    _, la, _ = hmm.random_dense(K, 1, 77)
    lp = rng.normal(size=K).astype(np.float32)
    lbs = [rng.normal(size=(T, K)).astype(np.float32) for T in lens]
    batch = fv.Batch([_dev(x) if len(x) else torch.empty((0, K), device="cuda") for x in lbs])
    fv.decode_batch(_dev(la), batch, _dev(lp), method="beam", P=P, B=B)
    torch.cuda.synchronize()
    paths, scores, status = batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()
    for b, T in enumerate(lens):
        if T == 0:
            assert status[b] == fv.FV_OK and scores[b] == 0.0
            continue
        po, so, rc, _ = oracle.beam(lp, la, lbs[b], B, P)
        assert status[b] == rc and (paths[b, :T] == po).all() and _bits(scores[b]) == _bits(so), b


def test_beam_dirichlet_k1024(fv):
    """Beam widths 64 and 256 on the batched workload's model (K = 1024,
    Dirichlet(0.1) rows) and one of its emission streams."""
    wl = hmm.batched_flash_workload(n=4)
    lb = wl.log_b(0)[:1500]
    for B in (64, 256):
        _check(fv, wl.log_pi, wl.log_a, lb, B, 16, f"beam K=1024 T=1500 B={B}")


def test_beam_large_k(fv):
    """The beam code's largest K: 16384 states, B = 16, P = 16."""
    K, T = 16384, 120
    rng = np.random.default_rng(8)
    la = (rng.standard_normal((K, K), dtype=np.float32) * np.float32(3.0)) - np.float32(10.0)
    lb = rng.standard_normal((T, K), dtype=np.float32) * np.float32(3.0)
    lp = np.full(K, -np.log(K), np.float32)
    _check(fv, lp, la, lb, 16, 16, "beam K=16384 T=120 B=16")


@pytest.mark.parametrize("K,T,B,P", [(1024, 700, 16, 4), (600, 900, 8, 2)])
def test_beam_fewer_parts_with_many_rows(fv, K, T, B, P):
    """One sequence: its beam steps are planned in several parts (one block
    each), but once many subtasks are in flight each step runs fewer parts
    per row; the rebuilt beam and the result must not change."""
    lp, la, lb = hmm.random_dense(K, T, 1000 + K)
    _check(fv, lp, la, lb, B, P, f"beam parts K={K} T={T} B={B} P={P}")
