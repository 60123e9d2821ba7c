"""GPU parity of sparse (CSR) transition models against the CPU oracle.

Vanilla and FLASH must reproduce the oracle's CSR Viterbi path and score bit
for bit (FLASH is exact for every P); FLASH-BS must reproduce the oracle's
CSR beam procedure (same path, re-summed score and status).  Instances cover
variable out-degrees, destinations without in-edges, duplicate edges, rows
listed out of column order, K not a multiple of 64, T = 1, batches of uneven
length, malformed CSR arrays, and the map-matching workload's shape.
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


def _model(fv, row_ptr, col, val):
    return fv.CsrModel(_dev(np.asarray(row_ptr, np.int32)), _dev(np.asarray(col, np.int32)),
                       _dev(np.asarray(val, np.float32)))


def _run(fv, model, lp, lb, method, P=16, B=0, leaves=True):
    path, score, status = fv.decode(model, _dev(lb), _dev(lp), method=method, P=P, B=B, leaves=leaves)
    torch.cuda.synchronize()
    return path.cpu().numpy(), score.cpu().numpy(), int(status.cpu()[0])


def _check_exact(fv, inst, tag, Ps=(1, 2, 5, 16)):
    """Vanilla, FLASH at each P (subtasks split 8 ways) and FLASH with
    FV_FLAG_NO_LEAVES (Alg. 1's bisection) against the oracle."""
    lp, rp, col, val, lb = inst
    print(tag, flush=True)
    po, so, rc = oracle.vanilla_csr(lp, rp, col, val, lb)
    model = _model(fv, rp, col, val)
    runs = [("vanilla", 1, True)] + [("flash", P, True) for P in Ps] + [("flash", Ps[-1], False)]
    for method, P, leaves in runs:
        p, s, st = _run(fv, model, lp, lb, method, P, leaves=leaves)
        assert st == rc, (method, P, leaves, st, rc)
        assert (p == po).all(), (method, P, leaves, np.flatnonzero(p != po)[:10])
        assert (_bits(s) == _bits(so)).all(), (method, P, leaves, s, so)


def _check_beam(fv, inst, B, P, tag):
    lp, rp, col, val, lb = inst
    print(tag, flush=True)
    po, so, rc, _ = oracle.beam_csr(lp, rp, col, val, lb, B, P)
    p, s, st = _run(fv, _model(fv, rp, col, val), lp, lb, "beam", P, B)
    assert st == rc, (st, rc)
    assert (p == po).all(), np.flatnonzero(p != po)[:10]
    assert (_bits(s) == _bits(so)).all(), (s, so)


SHAPES = [(1, 5), (2, 9), (7, 1), (13, 40), (64, 33), (65, 50), (130, 77), (300, 25)]


@pytest.mark.parametrize("K,T", SHAPES)
def test_sparse_exact_matches_oracle(fv, K, T):
    inst = hmm.random_csr(K, T, 3 * K + T, deg_lo=1, deg_hi=8)
    _check_exact(fv, inst, f"sparse K={K} T={T}")


@pytest.mark.parametrize("K,T", [(9, 30), (40, 60), (100, 41)])
def test_sparse_integer_ties_and_duplicates(fv, K, T):
    inst = hmm.random_csr(K, T, 7 * K + T, deg_lo=0, deg_hi=5, integer=True, dup_frac=0.3)
    _check_exact(fv, inst, f"sparse ties K={K} T={T}")


def test_sparse_no_self_loops_and_sources_without_edges(fv):
    inst = hmm.random_csr(50, 70, 11, deg_lo=0, deg_hi=3, self_loops=False)
    _check_exact(fv, inst, "sparse without self loops")


def test_sparse_without_pi(fv):
    inst = hmm.random_csr(33, 44, 12, with_pi=False)
    _check_exact(fv, inst, "sparse no pi")


def test_sparse_infeasible(fv):
    # no edges at all: every step after the first is -inf
    K, T = 10, 6
    lp, _, _, _, lb = hmm.random_csr(K, T, 13)
    rp, col, val = np.zeros(K + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32)
    po, so, rc = oracle.vanilla_csr(lp, rp, col, val, lb)
    assert rc == oracle.INFEASIBLE
    model = _model(fv, rp, col, val)
    for method in ("vanilla", "flash"):
        p, s, st = _run(fv, model, lp, lb, method, 3)
        assert st == fv.FV_E_INFEASIBLE and (p == -1).all() and s[0] == -np.inf


def test_sparse_malformed_csr_reports_invalid(fv):
    lp, rp, col, val, lb = hmm.random_csr(20, 10, 14)
    bad = [rp.copy() for _ in range(3)]
    bad[0][5] = bad[0][6] + 3          # decreasing
    bad[1][-1] += 1                    # last entry != nnz
    bad[2][0] = -1                     # negative start
    for r in bad:
        for method in ("vanilla", "flash", "beam"):
            _, _, st = _run(fv, _model(fv, r, col, val), lp, lb, method, 4, 3)
            assert st == fv.FV_E_INVALID_ARG, (method, st)


def test_sparse_batch_uneven(fv):
    K = 150
    lp, rp, col, val, _ = hmm.random_csr(K, 1, 15, deg_lo=1, deg_hi=9)
    lens = [0, 1, 2, 3, 17, 64, 200, 333]
    rng = np.random.default_rng(16)
    lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in lens]
    model = _model(fv, rp, col, val)
    for method, P, B in (("vanilla", 1, 0), ("flash", 4, 0), ("flash", 16, 0), ("beam", 4, 6)):
        batch = fv.Batch([_dev(x) if len(x) else torch.empty((0, K), device="cuda") for x in lbs])
        fv.decode_batch(model, batch, _dev(lp), method=method, P=P, B=B)
        torch.cuda.synchronize()
        paths, scores, status = batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()
        for b, T in enumerate(lens):
            if T == 0:
                assert status[b] == fv.FV_OK and scores[b] == 0.0
                continue
            if method == "beam":
                po, so, rc, _ = oracle.beam_csr(lp, rp, col, val, lbs[b], B, P)
            else:
                po, so, rc = oracle.vanilla_csr(lp, rp, col, val, lbs[b])
            assert status[b] == rc and (paths[b, :T] == po).all() and _bits(scores[b]) == _bits(so), (method, b)


@pytest.mark.parametrize("K,T", [(9, 30), (64, 50), (130, 40), (300, 60)])
@pytest.mark.parametrize("P", [1, 3, 16])
def test_sparse_beam_matches_oracle(fv, K, T, P):
    inst = hmm.random_csr(K, T, 5 * K + T, deg_lo=1, deg_hi=7)
    for B in sorted({1, 2, 5, K // 3, K - 1}):
        if 1 <= B < K:
            _check_beam(fv, inst, B, P, f"sparse beam K={K} T={T} B={B} P={P}")


@pytest.mark.parametrize("K,T", [(12, 40), (40, 30)])
def test_sparse_beam_ties_duplicates_fallbacks(fv, K, T):
    for seed in range(6):
        inst = hmm.random_csr(K, T, 100 * seed + K, deg_lo=0, deg_hi=3, integer=True, dup_frac=0.25,
                              self_loops=seed % 2 == 0)
        for B, P in ((1, 2), (2, 3), (3, 1)):
            _check_beam(fv, inst, B, P, f"sparse beam ties seed={seed} K={K} B={B} P={P}")


def test_sparse_beam_full_width_is_flash(fv):
    inst = hmm.random_csr(50, 40, 21, deg_lo=1, deg_hi=6)
    lp, rp, col, val, lb = inst
    po, so, rc = oracle.vanilla_csr(lp, rp, col, val, lb)
    p, s, st = _run(fv, _model(fv, rp, col, val), lp, lb, "beam", 4, 50)
    assert st == rc and (p == po).all() and (_bits(s) == _bits(so)).all()


def test_sparse_beam_too_many_candidates_is_reported(fv):
    # every state reaches all K = 600 states: a beam of 16 pushes 9600 > 4096 candidates
    K, T = 600, 5
    r = np.random.default_rng(22)
    rp = (np.arange(K + 1) * K).astype(np.int32)
    col = np.tile(np.arange(K, dtype=np.int32), K)
    val = (r.standard_normal(K * K) - 2).astype(np.float32)
    lb = r.standard_normal((T, K)).astype(np.float32)
    _, _, st = _run(fv, _model(fv, rp, col, val), None, lb, "beam", 2, 16)
    assert st == fv.FV_E_UNSUPPORTED


def test_map_matching_small(fv):
    """The map-matching workload's construction at K = 3000, 4 trajectories."""
    wl = hmm.map_matching_workload(K=3000, n=4, t_lo=50, t_hi=300)
    model = _model(fv, wl.row_ptr, wl.col, wl.val)
    lbs = [wl.log_b(b, "cuda") for b in range(wl.n)]
    for b in range(wl.n):
        lb = lbs[b].cpu().numpy()
        po, so, rc = oracle.vanilla_csr(wl.log_pi, wl.row_ptr, wl.col, wl.val, lb)
        bo, bso, brc, _ = oracle.beam_csr(wl.log_pi, wl.row_ptr, wl.col, wl.val, lb, 128, 16)
        for method, P, B in (("vanilla", 1, 0), ("flash", 16, 0)):
            p, s, st = _run(fv, model, wl.log_pi, lb, method, P, B)
            assert st == rc and (p == po).all() and _bits(s) == _bits(so), (b, method)
        p, s, st = _run(fv, model, wl.log_pi, lb, "beam", 16, 128)
        assert st == brc and (p == bo).all() and _bits(s) == _bits(bso), (b, "beam")
