"""GPU parity of the dense decoders against the CPU oracle.

Paths are compared element by element and scores bit for bit (every
candidate is one float32 add, so the GPU must reproduce the oracle exactly).
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


def _run(fv, lp, la, lb, method, P=16, B=0):
    path, score, status = fv.decode(_dev(la), _dev(lb), _dev(lp), method=method, P=P, B=B)
    torch.cuda.synchronize()
    return path.cpu().numpy(), score.cpu().numpy(), int(status.cpu()[0])


SHAPES = [(1, 1), (1, 6), (2, 1), (2, 2), (3, 3), (5, 7), (17, 40), (63, 33), (64, 64), (65, 50),
          (130, 21), (200, 9)]


@pytest.mark.parametrize("K,T", SHAPES)
def test_vanilla_matches_oracle(fv, K, T):
    lp, la, lb = hmm.random_dense(K, T, 11 * K + T)
    print(f"vanilla K={K} T={T}", flush=True)
    p, s, st = _run(fv, lp, la, lb, "vanilla")
    po, so, _ = oracle.vanilla(lp, la, lb)
    assert st == fv.FV_OK
    assert (p == po).all()
    assert (_bits(s) == _bits(so)).all()


@pytest.mark.parametrize("K,T", SHAPES)
@pytest.mark.parametrize("P", [1, 2, 3, 7, 16, 1000])
def test_flash_matches_oracle(fv, K, T, P):
    lp, la, lb = hmm.random_dense(K, T, 13 * K + T)
    print(f"flash K={K} T={T} P={P}", flush=True)
    p, s, st = _run(fv, lp, la, lb, "flash", P=P)
    po, so, _ = oracle.vanilla(lp, la, lb)
    assert st == fv.FV_OK
    assert (p == po).all()
    assert (_bits(s) == _bits(so)).all()


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("method,P", [("vanilla", 1), ("flash", 1), ("flash", 5)])
def test_integer_ties(fv, seed, method, P):
    K, T = 70, 37
    lp, la, lb = hmm.random_dense(K, T, seed, integer=True, lo=-2, hi=0)
    print(f"ties {method} seed={seed} P={P}", flush=True)
    p, s, _ = _run(fv, lp, la, lb, method, P=P)
    po, so, _ = oracle.vanilla(lp, la, lb)
    assert (p == po).all() and s[0] == so


def test_without_pi(fv):
    _, la, lb = hmm.random_dense(40, 30, 5, with_pi=False)
    for method in ("vanilla", "flash"):
        p, s, _ = _run(fv, None, la, lb, method, P=4)
        po, so, _ = oracle.vanilla(None, la, lb)
        assert (p == po).all() and (_bits(s) == _bits(so)).all()


def test_anchor_at_large_magnitude(fv):
    """Near-ties created by float32 rounding at |score| ~ 1e6: the anchored
    subtask start must reproduce vanilla's rounding."""
    K, T = 16, 1200
    r = np.random.default_rng(5)
    la = (np.float32(-np.log(K)) + 0.01 * r.standard_normal((K, K))).astype(np.float32)
    lb = (-1000.0 + 0.02 * r.standard_normal((T, K))).astype(np.float32)
    lp = hmm.uniform_log_pi(K)
    po, so, _ = oracle.vanilla(lp, la, lb)
    for method, P in (("vanilla", 1), ("flash", 1), ("flash", 16)):
        p, s, _ = _run(fv, lp, la, lb, method, P=P)
        assert (p == po).all() and (_bits(s) == _bits(so)).all()


def test_infeasible(fv):
    lp, la, lb = hmm.random_dense(20, 9, 3)
    la[:] = -np.inf
    for method in ("vanilla", "flash"):
        p, s, st = _run(fv, lp, la, lb, method, P=3)
        assert st == fv.FV_E_INFEASIBLE and (p == -1).all() and s[0] == -np.inf


def test_signed_zero(fv):
    lp = np.array([-0.0, 0.0], np.float32)
    la = np.array([[-0.0, -0.0], [0.0, 0.0]], np.float32)
    lb = np.array([[-0.0, -0.0], [-0.0, -0.0]], np.float32)
    po, so, _ = oracle.vanilla(lp, la, lb)
    for method in ("vanilla", "flash"):
        p, s, _ = _run(fv, lp, la, lb, method, P=2)
        assert (p == po).all() and (_bits(s) == _bits(so)).all()


@pytest.mark.parametrize("K,T", [(64, 300), (65, 1), (65, 300), (96, 257), (127, 64), (128, 700), (129, 40),
                                 (200, 300), (256, 129)])
def test_single_vanilla_two_columns_per_lane(fv, K, T):
    """Single vanilla decodes with 64 <= K <= 256 (the one-wave kernel at 64,
    the two- and four-wave kernels above): random, integer-tie, start-free
    and infeasible inputs, bit for bit against the oracle."""
    print(f"one-wave vanilla K={K} T={T}", flush=True)
    lp, la, lb = hmm.random_dense(K, T, 7 * K + T)
    p, s, st = _run(fv, lp, la, lb, "vanilla")
    po, so, _ = oracle.vanilla(lp, la, lb)
    assert st == fv.FV_OK and (p == po).all() and (_bits(s) == _bits(so)).all()
    lp, la, lb = hmm.random_dense(K, T, K + 3 * T, integer=True, lo=-2, hi=0)
    p, s, _ = _run(fv, lp, la, lb, "vanilla")
    po, so, _ = oracle.vanilla(lp, la, lb)
    assert (p == po).all() and (_bits(s) == _bits(so)).all()
    p, s, _ = _run(fv, None, la, lb, "vanilla")
    po, so, _ = oracle.vanilla(None, la, lb)
    assert (p == po).all() and (_bits(s) == _bits(so)).all()
    if T > 1:
        la[:] = -np.inf
        p, s, st = _run(fv, lp, la, lb, "vanilla")
        assert st == fv.FV_E_INFEASIBLE and (p == -1).all() and s[0] == -np.inf


@pytest.mark.parametrize("T", [1, 2])
def test_single_vanilla_signed_zero_across_lanes(fv, T):
    """Final scores -0 (state 70) and +0 (state 90) on both sides of the
    lane-64 split, all other states lower: -0 and +0 are equal, so the lower
    index wins and its score keeps its sign, as in the oracle."""
    K = 100
    lp = np.full(K, -5.0, np.float32)
    lp[70], lp[90] = -0.0, 0.0
    la = np.full((K, K), -np.inf, np.float32)
    la[70, 70], la[90, 90] = -0.0, 0.0
    lb = np.full((T, K), -1.0, np.float32)
    lb[:, 70], lb[:, 90] = -0.0, 0.0
    po, so, _ = oracle.vanilla(lp, la, lb)
    assert po[-1] == 70 and _bits(so)[0] == 0x80000000
    p, s, _ = _run(fv, lp, la, lb, "vanilla")
    assert (p == po).all() and (_bits(s) == _bits(so)).all()


@pytest.mark.parametrize("K,T", [(1, 5), (7, 1), (7, 2), (7, 3), (33, 129), (64, 700), (64, 3000), (65, 2),
                                 (65, 300), (100, 129), (128, 1000), (129, 130), (200, 257), (256, 150)])
def test_single_flash_one_wave(fv, K, T):
    """Single FLASH decodes with K <= 256 (the one- and multi-wave FLASH kernels): every
    P' from 2 to T (and beyond), with and without leaf subtasks, bit for bit
    against the oracle's vanilla result and the oracle's FLASH."""
    lp, la, lb = hmm.random_dense(K, T, 5 * K + T)
    po, so, _ = oracle.vanilla(lp, la, lb)
    for P in (1, 2, 5, 16, 64, 5000):
        pf, sf, rc, _ = oracle.flash(lp, la, lb, P)
        assert rc == 0 and (pf == po).all() and _bits(sf) == _bits(so)
        for leaves in (True, False):
            print(f"one-wave flash K={K} T={T} P={P} leaves={leaves}", flush=True)
            path, score, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="flash", P=P, leaves=leaves)
            torch.cuda.synchronize()
            assert int(st.cpu()[0]) == fv.FV_OK
            assert (path.cpu().numpy() == po).all(), (P, leaves)
            assert (_bits(score.cpu().numpy()) == _bits(so)).all()


@pytest.mark.parametrize("K", [50, 120, 250])
def test_single_flash_one_wave_ties_and_edges(fv, K):
    """Integer ties, no start vector, -0 against +0 and an infeasible model
    through the one-wave FLASH kernel (one and two destinations per lane)."""
    T = 300
    lp, la, lb = hmm.random_dense(K, T, 12, integer=True, lo=-2, hi=0)
    for P in (3, 16):
        po, so, _ = oracle.vanilla(lp, la, lb)
        p, s, _ = _run(fv, lp, la, lb, "flash", P=P)
        assert (p == po).all() and (_bits(s) == _bits(so)).all()
        po, so, _ = oracle.vanilla(None, la, lb)
        p, s, _ = _run(fv, None, la, lb, "flash", P=P)
        assert (p == po).all() and (_bits(s) == _bits(so)).all()
    lp = np.full(K, -5.0, np.float32)
    lp[20], lp[40] = -0.0, 0.0
    zla = np.full((K, K), -np.inf, np.float32)
    zla[20, 20], zla[40, 40] = -0.0, 0.0
    zlb = np.full((9, K), -1.0, np.float32)
    zlb[:, 20], zlb[:, 40] = -0.0, 0.0
    po, so, _ = oracle.vanilla(lp, zla, zlb)
    p, s, _ = _run(fv, lp, zla, zlb, "flash", P=4)
    assert po[-1] == 20 and (p == po).all() and (_bits(s) == _bits(so)).all()
    la[:] = -np.inf
    p, s, st = _run(fv, lp, la, lb, "flash", P=4)
    assert st == fv.FV_E_INFEASIBLE and (p == -1).all() and s[0] == -np.inf


@pytest.mark.parametrize("K,seed", [(40, 40), (100, 1), (128, 3)])
def test_single_flash_one_wave_relative_init(fv, K, seed):
    """The relative subtask start through the one-wave FLASH kernel equals
    the oracle's same procedure bit for bit (for K = 100 and 128 these seeds
    give paths that differ from vanilla's)."""
    lp, la, lb = hmm.random_dense(K, 2000, seed)
    lb = (lb * 20).astype(np.float32)
    for P in (2, 16):
        pr, sr, rc, _ = oracle.flash(lp, la, lb, P, relative_init=True)
        path, score, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="flash", P=P, relative_init=True)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == rc == 0
        assert (path.cpu().numpy() == pr).all() and (_bits(score.cpu().numpy()) == _bits(sr)).all()


@pytest.mark.parametrize("K", [20, 64, 100])
def test_batch_small_models_one_wave_per_sequence(fv, K):
    """Batches of one small dense model (one wave per sequence): ragged
    lengths with empty sequences, vanilla and FLASH (several P, leaves on and
    off, the relative start), each sequence bit for bit against the oracle."""
    r = np.random.default_rng(K)
    lengths = [int(x) for x in r.integers(0, 400, size=150)]
    lengths[:4] = [0, 1, 2, 399]
    _, la, _ = hmm.random_dense(K, 1, 300 + K)
    lp = hmm.uniform_log_pi(K)
    lbs = [(r.standard_normal((T, K)) * 2).astype(np.float32) for T in lengths]
    ref = [oracle.vanilla(lp, la, x) if x.shape[0] else None for x in lbs]
    runs = [("vanilla", 1, True, False), ("flash", 1, True, False), ("flash", 4, False, False),
            ("flash", 64, True, False), ("flash", 16, True, True)]
    for method, P, leaves, rel in runs:
        print(f"batch K={K} {method} P={P} leaves={leaves} relative={rel}", flush=True)
        batch = fv.Batch([_dev(x) if x.shape[0] else torch.empty((0, K), device="cuda") for x in lbs])
        fv.decode_batch(_dev(la), batch, _dev(lp), method=method, P=P, leaves=leaves, relative_init=rel)
        torch.cuda.synchronize()
        paths, scores, status = batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()
        for b, T in enumerate(lengths):
            assert status[b] == 0, (method, P, b)
            if T == 0:
                assert scores[b] == 0.0
                continue
            if rel:
                po, so, _, _ = oracle.flash(lp, la, lbs[b], P, relative_init=True)
            else:
                po, so, _ = ref[b]
            assert (paths[b, :T] == po).all(), (method, P, b)
            assert _bits(scores[b]) == _bits(so), (method, P, b)


def test_batch_k200_four_waves_per_sequence(fv):
    """A ragged batch on one K = 200 model (four waves per sequence): vanilla,
    FLASH with and without leaves, and the relative start."""
    K = 200
    r = np.random.default_rng(200)
    lengths = [int(x) for x in r.integers(0, 200, size=40)]
    lengths[:3] = [0, 1, 199]
    _, la, _ = hmm.random_dense(K, 1, 201)
    lp = hmm.uniform_log_pi(K)
    lbs = [(r.standard_normal((T, K)) * 2).astype(np.float32) for T in lengths]
    ref = [oracle.vanilla(lp, la, x) if x.shape[0] else None for x in lbs]
    for method, P, leaves, rel in (("vanilla", 1, True, False), ("flash", 4, True, False),
                                   ("flash", 4, False, False), ("flash", 16, True, True)):
        print(f"batch K={K} {method} P={P} leaves={leaves} relative={rel}", flush=True)
        batch = fv.Batch([_dev(x) if x.shape[0] else torch.empty((0, K), device="cuda") for x in lbs])
        fv.decode_batch(_dev(la), batch, _dev(lp), method=method, P=P, leaves=leaves, relative_init=rel)
        torch.cuda.synchronize()
        paths, scores, status = batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()
        for b, T in enumerate(lengths):
            assert status[b] == 0, (method, P, b)
            if T == 0:
                assert scores[b] == 0.0
                continue
            if rel:
                po, so, _, _ = oracle.flash(lp, la, lbs[b], P, relative_init=True)
            else:
                po, so, _ = ref[b]
            assert (paths[b, :T] == po).all(), (method, P, b)
            assert _bits(scores[b]) == _bits(so), (method, P, b)


def test_discrete_hmm_k64_t1000(fv):
    """Single discrete HMM: K=64, V=128, T=1000, Dirichlet rows, emissions
    gathered on the device."""
    h = hmm.discrete_hmm(K=64, V=128, T=1000, seed=1)
    lb_ref = oracle.gather_emissions(h.log_e, h.obs)
    lb = torch.empty((h.T, h.K), dtype=torch.float32, device="cuda")
    log_e, obs = _dev(h.log_e), _dev(h.obs)   # keep the inputs alive until the kernel ran
    rc = fv.lib().fv_gather_emissions(h.K, h.V, log_e.data_ptr(), obs.data_ptr(), h.T,
                                      lb.data_ptr(), h.K, torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    assert (lb.cpu().numpy() == lb_ref).all()
    po, so, _ = oracle.vanilla(h.log_pi, h.log_a, lb_ref)
    for method, P in (("vanilla", 1), ("flash", 1), ("flash", 4), ("flash", 16)):
        path, score, st = fv.decode(_dev(h.log_a), lb, _dev(h.log_pi), method=method, P=P)
        assert (path.cpu().numpy() == po).all() and (_bits(score.cpu().numpy()) == _bits(so)).all()


def test_batch_uneven_lengths(fv):
    K = 96
    r = np.random.default_rng(3)
    lengths = [0, 1, 2, 3, 5, 64, 100, 257, 31]
    _, la, _ = hmm.random_dense(K, 1, 77)
    lp = hmm.uniform_log_pi(K)
    lbs = [(r.standard_normal((T, K)) * 2).astype(np.float32) for T in lengths]
    for method, P in (("vanilla", 1), ("flash", 1), ("flash", 4), ("flash", 64)):
        batch = fv.Batch([_dev(x) if x.shape[0] else torch.empty((0, K), device="cuda") for x in lbs])
        fv.decode_batch(_dev(la), batch, _dev(lp), method=method, P=P)
        torch.cuda.synchronize()
        paths = batch.paths.cpu().numpy()
        scores = batch.scores.cpu().numpy()
        status = batch.status.cpu().numpy()
        for b, T in enumerate(lengths):
            assert status[b] == 0, (method, P, b)
            if T == 0:
                assert scores[b] == 0.0
                continue
            po, so, _ = oracle.vanilla(lp, la, lbs[b])
            assert (paths[b, :T] == po).all(), (method, P, b)
            assert _bits(scores[b]) == _bits(so)


@pytest.mark.parametrize("method,P", [("vanilla", 1), ("flash", 4)])
def test_batch_column_items_ragged_width(fv, method, P):
    """About 100 short sequences at K = 300 (padded width 320, so the last
    128-destination chunk holds one destination per lane): every XCD has
    more than one 8-row group of few-row column items."""
    K = 300
    r = np.random.default_rng(11)
    lengths = r.integers(5, 61, size=100)
    _, la, _ = hmm.random_dense(K, 1, 91)
    lp = hmm.uniform_log_pi(K)
    lbs = [(r.standard_normal((int(T), K)) * 2).astype(np.float32) for T in lengths]
    batch = fv.Batch([_dev(x) for x in lbs])
    fv.decode_batch(_dev(la), batch, _dev(lp), method=method, P=P)
    torch.cuda.synchronize()
    paths, scores, status = batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()
    for b, T in enumerate(lengths):
        po, so, _ = oracle.vanilla(lp, la, lbs[b])
        assert status[b] == 0 and (paths[b, :T] == po).all(), (method, P, b)
        assert _bits(scores[b]) == _bits(so)


@pytest.mark.parametrize("seed", [3, 4])
def test_relative_init_matches_oracle(fv, seed):
    """FV_FLAG_RELATIVE_INIT (the paper's displayed subtask start, carried
    score dropped): on inputs where its path differs from vanilla's, FLASH
    and FLASH-BS must still equal the oracle's same procedure bit for bit."""
    lp, la, lb = hmm.random_dense(64, 2000, seed)
    lb = (lb * 20).astype(np.float32)
    po, _, _ = oracle.vanilla(lp, la, lb)
    diverged = False
    for P in (4, 16):
        pr, sr, rc, _ = oracle.flash(lp, la, lb, P, relative_init=True)
        diverged |= bool((pr != po).any())
        path, score, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="flash", P=P, relative_init=True)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == rc
        assert (path.cpu().numpy() == pr).all(), np.flatnonzero(path.cpu().numpy() != pr)[:10]
        assert _bits(score.cpu().numpy()) == _bits(sr)
    assert diverged
    for B in (8, 32):
        pr, sr, rc, _ = oracle.beam(lp, la, lb, B, 4, relative_init=True)
        path, score, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="beam", P=4, B=B, relative_init=True)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == rc
        assert (path.cpu().numpy() == pr).all(), (B, np.flatnonzero(path.cpu().numpy() != pr)[:10])
        assert _bits(score.cpu().numpy()) == _bits(np.float32(sr))


def test_relative_init_batched(fv):
    """The flag through fv_decode_batch (uneven lengths, one launch)."""
    K = 96
    r = np.random.default_rng(21)
    _, la, _ = hmm.random_dense(K, 1, 31)
    lp = hmm.uniform_log_pi(K)
    lbs = [(r.standard_normal((T, K)) * 40).astype(np.float32) for T in (300, 1200, 77, 900)]
    batch = fv.Batch([_dev(x) for x in lbs])
    fv.decode_batch(_dev(la), batch, _dev(lp), method="flash", P=8, relative_init=True)
    torch.cuda.synchronize()
    paths, scores = batch.paths.cpu().numpy(), batch.scores.cpu().numpy()
    for b, x in enumerate(lbs):
        pr, sr, rc, _ = oracle.flash(lp, la, x, 8, relative_init=True)
        assert (paths[b, :x.shape[0]] == pr).all() and _bits(scores[b]) == _bits(sr)


def test_relative_init_full_width_beam_is_flash(fv):
    """A beam of width >= K is decoded as FLASH; with FV_FLAG_RELATIVE_INIT
    it returns the oracle's FLASH result (on these inputs the beam procedure
    at full width reports another score: the re-summed score of its path,
    where FLASH reports the root pass's maximum)."""
    lp, la, lb = hmm.random_dense(64, 2000, 9)
    lb = (lb * 20).astype(np.float32)
    pf, sf, rc, _ = oracle.flash(lp, la, lb, 4, relative_init=True)
    pb, sb, _, _ = oracle.beam(lp, la, lb, 64, 4, relative_init=True)
    assert (pb != pf).any() or _bits(sb) != _bits(sf)
    path, score, st = fv.decode(_dev(la), _dev(lb), _dev(lp), method="beam", P=4, B=64, relative_init=True)
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == rc and (path.cpu().numpy() == pf).all()
    assert _bits(score.cpu().numpy()) == _bits(sf)
