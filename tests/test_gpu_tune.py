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


@pytest.mark.parametrize("K,method,P,step,engine", [
    (1024, "flash", 16, "items", False), (1024, "flash", 16, "tiles", False), (1024, "vanilla", 1, "tiles", False),
    (512, "flash", 4, "items", False), (600, "flash", 8, "tiles", False),
    (96, "flash", 16, "auto", True), (96, "vanilla", 1, "auto", True), (200, "flash", 4, "tiles", True)])
def test_kernel_choices_are_exact(fv, K, method, P, step, engine):
    """Every step kernel (column slabs, column items, lane tiles) and the
    persistent engine for small models give the oracle's paths and scores."""
    lp, la, _ = hmm.random_dense(K, 1, 80 + K)
    rng = np.random.default_rng(81 + K)
    lens = [130, 1, 257, 40]
    lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in lens]
    batch = fv.Batch([_dev(x) for x in lbs])
    print(f"kernel choice K={K} {method} P={P} step={step} engine={engine}", flush=True)
    fv.decode_batch(_dev(la), batch, _dev(lp), method=method, P=P, rows="local", step=step, engine=engine)
    torch.cuda.synchronize()
    assert (batch.status.cpu().numpy() == fv.FV_OK).all()
    for b, T in enumerate(lens):
        po, so, _ = oracle.vanilla(lp, la, lbs[b])
        assert (batch.paths[b, :T].cpu().numpy() == po).all(), b
        assert _bits(batch.scores[b].cpu().numpy()) == _bits(so)


def test_conflicting_step_flags_are_rejected(fv):
    """FV_FLAG_STEP_ITEMS and FV_FLAG_STEP_TILES exclude each other: the call
    returns FV_E_INVALID_ARG and enqueues nothing."""
    import ctypes as C
    K, T = 64, 5
    lp, la, lb = hmm.random_dense(K, T, 1)
    la_d, lb_d, lp_d = _dev(la), _dev(lb), _dev(lp)
    path = torch.full((T,), -3, dtype=torch.int32, device="cuda")
    score = torch.zeros(1, device="cuda")
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    model = fv.dense_model(la_d)
    flags = fv._lib.FV_FLAG_STEP_ITEMS | fv._lib.FV_FLAG_STEP_TILES
    rc = fv.lib().fv_decode_flash(C.byref(model), lp_d.data_ptr(), lb_d.data_ptr(), K, T, 4, path.data_ptr(),
                                  score.data_ptr(), None, flags, ws.data_ptr(), ws.numel(),
                                  torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rc == fv.FV_E_INVALID_ARG
    assert (path.cpu().numpy() == -3).all()


def test_tuner_caches_and_keeps_results(fv, tmp_path):
    """The tuner's search decodes exactly; its choice is written to the cache
    file and a second call returns it without decoding."""
    K = 600
    lp, la, _ = hmm.random_dense(K, 1, 90)
    rng = np.random.default_rng(91)
    lens = [300, 41, 500]
    lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in lens]
    batch = fv.Batch([_dev(x) for x in lbs])
    path = str(tmp_path / "tune.json")
    cfg, timings = fv.tune(_dev(la), batch, _dev(lp), method="flash", P_candidates=(4, 16), path=path)
    assert set(cfg) == {"P", "rows", "step", "leaves", "engine"} and len(timings) >= 5
    torch.cuda.synchronize()
    for b, T in enumerate(lens):
        po, so, _ = oracle.vanilla(lp, la, lbs[b])
        assert (batch.paths[b, :T].cpu().numpy() == po).all()
    batch.paths.fill_(-3)
    cfg2, _ = fv.tune(_dev(la), batch, _dev(lp), method="flash", P_candidates=(4, 16), path=path)
    torch.cuda.synchronize()
    assert cfg2 == cfg and (batch.paths.cpu().numpy() == -3).all()   # cache hit: nothing decoded
    fv.decode_batch(_dev(la), batch, _dev(lp), method="flash", **cfg)
    torch.cuda.synchronize()
    for b, T in enumerate(lens):
        po, so, _ = oracle.vanilla(lp, la, lbs[b])
        assert (batch.paths[b, :T].cpu().numpy() == po).all()
        assert _bits(batch.scores[b].cpu().numpy()) == _bits(so)
