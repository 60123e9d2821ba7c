"""GPU checks of entry points and engine paths that the parity files do not
reach on their own:

- fv_rescore (the path score of Sec. III-A re-summed in time order) against
  the oracle's re-sum, bit for bit, on decoded and on random paths;
- HIP-graph capture of the persistent engine running a FLASH decode
  (K = 600, above the one-block-per-sequence kernels' range): every replay
  must reproduce the eager result, with unrelated eager work between
  replays;
- the engine's watchdog, forced from the host through
  fv_debug_engine_limits: a step bound or a barrier-wait bound far below
  what the decode needs makes every block stop normally and every status
  FV_E_DEVICE; the next decode with the default limits is exact again."""
import ctypes as C

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


@pytest.mark.parametrize("with_pi", [True, False])
def test_rescore_matches_oracle(fv, with_pi):
    K = 300
    rng = np.random.default_rng(31)
    lp, la, _ = hmm.random_dense(K, 1, 32, with_pi=with_pi)
    lens = [1, 2, 57, 640, 3]
    lbs_h = [(rng.standard_normal((T, K)) * 3).astype(np.float32) for T in lens]
    lbs = [_dev(x) for x in lbs_h]
    batch = fv.Batch(lbs)
    # decoded paths for the first three, random paths for the others
    fv.decode_batch(_dev(la), batch, _dev(lp), method="vanilla")
    torch.cuda.synchronize()
    paths = batch.paths.cpu().numpy().copy()
    for b in (3, 4):
        paths[b, :lens[b]] = rng.integers(0, K, lens[b])
    batch.paths.copy_(torch.from_numpy(paths))
    out = torch.full((len(lens),), 7.0, device="cuda")
    lib = fv.lib()
    la_d = _dev(la)
    model = fv.dense_model(la_d)
    lp_d = _dev(lp)
    fv._lib.check(lib.fv_rescore(C.byref(model), lp_d.data_ptr() if lp_d is not None else None,
                                 batch.desc.data_ptr(), len(lens), out.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream), "fv_rescore")
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for b, T in enumerate(lens):
        ref = oracle.rescore(lp, la, lbs_h[b], paths[b, :T])
        assert _bits(got[b]) == _bits(ref), (b, got[b], ref)


def test_rescore_out_of_range_state(fv):
    K, T = 40, 9
    lp, la, lb = hmm.random_dense(K, T, 33)
    batch = fv.Batch([_dev(lb)])
    p = np.arange(T, dtype=np.int32) % K
    p[4] = K   # outside [0, K)
    batch.paths.copy_(torch.from_numpy(p[None, :]))
    out = torch.zeros(1, device="cuda")
    la_d, lp_d = _dev(la), _dev(lp)
    model = fv.dense_model(la_d)
    fv._lib.check(fv.lib().fv_rescore(C.byref(model), lp_d.data_ptr(), batch.desc.data_ptr(), 1, out.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream), "fv_rescore")
    torch.cuda.synchronize()
    assert out.item() == -np.inf


@pytest.mark.parametrize("method,P", [("flash", 16), ("vanilla", 1)])
def test_engine_graph_replay(fv, method, P):
    K = 600
    lp, la, _ = hmm.random_dense(K, 1, 34)
    rng = np.random.default_rng(35)
    lens = [300, 41, 777, 2, 128]
    lbs_h = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in lens]
    lbs = [_dev(x) for x in lbs_h]
    la_d, lp_d = _dev(la), _dev(lp)
    eager = fv.Batch(lbs)
    ws = fv.decode_batch(la_d, eager, lp_d, method=method, P=P)
    torch.cuda.synchronize()
    ref_p, ref_s, ref_st = eager.paths.clone(), eager.scores.clone(), eager.status.clone()
    assert (ref_st.cpu().numpy() == fv.FV_OK).all()
    for b, T in enumerate(lens[:2]):
        po, so, _ = oracle.vanilla(lp, la, lbs_h[b])
        assert (ref_p[b, :T].cpu().numpy() == po).all()
        assert _bits(ref_s[b].cpu().numpy()) == _bits(so)

    batch = fv.Batch(lbs)
    ws2 = torch.empty_like(ws)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fv.decode_batch(la_d, batch, lp_d, method=method, P=P, ws=ws2)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fv.decode_batch(la_d, batch, lp_d, method=method, P=P, ws=ws2)
    for rep in range(3):
        batch.paths.fill_(-1)
        batch.scores.fill_(123.0)
        batch.status.fill_(99)
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(batch.paths, ref_p), rep
        assert torch.equal(batch.scores.view(torch.int32), ref_s.view(torch.int32)), rep
        assert torch.equal(batch.status, ref_st), rep


@pytest.mark.parametrize("max_steps,spin_limit", [(5, 0), (0, 1)])
def test_watchdog_stops_engine(fv, max_steps, spin_limit):
    K = 600
    lp, la, _ = hmm.random_dense(K, 1, 36)
    rng = np.random.default_rng(37)
    lens = [300, 200, 64]
    lbs_h = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in lens]
    lbs = [_dev(x) for x in lbs_h]
    la_d, lp_d = _dev(la), _dev(lp)
    lib = fv.lib()
    batch = fv.Batch(lbs)
    print(f"watchdog: max_steps={max_steps} spin_limit={spin_limit}", flush=True)
    fv._lib.check(lib.fv_debug_engine_limits(max_steps, spin_limit), "fv_debug_engine_limits")
    try:
        fv.decode_batch(la_d, batch, lp_d, method="flash", P=8)
        torch.cuda.synchronize()
    finally:
        fv._lib.check(lib.fv_debug_engine_limits(0, 0), "fv_debug_engine_limits")
    st = batch.status.cpu().numpy()
    assert (st == fv.FV_E_DEVICE).all(), st
    # the default limits again: the same batch decodes exactly
    fv.decode_batch(la_d, batch, lp_d, method="flash", P=8)
    torch.cuda.synchronize()
    assert (batch.status.cpu().numpy() == fv.FV_OK).all()
    po, so, _ = oracle.vanilla(lp, la, lbs_h[0])
    assert (batch.paths[0, :lens[0]].cpu().numpy() == po).all()
    assert _bits(batch.scores[0].cpu().numpy()) == _bits(so)


def test_debug_limits_reject_negative(fv):
    with pytest.raises(fv.FvError):
        fv._lib.check(fv.lib().fv_debug_engine_limits(-1, 0), "fv_debug_engine_limits")
