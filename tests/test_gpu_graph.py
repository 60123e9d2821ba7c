"""A decode call only enqueues work on the caller's stream (no allocation,
no host synchronisation, no memset), so it can be captured in a HIP graph
and replayed: every replay must reproduce the eager results bit for bit,
with unrelated eager work and synchronisations between the replays."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("method,P,B", [("vanilla", 1, 0), ("flash", 8, 0), ("beam", 4, 6)])
def test_graph_replay_matches_eager(fv, method, P, B):
    K = 72
    lp, la, _ = hmm.random_dense(K, 1, 80)
    rng = np.random.default_rng(81)
    lens = [40, 130, 7, 300]
    lbs = [_dev((rng.standard_normal((T, K)) * 2).astype(np.float32)) for T in lens]
    la_d, lp_d = _dev(la), _dev(lp)
    eager = fv.Batch(lbs)
    ws = fv.decode_batch(la_d, eager, lp_d, method=method, P=P, B=B)
    torch.cuda.synchronize()
    ref_p, ref_s, ref_st = eager.paths.clone(), eager.scores.clone(), eager.status.clone()

    batch = fv.Batch(lbs)
    ws2 = torch.empty_like(ws)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):   # warm-up on the capture stream
        fv.decode_batch(la_d, batch, lp_d, method=method, P=P, B=B, ws=ws2)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fv.decode_batch(la_d, batch, lp_d, method=method, P=P, B=B, ws=ws2)
    for rep in range(3):
        batch.paths.fill_(-1)            # entries past each length are never written
        batch.paths[:, 0] = -7
        batch.scores.fill_(123.0)
        batch.status.fill_(99)
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()               # unrelated eager work, synchronised
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(batch.paths, ref_p), rep
        assert torch.equal(batch.scores.view(torch.int32), ref_s.view(torch.int32)), rep
        assert torch.equal(batch.status, ref_st), rep
