"""Full-size parity on the map-matching workload: K = 100000 states on a
9-nearest-neighbour graph (CSR), 64 trajectories of length U[200, 2000],
Gaussian GPS emissions.  The whole batch is decoded in one launch per method
(vanilla, FLASH P = 16, FLASH-BS B = 128 P = 16), exactly as the benchmark
runs it; the oracle then recomputes sampled trajectories one by one (the
shortest, a median one and the longest) and every returned path and score
must match bit for bit.  Every trajectory's status must be FV_OK."""
import numpy as np
import pytest

import oracle
from workloads import hmm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2510_19301_amd as fv
    fv.lib()
    wl = hmm.map_matching_workload()
    dev = torch.device("cuda", 0)
    lbs = [wl.log_b(b, dev) for b in range(wl.n)]
    model = fv.CsrModel(torch.from_numpy(wl.row_ptr).to(dev), torch.from_numpy(wl.col).to(dev),
                        torch.from_numpy(wl.val).to(dev))
    lp = torch.from_numpy(wl.log_pi).to(dev)
    order = np.argsort(wl.lengths, kind="stable")
    sample = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    yield fv, wl, lbs, model, lp, sample
    del lbs
    torch.cuda.empty_cache()


def _bits(x):
    return np.asarray(x, np.float32).reshape(-1).view(np.uint32)


def _decode(fv, model, lbs, lp, method, P, B):
    batch = fv.Batch(lbs)
    fv.decode_batch(model, batch, lp, method=method, P=P, B=B)
    torch.cuda.synchronize()
    return batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()


@pytest.mark.parametrize("method,P,B", [("vanilla", 1, 0), ("flash", 16, 0), ("beam", 16, 128)])
def test_map_matching_full_size(setup, method, P, B):
    fv, wl, lbs, model, lp, sample = setup
    print(f"map matching K={wl.K} n={wl.n} {method} P={P} B={B}", flush=True)
    paths, scores, status = _decode(fv, model, lbs, lp, method, P, B)
    assert (status == fv.FV_OK).all(), np.unique(status, return_counts=True)
    for b in sample:
        T = int(wl.lengths[b])
        lb = lbs[b].cpu().numpy()
        print(f"  oracle trajectory {b} (T={T})", flush=True)
        if method == "beam":
            po, so, rc, _ = oracle.beam_csr(wl.log_pi, wl.row_ptr, wl.col, wl.val, lb, B, P)
        else:
            po, so, rc = oracle.vanilla_csr(wl.log_pi, wl.row_ptr, wl.col, wl.val, lb)
        assert rc == oracle.OK
        assert (paths[b, :T] == po).all(), (b, np.flatnonzero(paths[b, :T] != po)[:10])
        assert _bits(scores[b]) == _bits(so), (b, scores[b], so)
