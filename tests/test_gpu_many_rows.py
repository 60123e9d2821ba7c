"""Parity with many rows in flight: 2048 sequences on one dense K = 512 model
(log A rows Dirichlet(0.1), emission scores N(0, 2^2)), lengths U[64, 200],
decoded in one launch with rows kept on their XCD (the default placement at
this K).  All 2048 roots are admitted at the first step, 256 per XCD, for at
least the first 64 steps; that is beyond the count up to which an XCD
computes its rows as column items, so the lane-tile kernel (lanes = rows,
log A read as wave-uniform scalars) carries those steps.  Every sequence is
checked against the oracle's vanilla decode (FLASH = vanilla for every P,
Sec. V-B Def. 3), paths element by element and scores bit for bit."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from workloads import hmm

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(300)]

torch = pytest.importorskip("torch")

N, KM = 2048, 512


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2510_19301_amd as fv
    fv.lib()
    wl = hmm.dense_batch(KM, N, 64, 200, alpha=0.1, sigma=2.0, seed=21)
    print(f"many rows: n={wl.n} K={wl.K} sum T={wl.total_steps()}", flush=True)
    host = [wl.log_b(b) for b in range(wl.n)]
    ex = ThreadPoolExecutor(max_workers=8)
    refs = [ex.submit(oracle.vanilla, wl.log_pi, wl.log_a, host[b]) for b in range(wl.n)]
    dev = torch.device("cuda", 0)
    lbs = [torch.from_numpy(x).to(dev) for x in host]
    la = torch.from_numpy(wl.log_a).to(dev)
    lp = torch.from_numpy(wl.log_pi).to(dev)
    batch = fv.Batch(lbs)
    torch.cuda.synchronize()
    yield fv, wl, la, lp, batch, refs
    ex.shutdown(wait=True)
    del lbs, batch
    torch.cuda.empty_cache()


def _bits(x):
    return np.asarray(x, np.float32).reshape(-1).view(np.uint32)


@pytest.mark.parametrize("method,P", [("vanilla", 1), ("flash", 16), ("flash", 4)])
def test_many_rows_every_sequence(setup, method, P):
    fv, wl, la, lp, batch, refs = setup
    print(f"many rows: {method} P={P}", flush=True)
    batch.paths.fill_(-7)
    fv.decode_batch(la, batch, lp, method=method, P=P, rows="local")
    torch.cuda.synchronize()
    status = batch.status.cpu().numpy()
    assert (status == fv.FV_OK).all(), np.unique(status, return_counts=True)
    paths, scores = batch.paths.cpu().numpy(), batch.scores.cpu().numpy()
    bad = []
    for b in range(wl.n):
        Tb = int(wl.lengths[b])
        po, so, rc = refs[b].result()
        assert rc == oracle.OK
        if not (paths[b, :Tb] == po).all() or _bits(scores[b]) != _bits(so):
            bad.append(b)
    assert not bad, (len(bad), bad[:10])
