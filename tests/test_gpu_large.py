"""Parity at the large dense model's full K: K = 16384 states (log A rows
Dirichlet(0.05), 1 GiB float32), emission scores N(0, 3^2), one sequence of
T = 192 (the full-size T = 10000 is benchmarked, not oracle-checked: the
oracle's vanilla decode costs about 0.2 s per step at this K).

Vanilla and FLASH (P = 16) run on wide rows (every block takes a 64-column
slice of log A, Sec. III-A recurrence) and must equal the oracle's vanilla
decode; FLASH-BS at B = K must too (a beam of every state is FLASH,
Sec. V-C).  FLASH-BS with P = 16 and B in {16, 64, 256} must equal the
oracle's FLASH-BS procedure.  Paths element by element, scores bit for bit.
Oracle runs start in a thread pool when the module's fixture is built, so
they overlap the GPU decodes."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from workloads import hmm

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(400)]

torch = pytest.importorskip("torch")

K, T = 16384, 192
BEAMS = (16, 64, 256)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2510_19301_amd as fv
    fv.lib()
    print(f"large model: K={K} T={T}", flush=True)
    wl = hmm.dense_batch(K, 1, T, T, alpha=0.05, sigma=3.0, seed=3)
    lb = wl.log_b(0)
    ex = ThreadPoolExecutor(max_workers=4)
    refs = {"vanilla": ex.submit(oracle.vanilla, wl.log_pi, wl.log_a, lb)}
    for B in BEAMS:
        refs[B] = ex.submit(oracle.beam, wl.log_pi, wl.log_a, lb, B, 16)
    dev = torch.device("cuda", 0)
    la = torch.from_numpy(wl.log_a).to(dev)
    lbd = torch.from_numpy(lb).to(dev)
    lp = torch.from_numpy(wl.log_pi).to(dev)
    torch.cuda.synchronize()
    yield fv, la, lbd, lp, refs
    ex.shutdown(wait=True)
    del la, lbd
    torch.cuda.empty_cache()


def _bits(x):
    return np.asarray(x, np.float32).reshape(-1).view(np.uint32)


@pytest.mark.parametrize("method,P,B", [("vanilla", 1, 0), ("flash", 16, 0), ("beam", 16, K),
                                        ("beam", 16, 16), ("beam", 16, 64), ("beam", 16, 256)])
def test_large_dense(setup, method, P, B):
    fv, la, lbd, lp, refs = setup
    print(f"large K={K} T={T}: {method} P={P} B={B}", flush=True)
    path, score, status = fv.decode(la, lbd, lp, method, P=P, B=B)
    torch.cuda.synchronize()
    assert int(status.item()) == fv.FV_OK
    got_p, got_s = path.cpu().numpy(), score.cpu().numpy()
    if method == "beam" and B < K:
        po, so, rc, _ = refs[B].result()
    else:
        po, so, rc = refs["vanilla"].result()
    assert rc == oracle.OK
    assert (got_p == po).all(), np.flatnonzero(got_p != po)[:10]
    assert _bits(got_s) == _bits(so), (got_s, so)
