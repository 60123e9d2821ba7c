"""Full-size parity on the batched workload the benchmark times: 256
sequences sharing a dense K = 1024 model (log A rows Dirichlet(0.1)),
lengths U[500, 8000], emission scores N(0, 2^2).

Each method decodes the whole batch in one launch, exactly as bench.py runs
it (same workload generator, same ``decode_batch`` call, default placement
and leaf schedule): vanilla, FLASH with P in {1, 4, 16, 64} and FLASH-BS with
P = 16, B in {64, 256}.  Every sequence's status must be FV_OK.  The oracle
then decodes a fixed sample one by one (the shortest, median and longest
sequences plus five seeded picks) and every sampled path must match element
by element and every sampled score bit for bit.  FLASH is compared with the
oracle's vanilla decode (FLASH = vanilla for every P under the anchored
start, Sec. V-B Def. 3); FLASH-BS with the oracle's FLASH-BS procedure at the
same B and P (Sec. V-C).  Oracle runs go to a thread pool (ctypes releases
the GIL) and are cached per (method, sequence)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from workloads import hmm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_EXTRA = 5


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2510_19301_amd as fv
    fv.lib()
    wl = hmm.batched_flash_workload()
    dev = torch.device("cuda", 0)
    order = np.argsort(wl.lengths, kind="stable")
    fixed = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    rest = [b for b in range(wl.n) if b not in fixed]
    extra = np.random.default_rng(20251019).choice(rest, N_EXTRA, replace=False)
    sample = fixed + [int(b) for b in extra]
    print(f"headline workload: n={wl.n} K={wl.K} sum T={wl.total_steps()} sample={sample}", flush=True)
    host = {}
    with ThreadPoolExecutor(max_workers=8) as ex:
        arrays = list(ex.map(wl.log_b, range(wl.n)))
    lbs = []
    for b, x in enumerate(arrays):
        lbs.append(torch.from_numpy(x).to(dev))
        if b in sample:
            host[b] = x
    del arrays
    la = torch.from_numpy(wl.log_a).to(dev)
    lp = torch.from_numpy(wl.log_pi).to(dev)
    batch = fv.Batch(lbs)
    torch.cuda.synchronize()
    cache = {}
    yield fv, wl, la, lp, batch, host, sample, cache
    del lbs, batch
    torch.cuda.empty_cache()


def _bits(x):
    return np.asarray(x, np.float32).reshape(-1).view(np.uint32)


def _oracle_refs(wl, host, sample, cache, method, P, B):
    key = ("vanilla", 0, 0) if method in ("vanilla", "flash") else (method, P, B)

    def one(b):
        if (key, b) in cache:
            return cache[(key, b)]
        if key[0] == "vanilla":
            po, so, rc = oracle.vanilla(wl.log_pi, wl.log_a, host[b])
        else:
            po, so, rc, _ = oracle.beam(wl.log_pi, wl.log_a, host[b], B, P)
        return po, so, rc

    with ThreadPoolExecutor(max_workers=8) as ex:
        refs = list(ex.map(one, sample))
    for b, r in zip(sample, refs):
        cache[(key, b)] = r
    return dict(zip(sample, refs))


@pytest.mark.parametrize("method,P,B", [("vanilla", 1, 0), ("flash", 1, 0), ("flash", 4, 0), ("flash", 16, 0),
                                        ("flash", 64, 0), ("beam", 16, 64), ("beam", 16, 256)])
def test_headline_batch_full_size(setup, method, P, B):
    fv, wl, la, lp, batch, host, sample, cache = setup
    print(f"headline batch: {method} P={P} B={B}", flush=True)
    batch.paths.fill_(-7)
    fv.decode_batch(la, batch, lp, method=method, P=P, B=B)
    torch.cuda.synchronize()
    status = batch.status.cpu().numpy()
    assert (status == fv.FV_OK).all(), np.unique(status, return_counts=True)
    paths = batch.paths.cpu().numpy()
    scores = batch.scores.cpu().numpy()
    # every position of every sequence was written with a valid state
    for b in range(wl.n):
        T = int(wl.lengths[b])
        row = paths[b, :T]
        assert row.min() >= 0 and row.max() < wl.K, (b, row.min(), row.max())
    print("  oracle on the sample", flush=True)
    refs = _oracle_refs(wl, host, sample, cache, method, P, B)
    for b in sample:
        T = int(wl.lengths[b])
        po, so, rc = refs[b]
        assert rc == oracle.OK
        assert (paths[b, :T] == po).all(), (b, T, np.flatnonzero(paths[b, :T] != po)[:10])
        assert _bits(scores[b]) == _bits(so), (b, scores[b], so)
