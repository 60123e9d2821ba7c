"""FV_FLAG_VALIDATE: NaN or +inf in a model's scores or in a sequence's
emissions makes the affected statuses FV_E_INVALID_ARG; clean sequences of
the same batch still decode exactly as the oracle does."""
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


def _batch(fv, la, lp, lbs, method, P=4, B=0, validate=True):
    batch = fv.Batch([_dev(x) for x in lbs])
    fv.decode_batch(la, batch, _dev(lp) if not isinstance(lp, torch.Tensor) else lp, method=method, P=P, B=B,
                    validate=validate)
    torch.cuda.synchronize()
    return batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()


@pytest.mark.parametrize("method,B", [("vanilla", 0), ("flash", 0), ("beam", 5)])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_bad_emission_flags_only_its_sequence(fv, method, B, bad):
    K = 40
    lp, la, _ = hmm.random_dense(K, 1, 60)
    rng = np.random.default_rng(61)
    lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in (30, 45, 12)]
    lbs[1][7, 3] = bad
    paths, scores, status = _batch(fv, _dev(la), lp, lbs, method, B=B)
    assert status[1] == fv.FV_E_INVALID_ARG
    for b in (0, 2):
        T = lbs[b].shape[0]
        if method == "beam":
            po, so, rc, _ = oracle.beam(lp, la, lbs[b], B, 4)
        else:
            po, so, rc = oracle.vanilla(lp, la, lbs[b])
        assert status[b] == rc and (paths[b, :T] == po).all() and _bits(scores[b]) == _bits(so)


@pytest.mark.parametrize("where", ["log_a", "log_pi"])
def test_bad_model_flags_every_sequence(fv, where):
    K = 33
    lp, la, _ = hmm.random_dense(K, 1, 62)
    if where == "log_a":
        la[5, 9] = np.nan
    else:
        lp[2] = np.inf
    rng = np.random.default_rng(63)
    lbs = [(rng.standard_normal((T, K)) * 2).astype(np.float32) for T in (10, 20)]
    for method in ("vanilla", "flash"):
        _, _, status = _batch(fv, _dev(la), lp, lbs, method)
        assert (status == fv.FV_E_INVALID_ARG).all()


def test_bad_csr_scores_and_clean_inputs(fv):
    lp, rp, col, val, lb = hmm.random_csr(50, 30, 64)
    model = fv.CsrModel(_dev(rp), _dev(col), _dev(val))
    # clean inputs: validation changes nothing
    po, so, rc = oracle.vanilla_csr(lp, rp, col, val, lb)
    for method in ("vanilla", "flash"):
        p, s, st = fv.decode(model, _dev(lb), _dev(lp), method=method, P=4, validate=True)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == rc and (p.cpu().numpy() == po).all() and _bits(s.cpu().numpy()) == _bits(so)
    val2 = val.copy()
    val2[len(val2) // 2] = np.nan
    model2 = fv.CsrModel(_dev(rp), _dev(col), _dev(val2))
    for method, B in (("vanilla", 0), ("flash", 0), ("beam", 4)):
        _, _, st = fv.decode(model2, _dev(lb), _dev(lp), method=method, P=4, B=B, validate=True)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == fv.FV_E_INVALID_ARG
