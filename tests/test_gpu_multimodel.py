"""One persistent launch over several transition models of different K
(dense and sparse mixed): every sequence's result must equal the oracle's
for its own model, bit for bit, for each method."""
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


def _models(fv):
    """Three dense models (K = 37, 64, 200) and one sparse model (K = 90)."""
    out = []
    for k, K in enumerate((37, 64, 200)):
        lp, la, _ = hmm.random_dense(K, 1, 40 + k)
        out.append(("dense", K, lp if k != 1 else None, la, _dev(la)))
    lp, rp, col, val, _ = hmm.random_csr(90, 1, 44, deg_lo=1, deg_hi=7)
    out.append(("csr", 90, lp, (rp, col, val), fv.CsrModel(_dev(rp), _dev(col), _dev(val))))
    return out


def _expected(kind, lp, A, lb, method, P, B):
    if kind == "dense":
        if method == "beam" and B < A.shape[0]:
            p, s, rc, _ = oracle.beam(lp, A, lb, B, P)
        else:
            p, s, rc = oracle.vanilla(lp, A, lb)
    else:
        rp, col, val = A
        if method == "beam" and B < rp.shape[0] - 1:
            p, s, rc, _ = oracle.beam_csr(lp, rp, col, val, lb, B, P)
        else:
            p, s, rc = oracle.vanilla_csr(lp, rp, col, val, lb)
    return p, s, rc


@pytest.mark.parametrize("method,P,B", [("vanilla", 1, 0), ("flash", 1, 0), ("flash", 8, 0), ("beam", 4, 5),
                                        ("beam", 2, 64)])
def test_multimodel_batch(fv, method, P, B):
    models = _models(fv)
    rng = np.random.default_rng(45)
    seq_models = [0, 1, 2, 3, 3, 2, 1, 0, 2, 2, 3, 1]
    lens = [30, 1, 77, 50, 0, 130, 12, 2, 64, 9, 101, 40]
    lbs = [(rng.standard_normal((T, models[m][1])) * 2).astype(np.float32) for m, T in zip(seq_models, lens)]
    batch = fv.Batch([_dev(x) if len(x) else torch.empty((0, models[m][1]), device="cuda")
                      for x, m in zip(lbs, seq_models)], models=seq_models)
    print(f"multi-model {method} P={P} B={B}", flush=True)
    fv.decode_batch([m[4] for m in models], batch, [_dev(m[2]) for m in models], method=method, P=P, B=B)
    torch.cuda.synchronize()
    paths, scores, status = batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()
    for b, (m, T) in enumerate(zip(seq_models, lens)):
        if T == 0:
            assert status[b] == fv.FV_OK and scores[b] == 0.0
            continue
        kind, K, lp, A, _ = models[m]
        po, so, rc = _expected(kind, lp, A, lbs[b], method, P, B)
        assert status[b] == rc, (b, status[b], rc)
        assert (paths[b, :T] == po).all(), (b, np.flatnonzero(paths[b, :T] != po)[:10])
        assert _bits(scores[b]) == _bits(so), (b, scores[b], so)


def test_multimodel_equals_single_model_calls(fv):
    """A mixed batch gives each sequence the result of a one-model batch."""
    models = _models(fv)
    rng = np.random.default_rng(46)
    seq_models = [2, 0, 2, 1, 3, 0]
    lens = [90, 33, 5, 70, 44, 61]
    lbs = [_dev((rng.standard_normal((T, models[m][1])) * 2).astype(np.float32)) for m, T in zip(seq_models, lens)]
    mixed = fv.Batch(lbs, models=seq_models)
    fv.decode_batch([m[4] for m in models], mixed, [_dev(m[2]) for m in models], method="flash", P=4)
    for b, m in enumerate(seq_models):
        one = fv.Batch([lbs[b]])
        fv.decode_batch(models[m][4], one, _dev(models[m][2]), method="flash", P=4)
        torch.cuda.synchronize()
        T = lens[b]
        assert (mixed.paths[b, :T].cpu() == one.paths[0, :T].cpu()).all()
        assert _bits(mixed.scores[b].cpu().numpy()) == _bits(one.scores[0].cpu().numpy())


def test_device_model_index_out_of_range_is_reported(fv):
    """The device descriptors name a model the call does not have: that
    sequence gets FV_E_INVALID_ARG, the host-side counts then disagree with
    the device's and the model's other sequences are refused too."""
    models = _models(fv)[:2]
    rng = np.random.default_rng(47)
    lbs = [_dev((rng.standard_normal((20, 37)) * 2).astype(np.float32)) for _ in range(3)]
    batch = fv.Batch(lbs, models=[0, 5, 0])      # device descriptors: the middle one says model 5
    lib = fv.lib()
    trans = (fv._lib.FvTrans * 2)(*[fv.model_descriptor(m[4]) for m in models])
    host_models = np.array([0, 0, 0], np.int32)
    lengths = np.ascontiguousarray(batch.lengths, np.int32)
    n = fv.workspace_bytes_models("flash", trans, 2, lengths, host_models, 4, 0)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    pis = (C.c_void_p * 2)(None, None)
    rc = lib.fv_decode_batch(trans, C.cast(pis, C.c_void_p), 2, batch.desc.data_ptr(), lengths.ctypes.data,
                             host_models.ctypes.data, 3, fv._lib.FV_FLASH, 4, 0, batch.status.data_ptr(), 0,
                             ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    assert (batch.status.cpu().numpy() == fv.FV_E_INVALID_ARG).all()


@pytest.mark.parametrize("method,P", [("vanilla", 1), ("flash", 1), ("flash", 8), ("beam", 4)])
def test_multimodel_small_dense(fv, method, P):
    """Dense models of K = 20, 64 and 100 only (vanilla and FLASH run one
    wave per sequence, one launch per model; beam with B >= K is FLASH):
    every sequence equals the oracle for its own model."""
    models = []
    for k, K in enumerate((20, 64, 100)):
        lp, la, _ = hmm.random_dense(K, 1, 70 + k)
        models.append(("dense", K, lp if k != 2 else None, la, _dev(la)))
    rng = np.random.default_rng(71)
    seq_models = [0, 1, 2, 2, 1, 0, 0, 2, 1, 1]
    lens = [40, 300, 1, 0, 77, 129, 2, 250, 64, 5]
    lbs = [(rng.standard_normal((T, models[m][1])) * 2).astype(np.float32) for m, T in zip(seq_models, lens)]
    batch = fv.Batch([_dev(x) if len(x) else torch.empty((0, models[m][1]), device="cuda")
                      for x, m in zip(lbs, seq_models)], models=seq_models)
    B = 128 if method == "beam" else 0
    print(f"multi-model small {method} P={P} B={B}", flush=True)
    fv.decode_batch([m[4] for m in models], batch, [_dev(m[2]) for m in models], method=method, P=P, B=B)
    torch.cuda.synchronize()
    paths, scores, status = batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()
    for b, (m, T) in enumerate(zip(seq_models, lens)):
        if T == 0:
            assert status[b] == fv.FV_OK and scores[b] == 0.0
            continue
        kind, K, lp, A, _ = models[m]
        po, so, rc = _expected(kind, lp, A, lbs[b], method, P, B)
        assert status[b] == rc, (b, status[b], rc)
        assert (paths[b, :T] == po).all(), (b, np.flatnonzero(paths[b, :T] != po)[:10])
        assert _bits(scores[b]) == _bits(so), (b, scores[b], so)
