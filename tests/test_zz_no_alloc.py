"""fv_decode_flash_noalloc: the FLASH decode without a workspace argument,
its scratch a fixed device array inside the library.  Called through the C
ABI and compared with fv_decode_flash (caller workspace) on the same inputs,
path element by element and score bit for bit, on two calls in a row, the
second with a smaller input (the fixed array keeps the first call's
contents), then a decode too large for the array must be refused with
FV_E_WORKSPACE and a message, and a later call must still be exact."""
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


def _bits(x):
    return np.asarray(x, np.float32).reshape(-1).view(np.uint32)


def _inputs(K, T, seed):
    wl = hmm.dense_batch(K, 1, T, T, alpha=0.1, sigma=2.0, seed=seed)
    dev = torch.device("cuda", 0)
    return (wl, torch.from_numpy(wl.log_a).to(dev), torch.from_numpy(wl.log_b(0)).to(dev),
            torch.from_numpy(wl.log_pi).to(dev))


def _noalloc(fv, la, lb, lp, P):
    T, K = lb.shape
    path = torch.full((T,), -9, dtype=torch.int32, device="cuda")
    score = torch.full((1,), 5.0, device="cuda")
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    model = fv.dense_model(la)
    rc = fv.lib().fv_decode_flash_noalloc(C.byref(model), lp.data_ptr(), lb.data_ptr(), lb.stride(0), T, P,
                                          path.data_ptr(), score.data_ptr(), status.data_ptr(), 0,
                                          torch.cuda.current_stream().cuda_stream)
    return rc, path, score, status


def _compare(fv, wl, la, lb, lp, P, check_oracle):
    rc, path, score, status = _noalloc(fv, la, lb, lp, P)
    fv._lib.check(rc, "fv_decode_flash_noalloc")
    ref_p, ref_s, ref_st = fv.decode(la, lb, lp, "flash", P=P)
    torch.cuda.synchronize()
    assert int(status.item()) == fv.FV_OK == int(ref_st.item())
    assert torch.equal(path, ref_p)
    assert _bits(score.cpu().numpy()) == _bits(ref_s.cpu().numpy())
    if check_oracle:
        po, so, _ = oracle.vanilla(wl.log_pi, wl.log_a, wl.log_b(0))
        assert (path.cpu().numpy() == po).all()
        assert _bits(score.cpu().numpy()) == _bits(so)


def test_noalloc_two_calls_then_smaller(fv):
    # first call: K = 1024, T = 3000, P = 64 (about 63 MB of scratch)
    wl, la, lb, lp = _inputs(1024, 3000, 41)
    print("noalloc call 1: K=1024 T=3000 P=64", flush=True)
    _compare(fv, wl, la, lb, lp, 64, check_oracle=True)
    # second call, smaller: K = 600, T = 400, P = 8
    wl2, la2, lb2, lp2 = _inputs(600, 400, 42)
    print("noalloc call 2: K=600 T=400 P=8", flush=True)
    _compare(fv, wl2, la2, lb2, lp2, 8, check_oracle=True)
    # a small dense model (one block per sequence) through the same array
    wl3, la3, lb3, lp3 = _inputs(96, 250, 43)
    print("noalloc call 3: K=96 T=250 P=16", flush=True)
    _compare(fv, wl3, la3, lb3, lp3, 16, check_oracle=True)


def test_noalloc_refuses_oversized(fv):
    K, T = 2048, 4000     # about 146 MB of scratch (leaf tables)
    need = fv.workspace_bytes("flash", K, [T], 16)
    assert need > (128 << 20)
    la = torch.zeros((K, K), device="cuda")
    lb = torch.zeros((T, K), device="cuda")
    lp = torch.zeros(K, device="cuda")
    rc, path, _, _ = _noalloc(fv, la, lb, lp, 16)
    torch.cuda.synchronize()
    assert rc == fv.FV_E_WORKSPACE
    msg = fv.lib().fv_last_error().decode()
    assert "scratch" in msg and str(need) in msg, msg
    assert (path.cpu().numpy() == -9).all()     # nothing was enqueued
    # the array still serves a decode that fits
    wl, la2, lb2, lp2 = _inputs(600, 400, 44)
    _compare(fv, wl, la2, lb2, lp2, 8, check_oracle=False)
