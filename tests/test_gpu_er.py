"""GPU parity on Erdos-Renyi HMMs (the paper's synthetic experiment shape:
edge probability p, |O| = 50 symbols, sampled observations), against the
CPU oracle: vanilla, FLASH and FLASH-BS paths element by element, scores
bit for bit."""
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
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _bits(x):
    return np.asarray(x, np.float32).reshape(-1).view(np.uint32)


@pytest.mark.parametrize("K,T,p", [(64, 80, 0.05), (96, 60, 0.253), (130, 45, 1.0), (200, 33, 0.1125)])
def test_er_exact_methods(fv, K, T, p):
    h = hmm.er_hmm(K=K, T=T, p=p, seed=K + T)
    lb = h.log_b()
    po, so, _ = oracle.vanilla(h.log_pi, h.log_a, lb)
    la, lbd, lp = _dev(h.log_a), _dev(lb), _dev(h.log_pi)
    for method, P, B in (("vanilla", 1, 0), ("flash", 1, 0), ("flash", 4, 0), ("flash", 16, 0)):
        path, score, st = fv.decode(la, lbd, lp, method=method, P=P, B=B)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == 0, (method, P)
        assert (path.cpu().numpy() == po).all(), (method, P)
        assert _bits(score.cpu().numpy()) == _bits(so), (method, P)


@pytest.mark.parametrize("K,T,p,B", [(96, 60, 0.253, 8), (128, 50, 0.05, 16), (160, 40, 1.0, 32)])
def test_er_beam(fv, K, T, p, B):
    h = hmm.er_hmm(K=K, T=T, p=p, seed=7 * K + B)
    lb = h.log_b()
    for P in (1, 4):
        ep, es, erc, _ = oracle.beam(h.log_pi, h.log_a, lb, B, P)
        path, score, st = fv.decode(_dev(h.log_a), _dev(lb), _dev(h.log_pi), method="beam", P=P, B=B)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == erc, (P, B)
        assert (path.cpu().numpy() == ep).all(), (P, B)
        assert _bits(score.cpu().numpy()) == _bits(np.float32(es)), (P, B)
