"""GPU parity of the Viterbi-score backward (fv_viterbi_backward) and of the
ViterbiScore autograd function against the CPU oracle, bit for bit."""
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


def _rand_paths(K, lengths, tmax, seed, bad_frac=0.0, sticky=0.0):
    rng = np.random.default_rng(seed)
    n = len(lengths)
    p = np.full((n, tmax), -1, np.int32)
    for b, T in enumerate(lengths):
        q = rng.integers(0, K, size=T).astype(np.int32)
        if sticky:   # repeated transitions: counts above one
            keep = rng.random(T) < sticky
            for t in range(1, T):
                if keep[t]:
                    q[t] = q[t - 1]
        if bad_frac:
            q[rng.random(T) < bad_frac] = -1
        p[b, :T] = q
    return p


def _run(fv, K, lengths, paths, g, init=None, want=(True, True, True)):
    dev = torch.device("cuda", 0)
    n, tmax = paths.shape
    L = torch.from_numpy(np.asarray(lengths, np.int32)).to(dev)
    P = torch.from_numpy(paths).to(dev)
    G = torch.from_numpy(np.asarray(g, np.float32)).to(dev)
    outs = []
    for k, shape in enumerate(((n, tmax, K), (K, K), (K,))):
        if not want[k]:
            outs.append(None)
        elif init is not None:
            outs.append(torch.from_numpy(init[k].copy()).to(dev))
        else:
            outs.append(torch.full(shape, np.float32(7.0), device=dev))   # overwritten
    fv.viterbi_backward(K, L, P, G, *outs, accumulate=init is not None)
    torch.cuda.synchronize()
    return [None if o is None else o.cpu().numpy() for o in outs]


def _same(a, b):
    assert a.shape == b.shape
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), np.argwhere(a.view(np.uint32) != b.view(np.uint32))[:5]


CASES = [
    # K, lengths, Tmax, g kind, sticky, bad
    (5, [0, 1, 2, 7], 7, "ones", 0.0, 0.0),
    (17, [9, 30, 1, 30, 0, 12], 30, "uniform", 0.5, 0.0),
    (64, [100, 257, 3], 257, "uniform", 0.9, 0.0),
    (33, [50, 40], 50, "signed", 0.3, 0.1),
    (256, [512] * 4 + [32, 77], 512, "uniform", 0.2, 0.0),
    (3, [2000, 1999], 2000, "uniform", 0.0, 0.0),          # few cells, many repeats
    (1, [10, 0, 3], 10, "ones", 0.0, 0.0),
]


@pytest.mark.parametrize("K,lengths,tmax,gk,sticky,bad", CASES)
def test_backward_matches_oracle(fv, K, lengths, tmax, gk, sticky, bad):
    rng = np.random.default_rng(K * 1000 + tmax)
    paths = _rand_paths(K, lengths, tmax, K + tmax, bad_frac=bad, sticky=sticky)
    n = len(lengths)
    g = {"ones": np.ones(n), "uniform": rng.random(n), "signed": rng.normal(size=n)}[gk].astype(np.float32)
    gb, ga, gp = _run(fv, K, lengths, paths, g)
    rb, ra, rp = oracle.backward(K, lengths, paths, g)
    _same(gb, rb)
    _same(ga, ra)
    _same(gp, rp)
    if gk == "ones" and not bad:
        assert ga.sum() == sum(max(T - 1, 0) for T in lengths)


def test_backward_accumulate_and_partial_outputs(fv):
    K, lengths, tmax = 40, [60, 1, 59, 0, 60], 60
    paths = _rand_paths(K, lengths, tmax, 3, sticky=0.6)
    rng = np.random.default_rng(4)
    g = rng.random(len(lengths)).astype(np.float32)
    init = [rng.normal(size=s).astype(np.float32) for s in ((len(lengths), tmax, K), (K, K), (K,))]
    gb, ga, gp = _run(fv, K, lengths, paths, g, init=init)
    rb, ra, rp = oracle.backward(K, lengths, paths, g, init_b=init[0], init_a=init[1], init_pi=init[2])
    _same(gb, rb)
    _same(ga, ra)
    _same(gp, rp)
    for want in ((True, False, False), (False, True, False), (False, False, True)):
        out = _run(fv, K, lengths, paths, g, want=want)
        ref = oracle.backward(K, lengths, paths, g)
        for o, r in zip(out, ref):
            if o is not None:
                _same(o, r)


def test_backward_is_deterministic(fv):
    K, tmax = 16, 300
    lengths = [300] * 64
    paths = _rand_paths(K, lengths, tmax, 9, sticky=0.3)
    g = np.random.default_rng(10).random(64).astype(np.float32)
    a = _run(fv, K, lengths, paths, g)
    b = _run(fv, K, lengths, paths, g)
    for x, y in zip(a, b):
        _same(x, y)


def test_crf_config_forward_and_backward(fv):
    """Linear-chain CRF workload: 512 sequences, K = 256, T in [32, 512],
    emissions from a random Linear(512 -> 256), transitions N(0, 0.1^2), no
    start scores.  Forward (vanilla and FLASH P = 16) on sampled sequences and
    the full backward against the oracle."""
    wl = hmm.crf_batch()
    dev = torch.device("cuda", 0)
    em = torch.from_numpy(wl.emissions).to(dev)
    tr = torch.from_numpy(wl.transitions).to(dev)
    n, tmax, K = em.shape
    sample = np.random.default_rng(11).choice(n, size=12, replace=False)
    paths = {}
    for method, P in (("vanilla", 1), ("flash", 16)):
        scores, p = fv.ViterbiScore.apply(em, wl.lengths, tr, None, method, P)
        torch.cuda.synchronize()
        paths[method] = p.cpu().numpy()
        sc = scores.cpu().numpy()
        for b in sample:
            T = int(wl.lengths[b])
            rp, rs, rc = oracle.vanilla(None, wl.transitions, wl.emissions[b, :T])
            assert rc == oracle.OK
            assert np.array_equal(paths[method][b, :T], rp), (method, b)
            assert sc[b].tobytes() == np.float32(rs).tobytes(), (method, b)
    assert np.array_equal(paths["vanilla"], paths["flash"])
    # backward with g = 1 (structured hinge) and g ~ U(0, 1)
    for gk in ("ones", "uniform"):
        g = np.ones(n, np.float32) if gk == "ones" else np.random.default_rng(12).random(n).astype(np.float32)
        gb, ga, gp = _run(fv, K, wl.lengths, paths["flash"], g, want=(True, True, False))
        rb, ra, _ = oracle.backward(K, wl.lengths, paths["flash"], g, want_pi=False)
        _same(gb, rb)
        _same(ga, ra)


def test_autograd_gradients(fv):
    dev = torch.device("cuda", 0)
    K, lengths = 24, [40, 1, 17, 40]
    n, tmax = len(lengths), max(lengths)
    rng = np.random.default_rng(13)
    em = rng.normal(size=(n, tmax, K)).astype(np.float32)
    tr = (rng.normal(size=(K, K)) * 0.5).astype(np.float32)
    st = rng.normal(size=K).astype(np.float32)
    E = torch.from_numpy(em).to(dev).requires_grad_(True)
    A = torch.from_numpy(tr).to(dev).requires_grad_(True)
    S = torch.from_numpy(st).to(dev).requires_grad_(True)
    scores, paths = fv.ViterbiScore.apply(E, lengths, A, S, "flash", 4)
    w = torch.from_numpy(rng.random(n).astype(np.float32)).to(dev)
    (scores * w).sum().backward()
    torch.cuda.synchronize()
    p = paths.cpu().numpy()
    for b, T in enumerate(lengths):
        rp, rs, _ = oracle.vanilla(st, tr, em[b, :T])
        assert np.array_equal(p[b, :T], rp)
        assert scores[b].item() == float(np.float32(rs))
    rb, ra, rpi = oracle.backward(K, lengths, p, w.cpu().numpy())
    _same(E.grad.cpu().numpy(), rb)
    _same(A.grad.cpu().numpy(), ra)
    _same(S.grad.cpu().numpy(), rpi)
    # the score moves by h along a path coordinate whose change keeps the path
    h = 1e-2
    b, t = 0, 5
    q = int(p[b, t])
    em2 = em.copy()
    em2[b, t, q] += h
    s2, p2 = fv.ViterbiScore.apply(torch.from_numpy(em2).to(dev), lengths, A.detach(), S.detach(), "flash", 4)
    assert np.array_equal(p2.cpu().numpy(), p)
    fd = (s2[b].item() - scores[b].item()) / h
    assert abs(fd - 1.0) < 2 * np.spacing(np.float32(abs(scores[b].item()))) / h + 1e-3


def test_central_finite_differences(fv):
    """CRF-style inputs with continuous noise (a unique arg max): central
    differences, h = 1e-3, of the Viterbi scores against the hand-written
    backward, for emission entries on and off the decoded paths (gradient 1
    and 0) and for transition entries (gradient = the pair's count along the
    paths).  Every perturbed decode must keep the paths; the tolerance is the
    float32 spacing of the scores involved over 2h, plus 1e-3."""
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(17)
    K, lengths = 32, [60, 47, 33, 58]
    n, tmax = len(lengths), max(lengths)
    em = np.zeros((n, tmax, K), np.float32)
    for b, T in enumerate(lengths):
        em[b, :T] = rng.normal(size=(T, K)).astype(np.float32)
    tr = (rng.normal(size=(K, K)) * 0.1).astype(np.float32)
    h = np.float32(1e-3)

    def decode(e, a):
        s, p = fv.ViterbiScore.apply(torch.from_numpy(e).to(dev), lengths, torch.from_numpy(a).to(dev), None,
                                     "flash", 4)
        torch.cuda.synchronize()
        return s.cpu().numpy().astype(np.float64), p.cpu().numpy()

    E = torch.from_numpy(em).to(dev).requires_grad_(True)
    A = torch.from_numpy(tr).to(dev).requires_grad_(True)
    scores, paths = fv.ViterbiScore.apply(E, lengths, A, None, "flash", 4)
    scores.sum().backward()
    torch.cuda.synchronize()
    p0 = paths.cpu().numpy()
    gE, gA = E.grad.cpu().numpy(), A.grad.cpu().numpy()

    def tol(s_plus, s_minus, seqs):
        sp = sum(np.spacing(np.float32(max(abs(s_plus[b]), abs(s_minus[b])))) for b in seqs)
        return 2 * float(sp) / (2 * float(h)) + 1e-3

    checked = 0
    for k in range(24):   # emissions: half on a path, half off it
        b = int(rng.integers(n))
        t = int(rng.integers(lengths[b]))
        j = int(p0[b, t]) if k % 2 == 0 else int((p0[b, t] + 1 + rng.integers(K - 1)) % K)
        ep, emn = em.copy(), em.copy()
        ep[b, t, j] += h
        emn[b, t, j] -= h
        sp, pp = decode(ep, tr)
        sm, pm = decode(emn, tr)
        assert np.array_equal(pp, p0) and np.array_equal(pm, p0)
        fd = (sp[b] - sm[b]) / (2 * float(h))
        assert abs(fd - gE[b, t, j]) <= tol(sp, sm, [b]), (b, t, j, fd, gE[b, t, j])
        checked += 1
    used = np.argwhere(gA > 0)
    cells = [tuple(used[i]) for i in rng.choice(len(used), size=8, replace=False)]
    cells += [(int(rng.integers(K)), int(rng.integers(K))) for _ in range(8)]
    for (i, j) in cells:   # transitions: counts along the paths (0 when unused)
        ap, am = tr.copy(), tr.copy()
        ap[i, j] += h
        am[i, j] -= h
        sp, pp = decode(em, ap)
        sm, pm = decode(em, am)
        assert np.array_equal(pp, p0) and np.array_equal(pm, p0)
        fd = (sp.sum() - sm.sum()) / (2 * float(h))
        assert abs(fd - gA[i, j]) <= tol(sp, sm, range(n)), (i, j, fd, gA[i, j])
        checked += 1
    assert checked == 40
