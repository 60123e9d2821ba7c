"""GPU parity of generated emissions (fv_decode_batch_emit, CSR models): the
Gaussian point model's scores (Sec. III: continuous observations) are
computed inside the decode from the state points and each sequence's
observed points instead of being read from log_b tables.

Expected results come from the oracle alone: its own evaluation of the
emission model (float64, one rounding per operation, then float32) feeds its
vanilla / FLASH-BS decoders, and every GPU path must equal the oracle's
element by element with the score bit for bit.  Cases: a small map-matching
workload with every method, exact ties on an integer grid (the lowest-index
rule decides), the full-size map-matching batch (sampled trajectories),
validation of non-finite coordinates, and the host-side argument checks."""
import ctypes as C
from concurrent.futures import ThreadPoolExecutor

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


def _csr(fv, row_ptr, col, val):
    return fv.CsrModel(torch.from_numpy(np.ascontiguousarray(row_ptr, np.int32)).cuda(),
                       torch.from_numpy(np.ascontiguousarray(col, np.int32)).cuda(),
                       torch.from_numpy(np.ascontiguousarray(val, np.float32)).cuda())


def _ref(lp, row_ptr, col, val, lb, method, P, B):
    if method == "beam":
        po, so, rc, _ = oracle.beam_csr(lp, row_ptr, col, val, lb, B, P)
    else:
        po, so, rc = oracle.vanilla_csr(lp, row_ptr, col, val, lb)
    return po, so, rc


def _decode_obs(fv, model, em, obs, lp, method, P, B, validate=False):
    batch = fv.Batch.observations([torch.from_numpy(np.ascontiguousarray(o)).cuda() for o in obs])
    fv.decode_batch(model, batch, None if lp is None else torch.from_numpy(lp).cuda(), method=method, P=P, B=B,
                    emission=em, validate=validate)
    torch.cuda.synchronize()
    return batch.paths.cpu().numpy(), batch.scores.cpu().numpy(), batch.status.cpu().numpy()


def _check(fv, paths, scores, status, refs, lens):
    for b, ((po, so, rc), T) in enumerate(zip(refs, lens)):
        if T == 0:
            assert status[b] == fv.FV_OK and _bits(scores[b]) == _bits(np.float32(0.0))
            continue
        assert status[b] == rc, (b, status[b], rc)   # the oracle's codes are the library's
        assert (paths[b, :T] == po).all(), (b, T, np.flatnonzero(paths[b, :T] != po)[:8])
        assert _bits(scores[b]) == _bits(so), (b, scores[b], so)


@pytest.fixture(scope="module")
def small_map():
    wl = hmm.map_matching_workload(seed=11, K=5000, n=10, t_lo=1, t_hi=400)
    lens = [int(x) for x in wl.lengths]
    lens[0], lens[1] = 1, 2   # the shortest cases
    obs = [wl.gps(b)[:lens[b]] for b in range(wl.n)]
    c2, c0 = oracle.gauss_coefficients(wl.sigma_gps)
    lbs = [oracle.gauss_emissions(wl.xy, o, c2, c0) for o in obs]
    return wl, obs, lens, lbs, c2, c0


@pytest.mark.parametrize("method,P,B", [("vanilla", 1, 0), ("flash", 16, 0), ("flash", 1, 0), ("flash", 64, 0),
                                        ("beam", 16, 64), ("beam", 4, 1), ("beam", 16, 5000)])
def test_generated_emission_matches_oracle(fv, small_map, method, P, B):
    wl, obs, lens, lbs, c2, c0 = small_map
    print(f"generated emission K={wl.K} {method} P={P} B={B}", flush=True)
    model = _csr(fv, wl.row_ptr, wl.col, wl.val)
    em = fv.GaussEmission(torch.from_numpy(wl.xy).cuda(), c2, c0)
    paths, scores, status = _decode_obs(fv, model, em, obs, wl.log_pi, method, P, B)
    with ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(lambda lb: _ref(wl.log_pi, wl.row_ptr, wl.col, wl.val, lb, method, P, B), lbs))
    _check(fv, paths, scores, status, refs, lens)


def _grid_model(side):
    """States on an integer grid side x side (state = y * side + x); edges to
    the 4-neighbours and to itself, every score 0 (all ties) or -1."""
    K = side * side
    rows, cols, vals = [], [], []
    for s in range(K):
        x, y = s % side, s // side
        nb = [(x, y), (x - 1, y), (x + 1, y), (x, y - 1), (x, y + 1)]
        for (u, v) in nb:
            if 0 <= u < side and 0 <= v < side:
                rows.append(s)
                cols.append(v * side + u)
                vals.append(0.0 if (u, v) == (x, y) or (u + v) % 2 == 0 else -1.0)
    order = np.lexsort((np.array(cols), np.array(rows)))
    rows, cols, vals = np.array(rows)[order], np.array(cols)[order], np.array(vals, np.float32)[order]
    row_ptr = np.zeros(K + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    xy = np.array([[s % side, s // side] for s in range(K)], np.float64)
    return K, np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32), vals, xy


@pytest.mark.parametrize("method,P,B", [("vanilla", 1, 0), ("flash", 8, 0), ("beam", 8, 16)])
def test_generated_emission_exact_ties(fv, method, P, B):
    """Observations on half-integer points sit at equal distances from
    several states; c2 = -1, c0 = 0 make every score an exact small number,
    so ties are everywhere and the lowest index must win, as in the oracle."""
    side = 40
    K, row_ptr, col, val, xy = _grid_model(side)
    rng = np.random.default_rng(21)
    lens = [1, 3, 50, 333, 0, 129]
    obs = [(rng.integers(0, 2 * side - 1, size=(T, 2)) * 0.5).astype(np.float64) for T in lens]
    lbs = [oracle.gauss_emissions(xy, o, -1.0, 0.0) for o in obs]
    model = _csr(fv, row_ptr, col, val)
    em = fv.GaussEmission(torch.from_numpy(xy).cuda(), -1.0, 0.0)
    print(f"grid ties K={K} {method} P={P} B={B}", flush=True)
    paths, scores, status = _decode_obs(fv, model, em, obs, None, method, P, B)
    refs = [_ref(None, row_ptr, col, val, lb, method, P, B) if lb.shape[0] else (None, None, oracle.OK)
            for lb in lbs]
    _check(fv, paths, scores, status, refs, lens)


@pytest.fixture(scope="module")
def full_map(fv):
    wl = hmm.map_matching_workload()
    dev = torch.device("cuda", 0)
    c2, c0 = oracle.gauss_coefficients(wl.sigma_gps)
    obs = [wl.gps(b) for b in range(wl.n)]
    model = _csr(fv, wl.row_ptr, wl.col, wl.val)
    em = fv.GaussEmission(torch.from_numpy(wl.xy).to(dev), c2, c0)
    order = np.argsort(wl.lengths, kind="stable")
    sample = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    return wl, obs, model, em, c2, c0, sample


@pytest.mark.timeout(600)
@pytest.mark.parametrize("method,P,B", [("vanilla", 1, 0), ("flash", 16, 0), ("beam", 16, 128)])
def test_generated_emission_full_size(fv, full_map, method, P, B):
    """The map-matching batch at full size (K = 100000, 64 trajectories of
    200 to 2000 points) in one launch, as the benchmark runs it: every
    status FV_OK; the shortest, a median and the longest trajectory equal
    the oracle's decode of the oracle's emission tables."""
    wl, obs, model, em, c2, c0, sample = full_map
    print(f"generated emission full size {method} P={P} B={B}", flush=True)
    paths, scores, status = _decode_obs(fv, model, em, obs, wl.log_pi, method, P, B)
    assert (status == fv.FV_OK).all(), np.unique(status, return_counts=True)
    for b in sample:
        T = int(wl.lengths[b])
        print(f"  oracle trajectory {b} (T={T})", flush=True)
        lb = oracle.gauss_emissions(wl.xy, obs[b], c2, c0)
        po, so, rc = _ref(wl.log_pi, wl.row_ptr, wl.col, wl.val, lb, method, P, B)
        assert rc == oracle.OK
        assert (paths[b, :T] == po).all(), (b, np.flatnonzero(paths[b, :T] != po)[:10])
        assert _bits(scores[b]) == _bits(so), (b, scores[b], so)


def test_generated_emission_validation(fv, small_map):
    """FV_FLAG_VALIDATE: a non-finite observation marks its own sequence
    FV_E_INVALID_ARG; a non-finite state point marks every sequence."""
    wl, obs, lens, lbs, c2, c0 = small_map
    model = _csr(fv, wl.row_ptr, wl.col, wl.val)
    em = fv.GaussEmission(torch.from_numpy(wl.xy).cuda(), c2, c0)
    bad = [o.copy() for o in obs]
    bad[4][min(3, lens[4] - 1), 1] = np.nan
    bad[6][0, 0] = np.inf
    paths, scores, status = _decode_obs(fv, model, em, bad, wl.log_pi, "flash", 16, 0, validate=True)
    for b in range(len(obs)):
        assert status[b] == (fv.FV_E_INVALID_ARG if b in (4, 6) else fv.FV_OK), (b, status[b])
    refs = [_ref(wl.log_pi, wl.row_ptr, wl.col, wl.val, lbs[b], "flash", 16, 0) for b in (0, 2)]
    for b, (po, so, _) in zip((0, 2), refs):
        assert (paths[b, :lens[b]] == po).all() and _bits(scores[b]) == _bits(so)
    xy = wl.xy.copy()
    xy[17, 0] = np.nan
    em_bad = fv.GaussEmission(torch.from_numpy(xy).cuda(), c2, c0)
    _, _, status = _decode_obs(fv, model, em_bad, obs, wl.log_pi, "vanilla", 1, 0, validate=True)
    assert (status == fv.FV_E_INVALID_ARG).all(), status


def test_generated_emission_argument_checks(fv, small_map):
    """Host-side rejections, returned before anything is enqueued."""
    wl, obs, lens, lbs, c2, c0 = small_map
    xy = torch.from_numpy(wl.xy).cuda()
    model = _csr(fv, wl.row_ptr, wl.col, wl.val)
    o = [torch.from_numpy(x).cuda() for x in obs[:2]]
    # a dense model cannot take a generated emission
    la = torch.zeros((wl.K, wl.K), dtype=torch.float32, device="cuda")
    with pytest.raises(fv.FvError) as e:
        fv.decode_batch(la, fv.Batch.observations(o), method="vanilla", emission=fv.GaussEmission(xy, c2, c0))
    assert "status -2" in str(e.value)
    del la
    # c2 > 0 (scores could reach +inf), c0 = NaN
    for cc2, cc0 in ((0.5, c0), (c2, float("nan")), (float("-inf"), c0)):
        with pytest.raises(fv.FvError) as e:
            fv.decode_batch(model, fv.Batch.observations(o), method="vanilla",
                            emission=fv.GaussEmission(xy, cc2, cc0))
        assert "status -1" in str(e.value)
    # an unknown emission kind, through the C ABI
    batch = fv.Batch.observations(o)
    desc = fv._lib.FvEmission(7, xy.data_ptr(), c2, c0)
    lengths = np.ascontiguousarray(batch.lengths, np.int32)
    ws = torch.empty(1 << 26, dtype=torch.uint8, device="cuda")
    rc = fv.lib().fv_decode_batch_emit(C.byref(model.trans), C.byref(desc), None, 1, batch.desc.data_ptr(),
                                       lengths.ctypes.data, None, batch.n, fv._lib.FV_VANILLA, 1, 0,
                                       batch.status.data_ptr(), 0, ws.data_ptr(), ws.numel(),
                                       torch.cuda.current_stream().cuda_stream)
    assert rc == fv.FV_E_INVALID_ARG
