"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here touches the GPU.  Each test would fail on a plausible slip in
the oracle: a dropped term, a wrong tie-break, a transposed operand, an
off-by-one in the task tree, a lost anchor.
"""
import heapq
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from workloads import hmm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _bits(x):
    return np.asarray(x, np.float32).view(np.uint32)


# ---------------------------------------------------------------- vanilla vs brute force
@pytest.mark.parametrize("K,T", [(1, 5), (2, 1), (2, 6), (3, 5), (4, 4), (5, 3), (7, 3)])
@pytest.mark.parametrize("seed", range(6))
def test_vanilla_equals_brute_force(K, T, seed):
    """Max over all K**T paths of the float32 path score equals the
    recurrence's score bit for bit (x -> fl(x + c) is monotone), and the
    decoded path is one of the maximisers (unique -> equal)."""
    lp, la, lb = hmm.random_dense(K, T, seed)
    path, score, rc = oracle.vanilla(lp, la, lb)
    assert rc == oracle.OK
    best, argset = brute.brute_force(lp, la, lb)
    assert _bits(score) == _bits(best)
    assert any((path == a).all() for a in argset)
    if len(argset) == 1:
        assert (path == argset[0]).all()


@pytest.mark.parametrize("K,T", [(2, 7), (3, 6), (4, 5), (6, 4)])
@pytest.mark.parametrize("seed", range(8))
def test_vanilla_tie_rule_integer_inputs(K, T, seed):
    """Small-integer inputs: every sum is exact and ties are everywhere.
    Lowest-index arg max at every step picks the maximiser that is smallest
    when compared from the last position backwards."""
    lp, la, lb = hmm.random_dense(K, T, seed, integer=True, lo=-3, hi=0)
    path, score, rc = oracle.vanilla(lp, la, lb)
    best, argset = brute.brute_force(lp, la, lb)
    assert score == best
    assert (path == brute.reverse_lex_min(argset)).all()


def test_vanilla_without_pi():
    lp, la, lb = hmm.random_dense(3, 5, 11, with_pi=False)
    path, score, _ = oracle.vanilla(None, la, lb)
    best, argset = brute.brute_force(None, la, lb)
    assert _bits(score) == _bits(best)
    assert any((path == a).all() for a in argset)


# ---------------------------------------------------------------- closed forms
def test_single_state_chain():
    """K = 1: the only path is all zeros and its score is the plain sum."""
    lp, la, lb = hmm.random_dense(1, 9, 3)
    path, score, _ = oracle.vanilla(lp, la, lb)
    assert (path == 0).all()
    s = np.float32(lp[0] + lb[0, 0])
    for t in range(1, 9):
        s = np.float32(np.float32(s + la[0, 0]) + lb[t, 0])
    assert _bits(score) == _bits(s)


def test_single_step():
    """T = 1: the path is the lowest arg max of log pi + log B_0."""
    lp, la, lb = hmm.random_dense(17, 1, 4, integer=True)
    path, score, _ = oracle.vanilla(lp, la, lb)
    v = (lp + lb[0]).astype(np.float32)
    assert path[0] == int(np.argmax(v)) and score == v.max()


def test_constant_transitions_decouple_steps():
    """log A = const: each state is the per-step arg max of log B_t
    (t >= 1), and q_0 the arg max of log pi + log B_0 (integer inputs,
    exact arithmetic)."""
    K, T = 6, 12
    lp, _, lb = hmm.random_dense(K, T, 5, integer=True, lo=-20, hi=0)
    la = np.full((K, K), -2.0, np.float32)
    path, _, _ = oracle.vanilla(lp, la, lb)
    assert path[0] == int(np.argmax(lp + lb[0]))
    for t in range(1, T):
        assert path[t] == int(np.argmax(lb[t]))


def test_diagonal_transitions_constant_path():
    """log A = 0 on the diagonal, -inf elsewhere: the path stays in the state
    maximising log pi + sum_t log B_t."""
    K, T = 7, 9
    lp, _, lb = hmm.random_dense(K, T, 6, integer=True, lo=-9, hi=0)
    la = np.full((K, K), -np.inf, np.float32)
    np.fill_diagonal(la, 0.0)
    path, score, _ = oracle.vanilla(lp, la, lb)
    tot = lp + lb.sum(axis=0)
    assert (path == int(np.argmax(tot))).all() and score == tot.max()


def test_infeasible_sequence():
    K, T = 3, 4
    lp, la, lb = hmm.random_dense(K, T, 7)
    la[:] = -np.inf
    path, score, rc = oracle.vanilla(lp, la, lb)
    assert rc == oracle.INFEASIBLE and (path == -1).all() and score == -np.inf


@pytest.mark.parametrize("seed", range(10))
def test_rescore_identity(seed):
    """The decoded path's step-by-step re-sum equals the returned score."""
    K, T = 1 + seed * 7, 40 + seed
    lp, la, lb = hmm.random_dense(K, T, 100 + seed)
    path, score, _ = oracle.vanilla(lp, la, lb)
    assert _bits(oracle.rescore(lp, la, lb, path)) == _bits(score)


def test_rescore_by_hand():
    lp = np.array([-1.0, -2.0], np.float32)
    la = np.array([[-0.5, -1.5], [-0.25, -3.0]], np.float32)
    lb = np.array([[-1.0, -2.0], [-0.5, -0.75], [-2.0, -0.125]], np.float32)
    # path 0 -> 1 -> 0: (-1-1) + (-1.5) + (-0.75) + (-0.25) + (-2.0)
    assert oracle.rescore(lp, la, lb, np.array([0, 1, 0])) == np.float32(-6.5)


def test_signed_zero_keeps_winning_candidate():
    """Candidates -0 and +0 tie; the first index wins and its own value
    (-0) is kept, so (-0) + (-0) stays -0 at the next step."""
    lp = np.array([-0.0, 0.0], np.float32)
    la = np.array([[-0.0, -0.0], [0.0, 0.0]], np.float32)
    lb = np.array([[-0.0, -0.0], [-0.0, -0.0]], np.float32)
    path, score, _ = oracle.vanilla(lp, la, lb)
    assert path.tolist() == [0, 0]
    assert np.signbit(score)


def test_float64_instantiation_agrees_on_separated_inputs():
    lp, la, lb = hmm.random_dense(12, 30, 8)
    p32, s32, _ = oracle.vanilla(lp, la, lb)
    p64, s64, _ = oracle.vanilla_f64(lp, la, lb)
    assert (p32 == p64).all()
    assert abs(s64 - s32) < 1e-4 * abs(s64)


def test_csr_matches_dense_with_neg_inf():
    K, T = 9, 30
    lp, la, lb = hmm.random_dense(K, T, 12, neg_inf_frac=0.6)
    np.fill_diagonal(la, -0.1)
    rows, cols = np.nonzero(np.isfinite(la))
    row_ptr = np.zeros(K + 1, np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    val = la[rows, cols]
    p1, s1, r1 = oracle.vanilla(lp, la, lb)
    p2, s2, r2 = oracle.vanilla_csr(lp, row_ptr, cols, val, lb)
    assert r1 == r2 == oracle.OK
    assert (p1 == p2).all() and _bits(s1) == _bits(s2)


def test_gather_emissions():
    h = hmm.discrete_hmm(K=8, V=5, T=20, seed=3)
    lb = oracle.gather_emissions(h.log_e, h.obs)
    for t in range(20):
        for j in range(8):
            assert lb[t, j] == h.log_e[j, h.obs[t]]


# ---------------------------------------------------------------- Gaussian point emissions (Sec. III)
def test_gauss_emissions_by_hand():
    """Points whose squared distances are short binary fractions: every
    score is exact, so each entry is fixed (a swapped axis, a dropped or
    sign-flipped constant, or transposed output changes one)."""
    xy = np.array([[0.0, 0.0], [3.0, 4.0], [1.0, 1.0], [-2.0, 0.5]])
    obs = np.array([[0.0, 0.0], [3.0, 0.0]])
    got = oracle.gauss_emissions(xy, obs, -0.5, 0.25)
    # squared distances: t = 0: 0, 25, 2, 4.25; t = 1: 9, 16, 5, 25.25
    want = np.array([[-0.25, -12.75, -1.25, -2.375], [-4.75, -8.25, -2.75, -12.875]], np.float32)
    assert got.shape == (2, 4)
    assert (_bits(got) == _bits(want)).all()
    # c2 * 0 is -0 for c2 < 0, and -0 - 0 stays -0
    z = oracle.gauss_emissions(xy[:1], obs[:1], -0.5, 0.0)
    assert _bits(z)[0, 0] == 0x80000000


def test_gauss_emissions_match_normal_log_density():
    """With c2 = -1/(2 sigma^2) and c0 = ln(sigma sqrt(2 pi)) the score is
    the normal log-density of the distance (scipy's), to float32 rounding."""
    from scipy.stats import norm
    rng = np.random.default_rng(5)
    xy, obs, sigma = rng.random((300, 2)), rng.random((40, 2)), 0.05
    c2, c0 = oracle.gauss_coefficients(sigma)
    got = oracle.gauss_emissions(xy, obs, c2, c0)
    d = np.hypot(xy[None, :, 0] - obs[:, None, 0], xy[None, :, 1] - obs[:, None, 1])
    ref = norm.logpdf(d, 0.0, sigma).astype(np.float32)
    np.testing.assert_array_max_ulp(got, ref, maxulp=1)
    # at distance sigma the density is exp(-1/2) of its peak
    on = oracle.gauss_emissions(np.array([[0.0, 0.0]]), np.array([[sigma, 0.0]]), c2, c0)
    assert abs(float(on[0, 0]) - (-0.5 - np.log(sigma * np.sqrt(2 * np.pi)))) < 1e-6


def test_gauss_emissions_equal_map_matching_tables():
    """The map-matching generator's own float64 tables equal the oracle's
    evaluation bit for bit (the table decodes and the generated-emission
    decodes see the same scores)."""
    wl = hmm.map_matching_workload(K=2000, n=3, t_lo=20, t_hi=50)
    c2, c0 = oracle.gauss_coefficients(wl.sigma_gps)
    for b in range(wl.n):
        got = oracle.gauss_emissions(wl.xy, wl.gps(b), c2, c0)
        assert (_bits(got) == _bits(wl.log_b(b).numpy())).all()


# ---------------------------------------------------------------- FLASH (Alg. 1 + Alg. 2)
def _ptilde(T, P):
    return min(max(P, 2), T) if T > 1 else 1


@pytest.mark.parametrize("K,T", [(1, 7), (2, 2), (3, 3), (4, 8), (5, 16), (8, 33), (16, 100), (33, 257)])
@pytest.mark.parametrize("P", [1, 2, 3, 4, 7, 16, 1000])
def test_flash_equals_vanilla(K, T, P):
    """Pruned, parallel D&C returns vanilla's path and score bit for bit
    (retained pruning, Thm. 1-2, with the anchored float32 start); the
    decoding-call count is T - P' + 1 and every position is resolved once."""
    lp, la, lb = hmm.random_dense(K, T, 1000 * K + T)
    pv, sv, _ = oracle.vanilla(lp, la, lb)
    pf, sf, rc, st = oracle.flash(lp, la, lb, P)
    assert rc == oracle.OK
    assert (pf == pv).all() and _bits(sf) == _bits(sv)
    assert st["tasks"] == T - _ptilde(T, P) + 1
    assert st["resolved_twice"] == 0


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("P", [1, 3, 8])
def test_flash_any_dequeue_order(seed, P):
    """Same-layer tasks are independent (Sec. V-A (ii)): a random dequeue
    order gives the identical result."""
    lp, la, lb = hmm.random_dense(6, 60, 50 + seed)
    p0, s0, _, _ = oracle.flash(lp, la, lb, P)
    p1, s1, _, st = oracle.flash(lp, la, lb, P, shuffle_seed=1234567 + seed)
    assert (p0 == p1).all() and _bits(s0) == _bits(s1) and st["resolved_twice"] == 0


@pytest.mark.parametrize("seed", range(6))
def test_flash_integer_ties(seed):
    lp, la, lb = hmm.random_dense(4, 23, seed, integer=True, lo=-2, hi=0)
    pv, sv, _ = oracle.vanilla(lp, la, lb)
    for P in (1, 2, 5, 23):
        pf, sf, _, _ = oracle.flash(lp, la, lb, P)
        assert (pf == pv).all() and sf == sv


def test_flash_large_scores_need_anchor():
    """Long sequence with large accumulated scores: the anchored start
    reproduces vanilla even where rounding depends on the running score."""
    K, T = 64, 1500
    lp, la, lb = hmm.random_dense(K, T, 77)
    lb = (lb * 40.0).astype(np.float32)
    pv, sv, _ = oracle.vanilla(lp, la, lb)
    for P in (1, 16):
        pf, sf, _, _ = oracle.flash(lp, la, lb, P)
        assert (pf == pv).all() and _bits(sf) == _bits(sv)


@pytest.mark.parametrize("P", [1, 4, 16])
def test_flash_anchor_matters_at_large_magnitude(P):
    """Running scores near -1e6 (float32 spacing 0.0625) with candidate gaps
    far below that spacing: vanilla's rounding merges candidates into ties.
    The anchored subtask start reproduces those roundings; a start that
    drops the carried score (complete pruning, Def. 4) decodes at small
    magnitude and breaks the ties differently."""
    K, T = 16, 1200
    r = np.random.default_rng(5)
    la = (np.float32(-np.log(K)) + 0.01 * r.standard_normal((K, K))).astype(np.float32)
    lb = (-1000.0 + 0.02 * r.standard_normal((T, K))).astype(np.float32)
    lp = hmm.uniform_log_pi(K)
    pv, sv, _ = oracle.vanilla(lp, la, lb)
    pf, sf, _, _ = oracle.flash(lp, la, lb, P)
    assert (pf == pv).all() and _bits(sf) == _bits(sv)


def test_emission_added_after_the_max():
    """Reading of where log B enters: c_t(j) = max_i (delta + log A) first,
    then + log B_t(j).  Candidates 0.25 and 0.5 are distinct, so psi picks
    the larger (index 1); adding log B = 2^24 inside the max would round
    both to 2^24 (spacing 2 there) and tie them to index 0."""
    lp = np.array([0.0, 0.0], np.float32)
    la = np.zeros((2, 2), np.float32)
    lb = np.array([[0.25, 0.5], [2.0 ** 24, -np.inf]], np.float32)
    path, score, _ = oracle.vanilla(lp, la, lb)
    assert path.tolist() == [1, 0]
    assert score == np.float32(2.0 ** 24)
    pf, sf, _, _ = oracle.flash(lp, la, lb, 1)
    assert pf.tolist() == [1, 0]


def test_flash_infeasible():
    lp, la, lb = hmm.random_dense(3, 6, 9)
    la[:] = -np.inf
    pf, sf, rc, _ = oracle.flash(lp, la, lb, 2)
    assert rc == oracle.INFEASIBLE and (pf == -1).all()


def _simulate_cycles(T, trace, P):
    """List-schedule the root (length T) and the subtasks on P workers; a
    task is ready when the smallest earlier interval containing it ends."""
    finish = {}
    workers = [T] * P        # everyone waits for the root
    heapq.heapify(workers)
    for k, (m, n) in enumerate(trace):
        parents = [finish[(a, b)] for (a, b) in trace[:k]
                   if a <= m and n <= b and (a, b) != (m, n)]
        ready = min(parents, key=lambda x: x[1])[0] if parents else T
        pw = heapq.heappop(workers)
        start = max(ready, pw)
        end = start + (n - m + 1)
        heapq.heappush(workers, end)
        finish[(m, n)] = (end, n - m)
    return max(workers) / T


def test_task_tree_matches_paper_structure():
    g = json.load(open(os.path.join(GOLDEN, "paper_task_tree.json")))
    for case in g["cases"]:
        T, P = case["T"], case["P"]
        lp, la, lb = hmm.random_dense(3, T, 5)
        _, _, _, st = oracle.flash(lp, la, lb, P, want_trace=True)
        tr = st["trace"]
        if "first_level" in case:
            assert [list(x) for x in tr[:len(case["first_level"])]] == case["first_level"]
        if "cycles" in case:
            assert _simulate_cycles(T, tr, P) == pytest.approx(case["cycles"])
        if "cycles_serial" in case:
            assert _simulate_cycles(T, tr, 1) == pytest.approx(case["cycles_serial"])


@pytest.mark.parametrize("T", [2, 3, 4, 5, 9, 16, 31, 64, 100])
@pytest.mark.parametrize("P", [1, 2, 3, 5, 8])
def test_task_tree_rules(T, P):
    """Children per Alg. 1: two when n-m > 2, only the left when n-m = 2,
    none otherwise; every subtask is a split of an earlier one."""
    lp, la, lb = hmm.random_dense(2, T, 3)
    _, _, _, st = oracle.flash(lp, la, lb, P, want_trace=True)
    tr = st["trace"]
    seen = set()
    for (m, n) in tr:
        assert n > m
        seen.add((m, n))
    for (m, n) in tr:
        tm = (m + n) // 2
        left, right = (m, tm), (tm + 1, n)
        if n - m > 2:
            assert left in seen and right in seen
        elif n - m == 2:
            assert left in seen and right not in seen
        else:
            assert left not in seen and right not in seen
    assert len(tr) == T - _ptilde(T, P)


# ---------------------------------------------------------------- FLASH-BS
@pytest.mark.parametrize("K,T", [(4, 9), (9, 40), (20, 64)])
@pytest.mark.parametrize("P", [1, 3, 8])
def test_beam_full_width_is_vanilla(K, T, P):
    lp, la, lb = hmm.random_dense(K, T, 3 * K + T)
    pv, sv, _ = oracle.vanilla(lp, la, lb)
    for B in (K, K + 5):
        pb, sb, rc, st = oracle.beam(lp, la, lb, B, P)
        assert rc == oracle.OK
        assert (pb == pv).all() and _bits(sb) == _bits(sv)
        assert _bits(st["root_score"]) == _bits(sv)


def test_beam_width_above_finite_states_is_vanilla():
    """Only states with a finite score matter: B >= that count is exact."""
    K, T = 12, 30
    lp, la, lb = hmm.random_dense(K, T, 21)
    la[:, 5:] = -np.inf                       # states 5.. are never reachable after t=0
    pv, sv, _ = oracle.vanilla(lp, la, lb)
    for P in (1, 4):
        pb, sb, _, _ = oracle.beam(lp, la, lb, 5, P)
        assert (pb == pv).all() and _bits(sb) == _bits(sv)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("P", [1, 3, 8])
def test_beam_width_one_is_greedy(seed, P):
    K, T = 7, 25
    lp, la, lb = hmm.random_dense(K, T, 300 + seed)
    gp, gs = brute.greedy_path(lp, la, lb)
    pb, sb, _, st = oracle.beam(lp, la, lb, 1, P)
    assert (pb == gp).all() and _bits(sb) == _bits(gs)


@pytest.mark.parametrize("seed", range(5))
def test_beam_is_a_valid_suboptimal_path(seed):
    K, T = 30, 50
    lp, la, lb = hmm.random_dense(K, T, 400 + seed)
    pv, sv, _ = oracle.vanilla(lp, la, lb)
    for B in (2, 4, 8):
        pb, sb, rc, st = oracle.beam(lp, la, lb, B, 4)
        assert rc in (oracle.OK, oracle.BEAM_FALLBACK)
        assert ((0 <= pb) & (pb < K)).all() and st["resolved_twice"] == 0
        assert _bits(sb) == _bits(oracle.rescore(lp, la, lb, pb))
        assert sb <= sv


def test_beam_order_independent():
    lp, la, lb = hmm.random_dense(10, 70, 31)
    p0, s0, _, _ = oracle.beam(lp, la, lb, 3, 5)
    p1, s1, _, _ = oracle.beam(lp, la, lb, 3, 5, shuffle_seed=99)
    assert (p0 == p1).all() and _bits(s0) == _bits(s1)


def test_beam_top_b_tie_rule():
    """With all scores tied the beam keeps the lowest states (score desc,
    state asc; an equal score never evicts, Sec. V-C insertion rule)."""
    K, T = 6, 3
    lp = np.zeros(K, np.float32)
    la = np.zeros((K, K), np.float32)
    lb = np.zeros((T, K), np.float32)
    pb, _, _, _ = oracle.beam(lp, la, lb, 2, 1)
    assert (pb == 0).all()


def test_beam_keeps_lowest_states_among_boundary_ties():
    """B = 2 with scores (5, 3, 3, 3): the beam is {0, 1}.  State 1 then
    leads to the best end only if it survived the tie at the boundary."""
    K = 4
    lp = np.zeros(K, np.float32)
    lb = np.array([[5, 3, 3, 3], [0, 0, 0, 0]], np.float32)
    la = np.full((K, K), -10.0, np.float32)
    la[1, 2] = 0.0          # 3 + 0 beats 5 - 10
    la[3, 3] = 1.0          # would win if state 3 had been kept instead
    pb, sb, _, _ = oracle.beam(lp, la, lb, 2, 1)
    assert pb.tolist() == [1, 2] and sb == 3.0


_sparse_integer_instance = hmm.sparse_integer_instance


def test_beam_fallback_when_end_unreachable():
    """A subtask restarted from its anchor can end with a narrow beam from
    which the known end state is unreachable (sparse transitions).  That task
    is re-decoded exactly and the call reports the fallback; the result is
    still a valid path whose re-sum is the returned score."""
    lp, la, lb = _sparse_integer_instance(610)
    pb, sb, rc, st = oracle.beam(lp, la, lb, 2, 1)
    assert rc == oracle.BEAM_FALLBACK and st["fallbacks"] == 1
    K = la.shape[0]
    assert ((0 <= pb) & (pb < K)).all()
    for t in range(1, len(pb)):
        assert np.isfinite(la[pb[t - 1], pb[t]])
    assert _bits(sb) == _bits(oracle.rescore(lp, la, lb, pb))
    pv, sv, _ = oracle.vanilla(lp, la, lb)
    assert sb <= sv


# ---------------------------------------------------------------- backward
def _random_paths(K, n, Tmax, seed):
    r = np.random.default_rng(seed)
    lengths = r.integers(0, Tmax + 1, size=n).astype(np.int32)
    paths = r.integers(0, K, size=(n, Tmax)).astype(np.int32)
    return lengths, paths


def test_backward_counts_by_hand():
    K = 3
    paths = np.array([[0, 1, 1, 2, 0], [2, 2, 0, 0, 0]], np.int32)
    lengths = np.array([5, 3], np.int32)
    g = np.array([1.0, 1.0], np.float32)
    gb, ga, gp = oracle.backward(K, lengths, paths, g)
    want = np.zeros((K, K), np.float32)
    for (i, j) in [(0, 1), (1, 1), (1, 2), (2, 0), (2, 2), (2, 0)]:
        want[i, j] += 1
    assert (ga == want).all()
    assert gp.tolist() == [1.0, 0.0, 1.0]
    assert gb[0, 3, 2] == 1.0 and gb[1, 3].sum() == 0 and gb[1, 2, 0] == 1.0


@pytest.mark.parametrize("seed", range(4))
def test_backward_invariants(seed):
    K, n, Tmax = 5, 20, 30
    lengths, paths = _random_paths(K, n, Tmax, seed)
    g = np.random.default_rng(seed + 9).random(n).astype(np.float32)
    gb, ga, gp = oracle.backward(K, lengths, paths, g)
    for b in range(n):
        for t in range(Tmax):
            row = gb[b, t]
            if t < lengths[b]:
                assert row[paths[b, t]] == g[b] and np.count_nonzero(row) == (g[b] != 0)
            else:
                assert not row.any()
    # counts: with g = 1 every entry is an exact integer count
    ones = np.ones(n, np.float32)
    _, ga1, gp1 = oracle.backward(K, lengths, paths, ones)
    cnt = np.zeros((K, K))
    for b in range(n):
        for t in range(1, lengths[b]):
            cnt[paths[b, t - 1], paths[b, t]] += 1
    assert (ga1 == cnt).all()
    assert ga1.sum() == sum(max(int(L) - 1, 0) for L in lengths)
    assert gp1.sum() == sum(1 for L in lengths if L > 0)
    # ordered float32 sum of fl(g_b * c_b) in increasing b
    want = np.zeros((K, K), np.float32)
    for b in range(n):
        c = np.zeros((K, K), np.float32)
        for t in range(1, lengths[b]):
            c[paths[b, t - 1], paths[b, t]] += 1
        nz = c != 0
        want[nz] = (want[nz] + (np.float32(g[b]) * c[nz]).astype(np.float32)).astype(np.float32)
    assert (_bits(ga) == _bits(want)).all()


def test_backward_skips_states_outside_range():
    """An infeasible decode leaves -1 in its path; such entries, and the
    transitions that touch them, carry no gradient."""
    K = 3
    paths = np.array([[0, -1, 1, 1, 2], [2, 2, 3, 0, 0]], np.int32)   # 3 is out of range too
    lengths = np.array([5, 5], np.int32)
    g = np.array([1.0, 2.0], np.float32)
    gb, ga, gp = oracle.backward(K, lengths, paths, g)
    want = np.zeros((K, K), np.float32)
    want[1, 1] += 1; want[1, 2] += 1          # sequence 0: (0,-1), (-1,1) dropped
    want[2, 2] += 2; want[0, 0] += 2          # sequence 1: (2,3), (3,0) dropped
    assert (ga == want).all()
    assert not gb[0, 1].any() and not gb[1, 2].any()
    assert gb[0, 2, 1] == 1.0 and gb[1, 3, 0] == 2.0
    assert gp.tolist() == [1.0, 0.0, 2.0]
    bad_start = np.array([[-1, 0, 0]], np.int32)
    _, _, gp2 = oracle.backward(K, np.array([3], np.int32), bad_start, np.ones(1, np.float32))
    assert not gp2.any()


def test_backward_accumulate():
    K, n, Tmax = 4, 6, 10
    lengths, paths = _random_paths(K, n, Tmax, 3)
    g = np.full(n, 0.5, np.float32)
    gb0, ga0, gp0 = oracle.backward(K, lengths, paths, g)
    init_a = np.full((K, K), 2.0, np.float32)
    init_b = np.full((n, Tmax, K), 1.0, np.float32)
    init_pi = np.full(K, 3.0, np.float32)
    gb1, ga1, gp1 = oracle.backward(K, lengths, paths, g, init_b=init_b, init_a=init_a, init_pi=init_pi)
    assert (ga1 == ga0 + 2.0).all() and (gp1 == gp0 + 3.0).all()
    assert (gb1 == gb0 + 1.0).all()


def test_backward_matches_finite_differences():
    """Central differences (h = 1e-3) of a float64 Viterbi: the score is
    piecewise linear in the inputs, so away from path changes the
    derivative is exactly the path indicator / transition count."""
    K, T = 6, 25
    lp, la, lb = hmm.random_dense(K, T, 61)
    la = la.astype(np.float64); lb = lb.astype(np.float64); lp = lp.astype(np.float64)
    path, s0, _ = oracle.vanilla_f64(lp, la, lb)
    gb, ga, gp = oracle.backward(K, np.array([T], np.int32), path[None, :], np.ones(1, np.float32))
    h = 1e-3
    r = np.random.default_rng(0)
    checked = 0
    for _ in range(40):
        t, j = int(r.integers(T)), int(r.integers(K))
        for sgn_arr, arr, g in (("b", lb, gb[0, t, j]),):
            up = lb.copy(); up[t, j] += h
            dn = lb.copy(); dn[t, j] -= h
            pu, su, _ = oracle.vanilla_f64(lp, la, up)
            pd, sd, _ = oracle.vanilla_f64(lp, la, dn)
            if (pu == path).all() and (pd == path).all():
                assert abs((su - sd) / (2 * h) - g) < 1e-6
                checked += 1
    for _ in range(40):
        i, j = int(r.integers(K)), int(r.integers(K))
        up = la.copy(); up[i, j] += h
        dn = la.copy(); dn[i, j] -= h
        pu, su, _ = oracle.vanilla_f64(lp, up, lb)
        pd, sd, _ = oracle.vanilla_f64(lp, dn, lb)
        if (pu == path).all() and (pd == path).all():
            assert abs((su - sd) / (2 * h) - ga[i, j]) < 1e-6
            checked += 1
    for j in range(K):
        up = lp.copy(); up[j] += h
        dn = lp.copy(); dn[j] -= h
        pu, su, _ = oracle.vanilla_f64(up, la, lb)
        pd, sd, _ = oracle.vanilla_f64(dn, la, lb)
        if (pu == path).all() and (pd == path).all():
            assert abs((su - sd) / (2 * h) - gp[j]) < 1e-6
            checked += 1
    assert checked > 60


# ---------------------------------------------------------------- generators
def test_log_dirichlet_rows_normalised_and_finite():
    r = np.random.default_rng(0)
    la = hmm.log_dirichlet_rows(r, 64, 256, 0.05)
    assert np.isfinite(la).all()
    s = np.exp(la.astype(np.float64)).sum(axis=1)
    assert np.allclose(s, 1.0, atol=1e-5)


def test_discrete_hmm_is_deterministic():
    a = hmm.discrete_hmm(K=16, V=8, T=50, seed=9)
    b = hmm.discrete_hmm(K=16, V=8, T=50, seed=9)
    assert (a.obs == b.obs).all() and (a.log_a == b.log_a).all()
    assert a.obs.min() >= 0 and a.obs.max() < 8


def _dense_from_csr(K, row_ptr, col, val):
    """log A with -inf for missing edges; duplicates keep their largest value."""
    la = np.full((K, K), -np.inf, np.float32)
    for i in range(K):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            la[i, col[e]] = max(la[i, col[e]], val[e])
    return la


@pytest.mark.parametrize("seed", range(8))
def test_beam_csr_matches_dense_beam(seed):
    """FLASH-BS on CSR out-edges (push) equals the dense procedure on the
    same matrix with -inf entries, for every B and P, duplicates included."""
    K, T = 15, 37
    lp, rp, col, val, lb = hmm.random_csr(K, T, seed, deg_lo=0, deg_hi=4, integer=seed % 2 == 0,
                                          dup_frac=0.2 if seed % 3 == 0 else 0.0)
    la = _dense_from_csr(K, rp, col, val)
    for B in (1, 2, 4, 14, 15):
        for P in (1, 3, 8):
            a = oracle.beam(lp, la, lb, B, P)
            b = oracle.beam_csr(lp, rp, col, val, lb, B, P)
            assert a[2] == b[2] and (a[0] == b[0]).all() and _bits(a[1]) == _bits(b[1]), (B, P)
            assert a[3]["fallbacks"] == b[3]["fallbacks"]


def test_beam_csr_full_width_is_vanilla_csr():
    lp, rp, col, val, lb = hmm.random_csr(30, 50, 3, deg_lo=1, deg_hi=5)
    po, so, rc = oracle.vanilla_csr(lp, rp, col, val, lb)
    for P in (1, 4, 50):
        p, s, r, _ = oracle.beam_csr(lp, rp, col, val, lb, 30, P)
        assert r == rc and (p == po).all() and _bits(s) == _bits(so)


def test_vanilla_csr_duplicates_take_the_largest_edge():
    """Parallel edges i -> j act as one edge with the largest score (the
    dense form's entry), on an instance where brute force is feasible."""
    from itertools import product
    K, T = 4, 5
    lp, rp, col, val, lb = hmm.random_csr(K, T, 9, deg_lo=1, deg_hi=3, dup_frac=0.5)
    la = _dense_from_csr(K, rp, col, val).astype(np.float64)
    best, arg = -np.inf, None
    for q in product(range(K), repeat=T):   # first maximum in lexicographic order
        s = lp[q[0]] + lb[0, q[0]] + sum(la[q[t - 1], q[t]] + lb[t, q[t]] for t in range(1, T))
        if s > best:
            best, arg = s, q
    p, s, rc = oracle.vanilla_csr(lp, rp, col, val, lb)
    assert rc == oracle.OK and abs(s - best) < 1e-4
    # the same path as the dense oracle (ties broken identically)
    pd, sd, _ = oracle.vanilla(lp, la.astype(np.float32), lb)
    assert (p == pd).all() and _bits(s) == _bits(sd)


# ---- the paper's displayed subtask initialisation (relative_init) ----------
# In exact arithmetic the carried score is a constant over a subtask's start
# scores and changes no arg max (Sec. V-B); integer-valued inputs keep every
# float32 sum exact, so there the literal initialisation must return
# vanilla's path (FLASH) and the anchored beam's result (FLASH-BS).

@pytest.mark.parametrize("seed", range(6))
def test_relative_init_exact_on_integer_inputs(seed):
    K, T = 5 + seed, 40 + 7 * seed
    lp, la, lb = hmm.random_dense(K, T, 500 + seed, integer=True)
    po, so, _ = oracle.vanilla(lp, la, lb)
    for P in (1, 3, 8):
        p, s, rc, _ = oracle.flash(lp, la, lb, P, relative_init=True)
        assert rc == 0 and (p == po).all() and s == so
        for B in (2, K):
            pa, sa, rca, _ = oracle.beam(lp, la, lb, B, P)
            pr, sr, rcr, _ = oracle.beam(lp, la, lb, B, P, relative_init=True)
            assert rcr == rca and (pr == pa).all() and sr == sa


def test_relative_init_diverges_in_float32():
    """With float scores the literal start rounds differently from the
    anchored one, and the path follows vanilla's near ties differently in
    some cases; the anchored start never does."""
    diverged = 0
    for seed in range(6):
        lp, la, lb = hmm.random_dense(64, 2000, seed)
        lb = (lb * 20).astype(np.float32)
        po, so, _ = oracle.vanilla(lp, la, lb)
        pa, _, _, _ = oracle.flash(lp, la, lb, 4)
        pr, sr, rc, _ = oracle.flash(lp, la, lb, 4, relative_init=True)
        assert (pa == po).all()
        assert rc == 0 and np.isfinite(oracle.rescore(lp, la, lb, pr))
        diverged += int((pr != po).any())
    assert diverged >= 1
