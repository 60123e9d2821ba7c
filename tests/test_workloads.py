"""Host checks of the seeded workload generators (no decoding arithmetic)."""
import numpy as np
import pytest

from workloads import hmm


@pytest.mark.parametrize("p", [0.05, 0.253, 1.0])
def test_er_hmm_graph_and_rows(p):
    h = hmm.er_hmm(K=300, T=40, p=p, M=50, seed=3)
    fin = np.isfinite(h.log_a)
    # every row has an edge; the density follows p (self-loops only fill empty rows)
    assert fin.any(axis=1).all()
    assert abs(fin.mean() - p) < 0.02 + (np.exp(-300 * p) if p < 1 else 0.0)
    pa = np.exp(h.log_a.astype(np.float64))
    assert np.allclose(pa.sum(axis=1), 1.0, atol=1e-5)
    pe = np.exp(h.log_e.astype(np.float64))
    assert h.log_e.shape == (300, 50) and np.allclose(pe.sum(axis=1), 1.0, atol=1e-5)
    assert h.obs.shape == (40,) and h.obs.min() >= 0 and h.obs.max() < 50
    # the sampled hidden path only uses edges of the graph
    assert fin[h.states[:-1], h.states[1:]].all()


def test_er_hmm_is_deterministic():
    a, b = hmm.er_hmm(64, 30, 0.2, seed=7), hmm.er_hmm(64, 30, 0.2, seed=7)
    assert a.log_a.tobytes() == b.log_a.tobytes() and (a.obs == b.obs).all()
    c = hmm.er_hmm(64, 30, 0.2, seed=8)
    assert c.log_a.tobytes() != a.log_a.tobytes()


def test_er_hmm_sparse_rows_get_a_self_loop():
    h = hmm.er_hmm(K=200, T=5, p=0.001, seed=1)
    fin = np.isfinite(h.log_a)
    lone = fin.sum(axis=1) == 1
    assert lone.any()
    idx = np.flatnonzero(lone)
    # a row with a single edge is either a drawn edge or the added self-loop
    assert fin.any(axis=1).all() and (fin[idx, idx] | (fin[idx].sum(axis=1) == 1)).all()


def test_sample_observations_deterministic_and_in_range():
    h = hmm.discrete_hmm(K=16, V=20, T=50, seed=3)
    a = hmm.sample_observations(h, 300, seed=7)
    b = hmm.sample_observations(h, 300, seed=7)
    c = hmm.sample_observations(h, 300, seed=8)
    assert a.dtype == np.int32 and a.shape == (300,)
    assert (a == b).all() and not (a == c).all()
    assert a.min() >= 0 and a.max() < h.V
