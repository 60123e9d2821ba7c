"""Seeded synthetic HMM workloads.

This module only draws random inputs; it contains none of the decoding
arithmetic.  Both the CPU oracle and the GPU library consume what it makes,
so the two sides always see identical bytes.

Every array comes from ``numpy.random.default_rng`` seeded with a
``SeedSequence``; each named array gets its own spawned child stream, so
asking for one sequence of a batch never depends on having drawn the others.

Log-Dirichlet rows are sampled in log space (Gamma(a) = Gamma(a+1) * U^(1/a),
so log Gamma(a) = log Gamma(a+1) + log(U)/a, with numpy's Marsaglia-Tsang
gamma sampler for Gamma(a+1)), then normalised with a float64 log-sum-exp and
cast once to float32.  This keeps small concentrations (a <= 0.1) free of
-inf entries that a linear-space sampler would produce by underflow.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(list(key)))


def log_dirichlet_rows(rng: np.random.Generator, n_rows: int, n_cols: int,
                       alpha: float, chunk_rows: int = 1024) -> np.ndarray:
    """float32 [n_rows, n_cols]; every row is log of a Dirichlet(alpha) draw."""
    out = np.empty((n_rows, n_cols), dtype=np.float32)
    for r0 in range(0, n_rows, chunk_rows):
        r1 = min(n_rows, r0 + chunk_rows)
        g = rng.standard_gamma(alpha + 1.0, size=(r1 - r0, n_cols))
        u = rng.random(size=(r1 - r0, n_cols))
        u = np.maximum(u, np.finfo(np.float64).tiny)
        lg = np.log(g) + np.log(u) / alpha
        mx = lg.max(axis=1, keepdims=True)
        lse = mx + np.log(np.exp(lg - mx).sum(axis=1, keepdims=True))
        out[r0:r1] = (lg - lse).astype(np.float32)
    return out


def uniform_log_pi(K: int) -> np.ndarray:
    return np.full(K, np.float32(-math.log(K)), dtype=np.float32)


def _categorical(rng: np.random.Generator, p: np.ndarray) -> int:
    c = np.cumsum(p)
    return int(min(np.searchsorted(c, rng.random() * c[-1], side="right"), len(p) - 1))


@dataclass
class DiscreteHMM:
    """Discrete-emission HMM plus one sampled observation sequence."""
    K: int
    V: int
    T: int
    log_pi: np.ndarray      # [K]
    log_a: np.ndarray       # [K, K], row = source state
    log_e: np.ndarray       # [K, V], row = state
    obs: np.ndarray         # [T] int32 symbols
    states: np.ndarray      # [T] int32 hidden states that generated obs

    def log_b(self) -> np.ndarray:
        """[T, K] emission scores log e[j, x_t] (plain indexing, test side)."""
        return np.ascontiguousarray(self.log_e[:, self.obs].T)


def discrete_hmm(K: int = 64, V: int = 128, T: int = 1000, alpha_a: float = 1.0,
                 alpha_e: float = 0.5, seed: int = 1) -> DiscreteHMM:
    """Single discrete HMM: Dirichlet transition/emission rows, uniform start,
    observations sampled from the model with float64 probabilities."""
    log_a = log_dirichlet_rows(_rng(seed, 0), K, K, alpha_a)
    log_e = log_dirichlet_rows(_rng(seed, 1), K, V, alpha_e)
    rs = _rng(seed, 2)
    pa = np.exp(log_a.astype(np.float64))
    pe = np.exp(log_e.astype(np.float64))
    states = np.empty(T, np.int32)
    obs = np.empty(T, np.int32)
    q = int(rs.integers(0, K))
    for t in range(T):
        states[t] = q
        obs[t] = _categorical(rs, pe[q])
        q = _categorical(rs, pa[q])
    return DiscreteHMM(K, V, T, uniform_log_pi(K), log_a, log_e, obs, states)


@dataclass
class DenseBatch:
    """Many sequences sharing one dense transition matrix; emission scores are
    given directly per sequence as float32 [T_b, K] matrices."""
    K: int
    log_pi: np.ndarray | None
    log_a: np.ndarray
    lengths: np.ndarray                      # [n] int32
    seed: int
    sigma: float
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def n(self) -> int:
        return int(self.lengths.shape[0])

    def log_b(self, b: int) -> np.ndarray:
        """float32 [T_b, K] ~ N(0, sigma^2), drawn from sequence b's own stream."""
        if b in self._cache:
            return self._cache[b]
        T = int(self.lengths[b])
        x = _rng(self.seed, 100, b).standard_normal((T, self.K), dtype=np.float32)
        x *= np.float32(self.sigma)
        return x

    def total_steps(self) -> int:
        return int(self.lengths.astype(np.int64).sum())


def dense_batch(K: int, n: int, t_lo: int, t_hi: int, alpha: float, sigma: float,
                seed: int, with_pi: bool = True) -> DenseBatch:
    log_a = log_dirichlet_rows(_rng(seed, 0), K, K, alpha)
    lengths = _rng(seed, 1).integers(t_lo, t_hi + 1, size=n).astype(np.int32)
    return DenseBatch(K, uniform_log_pi(K) if with_pi else None, log_a, lengths, seed, sigma)


def batched_flash_workload(seed: int = 2, n: int = 256, K: int = 1024,
                           t_lo: int = 500, t_hi: int = 8000) -> DenseBatch:
    """256 sequences, dense K=1024 log-transition rows ~ Dirichlet(0.1),
    lengths uniform in [500, 8000], emission scores N(0, 2^2)."""
    return dense_batch(K, n, t_lo, t_hi, alpha=0.1, sigma=2.0, seed=seed)


def large_dense_workload(seed: int = 3, K: int = 16384, T: int = 10000) -> DenseBatch:
    """One sequence on a K=16384 dense HMM, rows ~ Dirichlet(0.05), T=10000,
    emission scores N(0, 3^2)."""
    return dense_batch(K, 1, T, T, alpha=0.05, sigma=3.0, seed=seed)


def random_dense(K: int, T: int, seed: int, integer: bool = False, lo: int = -6,
                 hi: int = 0, with_pi: bool = True, neg_inf_frac: float = 0.0):
    """Small random instance (log_pi, log_a, log_b) for tests.

    integer=True draws small integers so that exact ties are common and every
    sum is exact in float32.  neg_inf_frac sets that fraction of log_a to -inf.
    """
    r = _rng(seed, 7, K, T)
    if integer:
        log_a = r.integers(lo, hi + 1, size=(K, K)).astype(np.float32)
        log_b = r.integers(lo, hi + 1, size=(T, K)).astype(np.float32)
        log_pi = r.integers(lo, hi + 1, size=K).astype(np.float32)
    else:
        log_a = log_dirichlet_rows(r, K, K, 0.5)
        log_b = (r.standard_normal((T, K)) * 2.0).astype(np.float32)
        log_pi = log_dirichlet_rows(r, 1, K, 1.0)[0]
    if neg_inf_frac > 0:
        m = r.random((K, K)) < neg_inf_frac
        log_a[m] = -np.inf
    return (log_pi if with_pi else None), log_a, log_b


@dataclass
class CRFBatch:
    """Linear-chain CRF batch: emissions from a random Linear(512 -> K) layer
    over N(0, 1) features, a learned-style K x K transition matrix N(0, 0.1^2),
    no start scores."""
    K: int
    lengths: np.ndarray       # [n]
    emissions: np.ndarray     # [n, Tmax, K] float32, zero past each length
    transitions: np.ndarray   # [K, K] float32


def crf_batch(n: int = 512, K: int = 256, t_lo: int = 32, t_hi: int = 512,
              d_in: int = 512, seed: int = 5) -> CRFBatch:
    import torch
    lengths = _rng(seed, 1).integers(t_lo, t_hi + 1, size=n).astype(np.int32)
    tmax = int(lengths.max())
    g = torch.Generator().manual_seed(seed)
    lin = torch.nn.Linear(d_in, K)
    with torch.no_grad():
        # default nn.Linear init, but from our own generator
        bound = 1.0 / math.sqrt(d_in)
        lin.weight.uniform_(-bound, bound, generator=g)
        lin.bias.uniform_(-bound, bound, generator=g)
        em = np.zeros((n, tmax, K), dtype=np.float32)
        for b in range(n):
            T = int(lengths[b])
            x = torch.randn(T, d_in, generator=g)
            em[b, :T] = lin(x).numpy()
        trans = (torch.randn(K, K, generator=g) * 0.1).numpy().astype(np.float32)
    return CRFBatch(K, lengths, em, trans)


def sparse_integer_instance(seed: int):
    """Tiny HMM with sparse integer transitions (about 45% of the entries
    finite, self-loops always present), integer start and emission scores:
    ties are common and narrow beams can lose a task's known end state."""
    r = np.random.default_rng(seed)
    K = int(r.integers(3, 7)); T = int(r.integers(4, 12))
    la = np.where(r.random((K, K)) < 0.45, r.integers(-4, 1, (K, K)).astype(np.float32),
                  -np.inf).astype(np.float32)
    np.fill_diagonal(la, -1.0)
    lp = r.integers(-3, 1, K).astype(np.float32)
    lb = r.integers(-4, 1, (T, K)).astype(np.float32)
    return lp, la, lb

