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


def sample_observations(h: DiscreteHMM, T: int, seed: int) -> np.ndarray:
    """Another observation sequence of length T from the model of h (uniform
    start state, then the same sampling as discrete_hmm), int32 [T]."""
    rs = _rng(seed, 3)
    pa = np.exp(h.log_a.astype(np.float64))
    pe = np.exp(h.log_e.astype(np.float64))
    obs = np.empty(T, np.int32)
    q = int(rs.integers(0, h.K))
    for t in range(T):
        obs[t] = _categorical(rs, pe[q])
        q = _categorical(rs, pa[q])
    return obs


def er_hmm(K: int = 512, T: int = 512, p: float = 0.253, M: int = 50, seed: int = 1) -> DiscreteHMM:
    """Discrete HMM on an Erdos-Renyi transition graph, the shape of the
    paper's synthetic experiments (Sec. VII): edge i -> j present with
    probability p; a row left without edges gets a self-loop; present edges
    get uniform (0, 1] weights normalised per row (float64), absent edges
    are -inf.  M observable symbols with Dirichlet(1) emission rows, uniform
    start, observations sampled from the model."""
    r = _rng(seed, 10, K, T)
    mask = r.random((K, K)) < p
    empty = ~mask.any(axis=1)
    mask[np.flatnonzero(empty), np.flatnonzero(empty)] = True
    w = np.where(mask, 1.0 - r.random((K, K)), 0.0)
    w /= w.sum(axis=1, keepdims=True)
    with np.errstate(divide="ignore"):
        log_a = np.where(mask, np.log(w), -np.inf).astype(np.float32)
    log_e = log_dirichlet_rows(_rng(seed, 11, K, M), K, M, 1.0)
    rs = _rng(seed, 12, K, T)
    pa = np.exp(log_a.astype(np.float64))
    pe = np.exp(log_e.astype(np.float64))
    states = np.empty(T, np.int32)
    obs = np.empty(T, np.int32)
    q = int(rs.integers(0, K))
    for t in range(T):
        states[t] = q
        obs[t] = _categorical(rs, pe[q])
        q = _categorical(rs, pa[q])
    return DiscreteHMM(K, M, T, uniform_log_pi(K), log_a, log_e, obs, states)


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



def random_csr(K: int, T: int, seed: int, deg_lo: int = 0, deg_hi: int = 6, integer: bool = False,
               dup_frac: float = 0.0, self_loops: bool = True, with_pi: bool = True,
               lo: int = -4, hi: int = 0):
    """Small random sparse instance (log_pi, row_ptr, col, val, log_b) for
    tests.  Source i gets a degree in [deg_lo, deg_hi] and random
    destinations in random order within its row; dup_frac of the edges repeat
    an earlier destination of the same row (with their own value); with
    self_loops every row also holds i -> i.  integer=True draws small
    integers (frequent exact ties, exact sums)."""
    r = _rng(seed, 11, K, T)
    rows = []
    for i in range(K):
        d = int(r.integers(deg_lo, deg_hi + 1))
        js = list(r.choice(K, size=min(d, K), replace=False)) if d > 0 else []
        if self_loops and i not in js:
            js.insert(int(r.integers(0, len(js) + 1)), i)
        n_dup = int(round(dup_frac * len(js)))
        for _ in range(n_dup):
            js.insert(int(r.integers(0, len(js) + 1)), js[int(r.integers(0, len(js)))])
        rows.append(js)
    row_ptr = np.zeros(K + 1, np.int32)
    row_ptr[1:] = np.cumsum([len(x) for x in rows])
    col = np.array([j for x in rows for j in x], np.int32)
    nnz = int(col.shape[0])
    if integer:
        val = r.integers(lo, hi + 1, size=nnz).astype(np.float32)
        log_b = r.integers(lo, hi + 1, size=(T, K)).astype(np.float32)
        log_pi = r.integers(lo, hi + 1, size=K).astype(np.float32)
    else:
        val = (r.standard_normal(nnz) * 1.5 - 2.0).astype(np.float32)
        log_b = (r.standard_normal((T, K)) * 2.0).astype(np.float32)
        log_pi = (r.standard_normal(K) - 3.0).astype(np.float32)
    return (log_pi if with_pi else None), row_ptr, col, val, log_b


@dataclass
class MapMatching:
    """Map-matching-shaped sparse HMM.  K states uniform in the unit square;
    state i's out-edges go to its 8 nearest neighbours and itself with
    log-probability -d/sigma_a log-normalised over the 9 (float64, then
    float32); trajectories are random walks on the graph (each step to a
    uniformly chosen neighbour other than the state itself) observed through
    GPS points = position + N(0, sigma_gps^2) per axis; the emission score of
    state j at time t is log N(dist(state j, gps_t); 0, sigma_gps^2)."""
    K: int
    xy: np.ndarray            # [K, 2] float64
    row_ptr: np.ndarray       # [K+1] int32, columns sorted within a row
    col: np.ndarray           # [9K] int32
    val: np.ndarray           # [9K] float32
    log_pi: np.ndarray        # [K] uniform
    lengths: np.ndarray       # [n] int32
    seed: int
    sigma_gps: float

    @property
    def n(self) -> int:
        return int(self.lengths.shape[0])

    def total_steps(self) -> int:
        return int(self.lengths.astype(np.int64).sum())

    def gps(self, b: int) -> np.ndarray:
        """float64 [T_b, 2] observations of trajectory b (its own stream)."""
        r = _rng(self.seed, 20, b)
        T = int(self.lengths[b])
        s = int(r.integers(0, self.K))
        pts = np.empty((T, 2), np.float64)
        for t in range(T):
            pts[t] = self.xy[s]
            nb = [j for j in self.col[self.row_ptr[s]:self.row_ptr[s + 1]] if j != s]
            s = int(nb[int(r.integers(0, len(nb)))])
        return pts + r.standard_normal((T, 2)) * self.sigma_gps

    def log_b(self, b: int, device="cpu", t0: int = 0, t1: int | None = None):
        """float32 [t1 - t0, K] torch tensor of emission scores on `device`
        (float64 arithmetic, one rounding per elementwise op, then float32)."""
        import torch
        g = self.gps(b)[t0:t1]
        xy = torch.from_numpy(self.xy).to(device)
        out = torch.empty((g.shape[0], self.K), dtype=torch.float32, device=device)
        s2 = self.sigma_gps * self.sigma_gps
        scale = -1.0 / (2.0 * s2)
        norm = math.log(self.sigma_gps * math.sqrt(2.0 * math.pi))
        for c0 in range(0, g.shape[0], 128):
            gp = torch.from_numpy(g[c0:c0 + 128]).to(device)
            dx = xy[None, :, 0] - gp[:, 0, None]
            dy = xy[None, :, 1] - gp[:, 1, None]
            d2 = dx * dx + dy * dy
            out[c0:c0 + gp.shape[0]] = (d2 * scale - norm).to(torch.float32)
        return out


def map_matching_workload(seed: int = 4, K: int = 100000, n: int = 64, t_lo: int = 200,
                          t_hi: int = 2000, sigma_a: float = 0.01,
                          sigma_gps: float = 0.005) -> MapMatching:
    """K=100000 states, 9 out-edges each, 64 trajectories of length uniform in
    [200, 2000]."""
    from scipy.spatial import cKDTree
    xy = _rng(seed, 0).random((K, 2))
    dist, idx = cKDTree(xy).query(xy, k=9)
    # per row: the 9 nearest by (distance, index), then listed by column
    order = np.lexsort((idx, dist), axis=1)
    idx = np.take_along_axis(idx, order, 1)
    dist = np.take_along_axis(dist, order, 1)
    lg = -dist / sigma_a
    mx = lg.max(axis=1, keepdims=True)
    lg = lg - (mx + np.log(np.exp(lg - mx).sum(axis=1, keepdims=True)))
    by_col = np.argsort(idx, axis=1, kind="stable")
    col = np.take_along_axis(idx, by_col, 1).astype(np.int32).reshape(-1)
    val = np.take_along_axis(lg, by_col, 1).astype(np.float32).reshape(-1)
    row_ptr = (np.arange(K + 1, dtype=np.int64) * 9).astype(np.int32)
    lengths = _rng(seed, 1).integers(t_lo, t_hi + 1, size=n).astype(np.int32)
    return MapMatching(K, xy, row_ptr, col, val, uniform_log_pi(K), lengths, seed, sigma_gps)
