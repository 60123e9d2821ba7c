"""Brute-force decoding by enumeration of all K**T paths (tiny cases only).

Test infrastructure.  This is the decoding problem's plain definition
(Sec. III-A): the optimal path maximises the path's log score over every
state sequence.  Each path is scored in float32 in the recurrence's order
(s_0 = log pi + log B_0, then (s + log A) + log B_t), vectorised over all
paths with numpy; it shares nothing with ``fv_oracle.c``.
"""
from __future__ import annotations

import itertools

import numpy as np


def all_path_scores(log_pi, log_a, log_b):
    """Returns (paths int32 [K**T, T], scores float32 [K**T]); paths are in
    lexicographic order of (q_0, ..., q_{T-1})."""
    log_a = np.asarray(log_a, np.float32)
    log_b = np.asarray(log_b, np.float32)
    K = log_a.shape[0]
    T = log_b.shape[0]
    n = K ** T
    assert n <= 4_000_000, "too many paths to enumerate"
    paths = np.array(list(itertools.product(range(K), repeat=T)), dtype=np.int32).reshape(n, T)
    s = log_b[0, paths[:, 0]].astype(np.float32)
    if log_pi is not None:
        s = (np.asarray(log_pi, np.float32)[paths[:, 0]] + log_b[0, paths[:, 0]]).astype(np.float32)
    for t in range(1, T):
        c = (s + log_a[paths[:, t - 1], paths[:, t]]).astype(np.float32)
        s = (c + log_b[t, paths[:, t]]).astype(np.float32)
    return paths, s


def brute_force(log_pi, log_a, log_b):
    """Returns (best score, argmax set as int32 [m, T])."""
    paths, s = all_path_scores(log_pi, log_a, log_b)
    best = s.max()
    return np.float32(best), paths[s == best]


def reverse_lex_min(paths):
    """The path that is smallest when compared from the last position back."""
    order = np.lexsort(tuple(paths[:, t] for t in range(paths.shape[1])))
    return paths[order[0]]


def greedy_path(log_pi, log_a, log_b):
    """Greedy decoding: q_0 = lowest arg max of log pi + log B_0, then at each
    step the lowest arg max of (s + log A(q_{t-1}, j)) + log B_t(j)."""
    log_a = np.asarray(log_a, np.float32)
    log_b = np.asarray(log_b, np.float32)
    T = log_b.shape[0]
    s = log_b[0].copy() if log_pi is None else (np.asarray(log_pi, np.float32) + log_b[0]).astype(np.float32)
    q = [int(np.argmax(s))]
    v = s[q[0]]
    for t in range(1, T):
        cand = ((v + log_a[q[-1]]).astype(np.float32) + log_b[t]).astype(np.float32)
        j = int(np.argmax(cand))
        q.append(j)
        v = cand[j]
    return np.array(q, np.int32), np.float32(v)
