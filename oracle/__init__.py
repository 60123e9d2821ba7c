"""CPU oracle for FLASH Viterbi -- test infrastructure.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product library never does; the two share
no code.  The arithmetic lives in ``fv_oracle.c`` (plain C, float32, one
rounding per add); this module only compiles it with gcc and marshals numpy
arrays.  ``brute.py`` enumerates all paths for tiny cases.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fv_oracle.c")
_LIB = os.path.join(_HERE, "libfv_oracle.so")
_lock = threading.Lock()
_lib = None

OK, INVALID, INFEASIBLE, BEAM_FALLBACK = 0, -1, -5, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wno-unused-result", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class Stats(C.Structure):
    _fields_ = [("tasks", C.c_int64), ("candidates", C.c_int64),
                ("resolved_twice", C.c_int64), ("max_queue", C.c_int64)]


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        f, i32, i64, u64, vp = C.c_float, C.c_int, C.c_int64, C.c_uint64, C.c_void_p
        lib.fvo_vanilla.argtypes = [i32, i32, vp, vp, vp, i64, vp, vp]
        lib.fvo_vanilla_f64.argtypes = [i32, i32, vp, vp, vp, i64, vp, vp]
        lib.fvo_vanilla_csr.argtypes = [i32, i32, vp, vp, vp, vp, vp, i64, vp, vp]
        lib.fvo_rescore.argtypes = [i32, i32, vp, vp, vp, i64, vp]
        lib.fvo_rescore.restype = f
        lib.fvo_gather_emissions.argtypes = [i32, i32, vp, vp, i32, vp, i64]
        lib.fvo_gauss_emissions.argtypes = [i32, vp, vp, i32, C.c_double, C.c_double, vp, i64]
        lib.fvo_gauss_emissions.restype = C.c_int
        lib.fvo_flash.argtypes = [i32, i32, i32, vp, vp, vp, i64, vp, vp, u64, C.POINTER(Stats), vp, i32]
        lib.fvo_beam.argtypes = [i32, i32, i32, i32, vp, vp, vp, i64, vp, vp, vp, u64,
                                 C.POINTER(Stats), vp, i32]
        lib.fvo_beam_csr.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, i64, vp, vp, vp, u64,
                                     C.POINTER(Stats), vp, i32]
        lib.fvo_backward.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, i32]
        for fn in (lib.fvo_vanilla, lib.fvo_vanilla_f64, lib.fvo_vanilla_csr, lib.fvo_flash,
                   lib.fvo_beam, lib.fvo_beam_csr, lib.fvo_backward, lib.fvo_gather_emissions):
            fn.restype = C.c_int
        _lib = lib
        return lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def _prep(log_pi, log_a, log_b):
    log_a = _f32(log_a)
    log_b = np.asarray(log_b, dtype=np.float32)
    if log_b.ndim != 2 or log_b.strides[1] != 4:
        log_b = np.ascontiguousarray(log_b)
    K = log_a.shape[0]
    assert log_a.shape == (K, K) and log_b.shape[1] >= K
    return _f32(log_pi), log_a, log_b, K, log_b.shape[0], log_b.strides[0] // 4


def vanilla(log_pi, log_a, log_b):
    """Vanilla Viterbi.  Returns (path int32[T], score float32, status)."""
    lib = _load()
    log_pi, log_a, log_b, K, T, ld = _prep(log_pi, log_a, log_b)
    path = np.empty(T, np.int32)
    score = np.zeros(1, np.float32)
    rc = lib.fvo_vanilla(K, T, _p(log_pi), _p(log_a), _p(log_b), ld, _p(path), _p(score))
    return path, score[0], rc


def vanilla_f64(log_pi, log_a, log_b):
    lib = _load()
    log_a = np.ascontiguousarray(log_a, dtype=np.float64)
    log_b = np.ascontiguousarray(log_b, dtype=np.float64)
    lp = None if log_pi is None else np.ascontiguousarray(log_pi, dtype=np.float64)
    K, T = log_a.shape[0], log_b.shape[0]
    path = np.empty(T, np.int32)
    score = np.zeros(1, np.float64)
    rc = lib.fvo_vanilla_f64(K, T, _p(lp), _p(log_a), _p(log_b), log_b.shape[1], _p(path), _p(score))
    return path, score[0], rc


def vanilla_csr(log_pi, row_ptr, col, val, log_b):
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    val = _f32(val)
    log_b = np.ascontiguousarray(log_b, np.float32)
    log_pi = _f32(log_pi)
    K, T = row_ptr.shape[0] - 1, log_b.shape[0]
    path = np.empty(T, np.int32)
    score = np.zeros(1, np.float32)
    rc = lib.fvo_vanilla_csr(K, T, _p(log_pi), _p(row_ptr), _p(col), _p(val), _p(log_b),
                             log_b.shape[1], _p(path), _p(score))
    return path, score[0], rc


def rescore(log_pi, log_a, log_b, path):
    lib = _load()
    log_pi, log_a, log_b, K, T, ld = _prep(log_pi, log_a, log_b)
    path = np.ascontiguousarray(path, np.int32)
    assert path.shape[0] == T
    return np.float32(lib.fvo_rescore(K, T, _p(log_pi), _p(log_a), _p(log_b), ld, _p(path)))


def gather_emissions(log_e, obs):
    lib = _load()
    log_e = _f32(log_e)
    obs = np.ascontiguousarray(obs, np.int32)
    K, V = log_e.shape
    out = np.empty((obs.shape[0], K), np.float32)
    rc = lib.fvo_gather_emissions(K, V, _p(log_e), _p(obs), obs.shape[0], _p(out), K)
    assert rc == OK
    return out


def gauss_emissions(xy, obs, c2, c0):
    """float32 [T, K] emission scores of a Gaussian observation model on
    points: xy float64 [K, 2] state points, obs float64 [T, 2] observations,
    log B_t(j) = c2 * |xy_j - obs_t|^2 - c0 in double, then float32."""
    lib = _load()
    xy = np.ascontiguousarray(xy, np.float64)
    obs = np.ascontiguousarray(obs, np.float64)
    K, T = xy.shape[0], obs.shape[0]
    assert xy.shape == (K, 2) and obs.shape == (T, 2)
    out = np.empty((T, K), np.float32)
    rc = lib.fvo_gauss_emissions(K, _p(xy), _p(obs), T, float(c2), float(c0), _p(out), K)
    assert rc == OK
    return out


def gauss_coefficients(sigma):
    """(c2, c0) of a Gaussian of standard deviation sigma on the distance:
    log N(d; 0, sigma^2) = c2 * d^2 - c0."""
    import math
    return -1.0 / (2.0 * (sigma * sigma)), math.log(sigma * math.sqrt(2.0 * math.pi))


def flash(log_pi, log_a, log_b, P, shuffle_seed=0, want_trace=False, relative_init=False):
    """FLASH Viterbi.  Returns (path, score, status, stats dict); with
    want_trace the stats hold 'trace', the (m, n) of every subtask in decode
    order.  relative_init: the paper's displayed subtask initialisation
    (Sec. V-B, the carried score dropped) instead of the anchored one."""
    lib = _load()
    log_pi, log_a, log_b, K, T, ld = _prep(log_pi, log_a, log_b)
    path = np.empty(T, np.int32)
    score = np.zeros(1, np.float32)
    st = Stats()
    tr = np.full(2 * T + 2, -1, np.int32) if want_trace else None
    rc = lib.fvo_flash(K, T, int(P), _p(log_pi), _p(log_a), _p(log_b), ld, _p(path), _p(score),
                       int(shuffle_seed), C.byref(st), _p(tr), int(bool(relative_init)))
    d = {k: getattr(st, k) for k, _ in Stats._fields_}
    if want_trace:
        d["trace"] = [(int(tr[2 * k]), int(tr[2 * k + 1])) for k in range(d["tasks"] - 1)]
    return path, score[0], rc, d


def beam(log_pi, log_a, log_b, B, P, shuffle_seed=0, relative_init=False):
    """FLASH-BS.  Returns (path, score, status, stats dict); stats also holds
    'root_score' and 'fallbacks'.  relative_init as in flash()."""
    lib = _load()
    log_pi, log_a, log_b, K, T, ld = _prep(log_pi, log_a, log_b)
    path = np.empty(T, np.int32)
    score = np.zeros(1, np.float32)
    root = np.zeros(1, np.float32)
    nfb = np.zeros(1, np.int32)
    st = Stats()
    rc = lib.fvo_beam(K, T, int(B), int(P), _p(log_pi), _p(log_a), _p(log_b), ld, _p(path),
                      _p(score), _p(root), int(shuffle_seed), C.byref(st), _p(nfb), int(bool(relative_init)))
    d = {k: getattr(st, k) for k, _ in Stats._fields_}
    d["root_score"] = root[0]
    d["fallbacks"] = int(nfb[0])
    return path, score[0], rc, d


def beam_csr(log_pi, row_ptr, col, val, log_b, B, P, shuffle_seed=0, relative_init=False):
    """FLASH-BS on a CSR model (out-edges; missing edges are -inf).  Returns
    (path, score, status, stats dict) like beam()."""
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    val = _f32(val)
    log_b = np.ascontiguousarray(log_b, np.float32)
    log_pi = _f32(log_pi)
    K, T = row_ptr.shape[0] - 1, log_b.shape[0]
    path = np.empty(T, np.int32)
    score = np.zeros(1, np.float32)
    root = np.zeros(1, np.float32)
    nfb = np.zeros(1, np.int32)
    st = Stats()
    rc = lib.fvo_beam_csr(K, T, int(B), int(P), _p(log_pi), _p(row_ptr), _p(col), _p(val), _p(log_b),
                          log_b.shape[1], _p(path), _p(score), _p(root), int(shuffle_seed), C.byref(st),
                          _p(nfb), int(bool(relative_init)))
    d = {k: getattr(st, k) for k, _ in Stats._fields_}
    d["root_score"] = root[0]
    d["fallbacks"] = int(nfb[0])
    return path, score[0], rc, d


def backward(K, lengths, paths, grad_score, want_b=True, want_a=True, want_pi=True,
             init_b=None, init_a=None, init_pi=None):
    """Gradients of the Viterbi scores (see fv_oracle.c).  paths: int32 [n, Tmax]."""
    lib = _load()
    lengths = np.ascontiguousarray(lengths, np.int32)
    paths = np.ascontiguousarray(paths, np.int32)
    g = _f32(grad_score)
    n, Tmax = paths.shape
    acc = int(init_b is not None or init_a is not None or init_pi is not None)
    gb = (np.array(init_b, np.float32, copy=True) if init_b is not None
          else np.zeros((n, Tmax, K), np.float32)) if want_b else None
    ga = (np.array(init_a, np.float32, copy=True) if init_a is not None
          else np.zeros((K, K), np.float32)) if want_a else None
    gp = (np.array(init_pi, np.float32, copy=True) if init_pi is not None
          else np.zeros(K, np.float32)) if want_pi else None
    rc = lib.fvo_backward(K, n, Tmax, _p(lengths), _p(paths), _p(g), _p(gb), _p(ga), _p(gp), acc)
    assert rc == OK, rc
    return gb, ga, gp
