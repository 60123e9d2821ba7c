"""Torch-facing wrappers of the C ABI (argument marshalling only).

torch supplies device memory (inputs, outputs, the workspace) and the current
HIP stream; every decoding step runs in libflashviterbi.so.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib as L


def _stream(dev) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _need(t: torch.Tensor, name: str, dtype=torch.float32):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


def dense_model(log_a: torch.Tensor) -> L.FvTrans:
    _need(log_a, "log_a")
    if log_a.dim() != 2 or log_a.shape[0] != log_a.shape[1] or not log_a.is_contiguous():
        raise ValueError("log_a must be a contiguous [K, K] tensor")
    return L.FvTrans(L.FV_DENSE, log_a.shape[0], log_a.data_ptr(), None, None, None, 0)


class CsrModel:
    """Sparse transition model: CSR out-edges of each source state, as device
    tensors row_ptr int32 [K+1], col int32 [nnz] (destination), val float32
    [nnz] (log A); missing edges are -inf.  The library builds the in-edge
    transpose in each decode's workspace."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor):
        _need(row_ptr, "row_ptr", torch.int32)
        _need(col, "col", torch.int32)
        _need(val, "val")
        for name, t in (("row_ptr", row_ptr), ("col", col), ("val", val)):
            if t.dim() != 1 or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous 1-D tensor")
        if col.numel() != val.numel():
            raise ValueError("col and val must have the same length")
        if row_ptr.numel() < 2:
            raise ValueError("row_ptr must have K+1 >= 2 entries")
        self.K = row_ptr.numel() - 1
        self.nnz = col.numel()
        self.device = row_ptr.device
        self.keep = (row_ptr, col, val)
        self.trans = L.FvTrans(L.FV_CSR, self.K, None, row_ptr.data_ptr(), col.data_ptr() if self.nnz else None,
                               val.data_ptr() if self.nnz else None, self.nnz)


def _model(log_a):
    """(FvTrans, K, device) of a dense [K, K] tensor or a CsrModel."""
    if isinstance(log_a, CsrModel):
        return log_a.trans, log_a.K, log_a.device
    return dense_model(log_a), log_a.shape[0], log_a.device


def workspace_bytes(method: str, K_or_model, lengths, P: int = 16, B: int = 0) -> int:
    """Workspace bytes for a decode of sequences with the given lengths.
    K_or_model: an FvTrans, or K (sizing never dereferences the model)."""
    if isinstance(K_or_model, L.FvTrans):
        model = K_or_model
    else:
        model = L.FvTrans(L.FV_DENSE, int(K_or_model), 1, None, None, None, 0)
    lengths = np.ascontiguousarray(np.asarray(lengths, dtype=np.int32).reshape(-1))
    out = C.c_size_t(0)
    L.check(L.lib().fv_workspace_size(L.METHODS[method], C.byref(model), 1,
                                      lengths.ctypes.data, None, lengths.shape[0], int(P),
                                      int(B or 0), C.byref(out)), "fv_workspace_size")
    return int(out.value)


def _workspace(n: int, dev) -> torch.Tensor:
    return torch.empty(max(n, 256), dtype=torch.uint8, device=dev)


ROWS = {"auto": 0, "wide": L.FV_FLAG_WIDE_ROWS, "local": L.FV_FLAG_LOCAL_ROWS}
STEPS = {"auto": 0, "items": L.FV_FLAG_STEP_ITEMS, "tiles": L.FV_FLAG_STEP_TILES}


def _flags(rows: str, validate: bool, leaves: bool = True, relative_init: bool = False, step: str = "auto",
           engine: bool = False) -> int:
    return (ROWS[rows] | (L.FV_FLAG_VALIDATE if validate else 0) | (0 if leaves else L.FV_FLAG_NO_LEAVES)
            | (L.FV_FLAG_RELATIVE_INIT if relative_init else 0) | STEPS[step]
            | (L.FV_FLAG_ENGINE if engine else 0))


def decode(log_a, log_b: torch.Tensor, log_pi: torch.Tensor | None = None,
           method: str = "vanilla", P: int = 16, B: int = 0, check_status: bool = True,
           rows: str = "auto", validate: bool = False, leaves: bool = True, relative_init: bool = False,
           step: str = "auto", engine: bool = False):
    """Decode one sequence.  log_a: dense [K, K] tensor or a CsrModel;
    log_b [T, >=K] (row stride = ld), log_pi [K] or None; all float32 CUDA
    tensors.  rows: "auto", "wide" or "local" row placement of dense models
    (same results).  validate: scan the inputs for NaN / +inf first (status
    FV_E_INVALID_ARG).  leaves=False: bisect every FLASH subtask (no leaf
    tables; same results).  relative_init: subtasks start from the paper's
    displayed initialisation (the carried score dropped; dense models; paths
    may differ from vanilla's at near ties).  step ("auto", "items", "tiles")
    and engine (True: the persistent engine even for K <= 256) choose kernels
    for tuning; results are the same.  Returns (path int32 [T], score
    float32 [1], status int32 [1]) on the device."""
    model, K, dev = _model(log_a)
    _need(log_b, "log_b")
    if log_b.dim() != 2 or log_b.stride(1) != 1:
        raise ValueError("log_b must be [T, ld] with unit column stride")
    if log_pi is not None:
        _need(log_pi, "log_pi")
        if not log_pi.is_contiguous() or log_pi.numel() != K:
            raise ValueError("log_pi must be a contiguous [K] tensor")
    T, ld = log_b.shape[0], log_b.stride(0)
    path = torch.empty(T, dtype=torch.int32, device=dev)
    score = torch.empty(1, dtype=torch.float32, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    n = workspace_bytes(method, model, [T], P, B)
    ws = _workspace(n, dev)
    pi = log_pi.data_ptr() if log_pi is not None else None
    lib = L.lib()
    flags = _flags(rows, validate, leaves, relative_init, step, engine)
    if method == "vanilla":
        rc = lib.fv_decode_vanilla(C.byref(model), pi, log_b.data_ptr(), ld, T, path.data_ptr(),
                                   score.data_ptr(), status.data_ptr(), flags, ws.data_ptr(),
                                   ws.numel(), _stream(dev))
    elif method == "flash":
        rc = lib.fv_decode_flash(C.byref(model), pi, log_b.data_ptr(), ld, T, int(P), path.data_ptr(),
                                 score.data_ptr(), status.data_ptr(), flags, ws.data_ptr(),
                                 ws.numel(), _stream(dev))
    elif method == "beam":
        rc = lib.fv_decode_beam(C.byref(model), pi, log_b.data_ptr(), ld, T, int(B), int(P),
                                path.data_ptr(), score.data_ptr(), status.data_ptr(), flags,
                                ws.data_ptr(), ws.numel(), _stream(dev))
    else:
        raise ValueError(method)
    L.check(rc, f"fv_decode_{method}")
    return path, score, status


class GaussEmission:
    """Emission model generated inside the decode (CSR models): state j sits
    at the point state_xy[j] (float64 [K, 2] CUDA tensor) and each
    observation is a point; log B_t(j) = c2 * |state_xy[j] - obs_t|^2 - c0 in
    float64 (each operation rounded once), then float32.  Sequences of such a
    model are given as observations (Batch.observations)."""

    def __init__(self, state_xy: torch.Tensor, c2: float, c0: float):
        _need(state_xy, "state_xy", torch.float64)
        if state_xy.dim() != 2 or state_xy.shape[1] != 2 or not state_xy.is_contiguous():
            raise ValueError("state_xy must be a contiguous [K, 2] tensor")
        self.K = state_xy.shape[0]
        self.keep = state_xy
        self.desc = L.FvEmission(L.FV_EMIT_GAUSS2D, state_xy.data_ptr(), float(c2), float(c0))

    @classmethod
    def from_sigma(cls, state_xy: torch.Tensor, sigma: float) -> "GaussEmission":
        """A Gaussian of standard deviation sigma on the distance:
        c2 = -1 / (2 sigma^2), c0 = ln(sigma sqrt(2 pi))."""
        return cls(state_xy, -1.0 / (2.0 * (sigma * sigma)), math.log(sigma * math.sqrt(2.0 * math.pi)))


class Batch:
    """Device descriptors of a batch of sequences.

    Either a list of [T_b, K_b] tensors or a padded [n, Tmax, K] tensor plus
    lengths.  models: per-sequence model index (host ints) for batches over
    several transition models (default: all 0).  Outputs are a padded int32
    [n, Tmax] path tensor (entries past each length untouched) and float32
    [n] scores.  Batch.observations builds a batch of observation sequences
    for models with a generated emission (GaussEmission).
    """

    @classmethod
    def observations(cls, obs, models=None) -> "Batch":
        """A batch of observation sequences: a list of float64 [T_b, 2]
        contiguous CUDA tensors (each row one observed point)."""
        seqs = list(obs)
        for k, x in enumerate(seqs):
            _need(x, f"obs[{k}]", torch.float64)
            if x.dim() != 2 or x.shape[1] != 2 or not x.is_contiguous():
                raise ValueError("each observation sequence must be a contiguous [T, 2] tensor")
        return cls(seqs, models=models, _observations=True)

    def __init__(self, log_b, lengths=None, models=None, _observations=False):
        self.is_observations = _observations
        if _observations:
            seqs = list(log_b)
            n = len(seqs)
            lengths = np.array([x.shape[0] for x in seqs], np.int32)
            tmax = int(lengths.max()) if n else 0
            ptrs = [x.data_ptr() for x in seqs]
            ld = [0] * n
            self.keep = seqs
            dev = seqs[0].device if n else torch.device("cuda")
        elif isinstance(log_b, torch.Tensor):
            _need(log_b, "log_b")
            if log_b.dim() != 3 or log_b.stride(2) != 1:
                raise ValueError("padded log_b must be [n, Tmax, ld] with unit column stride")
            n, tmax = log_b.shape[0], log_b.shape[1]
            lengths = np.asarray(lengths if lengths is not None else [tmax] * n, np.int32)
            if lengths.shape != (n,) or (lengths > tmax).any() or (lengths < 0).any():
                raise ValueError("bad lengths")
            ptrs = [log_b.data_ptr() + b * log_b.stride(0) * 4 for b in range(n)]
            ld = [log_b.stride(1)] * n
            self.keep = [log_b]
            dev = log_b.device
        else:
            seqs = list(log_b)
            n = len(seqs)
            for k, x in enumerate(seqs):
                _need(x, f"log_b[{k}]")
                if x.dim() != 2 or x.stride(1) != 1:
                    raise ValueError("each log_b must be [T, ld] with unit column stride")
            lengths = np.array([x.shape[0] for x in seqs], np.int32)
            tmax = int(lengths.max()) if n else 0
            ptrs = [x.data_ptr() for x in seqs]
            ld = [x.stride(0) for x in seqs]
            self.keep = seqs
            dev = seqs[0].device if n else torch.device("cuda")
        self.n, self.tmax, self.lengths, self.device = n, tmax, lengths, dev
        self.models = np.ascontiguousarray(np.zeros(n, np.int32) if models is None else np.asarray(models, np.int32))
        if self.models.shape != (n,):
            raise ValueError("models must give one model index per sequence")
        self.paths = torch.full((n, max(tmax, 1)), -1, dtype=torch.int32, device=dev)
        self.scores = torch.empty(n, dtype=torch.float32, device=dev)
        self.status = torch.empty(n, dtype=torch.int32, device=dev)
        arr = (L.FvSeq * max(n, 1))()
        for b in range(n):
            arr[b] = L.FvSeq(int(self.models[b]), int(lengths[b]), ptrs[b], int(ld[b]),
                             self.paths.data_ptr() + b * self.paths.stride(0) * 4,
                             self.scores.data_ptr() + b * 4)
        host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
        self.desc = host.to(dev)


def decode_batch(log_a, batch: Batch, log_pi=None, method: str = "flash", P: int = 16, B: int = 0,
                 ws: torch.Tensor | None = None, rows: str = "auto", validate: bool = False,
                 leaves: bool = True, relative_init: bool = False, step: str = "auto", engine: bool = False,
                 emission=None):
    """Decode all sequences of `batch` in one decode launch (the persistent
    engine, or one block per sequence for vanilla and FLASH when every dense
    model has K <= 256).  log_a: a
    dense [K, K] tensor or a CsrModel, or a list of them when the batch's
    sequences use several models (batch.models indexes it); log_pi: a [K]
    tensor or None, or a list matching log_a.  Results land in batch.paths
    / batch.scores / batch.status.  emission: a GaussEmission (or a list
    of them, one per model) whose scores are generated in the decode; the
    batch then holds observations (Batch.observations).  Returns the
    workspace tensor so callers can reuse it."""
    many = isinstance(log_a, (list, tuple))
    mods = list(log_a) if many else [log_a]
    pis = list(log_pi) if isinstance(log_pi, (list, tuple)) else [log_pi] * len(mods)
    if len(pis) != len(mods):
        raise ValueError("log_pi must match the list of models")
    if not many and (batch.models != 0).any():
        raise ValueError("batch.models refers to several models: pass a list of models")
    trans = (L.FvTrans * len(mods))()
    dev = None
    for m, x in enumerate(mods):
        t, _, d = _model(x)
        trans[m] = t
        dev = dev or d
    n = workspace_bytes_models(method, trans, len(mods), batch.lengths, batch.models, P, B)
    if ws is None or ws.numel() < n:
        ws = _workspace(n, dev)
    pa = (C.c_void_p * len(mods))(*[p.data_ptr() if p is not None else None for p in pis])
    lengths = np.ascontiguousarray(batch.lengths, np.int32)
    flags = _flags(rows, validate, leaves, relative_init, step, engine)
    if emission is None:
        if batch.is_observations:
            raise ValueError("a batch of observations needs an emission model")
        rc = L.lib().fv_decode_batch(trans, C.cast(pa, C.c_void_p), len(mods), batch.desc.data_ptr(),
                                     lengths.ctypes.data, batch.models.ctypes.data, batch.n, L.METHODS[method],
                                     int(P), int(B or 0), batch.status.data_ptr(), flags,
                                     ws.data_ptr(), ws.numel(), _stream(dev))
        L.check(rc, "fv_decode_batch")
        return ws
    ems = list(emission) if isinstance(emission, (list, tuple)) else [emission]
    if len(ems) != len(mods):
        raise ValueError("emission must match the list of models")
    if any(not isinstance(e, GaussEmission) for e in ems):
        raise TypeError("emission must be a GaussEmission or a list of them")
    if not batch.is_observations:
        raise ValueError("generated emissions need a batch of observations (Batch.observations)")
    desc = (L.FvEmission * len(mods))()
    for m, e in enumerate(ems):
        if e.K != trans[m].K:
            raise ValueError(f"model {m}: {e.K} state points for K = {trans[m].K}")
        desc[m] = e.desc
    rc = L.lib().fv_decode_batch_emit(trans, desc, C.cast(pa, C.c_void_p), len(mods), batch.desc.data_ptr(),
                                      lengths.ctypes.data, batch.models.ctypes.data, batch.n, L.METHODS[method],
                                      int(P), int(B or 0), batch.status.data_ptr(), flags,
                                      ws.data_ptr(), ws.numel(), _stream(dev))
    L.check(rc, "fv_decode_batch_emit")
    return ws


def model_descriptor(log_a) -> L.FvTrans:
    """The C descriptor of a dense [K, K] tensor or a CsrModel."""
    return _model(log_a)[0]


def workspace_bytes_models(method, trans, n_models, lengths, models, P, B) -> int:
    """Workspace bytes of a batch over n_models models (trans: an FvTrans
    array); models gives each sequence's model index."""
    lengths = np.ascontiguousarray(np.asarray(lengths, dtype=np.int32).reshape(-1))
    models = np.ascontiguousarray(np.asarray(models, dtype=np.int32).reshape(-1))
    out = C.c_size_t(0)
    L.check(L.lib().fv_workspace_size(L.METHODS[method], trans, n_models, lengths.ctypes.data,
                                      models.ctypes.data, lengths.shape[0], int(P), int(B or 0),
                                      C.byref(out)), "fv_workspace_size")
    return int(out.value)
