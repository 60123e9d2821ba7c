"""Viterbi score as a differentiable function (structured hinge / CRF use).

The forward pass decodes every sequence of a padded batch (vanilla or FLASH,
bit-identical results) and returns the decoded paths' scores; the backward
pass is fv_viterbi_backward: with the decoded path held fixed the score is
linear in the emission, transition and start scores, so its gradient is
the path's indicators and transition counts (a subgradient at ties).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .decode import Batch, _need, _stream, _workspace, decode_batch


def backward_workspace_bytes(K: int, n: int, Tmax: int) -> int:
    out = C.c_size_t(0)
    L.check(L.lib().fv_backward_workspace_size(int(K), int(n), int(Tmax), C.byref(out)),
            "fv_backward_workspace_size")
    return int(out.value)


def viterbi_backward(K: int, lengths: torch.Tensor, paths: torch.Tensor, grad_score: torch.Tensor,
                     grad_log_b: torch.Tensor | None = None, grad_log_a: torch.Tensor | None = None,
                     grad_log_pi: torch.Tensor | None = None, accumulate: bool = False,
                     ws: torch.Tensor | None = None) -> None:
    """Write (or add, accumulate=True) the gradients of the scores of `paths`
    into the given output tensors (any may be None).  lengths int32 [n],
    paths int32 [n, Tmax], grad_score float32 [n]; grad_log_b [n, Tmax, K],
    grad_log_a [K, K], grad_log_pi [K]; all contiguous CUDA tensors."""
    _need(lengths, "lengths", torch.int32)
    _need(paths, "paths", torch.int32)
    _need(grad_score, "grad_score")
    if paths.dim() != 2 or not paths.is_contiguous():
        raise ValueError("paths must be a contiguous [n, Tmax] int32 tensor")
    n, tmax = paths.shape
    if lengths.shape != (n,) or grad_score.shape != (n,):
        raise ValueError("lengths and grad_score must be [n]")
    shapes = {"grad_log_b": (n, tmax, K), "grad_log_a": (K, K), "grad_log_pi": (K,)}
    outs = {"grad_log_b": grad_log_b, "grad_log_a": grad_log_a, "grad_log_pi": grad_log_pi}
    for name, t in outs.items():
        if t is not None:
            _need(t, name)
            if tuple(t.shape) != shapes[name] or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {shapes[name]} float32 tensor")
    need = backward_workspace_bytes(K, n, tmax)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, paths.device)
    ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
    rc = L.lib().fv_viterbi_backward(int(K), int(n), int(tmax), lengths.data_ptr(), paths.data_ptr(),
                                     grad_score.data_ptr(), ptr(grad_log_b), ptr(grad_log_a),
                                     ptr(grad_log_pi), int(bool(accumulate)), ws.data_ptr(), ws.numel(),
                                     _stream(paths.device))
    L.check(rc, "fv_viterbi_backward")


class ViterbiScore(torch.autograd.Function):
    """scores, paths = ViterbiScore.apply(emissions, lengths, transitions, start, method, P)

    emissions [n, Tmax, K] float32 (entries past each length are ignored),
    lengths int [n] (host list/array or tensor), transitions [K, K] (row =
    source state), start [K] or None.  Returns the Viterbi scores [n]
    (float32) and the decoded paths [n, Tmax] (int32, -1 past each length;
    not differentiable)."""

    @staticmethod
    def forward(ctx, emissions, lengths, transitions, start=None, method="flash", P=16):
        _need(emissions, "emissions")
        _need(transitions, "transitions")
        if emissions.dim() != 3 or not emissions.is_contiguous():
            raise ValueError("emissions must be a contiguous [n, Tmax, K] tensor")
        n, tmax, K = emissions.shape
        if transitions.shape != (K, K) or not transitions.is_contiguous():
            raise ValueError("transitions must be a contiguous [K, K] tensor")
        if start is not None and (start.shape != (K,) or not start.is_contiguous()):
            raise ValueError("start must be a contiguous [K] tensor")
        lens = (lengths.detach().cpu().numpy() if isinstance(lengths, torch.Tensor)
                else np.asarray(lengths)).astype(np.int32)
        batch = Batch(emissions.detach(), lens)
        decode_batch(transitions.detach(), batch, None if start is None else start.detach(),
                     method=method, P=P)
        paths = batch.paths[:, :tmax] if tmax > 0 else batch.paths[:, :0]
        ctx.K, ctx.has_start = K, start is not None
        ctx.save_for_backward(paths, torch.from_numpy(lens).to(emissions.device))
        ctx.mark_non_differentiable(paths)
        return batch.scores, paths

    @staticmethod
    def backward(ctx, grad_scores, _grad_paths):
        paths, lens = ctx.saved_tensors
        n, tmax = paths.shape
        K = ctx.K
        dev = paths.device
        g = grad_scores.detach().to(torch.float32).contiguous()
        want_e, _, want_a, want_s = ctx.needs_input_grad[:4]
        ge = torch.empty((n, tmax, K), dtype=torch.float32, device=dev) if want_e else None
        ga = torch.empty((K, K), dtype=torch.float32, device=dev) if want_a else None
        gs = torch.empty(K, dtype=torch.float32, device=dev) if (want_s and ctx.has_start) else None
        if ge is not None or ga is not None or gs is not None:
            viterbi_backward(K, lens, paths.contiguous(), g, ge, ga, gs)
        return ge, None, ga, gs, None, None
