#!/usr/bin/env python3
"""Benchmark: batched FLASH Viterbi decoding on one MI355X.

Workload (synthetic, seeded): 256 sequences sharing a dense K=1024 float32
log-transition matrix (rows ~ Dirichlet(0.1), logged), lengths uniform in
[500, 8000], emission scores N(0, 2^2).  One "step" is one batched decode of
the whole workload (one persistent launch).  The metric is state-steps/s =
sum_b T_b * K / wall time, inputs resident in HBM before timing starts.

Prints ONE JSON line.  Besides the headline method it reports vanilla and
the other P values, the workspace memory of each, the engine kernel's
roofline fraction and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
CU, LANES, CLOCK_GHZ = 256, 64, 2.4
# max-plus: one candidate = one add + one max (2 flops).  If every lane
# evaluated one candidate per clock the chip would reach
# 256 CU x 64 lanes x 2.4 GHz = 39.3e12 candidates/s = 78.6 TFLOP/s.
PEAK_MAXPLUS_TFLOPS = CU * LANES * CLOCK_GHZ * 1e9 * 2 / 1e12
PEAK_FP32_VECTOR_TFLOPS = 157.3


# ------------------------------------------------------------------ work model
LEAF_LEN = 128  # subtasks of at most this many steps are leaves (the library's default schedule)


def _sub_candidates(m: int, n: int, K: int, memo: dict, leaf_len: int) -> int:
    """Candidates the GPU evaluates for subtask (m, n) and its descendants:
    anchored start (K, none at m = 0), full steps m+1..n-1 (K^2 each), the
    end-only last step (K).  A leaf (at most leaf_len steps) has no children."""
    key = (n - m, m == 0)
    if key in memo:
        return memo[key]
    c = (K if m > 0 else 0) + (n - m - 1) * K * K + K
    tmid = (m + n) // 2
    if n - m + 1 <= leaf_len:
        pass
    elif n - m > 2:
        c += _sub_candidates(m, tmid, K, memo, leaf_len) + _sub_candidates(tmid + 1, n, K, memo, leaf_len)
    elif n - m == 2:
        c += _sub_candidates(m, tmid, K, memo, leaf_len)
    memo[key] = c
    return c


def flash_candidates(T: int, P: int, K: int, leaf_len: int = 0) -> int:
    """Candidates of one FLASH decode: root pass + every subtask."""
    if T <= 1:
        return 0
    pp = min(max(P, 2), T)
    total = (T - 1) * K * K
    memo: dict = {}
    for d in range(pp):
        m = 0 if d == 0 else ((d * T - 1) // pp) + 1
        n = ((d + 1) * T - 1) // pp
        if n - m >= 1:
            total += _sub_candidates(m, n, K, memo, leaf_len)
    return total


def vanilla_candidates(T: int, K: int) -> int:
    return max(T - 1, 0) * K * K


# ------------------------------------------------------------------ counters
PROFILE = os.path.join(ROOT, "profiles", "fv_engine_kernel__batched_k1024_n256_flash_p64.md")


def engine_source_hash() -> str:
    """sha256 over the library's kernel sources (names and contents)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2510_19301_amd", "csrc", "*"))):
        if f.endswith((".hip", ".h")):
            h.update(os.path.basename(f).encode())
            h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per engine launch from the committed counter summary, or
    None when the kernel sources changed since the counters were taken."""
    if not os.path.exists(PROFILE):
        return None
    fields = {}
    for line in open(PROFILE):
        if ":" in line and line.startswith("- "):
            k, _, v = line[2:].partition(":")
            fields[k.strip()] = v.strip()
    if fields.get("engine_source_sha256") != engine_source_hash():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ------------------------------------------------------------------ helpers
def _make_inputs(wl, torch, dev):
    with ThreadPoolExecutor(max_workers=8) as ex:
        host = list(ex.map(wl.log_b, range(wl.n)))
    return [torch.from_numpy(x).to(dev) for x in host]


def _time_method(fv, torch, la, lp, batch, method, P, B, steps, warmup, ws=None, leaves=True, emission=None):
    """Mean ms per decode over `steps` timed decodes (torch events on the
    current stream, which is the stream the library launches on) and the
    engine kernel's own duration in the last timed decode (HIP events the
    library records around that launch)."""
    import ctypes as C
    lib = fv.lib()
    for _ in range(warmup):
        ws = fv.decode_batch(la, batch, lp, method=method, P=P, B=B, ws=ws, leaves=leaves, emission=emission)
    torch.cuda.synchronize()
    fv._lib.check(lib.fv_profile_engine(1), "fv_profile_engine")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        ws = fv.decode_batch(la, batch, lp, method=method, P=P, B=B, ws=ws, leaves=leaves, emission=emission)
    stop.record()
    torch.cuda.synchronize()
    ms = C.c_float(0)
    fv._lib.check(lib.fv_profile_engine_ms(C.byref(ms)), "fv_profile_engine_ms")
    lib.fv_profile_engine(0)
    st = batch.status.cpu().numpy()
    return start.elapsed_time(stop) / steps, float(ms.value), ws, int((st != 0).sum())


def relative_divergence(fv, torch, la, lp, batch, lengths, P):
    """FV_FLAG_RELATIVE_INIT (the paper's displayed subtask start, carried
    score dropped) against vanilla on the same batch: sequences and positions
    whose decoded state differs, and the decode time."""
    fv.decode_batch(la, batch, lp, method="vanilla")
    torch.cuda.synchronize()
    ref = batch.paths.cpu().numpy().copy()
    fv.decode_batch(la, batch, lp, method="flash", P=P, relative_init=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fv.decode_batch(la, batch, lp, method="flash", P=P, relative_init=True)
    e1.record()
    torch.cuda.synchronize()
    got = batch.paths.cpu().numpy()
    seqs = pos = 0
    for b, T in enumerate(lengths):
        d = int((got[b, :T] != ref[b, :T]).sum())
        seqs += d > 0
        pos += d
    return {"method": f"flash_P{P} with FV_FLAG_RELATIVE_INIT", "ms": round(e0.elapsed_time(e1), 1),
            "sequences_differing_from_vanilla": int(seqs), "n_seqs": len(lengths),
            "positions_differing": int(pos), "positions": int(np.sum(lengths))}


def large_runs(fv, torch, hmm, dev):
    """One sequence on a large dense HMM: K = 16384 (log A rows
    Dirichlet(0.05), 1 GiB), T = 10000, log B ~ N(0, 3^2).  Vanilla and FLASH
    stream all of log A from HBM every step (wide rows); FLASH-BS reads only
    the B beam rows of log A per step."""
    wl = hmm.large_dense_workload()
    K, T = wl.K, int(wl.lengths[0])
    print(f"[bench] large: K={K} T={T}", file=sys.stderr, flush=True)
    la = torch.from_numpy(wl.log_a).to(dev)
    lb = torch.from_numpy(wl.log_b(0)).to(dev)
    lp = torch.from_numpy(wl.log_pi).to(dev)
    del wl
    res = {"workload": f"one sequence, dense K={K} (log A rows Dirichlet(0.05)), T={T}, log B ~ N(0,3^2)"}
    # FLASH at several P: a larger P stores more division copies in the root
    # pass and leaves fewer levels of subtasks (time against memory)
    for method, P, B in (("vanilla", 1, 0), ("flash", 16, 0), ("flash", 64, 0), ("flash", 256, 0),
                         ("beam", 16, 16), ("beam", 16, 64), ("beam", 16, 256)):
        fv.decode(la, lb, lp, method, P=P, B=B)   # warm-up (also sizes the workspace)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        path, score, status = fv.decode(la, lb, lp, method, P=P, B=B)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        key = {"flash": f"flash_P{P}", "vanilla": "vanilla", "beam": f"beam_P{P}_B{B}"}[method]
        entry = {"ms": round(ms, 1), "state_steps_per_s": T * K / (ms / 1e3), "status": int(status.item()),
                 "workspace_bytes": fv.workspace_bytes(method, K, [T], P, B)}
        if method == "vanilla":   # HBM bound: log A (K*K*4 bytes) every step
            gbs = (T - 1) * K * K * 4 / (ms / 1e3) / 1e9
            entry["hbm_roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                                     "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 3)}
        if method == "vanilla":
            ref = path.cpu().numpy().copy()
            ref_score = score.cpu().numpy().copy()
        elif method == "flash":   # exact: the same path and score bits as vanilla
            entry["same_as_vanilla"] = bool((path.cpu().numpy() == ref).all() and
                                            (score.cpu().numpy().reshape(-1).view("u4") ==
                                             ref_score.reshape(-1).view("u4")).all())
        res[key] = entry
        print(f"[bench] large {key}: {ms:.1f} ms", file=sys.stderr, flush=True)
    path, _, status = fv.decode(la, lb, lp, "flash", P=16, relative_init=True)
    d = int((path.cpu().numpy() != ref).sum())
    res["flash_P16_relative_init"] = {"status": int(status.item()), "positions_differing_from_vanilla": d,
                                      "positions": T}
    print(f"[bench] large flash_P16 relative init: {d} of {T} positions differ from vanilla",
          file=sys.stderr, flush=True)
    return res


def sparse_runs(fv, torch, hmm, dev):
    """The map-matching workload: K = 100000 states on a 9-nearest-neighbour
    CSR graph, 64 trajectories of length U[200, 2000], Gaussian GPS
    emissions: first as log B tables (produced on the device by torch before
    the timed decodes), then generated inside the decode from the GPS points.
    Vanilla and FLASH pull over in-edges; FLASH-BS pushes the beam's
    out-edges."""
    wl = hmm.map_matching_workload()
    print(f"[bench] sparse: K={wl.K} n={wl.n} sum T={wl.total_steps()}", file=sys.stderr, flush=True)
    lbs = [wl.log_b(b, dev) for b in range(wl.n)]
    model = fv.CsrModel(torch.from_numpy(wl.row_ptr).to(dev), torch.from_numpy(wl.col).to(dev),
                        torch.from_numpy(wl.val).to(dev))
    lp = torch.from_numpy(wl.log_pi).to(dev)
    batch = fv.Batch(lbs)
    torch.cuda.synchronize()
    res = {"workload": f"map matching: K={wl.K} states, 9-NN CSR graph ({len(wl.col)} edges), {wl.n} "
                       f"trajectories T~U[200,2000] (sum T={wl.total_steps()}), Gaussian GPS emissions"}
    steps = wl.total_steps() * wl.K
    for method, P, B in (("beam", 16, 128), ("flash", 16, 0), ("vanilla", 1, 0)):
        ms, eng_ms, ws, bad = _time_method(fv, torch, model, lp, batch, method, P, B, 1, 1)
        key = {"flash": f"flash_P{P}", "vanilla": "vanilla", "beam": f"beam_P{P}_B{B}"}[method]
        res[key] = {"ms": round(ms, 1), "engine_ms": round(eng_ms, 1), "state_steps_per_s": steps / (ms / 1e3),
                    "workspace_bytes": int(ws.numel()), "bad_status": bad}
        print(f"[bench] sparse {key}: {ms:.1f} ms", file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()
    del lbs, batch
    torch.cuda.empty_cache()
    # the same decodes with the emission generated inside the decode from
    # the GPS points (no log B tables: 28.6 GB less to produce and stream)
    em = fv.GaussEmission.from_sigma(torch.from_numpy(wl.xy).to(dev), wl.sigma_gps)
    obs = fv.Batch.observations([torch.from_numpy(wl.gps(b)).to(dev) for b in range(wl.n)])
    for method, P, B in (("beam", 16, 128), ("flash", 16, 0), ("vanilla", 1, 0)):
        ms, eng_ms, ws, bad = _time_method(fv, torch, model, lp, obs, method, P, B, 1, 1, emission=em)
        key = {"flash": f"flash_P{P}", "vanilla": "vanilla", "beam": f"beam_P{P}_B{B}"}[method] + "_generated_emission"
        res[key] = {"ms": round(ms, 1), "engine_ms": round(eng_ms, 1), "state_steps_per_s": steps / (ms / 1e3),
                    "workspace_bytes": int(ws.numel()), "bad_status": bad}
        print(f"[bench] sparse {key}: {ms:.1f} ms", file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()
    return res


def er_runs(fv, torch, hmm, dev):
    """The paper's synthetic sweeps (Sec. VII) on single sequences: Erdos-Renyi
    transition graphs, |O| = 50, defaults p = 0.253, K = 512, T = 512; p from
    0.05 up by x1.5 (and 1), K and T from 32 to 2048, and a beam-width sweep
    B = 1024..32 at K = 2048 (an ER model standing in for the paper's
    forced-alignment data).  Decode time in ms (emission scores already on the
    device) and workspace bytes; FLASH with P = 16."""
    lib = fv.lib()

    def one(h, runs):
        la = torch.from_numpy(h.log_a).to(dev)
        lp = torch.from_numpy(h.log_pi).to(dev)
        log_e = torch.from_numpy(h.log_e).to(dev)
        obs = torch.from_numpy(h.obs).to(dev)
        lb = torch.empty((h.T, h.K), dtype=torch.float32, device=dev)
        fv._lib.check(lib.fv_gather_emissions(h.K, h.V, log_e.data_ptr(), obs.data_ptr(), h.T, lb.data_ptr(),
                                              h.K, torch.cuda.current_stream().cuda_stream), "fv_gather_emissions")
        out = {}
        for method, P, B in runs:
            fv.decode(la, lb, lp, method, P=P, B=B)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            _, _, status = fv.decode(la, lb, lp, method, P=P, B=B)
            e1.record()
            torch.cuda.synchronize()
            key = {"vanilla": "vanilla", "flash": f"flash_P{P}", "beam": f"beam_B{B}"}[method]
            out[key] = {"ms": round(e0.elapsed_time(e1), 3), "status": int(status.item()),
                        "workspace_bytes": fv.workspace_bytes(method, h.K, [h.T], P, B)}
        return out

    exact = (("vanilla", 1, 0), ("flash", 16, 0))
    res = {"workload": "single sequences on Erdos-Renyi HMMs, |O|=50, uniform start, emission rows Dirichlet(1), "
                       "observations sampled from the model; defaults p=0.253, K=512, T=512"}
    res["p_sweep"] = []
    for k in range(9):
        p = 1.0 if k == 8 else 0.05 * 1.5 ** k
        res["p_sweep"].append({"p": round(p, 4), **one(hmm.er_hmm(512, 512, p, seed=100 + k), exact)})
    res["K_sweep"] = [{"K": K, **one(hmm.er_hmm(K, 512, 0.253, seed=200 + K), exact)}
                      for K in (32, 64, 128, 256, 512, 1024, 2048)]
    res["T_sweep"] = [{"T": T, **one(hmm.er_hmm(512, T, 0.253, seed=300 + T), exact)}
                      for T in (32, 64, 128, 256, 512, 1024, 2048)]
    beams = [("beam", 16, B) for B in (1024, 512, 256, 128, 64, 32)]
    res["B_sweep"] = {"K": 2048, "T": 512, "p": 0.253,
                      **one(hmm.er_hmm(2048, 512, 0.253, seed=400), [("vanilla", 1, 0), ("flash", 16, 0)] + beams)}
    print(f"[bench] ER sweeps: default point vanilla {res['K_sweep'][4]['vanilla']['ms']} ms, "
          f"FLASH {res['K_sweep'][4]['flash_P16']['ms']} ms", file=sys.stderr, flush=True)
    return res


def small_runs(fv, torch, hmm, dev):
    """Latency-bound decodes: one discrete HMM (K = 64, V = 128, T = 1000;
    microseconds per step of the single sequence), a batch of 256 sequences
    on the same model, and the CRF training step
    (512 sequences, K = 256, T ~ U[32, 512]: ViterbiScore forward + the
    hand-written backward)."""
    res = {}
    h = hmm.discrete_hmm(K=64, V=128, T=1000, seed=1)
    log_e = torch.from_numpy(h.log_e).to(dev)
    obs = torch.from_numpy(h.obs).to(dev)
    la = torch.from_numpy(h.log_a).to(dev)
    lp = torch.from_numpy(h.log_pi).to(dev)
    lb = torch.empty((h.T, h.K), dtype=torch.float32, device=dev)
    lib = fv.lib()
    stream = torch.cuda.current_stream().cuda_stream
    entry = {"workload": "discrete HMM: K=64, V=128, T=1000 (Dirichlet(1) transitions, Dirichlet(0.5) emissions)"}
    for method, P in (("vanilla", 1), ("flash", 16)):
        for rep in range(2):   # warm-up, then timed
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fv._lib.check(lib.fv_gather_emissions(h.K, h.V, log_e.data_ptr(), obs.data_ptr(), h.T, lb.data_ptr(),
                                                  h.K, stream), "fv_gather_emissions")
            fv.decode(la, lb, lp, method, P=P)
            e1.record()
            torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        entry[f"{method}_P{P}" if method == "flash" else method] = {"ms": round(ms, 3),
                                                                     "us_per_step": round(ms * 1e3 / h.T, 2)}
    res["discrete"] = entry
    # a batch of discrete HMM sequences sharing the model: one wave per sequence
    n_b, T_b = 256, 1000
    obs_b = torch.from_numpy(np.stack([hmm.sample_observations(h, T_b, seed=1000 + i) for i in range(n_b)])).to(dev)
    lbs = [torch.empty((T_b, h.K), dtype=torch.float32, device=dev) for _ in range(n_b)]
    for i in range(n_b):
        fv._lib.check(lib.fv_gather_emissions(h.K, h.V, log_e.data_ptr(), obs_b[i].data_ptr(), T_b,
                                              lbs[i].data_ptr(), h.K, stream), "fv_gather_emissions")
    entry = {"workload": f"discrete HMM batch: {n_b} sequences of T={T_b} sharing the K=64, V=128 model "
                         f"(observations sampled from it, one seed per sequence), decode only"}
    for method, P in (("vanilla", 1), ("flash", 16)):
        batch = fv.Batch(lbs)
        for rep in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fv.decode_batch(la, batch, lp, method=method, P=P)
            e1.record()
            torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        bad = int((batch.status != 0).sum().item())
        entry[f"{method}_P{P}" if method == "flash" else method] = {
            "ms": round(ms, 3), "state_steps_per_s": n_b * T_b * h.K / (ms / 1e3), "bad_status": bad}
    res["discrete_batch"] = entry
    wl = hmm.crf_batch()
    em = torch.from_numpy(wl.emissions).to(dev).requires_grad_(True)
    tr = torch.from_numpy(wl.transitions).to(dev).requires_grad_(True)
    entry = {"workload": f"CRF step: {len(wl.lengths)} sequences, K={wl.K}, T~U[32,512], "
                         f"Linear(512->256) emissions, no start scores"}
    for method, P in (("vanilla", 1), ("flash", 16)):
        for rep in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            scores, _ = fv.ViterbiScore.apply(em, wl.lengths, tr, None, method, P)
            scores.sum().backward()
            e1.record()
            torch.cuda.synchronize()
            em.grad = None
            tr.grad = None
        steps = int(np.asarray(wl.lengths, np.int64).sum()) * wl.K
        ms = e0.elapsed_time(e1)
        entry[f"{method}_P{P}" if method == "flash" else method] = {
            "ms_forward_backward": round(ms, 3), "state_steps_per_s": steps / (ms / 1e3)}
    res["crf"] = entry
    return res


def _oracle_sample(wl, budget_cand: float, cand_of):
    """Sequences 0..n-1 of the workload whose summed work fits the budget
    (at least one)."""
    chosen, cand = [], 0
    for b in range(wl.n):
        c = cand_of(int(wl.lengths[b]))
        if chosen and cand + c > budget_cand:
            break
        chosen.append(b)
        cand += c
    return chosen


def _time_oracle(wl, chosen, cores, fn):
    lbs = {b: wl.log_b(b) for b in chosen}
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(lambda b: fn(lbs[b]), chosen))
    return time.perf_counter() - t0


def cpu_baseline(wl, budget_s: float, P: int):
    """The oracle on a prefix of the workload's sequences, all host cores in
    parallel (one sequence per thread at a time): its FLASH procedure (Alg. 1
    and 2, every subtask bisected) at the headline's P, the headline figure,
    and its vanilla decode beside it."""
    import oracle
    cores = min(os.cpu_count() or 1, 16)
    per_core_rate = 2.2e9  # candidates/s per core (measured), for sizing the samples only
    budget = budget_s * cores * per_core_rate
    fl = _oracle_sample(wl, 0.6 * budget, lambda T: flash_candidates(T, P, wl.K, 0))
    dt_f = _time_oracle(wl, fl, cores, lambda lb: oracle.flash(wl.log_pi, wl.log_a, lb, P))
    va = _oracle_sample(wl, 0.4 * budget, lambda T: vanilla_candidates(T, wl.K))
    dt_v = _time_oracle(wl, va, cores, lambda lb: oracle.vanilla(wl.log_pi, wl.log_a, lb))
    steps_f = int(sum(int(wl.lengths[b]) for b in fl))
    steps_v = int(sum(int(wl.lengths[b]) for b in va))
    return {"value": steps_f * wl.K / dt_f, "unit": "state-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"FLASH oracle (plain C, float32; Alg. 1 and 2, P={P}, every subtask bisected) on "
                      f"sequences 0..{len(fl) - 1} ({len(fl)} of {wl.n}, sum T = {steps_f}), one sequence "
                      f"per thread",
            "seconds": round(dt_f, 3),
            "vanilla": {"value": steps_v * wl.K / dt_v, "unit": "state-steps/s",
                        "sample": f"vanilla oracle on sequences 0..{len(va) - 1} ({len(va)} of {wl.n}, "
                                  f"sum T = {steps_v})", "seconds": round(dt_v, 3)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--P", type=int, default=64, help="FLASH parallelism of the headline run")
    ap.add_argument("--sweep", default="vanilla,flash:1,flash:4,flash:16,beam:16:64,beam:16:256",
                    help="extra methods timed once each (method[:P[:B]])")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the K=16384, T=10000 single-sequence runs")
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the K=100000 map-matching (CSR) runs")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the discrete-HMM and CRF-step runs")
    ap.add_argument("--no-relative", action="store_true",
                    help="skip the FV_FLAG_RELATIVE_INIT divergence measurement")
    ap.add_argument("--no-er", action="store_true",
                    help="skip the Erdos-Renyi sweeps (p, K, T, beam width)")
    ap.add_argument("--no-headline", action="store_true",
                    help="skip the batched workload (headline and sweep): a profiling mode for the other "
                         "parts; the JSON line then carries only those parts")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device copy of GIB GiB (torch copy kernel), three times: "
                         "the reference point for the HBM byte counters")
    ap.add_argument("--with-copy", type=float, default=0.0, metavar="GIB",
                    help="run that plain copy once before the benchmark (same process, so one "
                         "counter pass covers both kernels)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library decodes "
              "on one GPU; sequences would shard across GPUs with no exchange between them)", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 30)) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))
        return

    if args.with_copy > 0:
        n = int(args.with_copy * (1 << 30)) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] plain copy of {n * 4} bytes done", file=sys.stderr, flush=True)
        del src, dst
        torch.cuda.empty_cache()

    import paper_2510_19301_amd as fv
    from workloads import hmm
    if args.no_headline:
        out = {"profiling_mode": "no headline"}
        _other_parts(args, out, fv, torch, hmm, dev)
        print(json.dumps(out), flush=True)
        torch.cuda.synchronize()
        return
    wl = hmm.batched_flash_workload(n=args.n)
    K = wl.K
    print(f"[bench] generating workload: {wl.n} sequences, K={K}, sum T={wl.total_steps()}", file=sys.stderr, flush=True)
    lbs = _make_inputs(wl, torch, dev)
    la = torch.from_numpy(wl.log_a).to(dev)
    lp = torch.from_numpy(wl.log_pi).to(dev)
    batch = fv.Batch(lbs)
    torch.cuda.synchronize()
    state_steps = wl.total_steps() * K

    results = {}
    ws = None
    runs = [("flash", args.P, 0, args.steps, args.warmup)]
    for item in [s for s in args.sweep.split(",") if s]:
        parts = item.split(":")
        runs.append((parts[0], int(parts[1]) if len(parts) > 1 else 1,
                     int(parts[2]) if len(parts) > 2 else 0, 1, 1))
    for name, P, B, steps, warmup in runs:
        # "flash-bisect": FLASH with every subtask bisected (no leaf tables)
        method, leaves = ("flash", False) if name == "flash-bisect" else (name, True)
        print(f"[bench] {name} P={P} B={B}: warmup {warmup}, timed {steps}", file=sys.stderr, flush=True)
        ms, eng_ms, ws_new, bad = _time_method(fv, torch, la, lp, batch, method, P, B, steps, warmup, leaves=leaves)
        if ws is None or ws_new.numel() > ws.numel():
            ws = ws_new
        entry = {"ms_per_step": round(ms, 3), "engine_ms": round(eng_ms, 3),
                 "state_steps_per_s": state_steps / (ms / 1e3),
                 "workspace_bytes": fv.workspace_bytes(method, K, wl.lengths, P, B),
                 "bad_status": bad}
        if method in ("flash", "vanilla"):
            leaf = LEAF_LEN if (leaves and K <= 2048) else 0
            cand = (sum(flash_candidates(int(T), P, K, leaf) for T in wl.lengths) if method == "flash"
                    else sum(vanilla_candidates(int(T), K) for T in wl.lengths))
            entry.update({"candidates": cand, "candidates_per_s": cand / (eng_ms / 1e3)})
        key = {"flash": f"flash_P{P}", "flash-bisect": f"flash_bisect_P{P}", "vanilla": "vanilla",
               "beam": f"beam_P{P}_B{B}"}[name]
        results[key] = entry
        print(f"[bench] {name} P={P} B={B}: {ms:.2f} ms/step, engine {eng_ms:.2f} ms", file=sys.stderr, flush=True)

    rel = None
    if not args.no_relative:
        rel = relative_divergence(fv, torch, la, lp, batch, wl.lengths, args.P)
        print(f"[bench] relative init: {rel['sequences_differing_from_vanilla']} of {wl.n} sequences, "
              f"{rel['positions_differing']} positions differ from vanilla", file=sys.stderr, flush=True)
    head = results[f"flash_P{args.P}"]
    ach_tflops = head["candidates"] * 2 / (head["engine_ms"] / 1e3) / 1e12
    out = {
        "metric": "state-steps/s (sum T*K /s), FLASH & beam vs vanilla GPU, bit-exact paths",
        "value": head["state_steps_per_s"],
        "unit": "state-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded generators; no dataset)",
        "config": {"workload": f"batched FLASH decode: {wl.n} sequences, dense K={K}, "
                               f"T~U[500,8000] (sum T={wl.total_steps()}), log A rows Dirichlet(0.1), "
                               f"log B ~ N(0,2^2); FLASH P={args.P}, one persistent launch",
                   "method": "flash", "P": args.P, "K": K, "n_seqs": wl.n, "sum_T": wl.total_steps()},
        "roofline": {"bound": "alu", "achieved": round(ach_tflops, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(ach_tflops / PEAK_FP32_VECTOR_TFLOPS, 4),
                     "traffic": measured_traffic(),
                     "kernel": "fv_engine_kernel",
                     "flops_per_candidate": 2,
                     "frac_of_lane_issue_peak": round(ach_tflops / PEAK_MAXPLUS_TFLOPS, 4)},
        "methods": results,
    }
    if rel is not None:
        out["relative_init"] = rel
    del lbs, batch, ws
    torch.cuda.empty_cache()
    _other_parts(args, out, fv, torch, hmm, dev)
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, args.P)
    print(json.dumps(out), flush=True)
    torch.cuda.synchronize()


def _other_parts(args, out, fv, torch, hmm, dev):
    """The runs beside the headline: large dense, sparse, small, sweeps."""
    if not args.no_large:
        out["large"] = large_runs(fv, torch, hmm, dev)
    if not args.no_sparse:
        torch.cuda.empty_cache()
        out["sparse"] = sparse_runs(fv, torch, hmm, dev)
    if not args.no_small:
        out.update(small_runs(fv, torch, hmm, dev))
    if not args.no_er:
        out["er_sweeps"] = er_runs(fv, torch, hmm, dev)


def _release_device():
    """Leave no device work or cached buffers to process teardown: main()'s
    tensors are gone once it returns; return their memory and wait."""
    import gc
    gc.collect()
    if "torch" in sys.modules:
        torch = sys.modules["torch"]
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            torch.cuda.synchronize()


if __name__ == "__main__":
    main()
    _release_device()
