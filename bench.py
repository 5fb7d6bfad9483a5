#!/usr/bin/env python3
"""Benchmark of the greedy column subset selection hot path on one MI355X.

One step = the whole path on one synthetic input already resident in HBM:
target preparation (B = A Omega, or the Gram matrix for B = A), initial
scores, the k-step selection loop, and the reconstruction error of the picks.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--dtype D]

Prints one JSON line.  value = n*k / t_step (score updates per second over
the whole step) of the workload (default: A 2048 x 2^20 binary32, B = A Omega
with r = 256, k = 100), plus the roofline of the fused streaming kernel (HBM
bytes per launch over its event-timed duration) and the FP64 CPU oracle
timed on a bounded sample of the same workload.  For that default workload
the line also carries two legs of the same comparison:
  * "bf16": the same matrix stored as bfloat16 (same Omega), timed the same
    way, with its own roofline and the FP64 error of its picks against the
    binary32 picks, both scored on the binary32 matrix and its own target;
  * "batched": Algorithm 4 on one GPU (m = 1024, 64 column blocks of uneven
    width, one shared B = A Omega with r = 128, 20 picks per block, merge
    of 100), against the same blocks solved one after another, with the
    roofline of the batched streaming pass and its own CPU baseline;
  * "batched_bf16": the same with the matrix stored as bfloat16.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "score updates/s (n·k/t)"
HEADLINE = "gcss_2048x1048576_r256_k100"
BATCHED = "batched_1024_64blocks_r128"

WORKLOADS = {
    # name: default storage dtype
    "gcss_2048x1048576_r256_k100": "f32",
    "css_4096x65536_k200": "f32",
    "css_500x1000_k20": "f32",
    "gcss_fp8_8192x262144_r512_k500": "fp8",
    "batched_1024_64blocks_r128": "f32",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(name, seed=0):
    """The binary32 matrix of a workload (and Omega for a projection target)."""
    import numpy as np
    import torch

    import synth

    w = synth.workload(name)
    m = w["m"]
    if "nblocks" in w:
        widths = synth.block_widths(w["nblocks"], w["wlo"], w["whi"], seed)
        w["col_off"] = [0] + list(map(int, np.cumsum(widths)))
        w["n"] = w["col_off"][-1]
        w["k"] = w["k_block"]
    n = w["n"]
    if w["kind"] == "gauss_scaled":
        A32 = synth.gauss_lowrank_torch(m, n, w["rank"], w["noise"], seed,
                                        scale=1.0 / math.sqrt(w["rank"]))
    elif w["kind"] == "spectral":
        A32 = synth.spectral_lowrank_torch(m, n, w["rank"], w["decay"], w["noise"], seed)
    else:
        A32 = synth.gauss_lowrank_torch(m, n, w["rank"], w["noise"], seed)
    Om = synth.omega_gauss_torch(n, w["r"], seed + 1) if w["target"] == "proj" else None
    torch.cuda.synchronize()
    return w, A32, Om


def store(A32, m, dtype):
    """The stored matrix the selection streams, and its FP8 scales."""
    import paper_1312_6838_amd as g
    if dtype == "f32":
        return A32, None
    return g.quantize_tensor(A32, m, dtype)


def algorithmic_bytes_per_column(m, dtype):
    # one read of the column + f, g read and written in FP64 (+ the FP8 scale)
    b = {"f32": 4, "bf16": 2, "fp8": 1}[dtype]
    return m * b + 32 + (4 if dtype == "fp8" else 0)


def _src_sha(name):
    src = open(os.path.join(ROOT, "paper_1312_6838_amd", "csrc", name), "rb").read()
    return hashlib.sha256(src).hexdigest()


def read_traffic(kernel, workload, dtype, src_sha):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{dtype}_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != src_sha:
        return None
    try:
        fetch = float(kv["fetch_kib_per_dispatch"]) / float(kv["copy_fetch_scale"])
        write = float(kv["write_kib_per_dispatch"]) / float(kv["copy_write_scale"])
    except (KeyError, ValueError, ZeroDivisionError):
        return None
    return (fetch + write) * 1024.0


def roofline(kernel_desc, kernel, src, workload, dtype, bytes_launch, prof):
    avg_ms = prof["stream_ms"] / max(prof["stream_launches"], 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {"bound": "hbm", "kernel": kernel_desc, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": read_traffic(kernel, workload, dtype, _src_sha(src)),
            "bytes_per_launch": bytes_launch, "avg_launch_ms": round(avg_ms, 5),
            "launches_timed": prof["stream_launches"]}


def _time_oracle(run, n, target_seconds, p0):
    """Grow a column sample until one oracle run takes about target_seconds:
    cost ~ ns^p with p from the last two runs."""
    ns = min(n, 1024)
    t, upd, desc = run(ns)
    p = p0
    for _ in range(3):
        if ns >= n or t >= 0.6 * target_seconds:
            break
        grow = (target_seconds / max(t, 1e-3)) ** (1.0 / p)
        ns_new = int(min(n, max(ns + 64, ns * grow)))
        ns_new = max(64, (ns_new // 64) * 64)
        t_new, upd_new, desc_new = run(ns_new)
        if t_new > t > 0 and ns_new > ns:
            p = min(2.0, max(1.0, math.log(t_new / t) / math.log(ns_new / ns)))
        ns, t, upd, desc = ns_new, t_new, upd_new, desc_new
    return t, upd, desc


def cpu_baseline(w, A32, Om, target_seconds=15.0):
    """The FP64 oracle on a smaller instance of the workload (first n_s columns)."""
    import numpy as np
    import torch

    import oracle

    m, n, k = w["m"], w["n"], w.get("k", 20)
    self_target = w["target"] == "self"
    r = w.get("r", 0)

    def run(ns):
        Acs = A32[:ns, :m].to(torch.float64).cpu().numpy()
        B = None
        if not self_target:
            Bs = (A32[:ns, :m].to(torch.float64).T @ Om[:ns].to(torch.float64)).cpu().numpy()
            B = np.ascontiguousarray(Bs.T)
        kk = min(k, ns)
        t0 = time.perf_counter()
        oracle.select(Acs, m, kk, B=B)
        desc = (f"first {ns} of {n} columns, m={m}, k={kk}, "
                + ("B = A" if self_target else f"B = A_s Omega_s (r={r})")
                + ", FP64 oracle incl. initial scores")
        return time.perf_counter() - t0, ns * kk, desc

    t, upd, desc = _time_oracle(run, n, target_seconds, 2.0 if self_target else 1.0)
    return {"value": upd / t, "unit": "score updates/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": desc, "seconds": round(t, 3)}


def cpu_baseline_batched(w, A32, Om, target_seconds=10.0):
    """The FP64 oracle's Algorithm 4 on the first blocks of the batched workload."""
    import numpy as np
    import torch

    import oracle

    m, off, kb, km, r = w["m"], w["col_off"], w["k_block"], w["k_merge"], w["r"]
    nb_all = len(off) - 1

    def run(nb):
        ns = off[nb]
        Acs = A32[:ns, :m].to(torch.float64).cpu().numpy()
        Bs = (A32[:ns, :m].to(torch.float64).T @ Om[:ns].to(torch.float64)).cpu().numpy()
        B = np.ascontiguousarray(Bs.T)
        kmm = min(km, nb * kb)
        t0 = time.perf_counter()
        oracle.select_distributed(Acs, m, B, np.asarray(off[:nb + 1], dtype=np.int64), kb, kmm)
        dt = time.perf_counter() - t0
        desc = (f"first {nb} of {nb_all} blocks ({ns} columns), m={m}, k_block={kb}, "
                f"merge k={kmm}, B = A_s Omega_s (r={r}), FP64 oracle incl. initial scores")
        return dt, ns * kb + nb * kb * kmm, desc

    nb, (t, upd, desc) = 1, run(1)
    while nb < nb_all and t < 0.5 * target_seconds:
        nb = min(nb_all, max(nb + 1, int(nb * target_seconds / max(t, 1e-3) * 0.8)))
        t, upd, desc = run(nb)
    return {"value": upd / t, "unit": "score updates/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": desc, "seconds": round(t, 3)}


def hbm_probe(args):
    """Achievable HBM read rate: the library's read-only pass over a 4 GiB
    buffer (beyond the 256 MB Infinity Cache), mean of 10 passes."""
    if args.no_probe:
        return None
    import torch

    import paper_1312_6838_amd as g
    buf = torch.zeros(4 << 30, dtype=torch.uint8, device="cuda")
    sec, _ = g.hbm_probe_tensor(buf, reps=10)
    rate = buf.numel() / sec / 1e9
    del buf
    return {"kernel": "k_hbm_read", "achieved": round(rate, 1), "unit": "GB/s",
            "buffer_bytes": 4 << 30, "passes": 10, "frac_of_peak": round(rate / HBM_PEAK_GBS, 4)}


# ---------------------------------------------------------------- one problem --
def run_single(args, name, w, A, scales, Om, dtype, steps, warmup, extras=True):
    """Time `steps` whole steps of one selection problem.  Returns (result
    dict, selector, last picks)."""
    import torch

    import paper_1312_6838_amd as g

    m, n, k = w["m"], w["n"], w["k"]
    self_target = w["target"] == "self"
    r = w.get("r", 0)
    sel = g.Selector(A, m, k_max=k, r_max=r, self_target=self_target, scales=scales)
    state = {}
    if extras and args.embedding:
        W = torch.empty(k, n, dtype=torch.float32, device="cuda")
        sel.set_embedding(W)

    def make_target():
        if self_target:
            sel.set_target(None)
        elif args.omega == "gauss":
            sel.project_target(Om, b_dtype=w.get("b_dtype", "f32"))
        else:
            sel.project_sign(1, r, density=1.0 if args.omega == "sign" else 1.0 / math.sqrt(n))

    def step():
        make_target()
        idx, obj, ns, st = sel.select(k)
        err = sel.reconstruction_error(idx[:ns])
        state.update(idx=idx, obj=obj, ns=ns, err=err)

    tuning = None
    if not args.no_tune:
        log(f"[bench] {name} ({dtype}): autotuning the streaming pass")
        make_target()
        tuning = sel.autotune(min(k, 32), reps=3, cache=args.tune_cache)
    log(f"[bench] {name} ({dtype}): warmup x{warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] {name} ({dtype}): timing x{steps}")
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / steps * 1e3
    # the streaming kernel's duration: HIP events around every streaming pass
    # on the context's stream, in the same steps repeated with event timing on
    # (the selection loop is then enqueued directly instead of replayed from
    # its graph; the kernels are the same)
    sel.profile(True)
    for _ in range(min(steps, 3)):
        step()
    torch.cuda.synchronize()
    prof = sel.profile()
    sel.profile(False)

    # phase split of one more (untimed) step
    torch.cuda.synchronize()
    ta = time.perf_counter()
    make_target()
    torch.cuda.synchronize()
    tb = time.perf_counter()
    idx, obj, ns, st = sel.select(k)
    tc = time.perf_counter()
    sel.reconstruction_error(idx[:ns])
    td = time.perf_counter()
    phases = {"target_and_initial_scores_ms": round((tb - ta) * 1e3, 3),
              "selection_loop_ms": round((tc - tb) * 1e3, 3),
              "reconstruction_error_ms": round((td - tc) * 1e3, 3)}

    roof = roofline("k_stream (fused A^T[q,z] pass + score update + argmax)", "k_stream",
                    "k_stream.hip", name, dtype, n * algorithmic_bytes_per_column(m, dtype), prof)
    out = {
        "metric": METRIC, "value": n * k / (ms_step / 1e3), "unit": "score updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": name, "m": m, "n": n, "k": k, "lda": int(A.shape[1]),
                   "target": "B = A" if self_target else f"B = A Omega, r = {r}",
                   "b_storage": None if self_target else w.get("b_dtype", "f32"),
                   "a_storage": dtype, "embedding": bool(extras and args.embedding),
                   "omega": None if self_target else args.omega},
        "roofline": roof,
        "roofline_note": "stream kernel event-timed in steps repeated right after the timed ones",
        "tuning": tuning,
        "loop_only": {"score_updates_per_s": n * k / (phases["selection_loop_ms"] * 1e-3),
                      "loop_ms": phases["selection_loop_ms"]},
        "phases": phases,
        "result": {"n_selected": int(state["ns"]), "objective_first": float(state["obj"][0]),
                   "objective_last": float(state["obj"][state["ns"]]),
                   "reconstruction_error": float(state["err"])},
    }
    return out, sel, state


def bf16_leg(args, w, A32, Om, sel32, state32, ms32):
    """The headline workload stored as bfloat16 (same Omega), and the quality
    of its picks against the binary32 picks on the binary32 matrix."""
    import torch

    Ab, _ = store(A32, w["m"], "bf16")
    res, sel, st = run_single(args, w["name"], w, Ab, None, Om, "bf16", args.steps, args.warmup,
                              extras=False)
    e32 = sel32.reconstruction_error(state32["idx"][:state32["ns"]])
    e16 = sel32.reconstruction_error(st["idx"][:st["ns"]])
    i32 = set(state32["idx"][:state32["ns"]].tolist())
    i16 = set(st["idx"][:st["ns"]].tolist())
    leg = {k: res[k] for k in ("value", "unit", "ms_per_step", "dtype", "roofline", "tuning",
                               "loop_only", "phases", "result")}
    leg["speedup_vs_f32"] = round(ms32 / res["ms_per_step"], 4)
    leg["quality_vs_f32"] = {
        "scored_on": "the binary32 matrix and its target B = A Omega (same Omega), FP64 error",
        "error_f32_picks": float(e32), "error_bf16_picks": float(e16),
        "rel_diff": float((e16 - e32) / e32) if e32 else None, "bound": 1e-3,
        "picks_in_common": len(i32 & i16)}
    sel.close()
    del Ab
    torch.cuda.synchronize()
    return leg


# ---------------------------------------------------------------- batched ------
def run_batched(args, name, dtype, steps, warmup, cpu=True):
    """Algorithm 4 on one GPU: all blocks in one captured lockstep loop, then
    the merge; against the same blocks solved one after another with the
    single-problem path."""
    import torch

    import paper_1312_6838_amd as g

    log(f"[bench] generating {name}")
    w, A32, Om = make_inputs(name)
    m, n, r = w["m"], w["n"], w["r"]
    A, scales = store(A32, m, dtype)
    off, kb, km = w["col_off"], w["k_block"], w["k_merge"]
    nb = len(off) - 1
    sel = g.Selector(A, m, k_max=kb, r_max=r, scales=scales, batched=(nb, kb, km))
    state = {}

    def step():
        sel.project_target(Om)
        ib, im, om, nm, st = sel.select_batched(off, kb, km)
        state.update(im=im, om=om, nm=nm)

    subs = [g.Selector(A[off[b]:off[b + 1]], m, k_max=kb, r_max=r,
                       scales=None if scales is None else scales[off[b]:off[b + 1]])
            for b in range(nb)]
    pool_max = nb * kb

    def step_seq():
        B = sel.project_target(Om)
        picks = []
        for b, sb in enumerate(subs):
            sb.set_target(B)
            idx, _, ns, _ = sb.select(kb)
            picks += [int(x) + off[b] for x in idx[:ns]]
        P = torch.tensor(picks, device=A.device)
        A0 = A.index_select(0, P).contiguous()
        s0 = g.Selector(A0, m, k_max=min(km, len(picks)), r_max=r,
                        scales=None if scales is None else scales.index_select(0, P).contiguous())
        s0.set_target(B)
        s0.select(min(km, len(picks)))
        s0.close()

    tuning = None
    if not args.no_tune:
        log(f"[bench] {name} ({dtype}): autotuning the batched pass")
        sel.project_target(Om)
        tuning = sel.autotune_batched(off, kb, km, reps=3, cache=args.tune_cache)
    log(f"[bench] {name} ({dtype}): warmup x{warmup}, timing x{steps}")
    for _ in range(warmup):
        step()
        step_seq()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        step_seq()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ms_b = (t1 - t0) / steps * 1e3
    ms_s = (t2 - t1) / steps * 1e3
    # the selection alone (both phases of Algorithm 4, target already set)
    sel.project_target(Om)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(steps):
        sel.select_batched(off, kb, km)
    torch.cuda.synchronize()
    ms_loop = (time.perf_counter() - t3) / steps * 1e3
    # the batched streaming pass's duration: the same call with event timing,
    # which enqueues the block loop directly instead of replaying its graph
    sel.profile(True)
    for _ in range(min(steps, 3)):
        step()
    torch.cuda.synchronize()
    prof = sel.profile()
    sel.profile(False)
    updates = n * kb + pool_max * km
    naive = None
    if args.naive:
        # the paper's naive distributed selection (each block against itself,
        # uniform budgets l/c), and both merged selections judged on A itself
        import numpy as np
        from paper_1312_6838_amd import distributed
        distributed.naive_select(A, m, off, nb * kb, k_merge=km, scales=scales)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rn = distributed.naive_select(A, m, off, nb * kb, k_merge=km, scales=scales)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        full = g.Selector(A, m, k_max=km, self_target=True, scales=scales)
        full.set_target(None)
        e_dist = full.reconstruction_error(state["im"][:state["nm"]])
        e_naive = full.reconstruction_error(rn["idx_merge"])
        e0 = full.reconstruction_error(np.zeros(0, dtype=np.int64))
        full.close()
        naive = {"ms": round((tb - ta) * 1e3, 3), "budget_per_block": int(kb),
                 "error_on_A_naive_merge": e_naive, "error_on_A_distgreedy_merge": e_dist,
                 "norm2_A": e0}
    roof = roofline("k_stream_b (batched fused pass over all blocks + per-group argmax)",
                    "k_stream_b", "k_batched.hip", name, dtype,
                    n * algorithmic_bytes_per_column(m, dtype), prof)
    out = {
        "metric": METRIC, "value": updates / (ms_b / 1e3), "unit": "score updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms_b, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": name, "m": m, "n": n, "blocks": nb, "k_block": kb,
                   "k_merge": km, "target": f"B = A Omega, r = {r}", "a_storage": dtype},
        "roofline": roof,
        "roofline_note": "event-timed in profiled calls right after the timed ones",
        "loop_only": {"score_updates_per_s": updates / (ms_loop / 1e3), "ms": round(ms_loop, 3),
                      "what": "gcss_select_batched alone (block phase and merge), target set"},
        "tuning": tuning,
        "naive_distributed": naive,
        "block_sequential": {"ms_per_step": round(ms_s, 3),
                             "value": updates / (ms_s / 1e3),
                             "batched_speedup": round(ms_s / ms_b, 3)},
        "result": {"n_merge": int(state["nm"]), "objective_first": float(state["om"][0]),
                   "objective_last": float(state["om"][state["nm"]])},
    }
    for s in subs:
        s.close()
    sel.close()
    out["cpu_baseline"] = None
    if cpu:
        log(f"[bench] {name}: cpu baseline (FP64 oracle, first blocks)")
        out["cpu_baseline"] = cpu_baseline_batched(w, A32, Om, args.cpu_seconds_legs)
    del A, A32, Om
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------- main ---------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=HEADLINE, choices=sorted(WORKLOADS))
    ap.add_argument("--dtype", default=None, choices=["f32", "bf16", "fp8"])
    ap.add_argument("--no-legs", action="store_true",
                    help="default workload: skip the bf16 and batched legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-seconds-legs", type=float, default=8.0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--omega", default="gauss", choices=["gauss", "sign", "ssgn"],
                    help="projection of B = A Omega workloads: Gaussian Omega from the host "
                         "(default), or random signs drawn on the GPU: dense +-1 (sign) or "
                         "sparse with density 1/sqrt(n) (ssgn)")
    ap.add_argument("--quality", type=int, default=0, metavar="L",
                    help="B = A workloads: after the timed steps, time the relative accuracy "
                         "(Section 7) of the first L picks against 10 uniform subsets and the "
                         "best rank-L error")
    ap.add_argument("--naive", action="store_true",
                    help="batched workload: also time the naive distributed selection (every "
                         "block against itself) and compare both merges' errors on A")
    ap.add_argument("--embedding", action="store_true",
                    help="the timed selections also write the embedding W = Q^T A")
    ap.add_argument("--rank-k", type=int, default=0, metavar="K",
                    help="with --embedding: time one rank-K approximation in the span of "
                         "the picks after the timed steps")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch setting of the streaming passes instead of "
                         "autotuning it before the warm-up")
    ap.add_argument("--tune-cache", default=os.environ.get("GCSS_TUNE_CACHE"),
                    help="JSON file of tuned settings (default $GCSS_TUNE_CACHE, else none)")
    ap.add_argument("--compare-f32", action="store_true",
                    help="BF16/FP8 storage: also select from the binary32 matrix it was stored "
                         "from, and score both pick sets against that matrix's own target "
                         "(untimed)")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the HBM read probe (achievable bandwidth ceiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one device-to-device copy of BYTES bytes (scales the "
                         "HBM traffic counters of a profiling run)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        nel = args.copy_calibration // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nel * 4}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the selection runs on one GPU; --gpus N > 1 is not supported "
              "(the column-sharded multi-GPU path is not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1312_6838_amd as g

    dtype = args.dtype or WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    g.load()
    if args.workload == BATCHED:
        out = run_batched(args, args.workload, dtype, args.steps, args.warmup,
                          cpu=not args.no_cpu_baseline)
        line = json.dumps(out)
        print(line, flush=True)
        if args.out:
            with open(args.out, "w") as f:
                f.write(line + "\n")
        return

    log(f"[bench] generating {args.workload}")
    w, A32, Om = make_inputs(args.workload)
    w["name"] = args.workload
    A, scales = store(A32, w["m"], dtype)
    out, sel, state = run_single(args, args.workload, w, A, scales, Om, dtype, args.steps,
                                 args.warmup)
    m, n, k = w["m"], w["n"], w["k"]
    self_target = w["target"] == "self"
    r = w.get("r", 0)

    if args.embedding:
        emb = {"written": True}
        if args.rank_k > 0:
            ns = int(state["ns"])
            kk = min(args.rank_k, ns)
            sel.rank_k(ns, kk)                      # warm (kernel load)
            torch.cuda.synchronize()
            te = time.perf_counter()
            U, sig, V, err_k = sel.rank_k(ns, kk)
            torch.cuda.synchronize()
            tf = time.perf_counter()
            emb.update({"rank_k": kk, "l": ns, "rank_k_ms": round((tf - te) * 1e3, 3),
                        "sigma_first": float(sig[0]), "sigma_last": float(sig[-1]),
                        "rank_k_error": float(err_k)})
            del U, V
        out["embedding"] = emb

    if args.quality > 0 and self_target:
        import synth
        from paper_1312_6838_amd import quality as gq
        lq = min(args.quality, int(state["ns"]))
        subsets = synth.uniform_subsets(n, lq, range(10))
        torch.cuda.synchronize()
        tq = time.perf_counter()
        q = gq.relative_accuracy(sel, state["idx"], subsets, l=lq, s=min(2 * lq, k, m),
                                 max_iters=60)
        torch.cuda.synchronize()
        out["quality"] = {"l": lq, "uniform_draws": 10,
                          "ms": round((time.perf_counter() - tq) * 1e3, 2),
                          "relative_accuracy_pct": q["relative_accuracy"], "err_s": q["err_s"],
                          "err_u_mean": float(sum(q["errs_u"]) / len(q["errs_u"])),
                          "err_l": q["err_l"], "eig_block": min(2 * lq, k, m),
                          "eig_iters": q["eig_iters"], "eig_change": q["eig_change"]}

    if args.compare_f32 and dtype != "f32":
        # both selections judged on the binary32 source and its target
        # (B = A, or B = A Omega with the same Omega), FP64 error evaluation
        s32 = g.Selector(A32, m, k_max=k, r_max=r, self_target=self_target)
        if self_target:
            s32.set_target(None)
        elif args.omega == "gauss":
            s32.project_target(Om)
        else:
            s32.project_sign(1, r, density=1.0 if args.omega == "sign" else 1.0 / math.sqrt(n))
        i32, o32, n32, _ = s32.select(k)
        e32 = s32.reconstruction_error(i32[:n32])
        elo = s32.reconstruction_error(state["idx"][:state["ns"]])
        out["vs_f32_on_f32_target"] = {
            "error_f32_picks": float(e32), "error_this_dtype_picks": float(elo),
            "rel_diff": float((elo - e32) / e32) if e32 else None,
            "picks_in_common": int(len(set(i32[:n32].tolist())
                                       & set(state["idx"][:state["ns"]].tolist())))}
        s32.close()

    probe = hbm_probe(args)
    if probe:
        probe["stream_frac_of_probe"] = round(out["roofline"]["achieved"] / probe["achieved"], 4)
    out["hbm_probe"] = probe

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (FP64 oracle, bounded sample)")
        out["cpu_baseline"] = cpu_baseline(w, A32, Om, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None

    legs = args.workload == HEADLINE and dtype == "f32" and not args.no_legs
    if legs:
        log("[bench] bf16 leg")
        out["bf16"] = bf16_leg(args, w, A32, Om, sel, state, out["ms_per_step"])
    sel.close()
    del A, A32, Om, sel
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if legs:
        out["batched"] = run_batched(args, BATCHED, "f32", args.steps, args.warmup,
                                     cpu=not args.no_cpu_baseline)
        # the same batched workload stored as bfloat16 (its CPU baseline is
        # the binary32 leg's: the oracle runs on FP64 either way)
        bb = run_batched(args, BATCHED, "bf16", args.steps, args.warmup, cpu=False)
        bb["speedup_vs_f32"] = round(out["batched"]["ms_per_step"] / bb["ms_per_step"], 4)
        out["batched_bf16"] = bb
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
