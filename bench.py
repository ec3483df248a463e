#!/usr/bin/env python3
"""Benchmark of SOAR assignment on one MI355X (gfx950).

A step is one full pass of the assignment hot path over the workload: primary assignment,
residual and SOAR spill of every point against a resident codebook, with the exact candidate
re-scoring (soar_assign).  The codebook is trained first on the same GPU (k-means++ and Lloyd
iterations; their times are reported under "train").  Inputs are resident in HBM before the timed
region starts.

--precision takes a comma list: the first form is the headline ("value"); every form is timed on
the same inputs and reported under "forms" with its speedup over FP32 and its index disagreement
and loss regret against the FP64 oracle on a sample of rows.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS_TFLOPS = {"fp32": 157.3, "bf16": 2516.0, "fp8": 5032.0}   # MI355X dense MFMA peaks

# HBM bytes per launch of the dominant kernel, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs
# (KiB per dispatch), each scaled by what the same counter reads for a plain 1 GiB device copy
# (bench.py --mode copy: FETCH_SIZE reads 524302.5 KiB, WRITE_SIZE 1048576 KiB, so the factors
# are 2.0 and 1.0), summed over the kernels of one step.  A figure holds only for the kernel
# sources it was taken on (sha256 below); after any change to them the traffic is reported as
# null until it is measured again.
COPY_SCALE = {"fetch": 1048576.0 / 524302.5, "write": 1.0}   # 1 GiB device copy
# L2-to-memory traffic of one whole call (rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE, KiB summed
# over the call's dispatches), valid while the sources of its kernels are unchanged.  Runs before
# the spill bound took K uniformly sampled rows as the codebook (--codebook sample); the BF16
# entry below was taken with the Lloyd-trained codebook of the default run (--codebook-file),
# since the rows the bound decides, and so the spill sweep's stream, depend on the codebook.
TRAFFIC = {
    # BF16, n=10M, d=96, K=40,000: codebook norms and packing, the spill bound's sample and
    # table, quantization, primary sweep, re-score, the bound's decisions, grouping of the rows
    # it left, grouped spill sweep over their residual rows, re-score
    ("bf16", "mix16384_n10m_d96"): dict(
        fetch_kib=62024592.5, write_kib=5048881.46875,
        sources={"paper_2404_00774_amd/csrc/assign_lowp.hip":
                 "f739b8c4c985ac40e434c23912d749241bc8439dd518f154db3ae775d98f5dcb",
                 "paper_2404_00774_amd/csrc/group.hip":
                 "4413a44cf489a8b77a65e6439b438c875b44e66230830bd7d03cce73d83c5198",
                 "paper_2404_00774_amd/csrc/common.h":
                 "9a129011de60ae36ab0840a680f6b957f22209852444aed35c9d039e2291cc27",
                 "paper_2404_00774_amd/csrc/soar_api.hip":
                 "d726c161aaec18f71ab2c0b2e681d42e2009e8cac74f51acf210522158b0da24",
                 "paper_2404_00774_amd/csrc/bound.hip":
                 "0d20dae175898ad1294ad2a29e74a5a5f2d540fe4041755794db3f749a133882"}),
    # FP8, same workload and the same stages (grouped spill over residual rows)
    ("fp8", "mix16384_n10m_d96"): dict(
        fetch_kib=80853062.9375, write_kib=4447144.65625,
        sources={"paper_2404_00774_amd/csrc/assign_lowp.hip":
                 "0a9b42cb0db6a6ab65ef03bbe158e7e7a68c1ba2084aae79fe7189b4c4ca486f",
                 "paper_2404_00774_amd/csrc/group.hip":
                 "4413a44cf489a8b77a65e6439b438c875b44e66230830bd7d03cce73d83c5198",
                 "paper_2404_00774_amd/csrc/common.h":
                 "08810850b969fa684bc36a9d5144497379e1c98575c4717106f79b1a8f596bcf",
                 "paper_2404_00774_amd/csrc/soar_api.hip":
                 "0f0bd156f3ebf639e438f7d74359f1e1a6c75b952566785d097956e6a548202d"}),
    # grouped FP32 pipeline, per step: codebook packing, primary pass, grouping by primary,
    # grouped spill pass, exact full scan
    ("fp32", "mix4096_n1m_d128"): dict(
        fetch_kib=519893.5, write_kib=87973.0625,
        sources={"paper_2404_00774_amd/csrc/assign_fp32.hip":
                 "d1ec9a821044596c233f27954c3f9d87d307d629d95deef8c1f5b8ce9c3e953a",
                 "paper_2404_00774_amd/csrc/group.hip":
                 "4413a44cf489a8b77a65e6439b438c875b44e66230830bd7d03cce73d83c5198",
                 "paper_2404_00774_amd/csrc/common.h":
                 "08810850b969fa684bc36a9d5144497379e1c98575c4717106f79b1a8f596bcf",
                 "paper_2404_00774_amd/csrc/soar_api.hip":
                 "0f0bd156f3ebf639e438f7d74359f1e1a6c75b952566785d097956e6a548202d"}),
    # FP32, n=2M, d=768, K=10,000 (rows in chunks of 128 dimensions): the same stages; the
    # 30.7 MB codebook does not fit an XCD's L2, so the sweeps refetch it past L2 (5 TB/s)
    ("fp32", "mix8192_n2m_d768_lognorm"): dict(
        fetch_kib=1858119085.1875, write_kib=227337.96875,
        sources={"paper_2404_00774_amd/csrc/assign_fp32.hip":
                 "d1ec9a821044596c233f27954c3f9d87d307d629d95deef8c1f5b8ce9c3e953a",
                 "paper_2404_00774_amd/csrc/group.hip":
                 "4413a44cf489a8b77a65e6439b438c875b44e66230830bd7d03cce73d83c5198",
                 "paper_2404_00774_amd/csrc/common.h":
                 "08810850b969fa684bc36a9d5144497379e1c98575c4717106f79b1a8f596bcf",
                 "paper_2404_00774_amd/csrc/soar_api.hip":
                 "0f0bd156f3ebf639e438f7d74359f1e1a6c75b952566785d097956e6a548202d"}),
}


def measured_traffic(prec, workload):
    """Bytes per launch, or None when not measured for this kernel source."""
    import hashlib
    t = TRAFFIC.get((prec, workload))
    if not t:
        return None
    for src, sha in t["sources"].items():
        path = os.path.join(ROOT, src)
        if not os.path.exists(path) or hashlib.sha256(open(path, "rb").read()).hexdigest() != sha:
            return None
    return (t["fetch_kib"] * COPY_SCALE["fetch"] + t["write_kib"] * COPY_SCALE["write"]) * 1024.0
METRIC = "SOAR-assigned points/sec and % MFMA peak, BF16/FP8 vs FP32 at ≤1e-3 regret"
DTYPE = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8_e4m3"}
KERNEL = {"fp32": "codebook packing, assign_f32_kernel (primary), grouping by primary, "
                  "assign_f32_spill_grouped (spill), exact full scan",
          "bf16": "quantization, centroid_knn_kernel (spill bound table), lowp_sweep_kernel "
                  "(primary), lowp_rescore_kernel (with the bound), grouping of the unbounded rows "
                  "by primary, lowp_sweep_kernel (spill), lowp_rescore_kernel",
          "fp8": "quantization, centroid_knn_kernel (spill bound table), lowp_sweep_kernel "
                 "(primary), lowp_rescore_kernel (with the bound), grouping of the unbounded rows "
                 "by primary, lowp_sweep_kernel (spill), lowp_rescore_kernel"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mix16384_n10m_d96")
    ap.add_argument("--lam", default=None,
                    help="comma list of lambdas (default: the workload's, 1.0 first); the first "
                         "is the headline, every one is timed and checked")
    ap.add_argument("--recall-queries", type=int, default=None,
                    help="queries of the recall@10 check (workloads that define queries; 0: off; "
                         "default: the workload's)")
    ap.add_argument("--precision", default="bf16,fp32,fp8",
                    help="comma list; the first is the headline form")
    ap.add_argument("--form-steps", type=int, default=3, help="timed steps of the other forms")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing (the oracle still checks a sample of every form)")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="rows of the oracle timing (default: the workload's, ~10-30 s of CPU)")
    ap.add_argument("--check-sample", type=int, default=None,
                    help="rows the oracle checks every form on (default: the workload's)")
    ap.add_argument("--codebook", default="train", choices=["train", "sample"],
                    help="sample: K uniformly sampled rows, no training (for short profiling runs)")
    ap.add_argument("--codebook-file", default=None,
                    help="train: load the trained codebook from this .npy when it exists, else "
                         "train and save it there (profiler runs that cannot trace the training)")
    ap.add_argument("--rows", type=int, default=0, help="use only the first N rows (profiling)")
    ap.add_argument("--mode", default="assign", choices=["assign", "serve", "copy"],
                    help="serve: the serving form (resident index, open-loop Poisson inserts); "
                         "copy: a plain device copy of --copy-mib MiB (calibrates the HBM byte "
                         "counters of a profiler)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--serve-base", type=int, default=20_000_000, help="rows of the base index")
    ap.add_argument("--serve-K", type=int, default=50_000)
    ap.add_argument("--serve-rates",
                    default="5000,20000,50000,100000,200000,500000,1000000,2000000",
                    help="offered insert rates, vectors/s")
    ap.add_argument("--serve-requests", type=int, default=10_000,
                    help="requests per offered rate (the window is the time they take to arrive)")
    ap.add_argument("--serve-max-seconds", type=float, default=60.0,
                    help="cap on the arrival window per rate")
    ap.add_argument("--serve-step-rows", type=int, default=16384, help="rows per step slot")
    ap.add_argument("--serve-train-rows", type=int, default=2_000_000,
                    help="rows (a prefix of the base) the serving codebook is trained on")
    ap.add_argument("--serve-kpp-rows", type=int, default=2_000_000,
                    help="rows (a prefix of the base) k-means++ seeds the serving codebook on")
    ap.add_argument("--serve-lloyd", type=int, default=10, help="Lloyd iterations of that codebook")
    ap.add_argument("--serve-precision", default="bf16", choices=["fp32", "bf16", "fp8"])
    return ap.parse_args()


def _threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except Exception:  # noqa: BLE001
        return max(1, min(16, os.cpu_count() or 1))


def oracle_reference(O, X, C, lam, idx, workers):
    """The oracle's answers on rows idx, computed over row chunks in parallel threads (the oracle
    is row-independent; BLAS runs single-threaded inside each worker)."""
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    chunks = [idx[i:i + 2000] for i in range(0, len(idx), 2000)]
    with threadpool_limits(1), ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(lambda r: O.reference(X[r], C, lam), chunks))
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def verify_form(O, X, C, lam, idx, outs, ref, workers, cands=None):
    """The acceptance rule and regret statistics of one GPU form on rows idx (oracle reference
    reused; rows whose GPU primary differs from the oracle's get the conditioned spill anew)."""
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    p, s, dp, ls = outs
    pos = np.arange(len(idx))
    chunks = [pos[i:i + 2000] for i in range(0, len(idx), 2000)]

    def one(r):
        sub = {k: v[r] for k, v in ref.items()}
        return O.verify(X[idx[r]], C, lam, p[r], s[r], dp[r], ls[r], ref=sub)
    with threadpool_limits(1), ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(one, chunks))
    cat = lambda k: np.concatenate([q[k] for q in parts])  # noqa: E731
    pr, sr = cat("primary_regret"), cat("spill_regret")
    p_star, s_star = cat("p_star"), cat("s_star")
    ok = cat("primary_ok") & cat("spill_ok")
    out = {"rows": int(len(idx)), "exact_by_rule": bool(ok.all()),
           "rows_outside_rule": int((~ok).sum()),
           "primary_index_disagreement": float((p != p_star).mean()),
           "spill_index_disagreement": float((s != s_star).mean()),
           "primary_regret_mean": float(pr.mean()), "primary_regret_p99": float(np.quantile(pr, .99)),
           "spill_regret_mean": float(sr.mean()), "spill_regret_p99": float(np.quantile(sr, .99)),
           "values_exact_at_index": bool(cat("pdist_ok").all() and cat("sloss_ok").all())}
    if cands is not None:
        # rows whose oracle best was not among the candidates the GPU re-scored
        pc, sc = cands
        out["candidate_misses_primary"] = int((~(pc == p_star[:, None]).any(1)).sum())
        out["candidate_misses_spill"] = int((~(sc == s_star[:, None]).any(1)).sum())
    return out


def cpu_baseline_leg(O, X, C, lam, rows):
    """The oracle as it stands, timed on a bounded sample of the workload (the CPU baseline)."""
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        threads = os.cpu_count() or 1
    Xs = X[rows]
    O.assign(Xs[:200], C, lam)                      # warm-up (BLAS threads, page faults)
    t0 = time.perf_counter()
    O.assign(Xs, C, lam)
    dt = time.perf_counter() - t0
    return {"value": len(Xs) / dt, "unit": "points/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(Xs)} uniformly sampled rows of the workload (FP64 screened oracle, "
                      f"lambda {lam}), {dt:.2f} s wall; BLAS on {threads} threads, the rest of "
                      "the oracle single-threaded"}


def lambda_trend(X64, C64, outs):
    """Mean cos^2(r, r') and mean ||r'||^2 of a form's answers (Figure 9's lambda trend)."""
    p, s_ = outs[0].astype(np.int64), outs[1].astype(np.int64)
    Rr, Rs = X64 - C64[p], X64 - C64[s_]
    rr, ss = (Rr * Rr).sum(1), (Rs * Rs).sum(1)
    ok = rr > 0
    cos2 = (Rr * Rs).sum(1)[ok] ** 2 / (rr[ok] * ss[ok])
    return {"mean_cos2_r_rspill": float(cos2.mean()), "mean_rspill_sq": float(ss.mean())}


def recall_leg(O, Q, X, C, ts, full, gt):
    """Recall@10 of top-t partition probing with and without the spilled assignment (Eq. 1)
    against brute force (gt: the oracle's exact MIPS top-10)."""
    rec = {"queries": int(len(Q)), "k": 10, "t": list(ts), "per_lambda": {}}
    for lam, (p, s_) in full.items():
        k0, n0 = O.kmr_curve(Q, X, C, [p], 10, ts, gt=gt)
        k1, n1 = O.kmr_curve(Q, X, C, [p, s_], 10, ts, gt=gt)
        rec["per_lambda"][str(lam)] = {
            "recall_unspilled": [float(v) for v in k0], "recall_spilled": [float(v) for v in k1],
            "points_searched_unspilled": [float(v) for v in n0],
            "points_searched_spilled": [float(v) for v in n1]}
    return rec


def search_leg(soar, torch, Xg, Cg, Qg, assign, ts, gt, reps=3):
    """Query-side probing on the GPU (soar_search over the lists built from the assignment):
    per probe depth t, queries/s over the whole query set and recall@10 against brute force,
    with the spilled lists and with the primary lists only."""
    K = Cg.shape[0]
    nq = Qg.shape[0]
    out = {}
    for name, lists in (("spilled", (assign[0], assign[1])), ("unspilled", (assign[0], None))):
        p = torch.from_numpy(lists[0].astype(np.int32)).cuda()
        s_ = None if lists[1] is None else torch.from_numpy(lists[1].astype(np.int32)).cuda()
        off, ids = soar.build_lists(p, s_, K)
        rows = []
        for t in ts:
            r = soar.search(Qg, Cg, Xg, off, ids, t, 10)     # warm-up (and the result)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                soar.search(Qg, Cg, Xg, off, ids, t, 10)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            got = r[0].cpu().numpy()
            recall = float(np.mean([len(set(a) & set(b)) / 10.0 for a, b in zip(got, gt)]))
            rows.append({"t": int(t), "queries_per_s": nq / dt, "ms": dt * 1e3, "recall_at_10": recall,
                         "points_searched": float(r[2].double().mean().item())})
        out[name] = rows
        del off, ids
    return out


def two_level_leg(soar, torch, Xg, Cg, Qg, assign, ts, gt, K2=64, t2s=(2, 8, 32), reps=3):
    """Two-level VQ probing (App. A.4.1, soar_search_two_level): an upper codebook of K2
    centroids trained on the partition centres (k-means++ and 10 Lloyd iterations on the GPU),
    each partition listed under its nearest upper centroid; per t2 and probe depth t, queries/s,
    recall@10 and the partitions probed, over the spilled lists."""
    K = Cg.shape[0]
    nq = Qg.shape[0]
    Ug, _, _ = soar.train_codebook(Cg, K2, 10)
    ua, _, _, _ = soar.assign(Cg, Ug, 0.0)
    uoff, uids = soar.build_lists(ua, None, K2)
    p = torch.from_numpy(assign[0].astype(np.int32)).cuda()
    s_ = torch.from_numpy(assign[1].astype(np.int32)).cuda()
    off, ids = soar.build_lists(p, s_, K)
    out = {"K2": K2, "upper_list_max": int((uoff[1:] - uoff[:-1]).max().item())}
    for t2 in t2s:
        rows = []
        for t in ts:
            r = soar.search_two_level(Qg, Ug, uoff, uids, t2, Cg, Xg, off, ids, t, 10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                soar.search_two_level(Qg, Ug, uoff, uids, t2, Cg, Xg, off, ids, t, 10)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            got = r[0].cpu().numpy()
            recall = float(np.mean([len(set(a) & set(b)) / 10.0 for a, b in zip(got, gt)]))
            rows.append({"t": int(t), "queries_per_s": nq / dt, "ms": dt * 1e3,
                         "recall_at_10": recall,
                         "points_searched": float(r[2].double().mean().item())})
        out[str(t2)] = rows
    return out


def search_pq_leg(soar, torch, Xg, Cg, Qg, assign, P, codes, ts, gt, Rs=(100, 1000), reps=3):
    """Search over the lists with PQ-coded copies (soar_search_pq): every probed copy estimated
    from its own residual's code, the R best points re-scored exactly; per re-rank size R and
    probe depth t, queries/s and recall@10, with the spilled lists and with the primary lists
    only."""
    return {str(R): _search_pq_rows(soar, torch, Xg, Cg, Qg, assign, P, codes, ts, gt, R, reps)
            for R in Rs}


def _search_pq_rows(soar, torch, Xg, Cg, Qg, assign, P, codes, ts, gt, R, reps):
    K = Cg.shape[0]
    nq = Qg.shape[0]
    out = {}
    for name, m in (("spilled", 2), ("unspilled", 1)):
        p = torch.from_numpy(assign[0].astype(np.int32)).cuda()
        s_ = torch.from_numpy(assign[1].astype(np.int32)).cuda() if m == 2 else None
        off, ids = soar.build_lists(p, s_, K)
        A = torch.from_numpy(np.stack(assign[:m], axis=1).astype(np.int32)).cuda()
        lc, _ = soar.list_codes(off, ids, A, codes[:, :m].contiguous())
        rows = []
        for t in ts:
            bound = soar.lists_probe_bound(off, t)
            r = soar.search_pq(Qg, Cg, Xg, off, ids, lc, P, bound, t, R, 10)   # warm-up, result
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                soar.search_pq(Qg, Cg, Xg, off, ids, lc, P, bound, t, R, 10)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            got = r[0].cpu().numpy()
            recall = float(np.mean([len(set(a) & set(b)) / 10.0 for a, b in zip(got, gt)]))
            rows.append({"t": int(t), "queries_per_s": nq / dt, "ms": dt * 1e3,
                         "recall_at_10": recall,
                         "copies_estimated": float(r[2].double().mean().item())})
        out[name] = rows
        del off, ids, lc
    return out


def further_leg(soar, torch, O, Xg, Cg, X, C, lam, assign, idx, steps, Q, ts, gt):
    """A third assignment per point given the primary and spill (Section 3.5.1, soar_spill_further,
    FP32): device time per call on resident inputs, algorithmic rate against the FP32 MFMA peak,
    the oracle's judgement of the check rows, and recall@10 with three lists per point."""
    n, d = Xg.shape
    K = Cg.shape[0]
    m = 2
    P = torch.from_numpy(np.stack(assign, axis=1).astype(np.int32)).to(Xg.device)
    soar.spill_further(Xg, Cg, P, lam)                      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev = []
    for _ in range(steps):
        nxt, loss, st = soar.spill_further(Xg, Cg, P, lam, stats=True)
        dev.append(st["device_ms"])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    dms = float(np.mean(dev))
    alg = 2.0 * n * K * d * (1 + m)
    nx, ls = nxt.cpu().numpy(), loss.cpu().numpy()
    Pn = P.cpu().numpy()
    j = O.verify_further(X[idx], C, lam, Pn[idx], nx[idx], ls[idx])
    out = {"earlier_assignments": m, "ms_per_call": wall, "device_ms": dms,
           "algorithmic_flops_per_call": alg, "algorithmic_tflops": alg / (dms / 1e3) / 1e12,
           "fp32_peak_frac": alg / (dms / 1e3) / 1e12 / PEAKS_TFLOPS["fp32"],
           "rows_full_scan": int(st["rows_full_scan"]), "rows_fp64": int(st["rows_fp64"]),
           "oracle_check": {"rows": int(len(idx)), "exact_by_rule": bool(j["all_ok"]),
                            "index_disagreement": float(j["mismatch"] / len(idx)),
                            "regret_mean": float(np.mean(j["regret"]))}}
    if Q is not None:
        k3, n3 = O.kmr_curve(Q, X, C, [assign[0], assign[1], nx], 10, ts, gt=gt)
        out["recall_three_lists"] = [float(v) for v in k3]
        out["points_searched_three_lists"] = [float(v) for v in n3]
    return out


def pq_leg(soar, torch, O, Xg, Cg, X, C, assign, idx, steps, s=2, train_rows=100_000):
    """PQ codes of both assignments' residuals (Section 3.5, soar_pq_encode): a PQ codebook of 16
    centres per subspace of s dimensions trained on the GPU from primary residuals of a row
    sample, the encode kernel's time against the HBM roofline, the oracle's codes on the check
    rows, each residual's relative reconstruction error, and the index bytes with and without the
    spilled copy (ids, codes and a float32 or int8 copy of every point)."""
    n, d = Xg.shape
    K = Cg.shape[0]
    A = torch.from_numpy(np.stack(assign, axis=1).astype(np.int32)).to(Xg.device)
    m = A.shape[1]
    rows = torch.from_numpy(np.sort(np.random.default_rng(11).choice(n, min(n, train_rows),
                                                                     replace=False))).to(Xg.device)
    R = (Xg[rows] - Cg[A[rows, 0].long()]).contiguous()
    t0 = time.perf_counter()
    P = soar.pq_train(R, s, iters=10)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del R
    codes = soar.pq_encode(Xg, Cg, A, P)                    # warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for _ in range(steps):
        codes = soar.pq_encode(Xg, Cg, A, P)
    ev[1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    dms = ev[0].elapsed_time(ev[1]) / steps
    nb = d // s // 2
    # algorithmic bytes: every point row and assignment once, the codebook once, the codes written
    alg = n * (4 * d + 4 * m + m * nb) + K * 4 * d
    cn, Pn = codes.cpu().numpy(), P.cpu().numpy()
    An = A.cpu().numpy()
    want = O.pq_pack(O.soar_pq_codes(X[idx], C, Pn, [An[idx, j] for j in range(m)]))
    agree = float(np.mean(cn[idx] == want))
    err = []
    for j in range(m):
        u = cn[idx, j].astype(np.int64)
        full = np.empty((len(idx), 2 * nb), np.int64)
        full[:, 0::2], full[:, 1::2] = u & 15, u >> 4
        r = X[idx].astype(np.float64) - C[An[idx, j]]
        q = O.pq_decode(full, Pn)
        err.append(float(((r - q) ** 2).sum() / (r ** 2).sum()))
    ids = 4
    mem = {}
    for name, hb in (("float32", 4), ("int8", 1)):
        one = n * (ids + nb) + n * hb * d
        two = n * m * (ids + nb) + n * hb * d
        mem[name] = {"bytes_one_assignment": int(one), "bytes_with_spill": int(two),
                     "growth": (two - one) / one,
                     "model_growth": O.spill_memory_overhead(d, s, hb),
                     "model_approx_1_over": 8 * s + 1 if hb == 4 else 2 * s + 1}
    return P, codes, {"s": s, "centres_per_subspace": 16, "subspaces": d // s, "code_bytes": nb,
            "train_rows": int(len(rows)), "train_s": t_train,
            "ms_per_call": wall, "device_ms": dms, "algorithmic_bytes_per_call": alg,
            "achieved_gbs": alg / (dms / 1e3) / 1e9, "hbm_peak_frac": alg / (dms / 1e3) / 8e12,
            "oracle_check": {"rows": int(len(idx)), "byte_agreement": agree},
            "relative_error_sum_sq": {"primary": err[0], "spill": err[1] if m > 1 else None},
            "index_memory": mem}


def time_form(soar, torch, Xg, Cg, lam, prec, steps, warmup, n, d, K, keep_candidates=False):
    """Warm-up, then `steps` timed blocking soar_assign calls on resident inputs.  The wall clock
    brackets the steps (torch.cuda.synchronize on both sides); the library's own HIP events on
    its stream give each call's device time and its split into phases."""
    dev = Xg.device
    out = tuple(torch.empty(n, dtype=t, device=dev)
                for t in (torch.int32, torch.int32, torch.float32, torch.float32))
    ws = torch.empty(soar.assign_workspace_size(n, d, K, lam, prec), dtype=torch.uint8, device=dev)
    for _ in range(warmup):
        soar.assign(Xg, Cg, lam, prec, out=out, workspace=ws)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        *_, st = soar.assign(Xg, Cg, lam, prec, out=out, workspace=ws, stats=True)
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cands = None
    if keep_candidates and prec != "fp32" and hasattr(soar, "assign_candidates"):
        cands = soar.assign_candidates(ws, n, d, K, lam, prec)
    phases = {k: float(np.mean([st["phase_ms"][k] for st in stats])) for k in stats[0]["phase_ms"]}
    r = dict(ms_per_step=wall * 1e3 / steps,
             device_ms=float(np.mean([st["device_ms"] for st in stats])),
             sweep_ms=float(np.mean([st["assign_kernel_ms"] for st in stats])),
             phase_ms=phases,
             rows_full_scan=int(np.mean([st["rows_full_scan"] for st in stats])),
             rows_fp64=int(np.mean([st["rows_fp64"] for st in stats])),
             rows_bounded=int(np.mean([st["rows_bounded"] for st in stats])),
             steps=steps, warmup=warmup,
             out=tuple(t.cpu().numpy() for t in out))
    if cands is not None:
        r["cands"] = tuple(c.cpu().numpy() for c in cands)
    del ws
    return r


def request_sizes(rng, count):
    """Insert request sizes floor(exp(U ln 4097)) clamped to [1, 4096] (log-uniform)."""
    return np.clip(np.floor(np.exp(rng.uniform(0.0, np.log(4097.0), count))), 1, 4096).astype(int)


def serve_main(args):
    """The serving form: a resident BF16 index (codebook + inverted lists of a base set) takes
    open-loop Poisson streams of insert requests; per offered rate, the achieved vectors/s and the
    latency from arrival to results in host memory."""
    import dataclasses
    import threading
    import queue
    from concurrent.futures import ThreadPoolExecutor
    from synth import WORKLOADS, gen_mixture, gen_queries

    spec = dataclasses.replace(WORKLOADS["mix4096_n1m_d128"]["spec"], n=args.serve_base)
    K, prec = args.serve_K, args.serve_precision
    lam = float(args.lam.split(",")[0]) if args.lam else 1.0
    rates = [float(r) for r in args.serve_rates.split(",") if r.strip()]
    CH = 1 << 20
    nch = (spec.n + CH - 1) // CH
    # all inputs are drawn before the GPU is touched (threads: numpy releases the GIL)
    print(f"[serve] generating base n={spec.n} d={spec.d} ({nch} chunks)", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        base = list(ex.map(lambda k: gen_mixture(spec, k * CH, min(spec.n, (k + 1) * CH)),
                           range(nch)))
    rng = np.random.default_rng(12345)
    mean_size = float(np.mean(request_sizes(np.random.default_rng(7), 200_000)))
    plans = []
    for rate in rates:
        req_rate = rate / mean_size
        window = min(args.serve_max_seconds, args.serve_requests / req_rate)
        nreq = max(1, int(np.ceil(req_rate * window * 1.2)) + 8)
        arr = np.cumsum(rng.exponential(1.0 / req_rate, nreq))
        arr = arr[arr < window]
        plans.append((rate, arr, request_sizes(rng, len(arr))))
    # request rows: windows of a pool of new rows from the same mixture (a stream separate from
    # the base), reused cyclically; every inserted vector still gets its own id
    pool_rows = 1 << 18
    pool = gen_queries(spec, pool_rows)
    print(f"[serve] inputs ready in {time.perf_counter() - t0:.1f} s; request pool {pool_rows} rows",
          file=sys.stderr, flush=True)

    import torch
    import paper_2404_00774_amd as soar
    dev = torch.device("cuda:0")
    # codebook: k-means++ on a prefix of the base, then Lloyd on a longer prefix
    ktr = min(args.serve_train_rows, spec.n)
    Xtr = torch.from_numpy(np.concatenate(base[:(ktr + CH - 1) // CH])[:ktr]).to(dev)
    t1 = time.perf_counter()
    C0, _ = soar.kmeanspp(Xtr[:min(args.serve_kpp_rows, ktr)].contiguous(), K, 0)
    Cg, _, _ = soar.train_codebook(Xtr, K, args.serve_lloyd, C_init=C0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    del Xtr, C0
    total_new = sum(int(sz.sum()) for _, _, sz in plans)
    cap = int(2 * (spec.n + total_new) * 1.05) + 64 * K
    ix = soar.SoarIndex(Cg, lam, precision=prec, max_step_rows=args.serve_step_rows,
                        list_capacity=cap)
    print(f"[serve] codebook K={K} in {t_train:.1f} s; arena {ix.arena.numel() / 2**30:.2f} GiB; "
          "building base lists", file=sys.stderr, flush=True)
    # base lists: the base rows go in through the same insert path, two requests in flight
    t2 = time.perf_counter()
    pend = []
    for k, Xc in enumerate(base):
        pend.append(ix.insert(Xc, k * CH))
        if len(pend) > 2:
            ix.wait(pend.pop(0))
    for t in pend:
        ix.wait(t)
    t_base = time.perf_counter() - t2
    base_rate = spec.n / t_base
    print(f"[serve] base {spec.n} rows in {t_base:.2f} s ({base_rate:.3g} vectors/s)",
          file=sys.stderr, flush=True)
    del base

    results = []
    next_id = spec.n
    for rate, arr, sizes in plans:
        q = queue.Queue()
        lat = np.zeros(len(arr))
        done_t = np.zeros(len(arr))
        offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]) % (pool_rows - 4096)

        def waiter():
            while True:
                item = q.get()
                if item is None:
                    return
                i, tk, t_arr = item
                ix.wait(tk)
                now = time.perf_counter()
                done_t[i] = now
                lat[i] = now - t_arr

        ws = [threading.Thread(target=waiter, daemon=True) for _ in range(4)]
        for w in ws:
            w.start()
        late = 0.0
        start = time.perf_counter() + 0.05
        for i, (ta, sz) in enumerate(zip(arr, sizes)):
            t_arr = start + ta
            dt = t_arr - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            else:
                late = max(late, -dt)
            o = int(offs[i])
            tk = ix.insert(pool[o:o + sz], next_id)
            next_id += int(sz)
            q.put((i, tk, t_arr))
        for _ in ws:
            q.put(None)
        for w in ws:
            w.join()
        nvec = int(sizes.sum())
        span = float(done_t.max() - start) if len(arr) else 0.0
        r = {"offered_vectors_per_s": rate, "requests": int(len(arr)), "vectors": nvec,
             "achieved_vectors_per_s": nvec / span if span > 0 else 0.0,
             "p50_ms": float(np.quantile(lat, 0.5) * 1e3), "p99_ms": float(np.quantile(lat, 0.99) * 1e3),
             "max_ms": float(lat.max() * 1e3), "mean_request_rows": float(sizes.mean()),
             "max_submit_lag_ms": late * 1e3}
        results.append(r)
        print(f"[serve] rate {rate:.0f}/s: {r['requests']} requests, p50 {r['p50_ms']:.3f} ms, "
              f"p99 {r['p99_ms']:.3f} ms, achieved {r['achieved_vectors_per_s']:.4g}/s",
              file=sys.stderr, flush=True)
    # every inserted vector sits in exactly two lists
    lens = np.array([ix.list_len(p) for p in range(K)], dtype=np.int64)
    ix.close()
    head = results[-1]
    rec = {
        "metric": "SOAR serving inserts: vectors/s with p50/p99 latency (arrival to results in "
                  "host memory)",
        "value": head["achieved_vectors_per_s"], "unit": "vectors/s", "n_gpus": 1,
        "steps": int(sum(r["requests"] for r in results)), "warmup": 0,
        "ms_per_step": head["p50_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": f"serve_mix4096_base{spec.n}_d128_K{K}", "n_base": spec.n, "d": spec.d,
                   "K": K, "lambda": lam, "precision": prec, "step_rows": args.serve_step_rows,
                   "arrivals": "open-loop Poisson per rate, request rows floor(exp(U ln 4097)) "
                               f"in [1, 4096], {args.serve_requests} requests or "
                               f"{args.serve_max_seconds} s per rate, whichever is shorter",
                   "codebook": f"k-means++ on {min(args.serve_kpp_rows, ktr)} rows, "
                               f"{args.serve_lloyd} Lloyd iterations on {ktr} rows (same GPU)"},
        "base_build": {"rows": spec.n, "seconds": t_base, "vectors_per_s": base_rate},
        "rates": results,
        "lists": {"total_ids": int(lens.sum()), "expected": int(2 * next_id),
                  "max_list": int(lens.max())},
        "train_s": t_train,
    }
    print(json.dumps(rec))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); every GPU box here "
              "has one GPU and the path's multi-GPU sharding is described, not run.",
              file=sys.stderr)
        sys.exit(2)
    if args.mode == "serve":
        serve_main(args)
        return
    if args.mode == "copy":
        import torch
        nbytes = args.copy_mib << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_copy": nbytes,
                          "bytes_written_per_copy": nbytes, "copies": args.steps}))
        return
    from concurrent.futures import ThreadPoolExecutor
    from synth import WORKLOADS, gen_mixture, gen_queries, sample_rows

    w = WORKLOADS[args.workload]
    spec, K, iters = w["spec"], w["K"], w["iters"]
    if args.rows:
        import dataclasses
        spec = dataclasses.replace(spec, n=min(args.rows, spec.n))
    n, d = spec.n, spec.d
    precs = [p.strip() for p in args.precision.split(",") if p.strip()]
    if args.lam:
        lams = [float(v) for v in args.lam.split(",") if v.strip()]
    else:
        lams = sorted(w["lambdas"], key=lambda v: (v != 1.0, v))
    check_rows = args.check_sample if args.check_sample is not None else w.get("check_rows", 5000)
    cpu_rows = args.cpu_sample if args.cpu_sample is not None else w.get("cpu_rows", 20_000)
    nq = w.get("queries", 0) if args.recall_queries is None else min(args.recall_queries,
                                                                       w.get("queries", 0))
    workers = _threads()
    # inputs are drawn before the GPU is touched (threads: numpy releases the GIL)
    print(f"[bench] generating {args.workload}: n={n} d={d} K={K}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    CH = 1 << 20
    X = np.empty((n, d), dtype=np.float32)

    def fill(k):
        X[k * CH:min(n, (k + 1) * CH)] = gen_mixture(spec, k * CH, min(n, (k + 1) * CH))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(fill, range((n + CH - 1) // CH)))
    Q = gen_queries(spec, nq) if nq else None
    print(f"[bench] inputs ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    import torch
    import paper_2404_00774_amd as soar
    dev = torch.device("cuda:0")
    Xg = torch.from_numpy(X).to(dev)
    torch.cuda.synchronize()

    # ---- codebook: k-means++ (on a subsample for the large workloads), then Lloyd on all rows
    sub = w.get("seed_subsample")
    t_kpp = t_lloyd = 0.0
    inertia = [float("nan")]
    if args.codebook == "sample":
        Cg = torch.from_numpy(X[sample_rows(spec, K)]).to(dev)
    elif args.codebook_file and os.path.exists(args.codebook_file):
        Cg = torch.from_numpy(np.load(args.codebook_file)).to(dev)
        if tuple(Cg.shape) != (K, d):
            raise SystemExit(f"{args.codebook_file}: shape {tuple(Cg.shape)}, not {(K, d)}")
        print(f"[bench] codebook loaded from {args.codebook_file}", file=sys.stderr, flush=True)
    else:
        print("[bench] training codebook", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        if sub and sub < n:
            Xs = torch.from_numpy(X[sample_rows(spec, sub)]).to(dev)
            C0, _ = soar.kmeanspp(Xs, K, 0)
            del Xs
        else:
            C0, _ = soar.kmeanspp(Xg, K, 0)
        torch.cuda.synchronize()
        t_kpp = time.perf_counter() - t0
        print(f"[bench] k-means++ {t_kpp:.2f} s; Lloyd x{iters}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        Cg, labels, inertia = soar.train_codebook(Xg, K, iters, C_init=C0)
        torch.cuda.synchronize()
        t_lloyd = time.perf_counter() - t0
        del labels, C0
        if args.codebook_file:
            np.save(args.codebook_file, Cg.cpu().numpy())
    C = Cg.cpu().numpy()
    idx = sample_rows(spec, check_rows)

    sweep, full = {}, {}
    alg = 4.0 * n * K * d
    for li, lam in enumerate(lams):
        forms = {}
        for k, prec in enumerate(precs):
            first = li == 0 and k == 0
            steps, warm = (args.steps, args.warmup) if first else (args.form_steps, 1)
            print(f"[bench] lambda {lam} {prec}: warmup {warm}, timing {steps} steps",
                  file=sys.stderr, flush=True)
            r = time_form(soar, torch, Xg, Cg, lam, prec, steps, warm, n, d, K,
                          keep_candidates=True)
            outs = r.pop("out")
            if k == 0 and (Q is not None or li == 0):
                full[lam] = (outs[0].copy(), outs[1].copy())
            r["out"] = tuple(a[idx] for a in outs)
            if "cands" in r:
                r["cands"] = tuple(c[idx] for c in r["cands"])
            r["value"] = n / (r["ms_per_step"] / 1e3)
            # whole call: algorithmic flops over the call's device time; sweeps alone beside it
            r["algorithmic_tflops"] = alg / (r["device_ms"] / 1e3) / 1e12
            r["mfma_peak_frac"] = r["algorithmic_tflops"] / PEAKS_TFLOPS[prec]
            r["sweeps_mfma_peak_frac"] = alg / (r["sweep_ms"] / 1e3) / 1e12 / PEAKS_TFLOPS[prec]
            if prec != "fp32":
                # MFMA work the call executes: the primary sweep over every row, the spill sweep
                # over the rows the spill bound left (stripes of 15 rows and the centroid: at
                # least 16/15 of them), the bound's table (FP32, 2 K^2 d)
                ex = 2.0 * n * K * d + 2.0 * (n - r["rows_bounded"]) * K * d * 16 / 15
                r["executed_mfma_flops"] = ex
                r["executed_tflops"] = ex / (r["device_ms"] / 1e3) / 1e12
                r["executed_frac"] = r["executed_tflops"] / PEAKS_TFLOPS[prec]
                r["table_flops_fp32"] = 2.0 * K * K * d
            print(f"[bench] lambda {lam} {prec}: {r['ms_per_step']:.3f} ms/step, device "
                  f"{r['device_ms']:.3f} ms, {r['mfma_peak_frac']:.3f} of peak; phases "
                  f"{ {k_: round(v, 3) for k_, v in r['phase_ms'].items()} }",
                  file=sys.stderr, flush=True)
            forms[prec] = r
        if "fp32" in forms:
            for prec, r in forms.items():
                r["speedup_vs_fp32"] = forms["fp32"]["ms_per_step"] / r["ms_per_step"]
        sweep[lam] = forms

    head = sweep[lams[0]][precs[0]]
    phases = head["phase_ms"]
    roofline = {"bound": "mfma", "achieved": head["algorithmic_tflops"],
                "peak": PEAKS_TFLOPS[precs[0]], "unit": "TFLOP/s", "frac": head["mfma_peak_frac"],
                "traffic": measured_traffic(precs[0], args.workload) if not args.rows else None,
                "kernel": "soar_assign, the whole call: " + KERNEL[precs[0]],
                "kernel_ms": head["device_ms"], "algorithmic_flops_per_launch": alg,
                "phase_ms": phases,
                "sweeps_frac": head["sweeps_mfma_peak_frac"]}
    if "executed_frac" in head:
        # the algorithmic 4 n K d counts both contractions over every row; the spill bound skips
        # the second for the rows it decides, so the MFMA work executed is smaller
        roofline.update(rows_bounded=head["rows_bounded"],
                        executed_mfma_flops=head["executed_mfma_flops"],
                        executed_frac=head["executed_frac"])

    # ---- oracle leg: reference answers on the check rows, every form judged against them
    import oracle as O
    print(f"[bench] oracle leg: {len(idx)} rows, {workers} threads", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    X64, C64 = X[idx].astype(np.float64), C.astype(np.float64)
    trend = {}
    for lam, forms in sweep.items():
        ref = oracle_reference(O, X, C, lam, idx, workers)
        for prec, r in forms.items():
            outs = r.pop("out")
            r["oracle_check"] = verify_form(O, X, C, lam, idx, outs, ref, workers,
                                            r.pop("cands", None))
            if prec == next(iter(forms)):
                trend[lam] = dict(form=prec, **lambda_trend(X64, C64, outs))
    lam_sorted = sorted(trend)
    trend_out = {"per_lambda": {str(l): trend[l] for l in lam_sorted},
                 "cos2_nonincreasing": all(trend[a]["mean_cos2_r_rspill"] >=
                                           trend[b]["mean_cos2_r_rspill"] - 1e-12
                                           for a, b in zip(lam_sorted, lam_sorted[1:])),
                 "rspill_nondecreasing": all(trend[a]["mean_rspill_sq"] <=
                                             trend[b]["mean_rspill_sq"] + 1e-12
                                             for a, b in zip(lam_sorted, lam_sorted[1:]))}
    print(f"[bench] oracle checks done in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    rec = None
    search = None
    if Q is not None:
        ts = (1, 2, 4, 8, 16, 32, 64, 128)
        print(f"[bench] recall@10 ground truth for {len(Q)} queries", file=sys.stderr, flush=True)
        gt = O.mips_topk(Q, X, 10)
        rec = recall_leg(O, Q, X, C, ts, full, gt)
        Qg = torch.from_numpy(Q).to(dev)
        search = {}
        for lam, assign in full.items():
            print(f"[bench] GPU search, lambda {lam}", file=sys.stderr, flush=True)
            search[str(lam)] = search_leg(soar, torch, Xg, Cg, Qg, assign, ts, gt)
        print(f"[bench] two-level probing, lambda {lams[0]}", file=sys.stderr, flush=True)
        search["two_level"] = two_level_leg(soar, torch, Xg, Cg, Qg, full[lams[0]], ts, gt)
    further = None
    if Q is not None and lams[0] in full:
        print(f"[bench] further spilled assignment (third list), lambda {lams[0]}",
              file=sys.stderr, flush=True)
        further = further_leg(soar, torch, O, Xg, Cg, X, C, lams[0], full[lams[0]], idx,
                              args.form_steps, Q, ts, gt)
        print(f"[bench] further: {further['device_ms']:.3f} ms, "
              f"{further['fp32_peak_frac']:.3f} of FP32 peak", file=sys.stderr, flush=True)
    pq = None
    if lams[0] in full and d % 4 == 0:
        print(f"[bench] PQ codes of both residuals, lambda {lams[0]}", file=sys.stderr,
              flush=True)
        P_pq, codes_pq, pq = pq_leg(soar, torch, O, Xg, Cg, X, C, full[lams[0]], idx,
                                    args.form_steps)
        print(f"[bench] PQ encode: {pq['device_ms']:.3f} ms, {pq['hbm_peak_frac']:.3f} of HBM "
              f"peak, byte agreement {pq['oracle_check']['byte_agreement']:.6f}",
              file=sys.stderr, flush=True)
        if Q is not None:
            print(f"[bench] GPU search over PQ-coded lists, lambda {lams[0]}", file=sys.stderr,
                  flush=True)
            pq["gpu_search_pq"] = search_pq_leg(soar, torch, Xg, Cg, Qg, full[lams[0]], P_pq,
                                                codes_pq, ts, gt)
        del P_pq, codes_pq
    cpu = None
    if not args.no_cpu_baseline and cpu_rows:
        print(f"[bench] CPU baseline: the oracle on {cpu_rows} rows", file=sys.stderr, flush=True)
        cpu = cpu_baseline_leg(O, X, C, lams[0], sample_rows(spec, cpu_rows))

    rec_out = {
        "metric": METRIC, "value": head["value"], "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[precs[0]], "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "K": K, "lambda": lams[0],
                   "precision": precs[0], "mixture_components": spec.components,
                   "lloyd_iters": iters,
                   "codebook": ("k-means++ + Lloyd on the same GPU" if args.codebook == "train"
                                else "uniformly sampled rows (profiling run)")},
        "mfma_peak_frac_algorithmic": head["mfma_peak_frac"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": sweep[lams[0]],
        "lambda_sweep": {str(l): sweep[l] for l in lams[1:]},
        "lambda_trend": trend_out,
        "recall_at_10": rec,
        "gpu_search": search,
        "further_assignment": further,
        "pq_codes": pq,
        "train": {"kmeanspp_s": t_kpp, "kmeanspp_rows": int(sub if sub and sub < n else n),
                  "lloyd_s": t_lloyd, "inertia_first": inertia[0], "inertia_last": inertia[-1]},
    }
    print(json.dumps(rec_out))


if __name__ == "__main__":
    main()
