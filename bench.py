#!/usr/bin/env python3
"""Benchmark of the MI355X sparse-permanent estimator: learned proposal
against the plain scaled method.

Set-up (untimed, reported): the learned proposal's network is trained on the
GPU from pairs recorded on 512 generated matrices (n = 1000, planted
permutation plus 5n uniform entries, avg degree 6) with the plain scaled
method (one local SK repair per step) as the teacher.

The job is the large sparse workload: n = 1e5 (planted random permutation
plus 7n uniform extra entries, avg degree 8), 1e5 trajectories of the
learned proposal.  Its trajectory ids are split evenly over the timed
steps: step k runs ids [k*M/K, (k+1)*M/K) (persistent trajectory kernel +
FP64 reduction); warmup steps run ids beyond M.  The metric is effective
samples per second over the whole job, ESS / T with ESS = (sum X)^2 /
sum X^2 pooled over all M trajectories (log-sum-exp over the per-step
ln X) and T the wall time of the K timed steps.  The plain scaled method
(one local SK repair per step, no inner filter) then runs the same ids in
the same chunks, timed the same way, and the ratio of the two is reported.
Launches run up to --streams at a time (one handle and HIP stream each,
default 3: one per hardware queue the runtime gives a process beside its
default stream), so that 5000-trajectory launches still fill the chip.
At n = 1e5 both ESS values collapse towards 1 (see "degenerate"), so the
same comparison also runs at n = 1e3 and 1e4 over five run seeds (mean
ratio, bootstrap interval, time to RSE 0.1 and 0.01), and on band matrices
of mean degree 8 whose permanent is known exactly (true error of each
estimate).

Prints one JSON line.  `--gpus N` with N > 1 is not supported: this build
runs on one GPU (see the design notes for how the work would shard).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective samples/sec at equal relative error, learned vs plain, n=1e5 avg deg 8"
HBM_PEAK_GBS = 8000.0

KERNEL_SOURCES = ["paper_2608_15390_amd/csrc/traj.hpp", "paper_2608_15390_amd/csrc/device.hpp",
                  "paper_2608_15390_amd/csrc/mlp.hpp", "paper_2608_15390_amd/csrc/rows.hpp",
                  "paper_2608_15390_amd/csrc/rows_learned.hpp", "paper_2608_15390_amd/csrc/reduce.hpp"]
MFMA_BF16_PEAK_TFLOPS = 2500.0
# the dominant kernel of each timed schedule on the large workload (one
# matrix of n = 1e5: four trajectories per wave for the network-only learned
# proposal, its min-tree's lowest level in the state slot, and for the
# unscaled plain estimator; one per wave for the local repair)
KERNEL_NAME = {"learned": "pe::traj_rows_learned_kernel<false, 1>", "local_nodm": "pe::traj_kernel<3, false, false>",
               "plain": "pe::traj_rows_kernel<false>"}
# algorithmic FLOPs of one 16-candidate tile through the network (8 -> 64 -> 64 -> 1)
FLOP_PER_TILE = 2 * 16 * (8 * 64 + 64 * 64 + 64)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(res: dict, n: int, m: int, scaled: bool) -> float:
    """Bytes the method must move in one launch (a lower bound independent of
    this data layout), from the launch's work counters and these per-unit
    figures:
      adjacency entry scanned at v or u (index + active check)       5 B
      scale gathered per entry of v's list (scaled or learned)      +4 B
      degree decrement with its O(1) bucket swap (deg, bstart RMW,
        arr read, two arr and two pos writes)                       36 B
      retire-chain link (a vertex of degree d takes d + 1 links;
        per step that is the decrements + 4)                        28 B
      trajectory state init (deg, arr, pos over 2n vertices)       24n B
      local-repair entry summed or gathered (index, scale, flag)     9 B
      local-repair value written                                     4 B
      full SK sweep over the residual (at most the whole matrix) 18m + 16n B
      inner filter call (augment + SCC, about three passes)        27m B
      output per trajectory (ln X, alive)                            9 B
    The learned proposal's feature reads beyond v's list (the candidates'
    own neighbours) are not counted: they are this proposal's extra work,
    not the method's."""
    steps = res["n_steps"]
    b = 5.0 * res["n_entries_scanned"]
    if scaled:
        b += 4.0 * res.get("n_entries_scanned_v", 0)
    b += 36.0 * res["n_decrements"]
    b += 28.0 * (res["n_decrements"] + 4 * steps)
    b += res["n_traj"] * (24.0 * n + 9.0)
    b += 9.0 * res["n_local_entries"] + 4.0 * res["n_local_values"]
    b += res["n_full_sk"] * (18.0 * m + 16.0 * n) + res["n_dm"] * 27.0 * m
    return float(b)


def load_traffic(workload: str, n_traj_launch: int):
    """HBM bytes per launch of `n_traj_launch` trajectories from committed
    rocprofv3 counter runs (scaled by the trajectory count when the counted
    launches had another size), or None when the kernel sources changed
    since the counters were taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_hash():
        return None
    per = d.get("n_traj_per_launch")
    if not per:
        return None
    return d["bytes_per_launch"] * n_traj_launch / per


def timed_run(est, first, n_traj, seed, sched, want=False):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = est.run(first, n_traj, seed, sched, want_logw=want, want_alive=want)
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def pooled(lw: np.ndarray, al: np.ndarray, secs: float, steps: int = 0) -> dict:
    """Statistics of one estimate over all its trajectories, in FP64 on the
    host from the per-trajectory ln X: S1 = sum X, S2 = sum X^2 by
    log-sum-exp, ESS = S1^2 / S2, RSE with the M - 1 denominator (zeros
    included), Var ln X over the survivors."""
    n_traj = int(lw.size)
    r = {"n_traj": n_traj, "n_alive": int(al.sum()), "p_match": float(al.mean()), "n_steps": steps,
         "ess": 0.0, "var_logw": float("nan"), "rse": float("nan"), "log_estimate": float("-inf")}
    if al.any():
        x = lw[al]
        top = x.max()
        ls1 = top + math.log(np.exp(x - top).sum())
        ls2 = 2 * top + math.log(np.exp(2 * (x - top)).sum())
        r["log_estimate"] = ls1 - math.log(n_traj)
        r["ess"] = math.exp(2 * ls1 - ls2)
        rel_var = max(0.0, math.exp(ls2 - 2 * ls1) * n_traj - 1.0) * n_traj / max(n_traj - 1, 1)
        r["rse"] = math.sqrt(rel_var / n_traj)
        r["var_logw"] = float(np.var(x, ddof=1)) if x.size > 1 else 0.0
    r["time_to_rse"] = time_to_rse(lw, al, secs)
    return r


def run_concurrent(ests, ranges, seed, sched, streams, label, want=True):
    """The launches of `ranges` [(first, count), ...] spread round-robin over
    the handles `ests` (one per stream), each handle driven by its own host
    thread on its own HIP stream, so that up to len(ests) launches are in
    flight together (a library call blocks only its own thread; results are
    identical per id whatever the grouping).  Returns the per-launch outputs
    in range order."""
    import threading

    import torch

    outs = [None] * len(ranges)
    errs = []
    done = [0]
    lock = threading.Lock()

    def worker(j):
        try:
            with torch.cuda.stream(streams[j]):
                for i in range(j, len(ranges), len(ests)):
                    first, cnt = ranges[i]
                    outs[i] = ests[j].run(first, cnt, seed, sched, want_logw=want, want_alive=want,
                                          stream=streams[j])
                    with lock:
                        done[0] += 1
                        if label:
                            print(f"[bench]   {label}: launch {done[0]}/{len(ranges)} done", file=sys.stderr,
                                  flush=True)
        except BaseException as e:  # re-raised in the caller
            errs.append(e)

    threads = [threading.Thread(target=worker, args=(j,)) for j in range(min(len(ests), len(ranges)))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    if errs:
        raise errs[0]
    return outs


def timed_concurrent(ests, ranges, seed, sched, streams, label):
    """run_concurrent bracketed by device synchronisation; the pooled
    statistics, the wall time and the per-launch results."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = run_concurrent(ests, ranges, seed, sched, streams, label)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    lw = np.concatenate([o["logw"].cpu().numpy() for o in outs])
    al = np.concatenate([o["alive"].cpu().numpy() for o in outs]).astype(bool)
    results = [o["result"] for o in outs]
    return pooled(lw, al, secs, sum(r["n_steps"] for r in results)), secs, results, lw, al


def launch_shape(r):
    """The launch shape a run used, from its result record."""
    return {"blocks": r["launch_blocks"], "waves_per_block": r["launch_waves_per_block"],
            "trajectories_per_wave": r["launch_trajectories_per_wave"],
            "blocks_per_cu": r["launch_blocks_per_cu"],
            "waves_per_cu": r["launch_blocks_per_cu"] * r["launch_waves_per_block"]}


def summary(r, secs):
    return {"ess": r["ess"], "ess_per_s": r["ess"] / secs, "seconds": secs, "traj_per_s": r["n_traj"] / secs,
            "var_logw": r["var_logw"], "p_match": r["p_match"], "rse": r["rse"],
            "log_estimate": r["log_estimate"], "steps_per_traj": r["n_steps"] / r["n_traj"]}


def prefix_rse(lw, al, m):
    """RSE of the estimate from the first m trajectories (zeros included)."""
    x = lw[:m][al[:m]]
    if x.size == 0 or m < 2:
        return math.inf
    top = x.max()
    ls1 = top + math.log(np.exp(x - top).sum())
    ls2 = 2 * top + math.log(np.exp(2 * (x - top)).sum())
    cv2 = m * (m * math.exp(ls2 - 2 * ls1) - 1.0) / (m - 1)
    return math.sqrt(max(cv2, 0.0) / m)


def time_to_rse(lw, al, secs, eps_list=(1e-1, 1e-2)):
    """Time to a target RSE: checkpoints after 2^k trajectories and at the
    end; the target counts as reached at the first checkpoint after the last
    one that misses it, and never if the last one misses it.  Every
    trajectory of a launch runs concurrently and costs about the same, so the
    time of a checkpoint is the launch time pro rata."""
    M = lw.size
    cps = [1 << k for k in range(1, 64) if (1 << k) < M] + [M]
    rses = [prefix_rse(lw, al, c) for c in cps]
    out = {}
    for eps in eps_list:
        bad = [i for i, r in enumerate(rses) if not r <= eps]
        if bad and bad[-1] == len(cps) - 1:
            out[f"{eps:g}"] = None
        else:
            c = cps[bad[-1] + 1] if bad else cps[0]
            out[f"{eps:g}"] = {"seconds": secs * c / M, "trajectories": c}
    return out


def bootstrap_ci(vals, reps=2000, seed=0):
    """95 % percentile bootstrap interval of the mean over replicates."""
    v = np.asarray(vals, dtype=np.float64)
    g = np.random.default_rng(seed)
    means = v[g.integers(0, v.size, size=(reps, v.size))].mean(axis=1)
    return [float(np.percentile(means, 2.5)), float(np.percentile(means, 97.5))]


def ladder(params, plain_sched, learned_sched, seeds, gated_sched=None):
    """The same comparison on smaller matrices of the same family, where the
    effective sample size does not collapse, replicated over run seeds; with
    `gated_sched`, the learned proposal with its gated fallback (local repair
    and the scaled proposal after a surprising step) runs the same seeds."""
    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import inputs as G
    from paper_2608_15390_amd import learned as LR

    methods = [("learned", learned_sched), ("plain", plain_sched)]
    if gated_sched is not None:
        methods.append(("gated", gated_sched))
    rows = []
    for n, cnt in ((1000, 100_000), (10_000, 20_000)):
        M = G.planted_uniform(n, 7 * n, 5)
        est = P.PermEst(M)
        est.set_model(params, LR.MIX_ALPHA)
        row = {"n": n, "n_traj": cnt, "seeds": list(seeds), "ratio": []}
        for name, _ in methods:
            row[name] = []
        if gated_sched is not None:
            row["ratio_gated"] = []
        for s in seeds:
            for name, sch in methods:
                est.run(0, 64, s, sch, want_logw=False, want_alive=False)
                out, secs = timed_run(est, 0, cnt, s, sch, want=True)
                rec = summary(out["result"], secs)
                rec["time_to_rse"] = time_to_rse(out["logw"].cpu().numpy(),
                                                 out["alive"].cpu().numpy().astype(bool), secs)
                row[name].append(rec)
            row["ratio"].append(row["learned"][-1]["ess_per_s"] / row["plain"][-1]["ess_per_s"])
            if gated_sched is not None:
                row["ratio_gated"].append(row["gated"][-1]["ess_per_s"] / row["plain"][-1]["ess_per_s"])
        print(f"[bench]   ladder n={n}: ratios {[round(r, 3) for r in row['ratio']]}", file=sys.stderr, flush=True)
        row["ratio_mean"] = float(np.mean(row["ratio"]))
        row["ratio_ci95"] = bootstrap_ci(row["ratio"])
        if gated_sched is not None:
            row["ratio_gated_mean"] = float(np.mean(row["ratio_gated"]))
            row["ratio_gated_ci95"] = bootstrap_ci(row["ratio_gated"])
        for name, _ in methods:
            row[f"{name}_ess_per_s_mean"] = float(np.mean([r["ess_per_s"] for r in row[name]]))
            row[f"{name}_var_logw_mean"] = float(np.mean([r["var_logw"] for r in row[name]]))
            row[f"{name}_traj_per_s_mean"] = float(np.mean([r["traj_per_s"] for r in row[name]]))
        rows.append(row)
        est.close()
    return rows


BAND_SIZES = ((1000, "1e3", 100_000), (10_000, "1e4", 20_000), (100_000, "1e5", 10_000))


def band_study(params, plain_sched, learned_sched, seed, cnt):
    """Both methods on band matrices of mean degree 8 whose permanent is known
    exactly (stored references, dynamic program over the band), at n = 1e3,
    1e4 (100000 and 20000 trajectories) and 1e5 (`cnt`): the true error of
    each estimate, so "equal relative error" can be read off directly."""
    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import inputs as G
    from paper_2608_15390_amd import learned as LR

    rows = []
    for n, tag, count in BAND_SIZES:
        count = cnt if n == 100_000 else count
        with open(os.path.join(ROOT, "tests", "golden", f"band_n{tag}_hw4.json")) as f:
            ref = json.load(f)
        M, _ = G.config_band(1, n=n)
        h = hashlib.sha256()
        for a in (M.row_ptr, M.col_idx, M.col_ptr, M.row_idx):
            h.update(a.astype("<i4").tobytes())
        if h.hexdigest() != ref["index_sha256"]:
            rows.append({"n": n, "error": "the generator no longer builds the stored band matrix"})
            continue
        lp = ref["log_permanent"]
        est = P.PermEst(M)
        est.set_model(params, LR.MIX_ALPHA)
        out = {"n": M.n, "nnz": M.nnz, "n_traj": count, "log_permanent": lp}
        for name, sch in (("learned", learned_sched), ("plain", plain_sched)):
            est.run(0, 64, seed, sch, want_logw=False, want_alive=False)
            res, secs = timed_run(est, 0, count, seed, sch)
            rec = summary(res["result"], secs)
            le = rec["log_estimate"]
            rec["log_error"] = le - lp
            rec["rel_error"] = math.expm1(le - lp) if math.isfinite(le) else -1.0
            out[name] = rec
            print(f"[bench]   band n={n} {name}: rel error {rec['rel_error']:.3g}, {secs:.1f} s",
                  file=sys.stderr, flush=True)
        est.close()
        rows.append(out)
    return rows


def pool_results(rs):
    """Pool per-launch statistics of the same matrix (disjoint trajectory
    sets or independent seeds) in log space: ln S1 = ln estimate + ln M,
    ln S2 = 2 ln S1 - ln ESS; ESS of the union = S1^2 / S2."""
    l1, l2 = [], []
    for r in rs:
        if r["n_alive"] > 0 and r["ess"] > 0:
            a = r["log_estimate"] + math.log(r["n_traj"])
            l1.append(a)
            l2.append(2 * a - math.log(r["ess"]))
    if not l1:
        return 0.0
    lse = lambda v: max(v) + math.log(sum(math.exp(x - max(v)) for x in v))  # noqa: E731
    return math.exp(2 * lse(l1) - lse(l2))


def batch_main(args) -> int:
    """Many small matrices in one launch (the batching row): 256 matrices,
    n ~ U{30..400}, mean degree ~ U[3, 12], planted permutation, 4096
    trajectories each, the given preset (default: adaptive SK with the
    threshold filter, the paper's adaptive_thr variant). The launch shape is
    picked by the library's autotuner and the launch sequence replayed as a
    captured graph; every step uses its own run seed. value = sum over
    matrices of each matrix's ESS pooled over the steps, per second."""
    import torch

    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import inputs as G
    from paper_2608_15390_amd import learned as LR

    stress = args.workload == "stress"
    if stress:
        # 64 power-law matrices, n log-uniform in [1e4, 1e6], learned proposal
        mats = G.config_stress(1)
        sched_name = args.batch_schedule if args.batch_schedule != "adaptive_threshold" else "learned"
        n_traj = args.n_traj or 256
        wname = "stress64_n1e4_1e6_powerlaw"
    else:
        mats = G.config_batch(1)
        sched_name = args.batch_schedule
        n_traj = args.n_traj or 4096
        wname = "batch256_n30_400"
    sched = P.preset(sched_name)
    bt = P.PermEstBatch(mats, device=0)
    if sched_name.startswith("learned"):
        print(f"[bench] training the proposal network ({args.train_epochs} epochs)", file=sys.stderr, flush=True)
        params, _ = LR.train_proposal(G.config_train(1), epochs=args.train_epochs, seed=args.seed)
        bt.set_model(params, LR.MIX_ALPHA)
    print(f"[bench] batch of {len(mats)} matrices (n {min(M.n for M in mats)}..{max(M.n for M in mats)}), "
          f"{n_traj} trajectories each, {sched_name}", file=sys.stderr, flush=True)
    # set-up: preprocessing, autotuning and graph capture happen on the first runs
    for w in range(max(1, args.warmup)):
        bt.run(n_traj, args.seed + 1000 + w, sched, want_logw=False, want_alive=False, autotune=True,
               graph=not args.no_graph)
        print(f"[bench]   warmup {w + 1} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = bt.run(n_traj, args.seed + k, sched, want_logw=False, want_alive=False, autotune=True,
                     graph=not args.no_graph)
        results.append(out["results"])
        print(f"[bench]   step {k + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ess = sum(pool_results([rs[b] for rs in results]) for b in range(len(mats)))
    steps = sum(r["n_steps"] for rs in results for r in rs)
    kern_s = sum(rs[0]["kernel_seconds"] for rs in results) / len(results)
    # algorithmic bytes per launch, matrix by matrix (work units are launch
    # totals, so the per-step and per-sweep terms use each matrix's counts)
    abytes = 0.0
    r0 = results[0]
    for M, r in zip(mats, r0):
        abytes += r["n_traj"] * (24.0 * M.n + 9.0)
        abytes += r["n_full_sk"] * (18.0 * M.nnz + 16.0 * M.n) + r["n_dm"] * 27.0 * M.nnz
    wt = dict(r0[0])
    wt.update(n_steps=sum(r["n_steps"] for r in r0), n_traj=0, n_full_sk=0, n_dm=0)
    abytes += algorithmic_bytes(wt, 0, 0, sched.sk_policy in (1, 2, 3, 4))
    achieved = abytes / kern_s / 1e9
    # where the waves' time goes (device wall clock, summed over trajectories)
    ws = sum(rs[0]["wave_seconds"] for rs in results)
    phases = {"wave_seconds_per_launch": ws / len(results)}
    for key, lab in (("wave_seconds_full_sk", "full_sk"), ("wave_seconds_dm", "inner_dm"),
                     ("wave_seconds_local", "local_repair")):
        phases[f"{lab}_frac"] = sum(rs[0][key] for rs in results) / ws if ws > 0 else None
    if ws > 0:
        phases["steps_frac"] = 1.0 - sum(v for k, v in phases.items() if k.endswith("_frac"))
    n_dm_all = sum(r["n_dm"] for rs in results for r in rs)
    phases["dm_entries_per_call"] = (sum(rs[0]["n_dm_entries"] for rs in results) / n_dm_all) if n_dm_all else None
    line = {
        "metric": f"effective samples/sec summed over a batch of {len(mats)} matrices",
        "value": ess / secs,
        "unit": "effective samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded generator)",
        "config": {"workload": wname, "matrices": len(mats), "n_traj_per_matrix": n_traj,
                   "n_total": int(sum(M.n for M in mats)), "nnz_total": int(sum(M.nnz for M in mats)),
                   "schedule": sched_name, "parallelism": "1 GPU", "autotune": True, "graph": not args.no_graph},
        "estimate": {"trajectories_per_s": len(mats) * n_traj * args.steps / secs,
                     "steps_per_s": steps / secs, "ess_sum": ess,
                     "p_match_mean": float(np.mean([r["p_match"] for r in results[0]])),
                     "n_dm": sum(r["n_dm"] for r in results[0]), "n_full_sk": sum(r["n_full_sk"] for r in results[0]),
                     "phases": phases},
        "launch": launch_shape(results[0][0]),
        "roofline": {"kernel": "pe::traj_kernel", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": abytes, "kernel_ms": kern_s * 1e3},
    }
    print(json.dumps(line), flush=True)
    bt.close()
    return 0


VARIANTS = ("fixed_all", "adaptive_threshold", "local_threshold", "adaptive_tracked", "local_tracked")


def est_time(cps, eps):
    """Time to target (Sec. 4 "Metrics"): the first checkpoint after the last
    one whose relative error exceeds eps; None if the final one exceeds it."""
    bad = [i for i, c in enumerate(cps) if not c["rel_error"] <= eps]
    if bad and bad[-1] == len(cps) - 1:
        return None
    return cps[bad[-1] + 1 if bad else 0]


def blocks_main(args) -> int:
    """The variant study on the hidden-block set (Sec. 4, "Matrices used";
    Sec. 4.2): the five variants of Sec. 4 on the 50 regenerated
    block-diagonal matrices of exactly known permanent (stored references),
    all 50 in one batched launch per checkpoint.  Each variant runs rounds of
    doubling trajectory counts per matrix (256, 256, 512, ...; a new run
    seed per round, estimates pooled over rounds) until its time budget is
    spent; after every round each matrix's relative error, RSE and p_match
    are logged with the variant's cumulative GPU time.  Reported per
    variant as in the paper's summary: error and RSE wins, median RSE,
    minimum p_match, median M, and the time to relative error 1e-3 and 1e-2
    (matrices stabilised, median time and trajectories)."""
    import torch

    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import inputs as G

    with open(os.path.join(ROOT, "tests", "golden", "blocks50.json")) as f:
        ref = {m["name"]: m for m in json.load(f)["matrices"]}
    sets = list(G.config_blocks())
    for name, M, _ in sets:
        r = ref[name]
        h = hashlib.sha256()
        for a in (M.row_ptr, M.col_idx, M.col_ptr, M.row_idx):
            h.update(a.astype("<i4").tobytes())
        if h.hexdigest() != r["index_sha256"]:
            raise SystemExit(f"bench.py: the generator no longer builds the stored block matrix {name}")
    mats = [M for _, M, _ in sets]
    names = [nm for nm, _, _ in sets]
    lp = np.array([ref[nm]["log_permanent"] for nm in names])
    per_var = {}
    # a batch is all 0/1 or all weighted: one batch of each per variant
    groups = [[b for b, M in enumerate(mats) if M.val is None], [b for b, M in enumerate(mats) if M.val is not None]]
    for vname in VARIANTS:
        sched = P.preset(vname)
        bts = [P.PermEstBatch([mats[b] for b in g], device=0) for g in groups]
        for bt in bts:
            bt.run(8, args.seed + 999, sched, want_logw=False, want_alive=False)  # preprocessing
        torch.cuda.synchronize()
        print(f"[bench]   blocks {vname}: preprocessing done", file=sys.stderr, flush=True)
        lws = [[] for _ in mats]
        als = [[] for _ in mats]
        cps = [[] for _ in mats]
        spent, rnd, count = 0.0, 0, 256
        while spent < args.block_seconds:
            outs = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for gi, bt in enumerate(bts):
                outs.append(bt.run(count, args.seed + rnd, sched))
                torch.cuda.synchronize()
                print(f"[bench]   blocks {vname}: round {rnd + 1}, {'binary' if gi == 0 else 'weighted'} "
                      f"batch done", file=sys.stderr, flush=True)
            spent += time.perf_counter() - t0
            for g, out in zip(groups, outs):
                lw = out["logw"].cpu().numpy()
                al = out["alive"].cpu().numpy().astype(bool)
                off = out["offsets"]
                for i, b in enumerate(g):
                    lws[b].append(lw[off[i]:off[i + 1]])
                    als[b].append(al[off[i]:off[i + 1]])
            for b in range(len(mats)):
                st = pooled(np.concatenate(lws[b]), np.concatenate(als[b]), spent)
                le = st["log_estimate"]
                cps[b].append({"seconds": spent, "trajectories": st["n_traj"],
                               "rel_error": abs(math.expm1(le - lp[b])) if math.isfinite(le) else 1.0,
                               "rse": st["rse"], "p_match": st["p_match"]})
            print(f"[bench]   blocks {vname}: round {rnd + 1}, {count} per matrix, {spent:.1f} s",
                  file=sys.stderr, flush=True)
            rnd += 1
            count = count if rnd == 1 else 2 * count
        for bt in bts:
            bt.close()
        per_var[vname] = cps
    # summary in the form of the paper's variant table
    V, B = len(VARIANTS), len(mats)
    fin_err = np.array([[per_var[v][b][-1]["rel_error"] for b in range(B)] for v in VARIANTS])
    fin_rse = np.array([[per_var[v][b][-1]["rse"] for b in range(B)] for v in VARIANTS])
    summary_rows = {}
    for i, v in enumerate(VARIANTS):
        row = {"error_wins": int(np.sum(np.argmin(fin_err, axis=0) == i)),
               "rse_wins": int(np.sum(np.nanargmin(np.where(np.isnan(fin_rse), np.inf, fin_rse), axis=0) == i)),
               "median_rse": float(np.nanmedian(fin_rse[i])),
               "min_p_match": float(min(per_var[v][b][-1]["p_match"] for b in range(B))),
               "median_M": float(np.median([per_var[v][b][-1]["trajectories"] for b in range(B)])),
               "seconds": per_var[v][0][-1]["seconds"]}
        for eps in (1e-3, 1e-2):
            hits = [est_time(per_var[v][b], eps) for b in range(B)]
            got = [h for h in hits if h is not None]
            row[f"est_{eps:g}"] = {"reached": len(got), "of": B,
                                   "median_seconds": float(np.median([h["seconds"] for h in got])) if got else None,
                                   "median_trajectories": float(np.median([h["trajectories"] for h in got]))
                                   if got else None}
        summary_rows[v] = row
        print(f"[bench]   {v}: {row}", file=sys.stderr, flush=True)
    line = {
        "metric": "hidden-block variant study: matrices stabilised at relative error 1e-3 within the budget",
        "value": summary_rows["local_threshold"]["est_0.001"]["reached"],
        "unit": "matrices of 50",
        "n_gpus": 1, "steps": None, "warmup": None, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator; exact permanents stored in tests/golden/blocks50.json)",
        "config": {"workload": "blocks50", "variants": list(VARIANTS), "budget_seconds_per_variant": args.block_seconds,
                   "launch": "per round one batched launch of the 25 binary and one of the 25 weighted "
                             "matrices"},
        "variants": summary_rows,
        "per_matrix_final": {v: [{"name": names[b], **per_var[v][b][-1]} for b in range(B)] for v in VARIANTS},
    }
    print(json.dumps(line), flush=True)
    return 0


CONSENSUS_SETS = {
    # the band of mean degree 8 at n = 1e3, whose permanent is known exactly
    # (stored reference): the diagnostics can be checked against the truth
    "band_n1e3": {"n": 1000, "variants": VARIANTS, "n_traj": 4096},
    # n = 1e3, the large workload's family (avg degree 8): the five variants of Sec. 4
    "n1e3": {"n": 1000, "variants": VARIANTS, "n_traj": 4096},
    # the large workload itself (n = 1e5): the methods that run there
    "n1e5": {"n": 100_000, "variants": ("local_nodm", "learned", "learned_gated"), "n_traj": 2000},
}


def consensus_main(args) -> int:
    """Multi-seed consensus diagnostics (Sec. 4.4): V variants x 5 run seeds
    on a band matrix of mean degree 8 at n = 1e3 whose permanent is known
    (so the diagnostics can be checked against the truth), on one matrix of
    the large workload's family at n = 1e3 (the five variants of Sec. 4) and
    on the n = 1e5 matrix itself (local repair, learned proposal with and
    without its gated fallback), each run a fixed number of trajectories;
    the library's perm_est_consensus gives the equal-variant consensus, its
    relative half-width, the variant ratio, D_max against the Bonferroni
    value and the provisional-consensus checks."""
    import torch

    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import inputs as G
    from paper_2608_15390_amd import learned as LR

    params = None
    out = {}
    for tag, cfg in CONSENSUS_SETS.items():
        exact = None
        if tag.startswith("band"):
            M, _ = G.config_band(1, n=cfg["n"])
            with open(os.path.join(ROOT, "tests", "golden", "band_n1e3_hw4.json")) as f:
                exact = json.load(f)["log_permanent"]
        elif cfg["n"] < 100_000:
            M = G.planted_uniform(cfg["n"], 7 * cfg["n"], 5)
        else:
            M = G.config_large(1)
        if any(v.startswith("learned") for v in cfg["variants"]) and params is None:
            params, _ = LR.train_proposal(G.config_train(1), epochs=args.train_epochs, seed=args.seed)
        est = P.PermEst(M, device=0)
        if params is not None:
            est.set_model(params, LR.MIX_ALPHA)
        runs, secs = [], {}
        for v in cfg["variants"]:
            sched = P.preset(v)
            est.run(0, 64, args.seed, sched, want_logw=False, want_alive=False)
            row, t = [], 0.0
            for r in range(args.consensus_seeds):
                res, s = timed_run(est, 0, cfg["n_traj"], 1000 + r, sched)
                row.append(res["result"])
                t += s
            runs.append(row)
            secs[v] = t
            print(f"[bench]   consensus {tag} {v}: {args.consensus_seeds} seeds, {t:.1f} s", file=sys.stderr,
                  flush=True)
        est.close()
        c = P.consensus(runs)
        c["variants"] = list(cfg["variants"])
        c["n"] = M.n
        c["n_traj_per_run"] = cfg["n_traj"]
        c["seconds_per_variant"] = secs
        if exact is not None:
            # the truth, for this check only: where it falls against the consensus interval
            c["exact_log_permanent"] = exact
            c["consensus_rel_error"] = math.expm1(c["log_p_con"] - exact)
            c["truth_within_half_width"] = abs(c["consensus_rel_error"]) <= c["rel_half_width"]
        c["runs"] = [[{k: r[k] for k in ("log_estimate", "rse", "ess", "p_match", "n_alive")} for r in row]
                     for row in runs]
        out[tag] = c
    line = {
        "metric": "multi-seed consensus: relative 95% half-width of the equal-variant consensus",
        "value": out["band_n1e3"]["rel_half_width"], "unit": "relative (band n = 1e3)", "n_gpus": 1,
        "higher_is_better": False, "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded generator)",
        "config": {"workload": "consensus", "seeds": args.consensus_seeds}, "consensus": out,
    }
    print(json.dumps(line), flush=True)
    return 0


def hubs_main(args) -> int:
    """The bounded-work local repair on hub vertices (Sec. 3.3): a power-law
    matrix (row degrees P(d) ~ d^-2.5 on [2, 200] plus a planted
    permutation), the plain scaled method (`local_nodm`) with the exact
    repair of Eq. (local) and with caps B on the list entries examined, the
    same trajectory ids and seed for each; per cap the trajectories/s, the
    entries examined per repair, ESS/s and Var ln X."""
    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import inputs as G

    n = args.hub_n
    M = G.power_law(n, 7)
    est = P.PermEst(M, device=0)
    count = args.n_traj or 20_000
    rows = []
    for cap in (0, 32, 16, 8, 4):
        sched = P.preset("local_nodm", local_cap=cap)
        est.run(count, 64, args.seed, sched, want_logw=False, want_alive=False)
        out, secs = timed_run(est, 0, count, args.seed, sched, want=True)
        r = out["result"]
        st = pooled(out["logw"].cpu().numpy(), out["alive"].cpu().numpy().astype(bool), secs, r["n_steps"])
        rows.append({"local_cap": cap, "seconds": secs, "traj_per_s": count / secs,
                     "entries_per_repair": r["n_local_entries"] / max(r["n_local_sk"], 1),
                     "values_per_repair": r["n_local_values"] / max(r["n_local_sk"], 1),
                     "ess": st["ess"], "ess_per_s": st["ess"] / secs, "var_logw": st["var_logw"],
                     "p_match": st["p_match"], "log_estimate": st["log_estimate"],
                     "local_seconds_frac": r["wave_seconds_local"] / r["wave_seconds"] if r["wave_seconds"] else None})
        print(f"[bench]   hubs cap={cap}: {rows[-1]['traj_per_s']:.0f} traj/s, "
              f"{rows[-1]['entries_per_repair']:.0f} entries/repair, ESS {st['ess']:.1f}", file=sys.stderr, flush=True)
    est.close()
    line = {
        "metric": "bounded-work local repair on a power-law matrix: trajectories/s by cap",
        "value": rows[2]["traj_per_s"], "unit": "trajectories/s (cap 16)", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded generator)",
        "config": {"workload": f"powerlaw_n{n}_dmax200", "n": M.n, "nnz": M.nnz, "n_traj": count,
                   "max_row_degree": int(np.diff(M.row_ptr).max()), "schedule": "local_nodm"},
        "caps": rows,
    }
    print(json.dumps(line), flush=True)
    return 0


def cpu_leg(args, M, params, sched_name, n_ids, gpu_logw, gpu_alive, ess_job, n_job):
    """The oracle as it stands, on the host's cores, over the first ids of the
    timed job (a bounded sample grown until about --cpu-seconds of work);
    its ESS/s = the job's ESS x oracle trajectories/s / the job's size."""
    from oracle import mlp as R
    from oracle import oracle as O
    from paper_2608_15390_amd import learned as LR

    print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
    A = O.OMatrix(M)
    osched = O.preset(sched_name)
    if sched_name.startswith("learned"):
        osched = osched.replace(model=R.quantize(params.cpu().numpy().astype(np.float64)), mix_alpha=LR.MIX_ALPHA)
    pre = O.prep(A, osched)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    count, elapsed = threads, 0.0
    while True:
        t = time.perf_counter()
        o = O.run(A, osched, seed=args.seed, first=0, count=count, nthreads=threads, pre=pre)
        elapsed = time.perf_counter() - t
        print(f"[bench]   oracle: {count} trajectories in {elapsed:.1f} s", file=sys.stderr, flush=True)
        if elapsed >= args.cpu_seconds / 4 or count >= n_ids:
            break
        count = min(n_ids, int(count * max(2.0, args.cpu_seconds / max(elapsed, 1e-3) / 2)))
    rate = count / elapsed
    k1 = max(1, min(count, int(2 * count / (elapsed * threads) + 1)))
    t = time.perf_counter()
    O.run(A, osched, seed=args.seed, first=0, count=k1, nthreads=1, pre=pre)
    rate1 = k1 / (time.perf_counter() - t)
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    lw = gpu_logw[:count]
    al = gpu_alive[:count]
    same = bool(np.array_equal(al, o["alive"]) and
                np.allclose(lw[al == 1], o["logw"][al == 1], rtol=1e-12, atol=0))
    return {
        "value": ess_job * rate / n_job,
        "unit": "effective samples/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"trajectory ids 0..{count - 1} of the timed job ({count} of {n_job}), "
                  f"{elapsed:.1f} s on {threads} threads; ESS/s = job ESS x oracle traj/s / job trajectories",
        "traj_per_s": rate,
        "single_thread_traj_per_s": rate1,
        "single_thread_ms_per_traj": 1e3 / rate1,
        "cpu_model": cpu_model,
        "host_cpus": os.cpu_count(),
        "matches_gpu": same,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed steps; the job's trajectory ids are split evenly over them")
    ap.add_argument("--warmup", type=int, default=1, help="untimed steps on trajectory ids beyond the job's")
    ap.add_argument("--workload", default="large",
                    choices=["large", "small", "batch", "stress", "blocks", "consensus", "hubs"],
                    help="batch: 256 matrices n in [30, 400] in one persistent, autotuned, graph-replayed launch; "
                         "blocks: the five variants on the 50-matrix hidden-block set (exact permanents); "
                         "consensus: multi-seed consensus diagnostics on matrices of unknown permanent")
    ap.add_argument("--block-seconds", type=float, default=30.0, help="GPU time budget per variant (blocks)")
    ap.add_argument("--consensus-seeds", type=int, default=5, help="run seeds per variant (consensus)")
    ap.add_argument("--hub-n", type=int, default=20_000, help="order of the power-law matrix (hubs)")
    ap.add_argument("--batch-schedule", default="adaptive_threshold")
    ap.add_argument("--no-graph", action="store_true", help="batch: eager launches instead of graph replay")
    ap.add_argument("--method", default="learned", choices=["learned", "plain"],
                    help="method whose job is timed as `value`")
    ap.add_argument("--plain-schedule", default="local_nodm")
    ap.add_argument("--learned-schedule", default="learned")
    ap.add_argument("--n-traj", type=int, default=None, help="trajectories of the whole job")
    ap.add_argument("--streams", type=int, default=3,
                    help="launches in flight together (one handle and HIP stream each)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--train-epochs", type=int, default=4)
    ap.add_argument("--no-compare", action="store_true", help="skip the other method, the ladder and the band")
    ap.add_argument("--no-ladder", action="store_true", help="skip the n = 1e3 / 1e4 ladder")
    ap.add_argument("--no-band", action="store_true", help="skip the band matrices of known permanent")
    ap.add_argument("--ladder-seeds", type=int, default=5, help="run seeds replicated at n = 1e3 and 1e4")
    ap.add_argument("--band-traj", type=int, default=10_000,
                    help="trajectories per method on the n = 1e5 band matrix of known permanent")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--save-model", default=None, help="write the trained network to this file (model_save)")
    ap.add_argument("--load-model", default=None, help="use this network file instead of training one")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (to scale HBM byte counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                                               "copies": 3}}), flush=True)
        return 0

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on exactly one GPU; N > 1 is not supported "
              "(trajectories shard trivially by id, see the design notes)", file=sys.stderr)
        return 2
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        return 2

    if args.workload in ("batch", "stress"):
        return batch_main(args)
    if args.workload == "blocks":
        return blocks_main(args)
    if args.workload == "consensus":
        return consensus_main(args)
    if args.workload == "hubs":
        return hubs_main(args)

    import torch

    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import inputs as G
    from paper_2608_15390_amd import learned as LR

    if args.workload == "large":
        M = G.config_large(1)
        n_job = args.n_traj or 100_000
        wname = "large_n1e5_deg8"
    else:
        M = G.config_small(1)
        n_job = args.n_traj or 10_000
        wname = "small_n20"
    learned_sched = P.preset(args.learned_schedule)
    plain_sched = P.preset(args.plain_schedule)
    sched = learned_sched if args.method == "learned" else plain_sched
    sched_name = args.learned_schedule if args.method == "learned" else args.plain_schedule

    # ---- set-up (untimed): train the proposal network on the GPU
    if args.load_model:
        p_host, _ = P.load_model(args.load_model)
        params = torch.as_tensor(p_host, device="cuda")
        tinfo = {"loaded_from": os.path.basename(args.load_model)}
    else:
        print(f"[bench] training the proposal network ({args.train_epochs} epochs)", file=sys.stderr, flush=True)
        params, tinfo = LR.train_proposal(G.config_train(1), epochs=args.train_epochs, seed=args.seed)
    if args.save_model:
        P.save_model(args.save_model, params, LR.MIX_ALPHA)
    # one handle per stream: launches on different handles run concurrently
    n_streams = max(1, min(args.streams, args.steps))
    ests = [P.PermEst(M, device=0) for _ in range(n_streams)]
    for e in ests:
        e.set_model(params, LR.MIX_ALPHA)
    streams = [torch.cuda.Stream() for _ in ests]
    est = ests[0]
    # the job's ids split over the timed steps; warmup on ids beyond the job
    chunk = -(-n_job // args.steps)
    ranges = [(k * chunk, min(chunk, n_job - k * chunk)) for k in range(args.steps) if k * chunk < n_job]
    # preprocessing (initial filter, outer SK, templates) happens on the first run
    for e in ests:
        e.run(n_job + args.warmup * chunk, 64, args.seed, sched, want_logw=False, want_alive=False)
    torch.cuda.synchronize()

    print(f"[bench] {args.warmup} warmup + {len(ranges)} timed steps of {chunk} trajectories, "
          f"{args.method} on {wname}, {n_streams} in flight", file=sys.stderr, flush=True)
    if args.warmup:
        wr = [(n_job + w * chunk, chunk) for w in range(args.warmup)]
        run_concurrent(ests, wr, args.seed, sched, streams, "warmup", want=False)
        torch.cuda.synchronize()
    job, secs, results, lw, al = timed_concurrent(ests, ranges, args.seed, sched, streams, "timed")
    ms_per_step = secs * 1e3 / len(ranges)
    value = job["ess"] / secs

    # roofline of the trajectory kernel.  Each launch's device time comes
    # from HIP events around the kernel on its own stream; with several
    # launches in flight they overlap, so the chip-wide rate is the
    # algorithmic bytes of all timed launches over the time the kernels
    # were in flight together (their summed device time over the launches
    # in flight, never more than the timed wall time)
    kern_s = sum(r["kernel_seconds"] for r in results) / len(results)
    in_flight = min(n_streams, len(ranges))
    busy_s = min(secs, sum(r["kernel_seconds"] for r in results) / in_flight)
    scaled = sched.sk_policy in (1, 2, 3, 4)
    abytes = sum(algorithmic_bytes(r, M.n, M.nnz, scaled) for r in results) / len(results)
    achieved = abytes * len(results) / busy_s / 1e9
    tiles = sum(r["n_mlp_tiles"] for r in results)
    mfma_tflops = tiles * FLOP_PER_TILE / busy_s / 1e12
    traffic = load_traffic(f"{wname}_{args.method}", chunk)
    mine = summary(job, secs)
    mine["time_to_rse"] = job["time_to_rse"]
    mine.update(n_local_sk=sum(r["n_local_sk"] for r in results), n_mlp_tiles=sum(r["n_mlp_tiles"] for r in results))

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "effective samples/s",
        "n_gpus": 1,
        "steps": len(ranges),
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator)",
        "config": {
            "workload": wname, "n": M.n, "nnz": M.nnz, "n_traj": n_job, "n_traj_per_step": chunk,
            "launches_in_flight": in_flight,
            "method": args.method, "schedule": sched_name, "parallelism": "1 GPU",
            "arithmetic": "f64 weights and statistics, f32 scaling, bf16 network on an exact grid",
        },
        "estimate": mine,
        "training": dict(tinfo, matrices="512 x (n=1000, avg degree 6)", teacher="local_nodm (local SK repair per step)",
                         mix_alpha=LR.MIX_ALPHA),
        "roofline": {
            "kernel": KERNEL_NAME.get(sched_name, "pe::traj_kernel"),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            # the measured HBM bytes of all timed launches over the same
            # in-flight time, and as a fraction of the peak (null with `traffic`)
            "traffic_gbs": traffic * len(results) / busy_s / 1e9 if traffic else None,
            "traffic_frac": traffic * len(results) / busy_s / 1e9 / HBM_PEAK_GBS if traffic else None,
            "algorithmic_bytes_per_launch": abytes,
            "n_traj_per_launch": chunk,
            "launches_in_flight": in_flight,
            "kernel_ms": kern_s * 1e3,
            "in_flight_seconds": busy_s,
            "launch": launch_shape(results[0]),
            "mfma_bf16_tflops": mfma_tflops,
            "mfma_frac": mfma_tflops / MFMA_BF16_PEAK_TFLOPS,
        },
    }

    if not args.no_compare and args.workload == "large":
        other = plain_sched if args.method == "learned" else learned_sched
        oname = "plain" if args.method == "learned" else "learned"
        print(f"[bench] comparison run: {oname}, same trajectory ids in the same steps", file=sys.stderr, flush=True)
        for e in ests:
            e.run(n_job + args.warmup * chunk, 64, args.seed, other, want_logw=False, want_alive=False)
        res_o, secs_o, _, _, _ = timed_concurrent(ests, ranges, args.seed, other, streams, oname)
        theirs = summary(res_o, secs_o)
        theirs["time_to_rse"] = res_o["time_to_rse"]
        learned_s, plain_s = (mine, theirs) if args.method == "learned" else (theirs, mine)
        cmp = {
            "plain_schedule": args.plain_schedule,
            "learned_schedule": args.learned_schedule,
            "learned": learned_s, "plain": plain_s,
            "ratio_learned_over_plain": learned_s["ess_per_s"] / plain_s["ess_per_s"],
            "degenerate": bool(learned_s["ess"] < 10 and plain_s["ess"] < 10),
        }
        if not args.no_ladder:
            print("[bench] ladder n=1e3, 1e4", file=sys.stderr, flush=True)
            cmp["ladder"] = ladder(params, plain_sched, learned_sched, [args.seed + i for i in range(args.ladder_seeds)],
                                   gated_sched=P.preset("learned_gated"))
        if not args.no_band:
            print("[bench] band matrices n=1e3, 1e4, 1e5 (exact permanent known)", file=sys.stderr, flush=True)
            cmp["band"] = band_study(params, plain_sched, learned_sched, args.seed, args.band_traj)
        line["compare"] = cmp

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_leg(args, M, params, sched_name, chunk, lw, al.astype(np.uint8),
                                       job["ess"], n_job)
    print(json.dumps(line), flush=True)
    for e in ests:
        e.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
