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
                  "paper_2608_15390_amd/csrc/rows_learned.hpp"]
MFMA_BF16_PEAK_TFLOPS = 2500.0
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


def chunked_run(est, ranges, seed, sched, label):
    """The trajectory ids of `ranges` [(first, count), ...] as consecutive
    launches (results are identical per id), each bracketed by device
    synchronisation; returns the pooled statistics, the wall time summed
    over the launches, and the per-launch results."""
    import torch

    lws, als, secs, steps, per_launch = [], [], 0.0, 0, []
    done, total = 0, sum(c for _, c in ranges)
    for first, c in ranges:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = est.run(first, c, seed, sched, want_logw=True, want_alive=True)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        lws.append(out["logw"].cpu().numpy())
        als.append(out["alive"].cpu().numpy())
        steps += out["result"]["n_steps"]
        per_launch.append(out["result"])
        done += c
        print(f"[bench]   {label}: {done}/{total} trajectories, {secs:.1f} s", file=sys.stderr, flush=True)
    r = pooled(np.concatenate(lws), np.concatenate(als).astype(bool), secs, steps)
    return r, secs, per_launch


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


def ladder(params, plain_sched, learned_sched, seeds):
    """The same comparison on smaller matrices of the same family, where the
    effective sample size does not collapse, replicated over run seeds."""
    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import inputs as G
    from paper_2608_15390_amd import learned as LR

    rows = []
    for n, cnt in ((1000, 100_000), (10_000, 20_000)):
        M = G.planted_uniform(n, 7 * n, 5)
        est = P.PermEst(M)
        est.set_model(params, LR.MIX_ALPHA)
        row = {"n": n, "n_traj": cnt, "seeds": list(seeds), "learned": [], "plain": [], "ratio": []}
        for s in seeds:
            for name, sch in (("learned", learned_sched), ("plain", plain_sched)):
                est.run(0, 64, s, sch, want_logw=False, want_alive=False)
                out, secs = timed_run(est, 0, cnt, s, sch, want=True)
                rec = summary(out["result"], secs)
                rec["time_to_rse"] = time_to_rse(out["logw"].cpu().numpy(),
                                                 out["alive"].cpu().numpy().astype(bool), secs)
                row[name].append(rec)
            row["ratio"].append(row["learned"][-1]["ess_per_s"] / row["plain"][-1]["ess_per_s"])
        print(f"[bench]   ladder n={n}: ratios {[round(r, 3) for r in row['ratio']]}", file=sys.stderr, flush=True)
        row["ratio_mean"] = float(np.mean(row["ratio"]))
        row["ratio_ci95"] = bootstrap_ci(row["ratio"])
        for name in ("learned", "plain"):
            row[f"{name}_ess_per_s_mean"] = float(np.mean([r["ess_per_s"] for r in row[name]]))
            row[f"{name}_var_logw_mean"] = float(np.mean([r["var_logw"] for r in row[name]]))
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

    mats = G.config_batch(1)
    n_traj = args.n_traj or 4096
    sched = P.preset(args.batch_schedule)
    bt = P.PermEstBatch(mats, device=0)
    print(f"[bench] batch of {len(mats)} matrices, {n_traj} trajectories each, {args.batch_schedule}",
          file=sys.stderr, flush=True)
    # set-up: preprocessing, autotuning and graph capture happen on the first runs
    for w in range(max(1, args.warmup)):
        bt.run(n_traj, args.seed + 1000 + w, sched, want_logw=False, want_alive=False, autotune=True, graph=True)
        print(f"[bench]   warmup {w + 1} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = bt.run(n_traj, args.seed + k, sched, want_logw=False, want_alive=False, autotune=True, graph=True)
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
        scaled = sched.sk_policy in (1, 2, 3)
        abytes += r["n_traj"] * (24.0 * M.n + 9.0)
        abytes += r["n_full_sk"] * (18.0 * M.nnz + 16.0 * M.n) + r["n_dm"] * 27.0 * M.nnz
    wt = dict(r0[0])
    wt.update(n_steps=sum(r["n_steps"] for r in r0), n_traj=0, n_full_sk=0, n_dm=0)
    abytes += algorithmic_bytes(wt, 0, 0, sched.sk_policy in (1, 2, 3))
    achieved = abytes / kern_s / 1e9
    line = {
        "metric": f"effective samples/sec summed over a batch of {len(mats)} matrices",
        "value": ess / secs,
        "unit": "effective samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded generator)",
        "config": {"workload": "batch256_n30_400", "matrices": len(mats), "n_traj_per_matrix": n_traj,
                   "schedule": args.batch_schedule, "parallelism": "1 GPU", "autotune": True, "graph": True},
        "estimate": {"trajectories_per_s": len(mats) * n_traj * args.steps / secs,
                     "steps_per_s": steps / secs, "ess_sum": ess,
                     "p_match_mean": float(np.mean([r["p_match"] for r in results[0]])),
                     "n_dm": sum(r["n_dm"] for r in results[0]), "n_full_sk": sum(r["n_full_sk"] for r in results[0])},
        "roofline": {"kernel": "pe::traj_kernel", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": abytes, "kernel_ms": kern_s * 1e3},
    }
    print(json.dumps(line), flush=True)
    bt.close()
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
    ap.add_argument("--workload", default="large", choices=["large", "small", "batch"],
                    help="batch: 256 matrices n in [30, 400] in one persistent, autotuned, graph-replayed launch")
    ap.add_argument("--batch-schedule", default="adaptive_threshold")
    ap.add_argument("--method", default="learned", choices=["learned", "plain"],
                    help="method whose job is timed as `value`")
    ap.add_argument("--plain-schedule", default="local_nodm")
    ap.add_argument("--learned-schedule", default="learned")
    ap.add_argument("--n-traj", type=int, default=None, help="trajectories of the whole job")
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

    if args.workload == "batch":
        return batch_main(args)

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
    est = P.PermEst(M, device=0)
    est.set_model(params, LR.MIX_ALPHA)
    # the job's ids split over the timed steps; warmup on ids beyond the job
    chunk = -(-n_job // args.steps)
    ranges = [(k * chunk, min(chunk, n_job - k * chunk)) for k in range(args.steps) if k * chunk < n_job]
    # preprocessing (initial filter, outer SK, templates) happens on the first run
    est.run(n_job + args.warmup * chunk, 64, args.seed, sched, want_logw=False, want_alive=False)
    torch.cuda.synchronize()

    print(f"[bench] {args.warmup} warmup + {len(ranges)} timed steps of {chunk} trajectories, "
          f"{args.method} on {wname}", file=sys.stderr, flush=True)
    for w in range(args.warmup):
        est.run(n_job + w * chunk, chunk, args.seed, sched, want_logw=False, want_alive=False)
        torch.cuda.synchronize()
        print(f"[bench]   warmup {w + 1}/{args.warmup}", file=sys.stderr, flush=True)
    outs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, (first, cnt) in enumerate(ranges):
        outs.append(est.run(first, cnt, args.seed, sched, want_logw=True, want_alive=True))
        if (k + 1) % max(1, len(ranges) // 10) == 0:
            print(f"[bench]   step {k + 1}/{len(ranges)}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    secs = t1 - t0
    ms_per_step = secs * 1e3 / len(ranges)
    lw = np.concatenate([o["logw"].cpu().numpy() for o in outs])
    al = np.concatenate([o["alive"].cpu().numpy() for o in outs]).astype(bool)
    results = [o["result"] for o in outs]
    job = pooled(lw, al, secs, sum(r["n_steps"] for r in results))
    value = job["ess"] / secs

    # roofline of the trajectory kernel: algorithmic bytes per launch over its
    # average device time (HIP events around the kernel on the run's stream)
    kern_s = sum(r["kernel_seconds"] for r in results) / len(results)
    scaled = sched.sk_policy in (1, 2, 3, 4)
    abytes = sum(algorithmic_bytes(r, M.n, M.nnz, scaled) for r in results) / len(results)
    achieved = abytes / kern_s / 1e9
    tiles = sum(r["n_mlp_tiles"] for r in results) / len(results)
    mfma_tflops = tiles * FLOP_PER_TILE / kern_s / 1e12
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
            "method": args.method, "schedule": sched_name, "parallelism": "1 GPU",
            "arithmetic": "f64 weights and statistics, f32 scaling, bf16 network on an exact grid",
        },
        "estimate": mine,
        "training": dict(tinfo, matrices="512 x (n=1000, avg degree 6)", teacher="local_nodm (local SK repair per step)",
                         mix_alpha=LR.MIX_ALPHA),
        "roofline": {
            "kernel": "pe::traj_kernel",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            # the measured HBM bytes over the same launch time, and as a
            # fraction of the peak (null with `traffic`)
            "traffic_gbs": traffic / kern_s / 1e9 if traffic else None,
            "traffic_frac": traffic / kern_s / 1e9 / HBM_PEAK_GBS if traffic else None,
            "algorithmic_bytes_per_launch": abytes,
            "n_traj_per_launch": chunk,
            "kernel_ms": kern_s * 1e3,
            "mfma_bf16_tflops": mfma_tflops,
            "mfma_frac": mfma_tflops / MFMA_BF16_PEAK_TFLOPS,
        },
    }

    if not args.no_compare and args.workload == "large":
        other = plain_sched if args.method == "learned" else learned_sched
        oname = "plain" if args.method == "learned" else "learned"
        print(f"[bench] comparison run: {oname}, same trajectory ids in the same steps", file=sys.stderr, flush=True)
        est.run(n_job + args.warmup * chunk, 64, args.seed, other, want_logw=False, want_alive=False)
        res_o, secs_o, _ = chunked_run(est, ranges, args.seed, other, oname)
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
            cmp["ladder"] = ladder(params, plain_sched, learned_sched, [args.seed + i for i in range(args.ladder_seeds)])
        if not args.no_band:
            print("[bench] band matrices n=1e3, 1e4, 1e5 (exact permanent known)", file=sys.stderr, flush=True)
            cmp["band"] = band_study(params, plain_sched, learned_sched, args.seed, args.band_traj)
        line["compare"] = cmp

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_leg(args, M, params, sched_name, chunk, lw, al.astype(np.uint8),
                                       job["ess"], n_job)
    print(json.dumps(line), flush=True)
    est.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
