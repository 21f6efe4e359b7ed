"""Benchmark: rank-k implicit SVD wall time to relative residual 1e-4 on one MI355X.

One step = one isvd_truncated_svd call in tolerance mode (every product,
orthonormalisation, Rayleigh-Ritz step and residual check of the method)
on a resident synthetic graph; the start block is drawn on the device
inside the call.  Default workload: Chung-Lu power-law graph, n = 2,000,000,
exponent 2.3, mean degree 25, M = (1/5) sum_{j=1..5} T^j - 0.05 (11^T - A),
k = 256, p = 32.  `value` is the time per step with FP32 blocks; the same
line carries the BF16-storage form (BF16 blocks with an FP32 finish) over a
fixed number of steps, and the singular-value errors and subspace angles of
both against an FP64 run of the library from the same start block at a
fixed q = 2.

`roofline` describes the sparse-pass kernel (the kernel that bounds every
product) over the FP32 passes of the timed steps: algorithmic bytes (every
gathered row counted each time it is gathered) over the summed HIP-event
durations of its launches; `traffic` is the measured bytes per launch from
hardware counters when they were taken on the current source.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload and scales it to one whole iSVD (extrapolated; see its `sample`).
Other modes: --config c2|c3|c5, --peaks, --products, --traffic-from,
--start-study, --learners, --dag, --ablation.
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c4", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--bf16-steps", type=int, default=5,
                    help="default workload: timed BF16-storage steps (after one warm-up)")
    ap.add_argument("--error-q", type=int, default=2,
                    help="default workload: power iterations of the FP64 / FP32 / BF16 error runs")
    ap.add_argument("--no-errors", action="store_true")
    ap.add_argument("--peaks", action="store_true",
                    help="measure the device's peak rates instead: streaming copy (HBM), repeated reads of a "
                         "96 MiB buffer (Infinity Cache), FP64 and FP32 MFMA; one JSON line")
    ap.add_argument("--products", type=int, default=0,
                    help="time this many product pairs (M Y, M^T Y) per block storage (FP32, BF16) on the "
                         "workload's operator instead of whole SVDs (a short run for hardware counters)")
    ap.add_argument("--orth", type=int, default=0,
                    help="time this many orthonormalisations (CholeskyQR2: two passes of Gram, Cholesky, "
                         "triangular solve) of an n x l Gaussian block of the workload's shape per block "
                         "storage (FP32, BF16) instead of whole SVDs (a short run for hardware counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="summarise two rocprofv3 --pmc counter files (FETCH_SIZE, WRITE_SIZE) of a "
                         "--products --calibrate-copy run into profiles/spmm_traffic_<workload>.json (no GPU)")
    ap.add_argument("--start-study", action="store_true",
                    help="on the n = 1,000,000 warm-start workload: iterations to rho <= tol from start blocks "
                         "built from the converged top singular vectors (all, leading, trailing, noisy), from "
                         "Gaussian rows restricted or weighted by node scores, and from the committed network "
                         "(one JSON line)")
    ap.add_argument("--oracle-runs", type=int, default=1,
                    help="--config c2/c3: timed runs of the FP64 oracle at fixed q on the GPU's start block "
                         "(median reported; 0 skips it)")
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16"])
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-iter", type=int, default=2000)
    ap.add_argument("--check-every", type=int, default=0)
    ap.add_argument("--fp32-switch-tol", type=float, default=1e-2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy a 1 GiB device buffer 3 times (a plain copy kernel of known size, "
                         "to scale hardware byte counters)")
    ap.add_argument("--traffic-json", default=None,
                    help="counter summary to read `traffic` from (default profiles/spmm_traffic_<workload>.json)")
    ap.add_argument("--warmstart", default=None,
                    help="trained warm-start parameters (.npy); each step then computes the features, the "
                         "network's start block and the iSVD from it, and the same steps with a Gaussian "
                         "start block are timed for comparison")
    ap.add_argument("--learners", action="store_true",
                    help="time the closed-form learners instead: Eq. 5 embeddings and pair scores on the "
                         "rank-128 SVD of the n = 200,000 NE workload, and the Eq. 8 least-norm model on the "
                         "rank-64 SVD of the n = 170,000 feature-propagation workload (one JSON line)")
    ap.add_argument("--dag", action="store_true",
                    help="time the symbolic form instead: the NE matrix of the n = 200,000 workload built as "
                         "Fig. 1 builds it (leaves A, D^-1 and a ones column), products and one iSVD step, "
                         "with and without the lazy cache, beside the fused operator (one JSON line)")
    ap.add_argument("--ablation", action="store_true",
                    help="Fig. 3-style ablation on the n = 200,000 NE workload: iSVD time to rho <= 1e-4 for "
                         "{Householder QR, Cholesky QR, CholeskyQR2 everywhere} x {fused form, DAG with the lazy "
                         "cache, DAG without it} (one JSON line)")
    ap.add_argument("--pairs", type=int, default=2_000_000)
    ap.add_argument("--label-frac", type=float, default=0.5)
    return ap.parse_args()


def _timed(lib, torch, name, fn, reps):
    """(mean call time, mean kernel time) in s of fn() over reps calls: host
    clock around each call with a device synchronisation, and the library's
    HIP events around the call's kernels on its stream."""
    torch.cuda.synchronize()
    lib.profile_spmm(True)
    t_call = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        t_call += time.perf_counter() - t0
    rec = lib.profile_learners_read()[name]
    lib.profile_spmm(False)
    assert rec[2] == reps, rec
    return t_call / reps, rec[0] / 1e3 / reps, rec[1] / reps


def dag_bench(args, lib, torch, np):
    """Symbolic form (Section 4) on the n = 200,000 NE workload.

    M = sum_j (1/10) t^j - 0.1 (1 1^T - A), t = D^-1 A, built from three
    leaves as in Fig. 1.  Per product pair (M Y and M^T Y, l = 144, FP32):
    device time (library HIP events over the sparse passes plus the host
    clock of the whole pair) and sparse passes, for the fused operator and
    for the DAG operator with and without the lazy cache; then one iSVD step
    to rho <= 1e-4 through the DAG with the cache."""
    import scipy.sparse as sp
    from synth import CONFIGS
    from synth.configs import make_graph

    cfg = CONFIGS["c2"]
    g = make_graph(cfg)
    a = sp.csr_matrix((np.ones(len(g.indices)), g.indices, g.indptr), shape=(g.n, g.n))
    deg = np.diff(a.indptr).astype(np.float64)
    dag = lib.Dag(lib.FP32)
    A = dag.sparse(a.indptr, a.indices, a.shape)
    t = dag.diag(np.where(deg > 0, 1.0 / np.maximum(deg, 1.0), 0.0)) @ A
    one = dag.dense(torch.ones((g.n, 1), dtype=torch.float32, device="cuda"))
    m = dag.sum([t ** j for j in range(1, cfg.K + 1)], cfg.coeffs) - cfg.lam * (one @ one.T - A)
    ops = {"fused": lib.Operator(g, form="ne", coeffs=cfg.coeffs, lam=cfg.lam, precision=lib.FP32),
           "dag_lazy_cache": dag.operator(m, lazy_cache=True),
           "dag_no_cache": dag.operator(m, lazy_cache=False)}
    y = lib.gaussian_block(g.n, cfg.l, seed=1)
    res = {}
    for name, op in ops.items():
        for _ in range(args.warmup):
            op.matmul(op.matmul(y), transpose=True)
        torch.cuda.synchronize()
        lib.profile_spmm(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            op.matmul(op.matmul(y), transpose=True)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        ms, gb, _, launches = lib.profile_spmm_read()
        lib.profile_spmm(False)
        res[name] = {"pair_ms": round(1e3 * wall, 3), "passes_per_pair": launches // args.steps,
                     "spmm_ms_per_pair": round(ms / args.steps, 3),
                     "spmm_gbps": round(gb / (ms / 1e3) / 1e9, 1) if ms > 0 else None}
        print(f"[bench] {name}: {res[name]}", file=sys.stderr, flush=True)
    svd = {}
    for name in ("fused", "dag_lazy_cache"):
        op = ops[name]
        op.truncated_svd(cfg.k, cfg.p, tol=1e-4, max_iter=2000, seed=1000)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, info = op.truncated_svd(cfg.k, cfg.p, tol=1e-4, max_iter=2000, seed=0)
        torch.cuda.synchronize()
        svd[name] = {"s": round(time.perf_counter() - t0, 4), "iterations": info.iterations,
                     "residual": info.residual}
        print(f"[bench] svd {name}: {svd[name]}", file=sys.stderr, flush=True)
    for op in ops.values():
        op.close()
    dag.close()
    line = {
        "metric": "symbolic-form product pair and iSVD step time vs the fused form (Section 4)",
        "value": svd["dag_lazy_cache"]["s"], "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "higher_is_better": False, "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name + "_fig1_dag", "n": g.n, "nnz": int(g.nnz), "K": cfg.K, "l": cfg.l,
                   "products": res, "svd": svd,
                   "lazy_cache_speedup": round(res["dag_no_cache"]["pair_ms"] / res["dag_lazy_cache"]["pair_ms"], 2)},
        "roofline": {"bound": "hbm", "kernel": "spmm_pass_kernel (in the DAG with the cache)",
                     "achieved": res["dag_lazy_cache"]["spmm_gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(res["dag_lazy_cache"]["spmm_gbps"] / HBM_PEAK_GBPS, 4), "traffic": None},
    }
    print(json.dumps(line), flush=True)


def ablation_bench(args, lib, torch, np):
    """Orthonormaliser x product evaluation, one iSVD each to rho <= 1e-4
    (after a one-iteration warm-up of the same configuration), on the
    n = 200,000 NE workload built both ways (fused operator; Fig. 1 DAG)."""
    import scipy.sparse as sp
    from synth import CONFIGS
    from synth.configs import make_graph

    cfg = CONFIGS["c2"]
    g = make_graph(cfg)
    a = sp.csr_matrix((np.ones(len(g.indices)), g.indices, g.indptr), shape=(g.n, g.n))
    deg = np.diff(a.indptr).astype(np.float64)
    dag = lib.Dag(lib.FP32)
    A = dag.sparse(a.indptr, a.indices, a.shape)
    t = dag.diag(np.where(deg > 0, 1.0 / np.maximum(deg, 1.0), 0.0)) @ A
    one = dag.dense(torch.ones((g.n, 1), dtype=torch.float32, device="cuda"))
    m = dag.sum([t ** j for j in range(1, cfg.K + 1)], cfg.coeffs) - cfg.lam * (one @ one.T - A)
    ops = {"fused": lib.Operator(g, form="ne", coeffs=cfg.coeffs, lam=cfg.lam, precision=lib.FP32),
           "dag_lazy_cache": dag.operator(m, lazy_cache=True),
           "dag_no_cache": dag.operator(m, lazy_cache=False)}
    orths = {"householder_qr": dict(orth_method=1), "cholesky_qr": dict(orth_method=0),
             "cholesky_qr2": dict(orth_method=0, orth_passes=2)}
    res = {}
    for pname, op in ops.items():
        for oname, kw in orths.items():
            op.truncated_svd(cfg.k, cfg.p, q=1, seed=1000, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, _, info = op.truncated_svd(cfg.k, cfg.p, tol=1e-4, max_iter=2000, seed=0,
                                             allow_not_converged=True, **kw)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            res[f"{pname}/{oname}"] = {"s": round(sec, 3), "iterations": info.iterations,
                                       "residual": info.residual, "status": info.status}
            print(f"[bench] {pname} / {oname}: {sec:.3f} s, {info.iterations} iterations, "
                  f"rho {info.residual:.2e}", file=sys.stderr, flush=True)
    for op in ops.values():
        op.close()
    dag.close()
    base = res["dag_no_cache/householder_qr"]["s"]
    line = {
        "metric": "iSVD time to rel. residual 1e-4 by orthonormaliser and product evaluation (Fig. 3 ablation)",
        "value": res["fused/cholesky_qr"]["s"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "higher_is_better": False, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": cfg.name + "_ablation", "n": g.n, "k": cfg.k, "p": cfg.p, "runs": res,
                   "ratio_to_no_cache_householder": {k: round(v["s"] / base, 3) for k, v in res.items()}},
    }
    print(json.dumps(line), flush=True)


def learners_bench(args, lib, torch, np):
    """Closed-form learners (Section 3) on resident SVD outputs.

    NE (Eq. 5): U, S, V of the n = 200,000 Chung-Lu NE matrix (k = 128,
    FP32); embeddings L, R and `--pairs` uniform random pair scores.  NC
    (Eq. 8): U, S, V of the n = 170,000 SBM feature-propagation matrix
    (d = 128, L = 3, k = 64, FP32), labels = the 40 planted blocks one-hot,
    `--label-frac` of the rows labelled (option (i)).  `value` sums the
    host-clocked call times (they include each call's synchronisation);
    the roofline takes the library's HIP events around the kernels of the
    call with the longest device time.  Algorithmic bytes:
    embeddings read and write U and V once; a score gathers one row of U
    and of V (+ two int64 indices, one FP64 score); the model reads the
    labelled rows of U and Y once, V once and writes W."""
    from synth import CONFIGS, block_features
    from synth.configs import make_graph

    out = {}
    c2 = CONFIGS["c2"]
    g = make_graph(c2)
    op = lib.Operator(g, form="ne", coeffs=c2.coeffs, lam=c2.lam, self_loops=c2.self_loops, precision=lib.FP32)
    U, S, V, info = op.truncated_svd(c2.k, c2.p, tol=1e-4, max_iter=2000, seed=0)
    op.close()
    n, k = U.shape
    es = 4
    rng = np.random.default_rng(5)
    pi = torch.as_tensor(rng.integers(0, n, args.pairs)).cuda()
    pj = torch.as_tensor(rng.integers(0, n, args.pairs)).cuda()
    for _ in range(args.warmup):
        lib.ne_embeddings(U, S, V)
        lib.ne_scores(U, S, V, pi, pj)
    c_emb, t_emb, b_emb = _timed(lib, torch, "ne_embeddings", lambda: lib.ne_embeddings(U, S, V), args.steps)
    c_sc, t_sc, b_sc = _timed(lib, torch, "ne_scores", lambda: lib.ne_scores(U, S, V, pi, pj), args.steps)
    out["ne_embeddings"] = {"workload": c2.name, "rows": [n, n], "k": k, "call_s": round(c_emb, 6),
                            "s": round(t_emb, 6), "bytes": round(b_emb), "gbps": round(b_emb / t_emb / 1e9, 1)}
    out["ne_scores"] = {"workload": c2.name, "pairs": args.pairs, "k": k, "call_s": round(c_sc, 6),
                        "s": round(t_sc, 6), "bytes": round(b_sc), "gbps": round(b_sc / t_sc / 1e9, 1),
                        "pairs_per_s": round(args.pairs / c_sc)}
    del U, V, pi, pj
    c3 = CONFIGS["c3"]
    g = make_graph(c3)
    x = block_features(g.blocks, c3.d, seed=1000 + c3.index)
    op = lib.Operator(g, form="featprop", X=torch.as_tensor(x).cuda(), L=c3.L, precision=lib.FP32)
    U, S, V, info = op.truncated_svd(c3.k, c3.p, tol=1e-4, max_iter=2000, seed=0)
    op.close()
    ny = int(g.blocks.max()) + 1
    y = np.zeros((g.n, ny), dtype=np.float32)
    y[np.arange(g.n), g.blocks] = 1.0
    Y = torch.as_tensor(y).cuda()
    nl = int(args.label_frac * g.n)
    rows = torch.as_tensor(np.sort(np.random.default_rng(6).choice(g.n, nl, replace=False))).cuda()
    for _ in range(args.warmup):
        lib.nc_fit(U, S, V, Y, rows=rows)
    c_nc, t_nc, b_nc = _timed(lib, torch, "nc_fit", lambda: lib.nc_fit(U, S, V, Y, rows=rows), args.steps)
    kk, d = U.shape[1], V.shape[0]
    out["nc_fit"] = {"workload": c3.name, "labelled_rows": nl, "k": kk, "classes": ny, "d": d,
                     "call_s": round(c_nc, 6), "s": round(t_nc, 6), "bytes": round(b_nc),
                     "gbps": round(b_nc / t_nc / 1e9, 1)}
    dom = max(out, key=lambda key: out[key]["s"])     # longest device time
    line = {
        "metric": "closed-form learner time on resident SVD outputs (Eq. 5 and Eq. 8)",
        "value": round(sum(v["call_s"] for v in out.values()), 6), "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": False, "vs_baseline": None,
        "dtype": "f32 in, f64 sums", "data": "synthetic",
        "config": {"workload": "learners_" + c2.name + "+" + c3.name, **out},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": out[dom]["gbps"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(out[dom]["gbps"] / HBM_PEAK_GBPS, 4), "traffic": None},
    }
    print(json.dumps(line), flush=True)



def host_info():
    """Host cores and CPU model of the machine the oracle runs on."""
    from threadpoolctl import threadpool_info
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"nproc": nproc, "blas_threads": blas, "cpu_model": model}


def infinity_cache_peak():
    """Infinity-Cache read rate measured by `bench.py --peaks` (GB/s), from
    the peaks record in profiles/, else the HBM figure."""
    try:
        with open(os.path.join(ROOT, "profiles", "peaks_mi355x.json")) as fh:
            return float(json.load(fh)["config"]["infinity_cache_read_gbps"])
    except (OSError, ValueError, KeyError):
        return HBM_PEAK_GBPS


def traffic_path(args, workload):
    return args.traffic_json or os.path.join(ROOT, "profiles", f"spmm_traffic_{workload}.json")


def spmm_source_hash():
    import hashlib
    with open(os.path.join(ROOT, "paper_2111_06312_amd", "csrc", "spmm.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def load_traffic(args, workload, storage):
    """Measured bytes per sparse pass over `storage` blocks, or None when no
    counter summary exists for this workload or it was taken on another
    version of the kernel's source."""
    path = traffic_path(args, workload)
    try:
        with open(path) as fh:
            tj = json.load(fh)
    except (OSError, ValueError):
        return None
    if tj.get("workload") != workload or tj.get("spmm_source_sha256_16") != spmm_source_hash():
        return None
    rec = tj.get("passes", {}).get(storage)
    return None if rec is None else rec.get("bytes_per_launch")


def pass_roofline(lib, storage, peak_gbps, bound, args, workload, steps_s):
    """Roofline object of the sparse passes over `storage` blocks recorded
    since profiling was enabled (the record is kept)."""
    ms, gather_b, comp_b, launches = lib.profile_spmm_read_storage(storage)
    if launches == 0:
        return None
    avg_s = ms / 1e3 / launches
    achieved = gather_b / launches / avg_s / 1e9
    name = {lib.FP32: "fp32", lib.BF16: "bf16", lib.FP64: "fp64"}[storage]
    traffic = load_traffic(args, workload, name)
    out = {"bound": bound, "achieved": round(achieved, 1), "peak": peak_gbps, "unit": "GB/s",
           "frac": round(achieved / peak_gbps, 4), "traffic": traffic,
           "kernel": "spmm_pass_kernel", "storage": name, "avg_launch_us": round(avg_s * 1e6, 2),
           "launches": launches, "bytes_per_launch": round(gather_b / launches),
           "compulsory_bytes_per_launch": round(comp_b / launches),
           "compulsory_gbps": round(comp_b / launches / avg_s / 1e9, 1),
           "share_of_steps": round(ms / 1e3 / steps_s, 4) if steps_s > 0 else None}
    if traffic:
        out["traffic_gbps"] = round(traffic / avg_s / 1e9, 1)
        out["traffic_frac"] = round(traffic / avg_s / 1e9 / peak_gbps, 4)
    return out


def subspace_angle(torch, Ua, Ub, k):
    """Largest principal angle (rad) between span(Ua[:, :k]) and span(Ub[:, :k])
    (device tensors; FP64 arithmetic): asin of the 2-norm of the part of Ub
    outside span(Ua), Ua orthonormal."""
    A = Ua[:, :k].double()
    B = Ub[:, :k].double()
    R = B - A @ (A.T @ B)
    w = torch.linalg.eigvalsh(R.T @ R)
    s = float(torch.sqrt(torch.clamp(w[-1], min=0.0)))
    import math
    return math.asin(min(s, 1.0))


def gapped_k(S, k, rel_gap=1e-3):
    """Largest k' <= k whose Ritz gap (s_k' - s_k'+1) / s_k' reaches rel_gap."""
    for kk in range(k, 0, -1):
        if kk == len(S) or (S[kk - 1] - S[kk]) / S[kk - 1] >= rel_gap:
            return kk
    return 1


def cpu_baseline_extrapolated(g, cfg, applies, orths, row_frac=1 / 16):
    """Oracle timing on a bounded sample of a large NE workload: one FP64 sparse
    product T[rows] @ P over a random sample of the rows (scaled by the nnz
    ratio) and one LAPACK Householder QR of a row sample of an n x l block
    (scaled linearly in the rows), scaled to the products and
    orthonormalisations of one GPU step."""
    import numpy as np

    from oracle.graph import adjacency, transition
    from oracle.isvd import orthonorm_qr

    rng = np.random.default_rng(0)
    a = adjacency(g.n, g.indptr, g.indices, add_self_loops=cfg.self_loops)
    t = transition(a)
    rows = np.sort(rng.choice(g.n, max(1, int(g.n * row_frac)), replace=False))
    ts = t[rows]
    p = rng.standard_normal((g.n, cfg.l))
    t0 = time.perf_counter()
    _ = ts @ p
    t_pass = (time.perf_counter() - t0) * t.nnz / max(ts.nnz, 1)
    nq = max(cfg.l, int(g.n * row_frac))
    t0 = time.perf_counter()
    _ = orthonorm_qr(p[:nq])
    t_qr = (time.perf_counter() - t0) * g.n / nq
    passes_per_apply = cfg.K + 1          # K powers of T plus the A product of the lambda term
    total = applies * passes_per_apply * t_pass + orths * t_qr
    h = host_info()
    return {
        "value": round(total, 2), "unit": "s", "cores": h["nproc"], "kind": "oracle", "extrapolated": True,
        "cpu_model": h["cpu_model"], "blas_threads": h["blas_threads"],
        "sample": (f"extrapolated: one FP64 scipy CSR product T[rows] @ P over {len(rows)} sampled rows "
                   f"({ts.nnz} of {t.nnz} stored entries, scaled to {t_pass:.2f} s for the whole T, "
                   f"single-threaded) and one LAPACK QR of {nq} x {cfg.l} (scaled to {t_qr:.2f} s for "
                   f"{g.n} rows, {h['blas_threads']} BLAS threads), scaled by {applies} products x "
                   f"{passes_per_apply} sparse passes and {orths} QRs of the GPU step"),
    }


def oracle_timed(g, cfg, omega_np, x=None, runs=1):
    """The FP64 oracle's Algorithm 1 at fixed q on the given start block (the
    GPU run's, as FP64), whole: every product, Householder QR and the final
    SVD.  Median wall time of `runs` runs and the oracle's singular values
    and left basis."""
    from oracle.isvd import isvd as oracle_isvd
    from oracle.operators import FeatPropDesignMatrix, NEDesignMatrix
    if cfg.form == "featprop":
        m = FeatPropDesignMatrix.from_graph(g, x, cfg.L)
    else:
        m = NEDesignMatrix.from_graph(g, cfg.coeffs, cfg.lam, add_self_loops=cfg.self_loops)
    times, out = [], None
    for _ in range(max(1, runs)):
        t0 = time.perf_counter()
        out = oracle_isvd(m, cfg.k, omega_np, cfg.q)
        times.append(time.perf_counter() - t0)
    return statistics.median(times), out


def peaks_bench(args, lib, torch):
    """Peak rates of this GPU for the rooflines (library kernels, HIP events)."""
    res = {}
    nb = 4 << 30                                  # 4 GiB copy: far beyond every cache
    src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    lib.peak_copy(src, dst, 1)
    ms = lib.peak_copy(src, dst, 5)
    res["hbm_copy_gbps"] = round(2 * 5 * nb / (ms / 1e3) / 1e9, 1)
    res["hbm_copy"] = f"5 copies of {nb >> 20} MiB, read + write bytes counted"
    rd_ms = lib.peak_read(src, 5)
    res["hbm_read_gbps"] = round(5 * nb / (rd_ms / 1e3) / 1e9, 1)
    del src, dst
    ic = 96 << 20                                 # > 8 x 4 MB of L2, < 256 MB Infinity Cache
    buf = torch.ones(ic // 4, dtype=torch.float32, device="cuda")
    lib.peak_read(buf, 5)
    reps = 200
    ms = lib.peak_read(buf, reps)
    res["infinity_cache_read_gbps"] = round(reps * ic / (ms / 1e3) / 1e9, 1)
    res["infinity_cache_read"] = f"{reps} passes over {ic >> 20} MiB in one launch"
    del buf
    for name, prec, iters in (("fp64", lib.FP64, 1000), ("fp32", lib.FP32, 2000)):
        lib.peak_mfma(prec, 20)
        fl, ms = lib.peak_mfma(prec, iters)
        res[f"mfma_{name}_tflops"] = round(fl / (ms / 1e3) / 1e12, 1)
    res["device"] = torch.cuda.get_device_name(0)
    line = {"metric": "device peak rates (roofline denominators)", "value": res["hbm_copy_gbps"],
            "unit": "GB/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": "peaks", **res},
            "datasheet": {"hbm_gbps": HBM_PEAK_GBPS, "mfma_fp64_tflops": 78.6, "mfma_fp32_tflops": 157.3}}
    print(json.dumps(line), flush=True)


def orth_bench(args, lib, torch):
    """`--orth` orthonormalisations (CholeskyQR2: Algorithm 2's Cholesky QR
    run twice, each pass a Gram, a Cholesky and a triangular solve) per block
    storage on an n x l block of the workload's shape, after one warm-up; one
    JSON line with the time per call (HIP events around each call) and the
    orthogonality of the result."""
    from synth import CONFIGS
    cfg = CONFIGS[args.config]
    n, l = cfg.n, cfg.l
    res = {}
    for name, dt in (("fp32", torch.float32), ("bf16", torch.bfloat16)):
        y0 = lib.gaussian_block(n, l, seed=3, dtype=torch.float64)
        y0 = (y0 * torch.logspace(0, 3, l, dtype=torch.float64, device="cuda")[None, :]).to(dt)
        y = y0.clone()
        lib.orthonormalize(y)
        torch.cuda.synchronize()
        ms = 0.0
        for _ in range(args.orth):
            y.copy_(y0)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            lib.orthonormalize(y)
            ev[1].record()
            torch.cuda.synchronize()
            ms += ev[0].elapsed_time(ev[1])
        qd = y.double()
        orth_err = float((qd.T @ qd - torch.eye(l, dtype=torch.float64, device="cuda")).abs().max())
        res[name] = {"ms_per_call": round(ms / args.orth, 3), "orthogonality": orth_err}
        print(f"[bench] orth {name}: {res[name]}", file=sys.stderr, flush=True)
        del y0, y, qd
    line = {"metric": "CholeskyQR2 time per block (two passes of Gram, Cholesky, triangular solve)",
            "value": res["fp32"]["ms_per_call"],
            "unit": "ms", "n_gpus": 1, "steps": args.orth, "higher_is_better": False, "data": "synthetic",
            "config": {"workload": f"{cfg.name}_orth", "n": n, "l": l,
                       "block": "Gaussian columns scaled by 10^(3 j / (l - 1))", **res}}
    print(json.dumps(line), flush=True)


def products_bench(args, lib, torch, np):
    """`--products` pairs (M Y then M^T Y) per block storage on the workload's
    operator, after one warm-up pair; one JSON line with the sparse-pass
    rates.  Short enough to run under hardware counters."""
    from synth import CONFIGS
    from synth.configs import make_graph
    cfg = CONFIGS[args.config]
    g = make_graph(cfg)
    storages = [("fp32", lib.FP32)] + ([("bf16", lib.BF16)] if cfg.form == "ne" else [])
    res = {}
    for name, prec in storages:
        if cfg.form == "featprop":
            from synth import block_features
            X = torch.as_tensor(block_features(g.blocks, cfg.d, seed=1000 + cfg.index)).cuda()
            op = lib.Operator(g, form="featprop", X=X, L=cfg.L, precision=prec)
        else:
            op = lib.Operator(g, form="ne", coeffs=cfg.coeffs, lam=cfg.lam, self_loops=cfg.self_loops,
                              precision=prec)
        y = lib.gaussian_block(op.shape[1], cfg.l, seed=1, dtype=op.dtype)
        op.matmul(op.matmul(y), transpose=True)
        torch.cuda.synchronize()
        print(f"[bench] products {name}: {args.products} pairs", file=sys.stderr, flush=True)
        lib.profile_spmm(True)
        t0 = time.perf_counter()
        for _ in range(args.products):
            op.matmul(op.matmul(y), transpose=True)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.products
        ms, gb, cb, launches = lib.profile_spmm_read()
        lib.profile_spmm(False)
        res[name] = {"pair_ms": round(1e3 * wall, 3), "passes": launches,
                     "avg_pass_us": round(1e3 * ms / max(launches, 1), 2),
                     "bytes_per_launch": round(gb / max(launches, 1)),
                     "gather_gbps": round(gb / (ms / 1e3) / 1e9, 1) if ms > 0 else None}
        print(f"[bench] products {name}: {res[name]}", file=sys.stderr, flush=True)
        op.close()
        del y
    line = {"metric": "sparse-pass rate over product pairs", "value": res["fp32"]["gather_gbps"], "unit": "GB/s",
            "n_gpus": 1, "steps": args.products, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": cfg.name, "n": g.n, "nnz": int(g.nnz), "l": cfg.l, **res}}
    print(json.dumps(line), flush=True)


def traffic_summary(args):
    """Counter files of a `--products N --calibrate-copy` run -> measured bytes
    per sparse pass, per block storage.  The copy kernel's dispatches (known
    bytes) scale each counter to bytes."""
    import csv
    from synth import CONFIGS
    cfg = CONFIGS[args.config]

    def per_dispatch(path, counter):
        vals = {}
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                key = (row.get("Dispatch_Id") or row.get("Correlation_Id"), row["Kernel_Name"])
                vals[key] = vals.get(key, 0.0) + float(row["Counter_Value"])
        return vals

    def split(vals):
        out = {"copy": [], "fp32": [], "bf16": [], "fp64": []}
        for (_, kname), v in vals.items():
            if "peak_copy_kernel" in kname:
                out["copy"].append(v)
            elif "spmm_pass_kernel<isvd::bf16" in kname:
                out["bf16"].append(v)
            elif "spmm_pass_kernel<float" in kname:
                out["fp32"].append(v)
            elif "spmm_pass_kernel<double" in kname:
                out["fp64"].append(v)
        return out

    fetch = split(per_dispatch(args.traffic_from[0], "FETCH_SIZE"))
    write = split(per_dispatch(args.traffic_from[1], "WRITE_SIZE"))
    copy_bytes = 1 << 30
    assert fetch["copy"] and write["copy"], "no copy-kernel dispatches: run with --calibrate-copy"
    f_scale = copy_bytes / (statistics.median(fetch["copy"]) * 1024.0)
    w_scale = copy_bytes / (statistics.median(write["copy"]) * 1024.0)
    passes = {}
    for name in ("fp32", "bf16", "fp64"):
        if not fetch[name]:
            continue
        fk = statistics.mean(fetch[name])
        wk = statistics.mean(write[name]) if write[name] else 0.0
        passes[name] = {"fetch_size_kib_per_dispatch": round(fk, 1), "write_size_kib_per_dispatch": round(wk, 1),
                        "dispatches": len(fetch[name]),
                        "bytes_per_launch": round(fk * 1024.0 * f_scale + wk * 1024.0 * w_scale)}
    out = {"workload": cfg.name, "kernel": "spmm_pass_kernel", "spmm_source_sha256_16": spmm_source_hash(),
           "calibration": f"copy kernel of {copy_bytes} bytes: FETCH_SIZE x {f_scale:.5f}, WRITE_SIZE x {w_scale:.5f}",
           "fetch_scale": round(f_scale, 5), "write_scale": round(w_scale, 5), "passes": passes,
           "note": ("FETCH_SIZE and WRITE_SIZE count the bytes that cross from the L2s to the memory side "
                    "(Infinity Cache and HBM); they do not separate Infinity-Cache hits from HBM reads"),
           "commands": [f"rocprofv3 --pmc {c} --output-format csv -d <dir> -o {args.config} -- "
                        f"python3 bench.py --config {args.config} --products 2 --calibrate-copy"
                        for c in ("FETCH_SIZE", "WRITE_SIZE")] +
                       [f"python3 bench.py --config {args.config} --traffic-from <FETCH_SIZE csv> <WRITE_SIZE csv>"]}
    path = traffic_path(args, cfg.name)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out))


def phase_summary(lib, steps, mean_step_s):
    """Per-step seconds of each phase of Algorithm 1 recorded since profiling
    was enabled (event-timed on the SVD's stream), and the rest of the step."""
    ph = lib.profile_phases_read()
    out = {name: round(ms / 1e3 / max(steps, 1), 4) for name, (ms, _) in ph.items()}
    out["between_phases"] = round(mean_step_s - sum(out.values()), 4)
    out["occurrences_per_step"] = {name: n // max(steps, 1) for name, (_, n) in ph.items()}
    return out


def headline(args, lib, torch, np):
    """The default line: the n = 2,000,000 NE workload with FP32 blocks to
    rho <= tol (`value`), the BF16-storage form beside it, and the errors of
    both against an FP64 run from the same start block at fixed q."""
    from synth import CONFIGS
    from synth.configs import make_graph
    cfg = CONFIGS["c4"]
    t0 = time.perf_counter()
    g = make_graph(cfg)
    print(f"[bench] graph {cfg.name}: n={g.n} nnz={g.nnz} ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    kw = dict(tol=args.tol, max_iter=args.max_iter, check_every=args.check_every)
    mk = lambda prec: lib.Operator(g, form="ne", coeffs=cfg.coeffs, lam=cfg.lam, self_loops=cfg.self_loops,
                                   precision=prec)
    op32 = mk(lib.FP32)
    for w in range(args.warmup):
        _, _, _, info = op32.truncated_svd(cfg.k, cfg.p, seed=1000 + w, allow_not_converged=True, **kw)
        print(f"[bench] warmup {w}: {info.seconds:.3f} s, iterations {info.iterations}, rho {info.residual:.2e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    lib.profile_spmm(True)
    times, infos = [], []
    t_start = time.perf_counter()
    for s_ in range(args.steps):
        ts = time.perf_counter()
        _, _, _, info = op32.truncated_svd(cfg.k, cfg.p, seed=s_, allow_not_converged=True, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        infos.append(info)
        print(f"[bench] step {s_}: {times[-1]:.3f} s, iterations {info.iterations}, applies {info.applies}, "
              f"rho {info.residual:.2e}, status {info.status}, ritz {info.ritz_steps}, fallback {info.used_fallback}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    roof32 = pass_roofline(lib, lib.FP32, HBM_PEAK_GBPS, "hbm", args, cfg.name, total)
    phases32 = phase_summary(lib, len(times), sum(times) / len(times))
    lib.profile_spmm_read()
    lib.profile_spmm(False)

    # BF16 storage with the FP32 finish, same tolerance
    op16 = mk(lib.BF16)
    kw16 = dict(kw, fp32_switch_tol=args.fp32_switch_tol)
    op16.truncated_svd(cfg.k, cfg.p, seed=2000, allow_not_converged=True, **kw16)
    torch.cuda.synchronize()
    lib.profile_spmm(True)
    t16, i16 = [], []
    tb = time.perf_counter()
    for s_ in range(args.bf16_steps):
        ts = time.perf_counter()
        _, _, _, info = op16.truncated_svd(cfg.k, cfg.p, seed=s_, allow_not_converged=True, **kw16)
        torch.cuda.synchronize()
        t16.append(time.perf_counter() - ts)
        i16.append(info)
        print(f"[bench] bf16 step {s_}: {t16[-1]:.3f} s, iterations {info.iterations} "
              f"({info.bf16_iterations} in BF16), rho {info.residual:.2e}, status {info.status}",
              file=sys.stderr, flush=True)
    total16 = time.perf_counter() - tb
    roof16 = pass_roofline(lib, lib.BF16, HBM_PEAK_GBPS, "hbm", args, cfg.name, total16)
    roof16_f = pass_roofline(lib, lib.FP32, HBM_PEAK_GBPS, "hbm", args, cfg.name, total16)
    phases16 = phase_summary(lib, len(t16), sum(t16) / len(t16)) if t16 else None
    lib.profile_spmm_read()
    lib.profile_spmm(False)
    mean32 = sum(times) / len(times)
    mean16 = sum(t16) / len(t16) if t16 else None
    bf16 = {"steps": len(t16), "mean_step_s": round(mean16, 4) if mean16 else None,
            "speedup_vs_fp32": round(mean32 / mean16, 3) if mean16 else None,
            "iterations": [i.iterations for i in i16], "bf16_iterations": [i.bf16_iterations for i in i16],
            "residual": [i.residual for i in i16], "converged": all(i.status == 0 for i in i16),
            "roofline_bf16_passes": roof16, "roofline_fp32_finish_passes": roof16_f, "phases_s": phases16}

    errors = None
    if not args.no_errors:
        # the same start block for all three: FP64 Philox draws, rounded to each storage
        q = args.error_q
        om = lib.gaussian_block(g.n, cfg.l, seed=cfg.omega_seed, dtype=torch.float64)
        op64 = mk(lib.FP64)
        te = time.perf_counter()
        U64, S64, _, _ = op64.truncated_svd(cfg.k, cfg.p, q=q, omega=om)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - te
        op64.close()
        del op64
        s64 = S64.cpu().numpy()
        kk = gapped_k(s64, cfg.k)
        errors = {"q": q, "start_block": f"Philox N(0,1) seed {cfg.omega_seed}, FP64, rounded per storage",
                  "fp64_s": round(t64, 3), "k_gapped": kk}
        for name, op, dt in (("fp32", op32, torch.float32), ("bf16", op16, torch.bfloat16)):
            U, S, _, _ = op.truncated_svd(cfg.k, cfg.p, q=q, omega=om.to(dt))
            s = S.cpu().numpy()
            errors[name] = {"sigma_max_rel_err": float(np.max(np.abs(s - s64) / s64)),
                            "subspace_angle_rad": subspace_angle(torch, U64, U, kk)}
            del U
            print(f"[bench] error run {name}: {errors[name]}", file=sys.stderr, flush=True)
        del U64, om
        # at the tolerance: each storage's own run to rho <= tol (BF16 with its FP32
        # finish) against an FP64 run to rho <= tol, all from the same seed's draws
        op64 = mk(lib.FP64)
        te = time.perf_counter()
        U64, S64, _, i64 = op64.truncated_svd(cfg.k, cfg.p, seed=7, allow_not_converged=True, **kw)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - te
        op64.close()
        del op64
        s64 = S64.cpu().numpy()
        kk = gapped_k(s64, cfg.k)
        at_tol = {"seed": 7, "fp64_s": round(t64, 3), "fp64_iterations": i64.iterations,
                  "fp64_residual": i64.residual, "k_gapped": kk}
        for name, op, kwx in (("fp32", op32, kw), ("bf16", op16, kw16)):
            U, S, _, inf = op.truncated_svd(cfg.k, cfg.p, seed=7, allow_not_converged=True, **kwx)
            s = S.cpu().numpy()
            at_tol[name] = {"sigma_max_rel_err": float(np.max(np.abs(s - s64) / s64)),
                            "subspace_angle_rad": subspace_angle(torch, U64, U, kk),
                            "iterations": inf.iterations, "residual": inf.residual}
            del U
            print(f"[bench] error run at tol {name}: {at_tol[name]}", file=sys.stderr, flush=True)
        errors["at_tolerance"] = at_tol
        del U64
    op16.close()

    converged = all(i.status == 0 for i in infos)
    line = {
        "metric": "rank-k iSVD wall time at rel. residual 1e-4; SpMM achieved HBM GB/s vs peak",
        "value": round(total / args.steps, 4), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * total / args.steps, 2), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": cfg.name, "n": g.n, "nnz": int(g.nnz), "k": cfg.k, "p": cfg.p, "K": cfg.K,
                   "lambda": cfg.lam, "tol": args.tol, "csr": "int64 offsets, int32 column ids, unit values "
                   "(A is 0/1; D^-1 applied as an FP32 row scale)",
                   "iterations": [i.iterations for i in infos], "applies": [i.applies for i in infos],
                   "residual": [i.residual for i in infos], "converged": converged,
                   "median_step_s": round(statistics.median(times), 4), "start_block": "gaussian",
                   "phases_s": phases32, "bf16_storage": bf16, "errors_vs_fp64": errors},
        "roofline": roof32,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        last = infos[-1]
        line["cpu_baseline"] = cpu_baseline_extrapolated(g, cfg, last.applies, last.applies)
    op32.close()
    print(json.dumps(line), flush=True)


def start_study(args, lib, torch, np):
    """Which start blocks save power iterations on the warm-start workload
    (n = 1,000,000 Chung-Lu, K = 10, lambda = 0.1, k = 128, p = 16)?  Each
    start block is passed to the SVD as `omega`; iterations to rho <= tol.
    V_k comes from a converged run from another seed.  One JSON line."""
    import math
    import scipy.sparse as sp
    from synth import CONFIGS
    from synth.configs import make_graph
    cfg = CONFIGS["c5"]
    g = make_graph(cfg)
    op = lib.Operator(g, form="ne", coeffs=cfg.coeffs, lam=cfg.lam, precision=lib.FP32)
    k, p, l, n = cfg.k, cfg.p, cfg.l, g.n
    kw = dict(tol=args.tol, max_iter=args.max_iter, allow_not_converged=True)
    res = {}

    def run(name, om):
        _, _, _, info = op.truncated_svd(k, p, omega=om.contiguous(), **kw)
        res.setdefault(name, []).append(info.iterations)
        print(f"[bench] start study: {name}: {info.iterations} iterations, rho {info.residual:.2e}",
              file=sys.stderr, flush=True)

    gen = torch.Generator(device="cuda")

    def gauss(cols, seed):
        gen.manual_seed(seed)
        return torch.randn((n, cols), generator=gen, device="cuda", dtype=torch.float32)

    _, _, V, _ = op.truncated_svd(k, p, seed=77, **kw)
    V = V.contiguous()
    sq = math.sqrt(n)            # columns scaled to the norm of the Gaussian ones
    lev = (V.double() ** 2).sum(1)
    deg = torch.as_tensor(np.diff(g.indptr).astype(np.float64), device="cuda")
    a = sp.csr_matrix((np.ones(len(g.indices)), g.indices, g.indptr), shape=(n, n))
    dd = np.maximum(np.diff(g.indptr), 1).astype(np.float64)
    tcol = torch.as_tensor(np.sqrt(a.T @ (1.0 / dd ** 2)), device="cuda")
    for s_ in range(2):
        run("gaussian", gauss(l, 1000 + s_))
    run("exact V_k + gaussian p", torch.cat([V * sq, gauss(p, 2000)], 1))
    for eps in (0.3, 1.0, 3.0):
        run(f"V_k + noise {eps}", torch.cat([(V + eps * gauss(k, 3000) / sq) * sq, gauss(p, 2000)], 1))
    for k0 in (16, 32, 64, 96, 112, 120):
        run(f"exact top {k0} + gaussian", torch.cat([V[:, :k0] * sq, gauss(l - k0, 11 + k0)], 1))
    for k0 in (64, 96):
        run(f"exact v_{k0 + 1}..v_{k} + gaussian", torch.cat([V[:, k0:] * sq, gauss(l - (k - k0), 21 + k0)], 1))
    for sname, score in (("leverage", lev), ("T column norm", tcol), ("degree", deg)):
        order = torch.argsort(score, descending=True)
        for H in (256, 1024, 4096, 16384):
            mask = torch.zeros(n, device="cuda", dtype=torch.float32)
            mask[order[:H]] = 1.0
            run(f"gaussian on the top {H} rows by {sname}",
                torch.cat([mask[:, None] * gauss(k, 7000 + H), gauss(p, 8000)], 1))
    run("gaussian weighted by sqrt(leverage)", torch.sqrt(lev + 1e-3 * lev.mean()).float()[:, None] * gauss(l, 4000))
    for a_ in (0.25, 0.5, 1.0):
        run(f"gaussian weighted by degree^{a_}", (deg + 1.0).pow(a_).float()[:, None] * gauss(l, 5000))
    try:
        ws = lib.WarmStart(k, seed=0)
        ws.set_params(np.load(os.path.join(ROOT, "paper_2111_06312_amd", "weights", "warmstart_k128.npy")))
        F = lib.features(op)
        Z = ws.forward(F)
        Zq, _ = lib.orthonormalize(Z.clone())
        sv = torch.linalg.svdvals(V.double().T @ Zq.double())
        span = float((sv ** 2).mean())
        for s_ in range(3):
            om, fb = ws.omega(op, F, p, seed=s_)
            run("learned (orthonormalised)", om)
        ws.close()
    except (OSError, ValueError):
        span = None
    op.close()
    pr = 1.0 / (V.double() ** 4).sum(0)
    order = torch.argsort(deg, descending=True)
    line = {"metric": "power iterations to rel. residual 1e-4 by start block", "value": res["gaussian"][0],
            "unit": "iterations", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
            "config": {"workload": cfg.name + "_start_study", "n": n, "k": k, "p": p, "tol": args.tol,
                       "iterations": res,
                       "leverage_on_top_0.1pct_by_degree": round(float(lev[order[: n // 1000]].sum()) / k, 3),
                       "participation_ratio_median": round(float(pr.median()), 1),
                       "learned_mean_cos2_to_Vk": span}}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU sharding of this path is a design note, not a measured configuration.",
              file=sys.stderr)
        sys.exit(2)
    if args.traffic_from:
        traffic_summary(args)
        return
    import numpy as np
    import torch

    from paper_2111_06312_amd import isvd as lib
    from synth import CONFIGS
    from synth.configs import make_graph

    lib.load()
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        lib.peak_copy(src, dst, 3)
        print("[bench] calibration copies: 3 x 1 GiB by the library's copy kernel", file=sys.stderr, flush=True)
        del src, dst
    if args.peaks:
        peaks_bench(args, lib, torch)
        return
    if args.products:
        products_bench(args, lib, torch, np)
        return
    if args.orth:
        orth_bench(args, lib, torch)
        return
    if args.start_study:
        start_study(args, lib, torch, np)
        return
    if args.learners:
        learners_bench(args, lib, torch, np)
        return
    if args.dag:
        dag_bench(args, lib, torch, np)
        return
    if args.ablation:
        ablation_bench(args, lib, torch, np)
        return
    if args.config == "c4" and args.precision is None and not args.warmstart:
        headline(args, lib, torch, np)
        return
    cfg = CONFIGS[args.config]
    prec_name = args.precision or ("bf16" if cfg.precision == "bf16" else "fp32")
    precision = lib.BF16 if prec_name == "bf16" else lib.FP32
    t0 = time.perf_counter()
    g = make_graph(cfg)
    print(f"[bench] graph {cfg.name}: n={g.n} nnz={g.nnz} ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    X = x_np = None
    if cfg.form == "featprop":
        from synth import block_features
        x_np = block_features(g.blocks, cfg.d, seed=1000 + cfg.index)
        X = torch.as_tensor(x_np).cuda()
        op = lib.Operator(g, form="featprop", X=X, L=cfg.L, precision=precision)
    else:
        op = lib.Operator(g, form="ne", coeffs=cfg.coeffs, lam=cfg.lam, self_loops=cfg.self_loops,
                          precision=precision)
    kw = dict(tol=args.tol, max_iter=args.max_iter, check_every=args.check_every,
              fp32_switch_tol=args.fp32_switch_tol if precision == lib.BF16 else 0.0)
    ws = None
    if args.warmstart:
        ws = lib.WarmStart(cfg.k, seed=0)
        ws.set_params(np.load(args.warmstart))

    def one_step(seed, warm):
        if warm:
            F = lib.features(op)
            om, fb = ws.omega(op, F, cfg.p, seed=seed)
            out = op.truncated_svd(cfg.k, cfg.p, omega=om, allow_not_converged=True, **kw)
            return out[3], fb
        return op.truncated_svd(cfg.k, cfg.p, seed=seed, allow_not_converged=True, **kw)[3], False

    gauss = None
    if ws is not None:
        # the Gaussian-start comparison: same seeds, same tolerance
        g_times, g_its = [], []
        for s_ in range(args.steps):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            info, _ = one_step(s_, False)
            torch.cuda.synchronize()
            g_times.append(time.perf_counter() - ts)
            g_its.append(info.iterations)
            print(f"[bench] gaussian start {s_}: {g_times[-1]:.3f} s, iterations {info.iterations}, "
                  f"rho {info.residual:.2e}", file=sys.stderr, flush=True)
        gauss = {"mean_s": round(sum(g_times) / len(g_times), 4), "iterations": g_its}
    infos = []
    for w in range(args.warmup):
        _, S, _, info = op.truncated_svd(cfg.k, cfg.p, seed=1000 + w, allow_not_converged=True, **kw)
        print(f"[bench] warmup {w}: {info.seconds:.3f} s, iterations {info.iterations}, rho {info.residual:.2e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    lib.profile_spmm(True)
    times = []
    t_start = time.perf_counter()
    fallbacks = 0
    for s in range(args.steps):
        ts = time.perf_counter()
        info, fb = one_step(s, ws is not None)
        fallbacks += int(fb)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        infos.append(info)
        print(f"[bench] step {s}: {times[-1]:.3f} s, iterations {info.iterations}, applies {info.applies}, "
              f"rho {info.residual:.2e}, status {info.status}, ritz {info.ritz_steps}, sweeps {info.jacobi_sweeps}, "
              f"bf16 iterations {info.bf16_iterations}, fallback {info.used_fallback}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    # blocks of n x l beyond the 256 MB Infinity Cache: rows come from HBM
    block_bytes = g.n * cfg.l * (2 if precision == lib.BF16 else 4)
    in_cache = block_bytes < 200e6
    peak = HBM_PEAK_GBPS
    bound = "hbm"
    if in_cache:
        bound = "infinity-cache"
        peak = infinity_cache_peak()
    roof = pass_roofline(lib, precision, peak, bound, args, cfg.name, total)
    phases = phase_summary(lib, len(times), sum(times) / len(times))
    lib.profile_spmm_read()
    lib.profile_spmm(False)
    ms_per_step = 1e3 * total / args.steps
    converged = all(i.status == 0 for i in infos)
    line = {
        "metric": "rank-k iSVD wall time at rel. residual 1e-4; SpMM achieved HBM GB/s vs peak",
        "value": round(ms_per_step / 1e3, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32" if precision == lib.BF16 else "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "n": g.n, "nnz": int(g.nnz), "k": cfg.k, "p": cfg.p,
                   **({"d": cfg.d, "L": cfg.L} if cfg.form == "featprop" else {"K": cfg.K, "lambda": cfg.lam}),
                   "tol": args.tol,
                   "iterations": [i.iterations for i in infos], "applies": [i.applies for i in infos],
                   **({"bf16_iterations": [i.bf16_iterations for i in infos]} if precision == lib.BF16 else {}),
                   "residual": [i.residual for i in infos], "converged": converged,
                   "median_step_s": round(statistics.median(times), 4), "phases_s": phases,
                   "start_block": "learned warm start" if ws is not None else "gaussian",
                   **({"gaussian_start": gauss, "warmstart_fallbacks": fallbacks,
                       "warmstart_weights": os.path.relpath(args.warmstart, ROOT)} if ws is not None else {})},
        "roofline": roof,
    }
    if not args.no_cpu_baseline and args.config in ("c2", "c3") and args.oracle_runs > 0 and ws is None:
        # the oracle run whole (Algorithm 1, Householder QR) at fixed q on the start block of a
        # fixed-q GPU run, both timed; errors of the GPU result against it
        om = lib.gaussian_block(op.shape[1], cfg.l, seed=cfg.omega_seed, dtype=torch.float64)
        om_np = om.cpu().numpy()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        U, S, _, ginfo = op.truncated_svd(cfg.k, cfg.p, q=cfg.q, omega=om.to(op.dtype))
        torch.cuda.synchronize()
        tg = time.perf_counter() - tg
        print(f"[bench] timing the CPU oracle: {args.oracle_runs} run(s) at q = {cfg.q}", file=sys.stderr,
              flush=True)
        t_or, (uo, so, _) = oracle_timed(g, cfg, om_np, x=x_np, runs=args.oracle_runs)
        s = S.cpu().numpy()
        kk = gapped_k(so, cfg.k)
        h = host_info()
        line["cpu_baseline"] = {
            "value": round(t_or, 2), "unit": "s", "cores": h["nproc"], "kind": "oracle", "extrapolated": False,
            "cpu_model": h["cpu_model"], "blas_threads": h["blas_threads"],
            "sample": (f"the whole FP64 oracle (Algorithm 1 with Householder QR, LAPACK SVD) at fixed q = {cfg.q} "
                       f"on the start block of a fixed-q GPU run (Philox seed {cfg.omega_seed}), median of "
                       f"{args.oracle_runs}; the GPU's tolerance-mode steps run about "
                       f"{infos[-1].iterations / max(cfg.q, 1):.0f} times as many iterations"),
            "gpu_fixed_q_s": round(tg, 4),
            "speedup_fixed_q": round(t_or / tg, 1),
            "sigma_max_rel_err": float(np.max(np.abs(s - so) / so)),
            "subspace_angle_rad": subspace_angle(torch, torch.as_tensor(uo, device="cuda"), U, kk),
            "k_gapped": kk,
        }
    elif not args.no_cpu_baseline and cfg.form == "ne":
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        last = infos[-1]
        line["cpu_baseline"] = cpu_baseline_extrapolated(g, cfg, last.applies, last.applies)
    op.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
