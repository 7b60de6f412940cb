"""Benchmark: Helmholtz solves/s to relative residual 1e-8 on one MI355X.

Default workload: P1 h = 1/256 (65,025 dofs), k = 80, lognormal coefficient, 16 x 16 subdomains,
FGMRES(150) (the mixed-precision configuration).  A step is one pass of the whole hot path for one
right-hand side with its inputs resident in device memory: the numeric setup (local blocks, local
H_k-GenEO eigenproblems, coarse space, coarse and local factors; hkgeneo_factor) followed by the
FGMRES solve.  The host analysis (partition, index sets, uploads) runs once before the timed
region.  Forms, each timed over the same steps:

  * mixed  - float32 local inverses (formed in float64) inside float64 FGMRES, solved by the
             batched engine (hkgeneo_batch_solve: graph-captured iteration).  This is `value`.
  * fp64   - everything in float64, same batched engine.
  * plain  - everything in float64, single-problem path (hkgeneo_gmres_solve).
  * pou    - the mixed form with the partition-of-unity weighted local prolongation (W_D = Xi_D).

The mixed form's timed region runs with the engine's measurement hook on: HIP events around every
batched local-solve launch on the engine's stream give the roofline of that kernel (the hook
launches the iteration directly instead of replaying its graph; the unprofiled step time is
reported beside it).  `iteration_roofline` prices the whole FGMRES iteration: the method's
algorithmic bytes per iteration times the iterations, over the solve time.  The line also carries
solve-only latency percentiles (factors resident), an 8-right-hand-side solve-only throughput, the
relative error of every form's solution against the float64 oracle's FGMRES solution, and the
oracle itself timed on the host cores (one full setup + solve).

Other workloads: --workload p1_h128_k40_8x8 (and the other named ones), --workload mix64 (64
independent problems in one batch, setup timed apart) and --workload serve (Poisson request stream
through the continuous-batching server).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--cpu-sample N]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Helmholtz solves/s to rel.res 1e-8 (mixed vs FP64); p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def local_solve_bytes(nI: np.ndarray, m: np.ndarray, word: int, nrhs: int = 1) -> int:
    """Algorithmic bytes of one batched local-solve launch: the local inverses (sum n_D^2 words, read
    once whatever nrhs), and per right-hand side the gathered residual entries with their indices,
    the weights, the output, and the coarse restriction fused into the same launch (Z_i^T: sum n_D m_i
    doubles read, m0 outputs written)."""
    s = int(nI.sum())
    nI64 = nI.astype(np.int64)
    per_rhs = s * (8 + 4) + s * 8 + s * 8 + 8 * int(m.sum())
    return int(word * int((nI64 ** 2).sum()) + 8 * int((nI64 * m.astype(np.int64)).sum()) + nrhs * per_rhs)


def iteration_bytes(n, nnz, nI, m, m0, word, j_mean):
    """Algorithmic bytes of one FGMRES iteration for one right-hand side (every term the method needs):
    local inverses (sum n_D^2 words), the coarse basis read twice (restriction Z^T r and prolongation
    Z y), the dense inverse of B_0, the CSR product, the gathers and scatters of the local vectors,
    classical Gram-Schmidt twice against the j current basis vectors, and the new z_j, v_{j+1}."""
    nI64 = nI.astype(np.int64)
    s = int(nI64.sum())
    return int(word * int((nI64 ** 2).sum()) + 16 * int((nI64 * m.astype(np.int64)).sum()) + 8 * m0 * m0
               + 12 * nnz + 20 * n + 24 * s + 8 * n + 32 * j_mean * n + 24 * n)


def progress(msg):
    """Progress of the longer workloads on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def sync():
    import torch
    torch.cuda.synchronize()


def timed_steps(S, solve, steps, warmup):
    """warmup + `steps` timed (factor, solve) passes; returns per-step lists."""
    for _ in range(warmup):
        S.factor()
        solve()
    sync()
    fac, sol, it, rel = [], [], [], []
    u = None
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        S.factor()
        b = time.perf_counter()
        info, u = solve()
        c = time.perf_counter()
        fac.append(1e3 * (b - a))
        sol.append(1e3 * (c - b))
        it.append(info["iters"])
        rel.append(info["relres_true"])
    sync()
    return dict(total_s=time.perf_counter() - t0, fac_ms=fac, sol_ms=sol, iters=it, relres=rel,
                u=u.cpu().numpy().ravel() if u is not None else None)


def kernel_source_hash() -> str:
    """sha256 of the batched kernels' source (the traffic figures below belong to one version)."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2406_06283_amd", "csrc", "batch.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def recorded_traffic(workload: str):
    """HBM bytes per local-solve launch from the committed counter summary of this workload, if it
    was taken on the current kernel source; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"traffic_k_b_local_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for ln in fh:
            if ln.startswith("- ") and ":" in ln:
                k, v = ln[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel source sha256") != kernel_source_hash():
        return None
    try:
        return int(vals["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def calibrate_copy(nbytes: int):
    """An elementwise copy of nbytes (read once, written once) for counter calibration."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    evict = torch.zeros(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB: pushes a out of L2 and MALL
    evict += 1.0
    torch.mul(a, 1.0, out=b)
    sync()
    progress(f"calibration copy: {nbytes} bytes read and written by one elementwise kernel")


def latency(solve, n):
    lat = []
    for _ in range(n):
        a = time.perf_counter()
        solve()
        lat.append(1e3 * (time.perf_counter() - a))
    return lat


def run_default(args, w, p):
    import torch
    from paper_2406_06283_amd import hkgeneo as H
    dev = torch.device("cuda:0")
    f = torch.from_numpy(p.f).to(dev)
    p8 = w.problem(seed=0, nrhs=8)
    f8 = torch.from_numpy(p8.f).to(dev)
    out = {}
    forms = args.forms.split(",") + ["mixed"]
    # plain float64 single-problem path
    if "plain" in forms:
        S = H.Solver(p, H.options_for(w, keep_workspace=1))

        def solve_plain():
            u, info, _ = S.solve(f)
            return info[0], u
        r = timed_steps(S, solve_plain, args.steps, args.warmup)
        r["lat"] = latency(lambda: S.solve(f), max(args.steps, args.lat_reps))
        r["lat8"] = latency(lambda: S.solve(f8), max(1, args.lat_reps // 4))
        r["m0"] = S.stats()["m0"]
        out["plain"] = r
        S.close()
    # batched engine, float64 and mixed
    for tag, prec, prolong in (("fp64", 64, H.HKG_PROLONG_AS), ("mixed", 32, H.HKG_PROLONG_AS),
                               ("pou", 32, H.HKG_PROLONG_POU)):
        if tag not in forms:
            continue
        S = H.Solver(p, H.options_for(w, local_prec=prec, prolong=prolong, keep_workspace=1))
        B = H.Batch([S], [1])
        B8 = H.Batch([S], [8])

        def solve():
            (u,), (info,), _ = B.solve([f])
            return info[0], u
        r = timed_steps(S, solve, args.steps, args.warmup)       # graph replay
        if tag == "mixed":
            B.profile(True)
            rp = timed_steps(S, solve, args.steps, 0)             # measurement hook on
            local_ms, launches = B.profile_read()
            B.profile(False)
            rp["local_ms"], rp["launches"], rp["waves"] = local_ms, launches, B.local_waves
            r["profiled"] = rp
            nI, _, m = S.subdomains()
            r["nI"], r["m"] = nI, m
        r["lat"] = latency(lambda: B.solve([f]), max(args.steps, args.lat_reps))
        r["lat8"] = latency(lambda: B8.solve([f8]), max(1, args.lat_reps // 4))
        r["m0"] = S.stats()["m0"]
        out[tag] = r
        B.close()
        B8.close()
        S.close()
    return out


def run_in_flight(w, n_flight: int, steps: int, warmup: int):
    """Independent problems of the same workload (seeds 0 .. n_flight-1) stepped concurrently, one host
    thread and one stream each: whole-device throughput when setups and solves of different problems
    overlap (each problem uses a fraction of the CUs in its latency-bound setup phases)."""
    import threading
    import torch
    from paper_2406_06283_amd import hkgeneo as H
    res, errs = {}, []
    bar = threading.Barrier(n_flight)

    def worker(seed):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                p = w.problem(seed=seed)
                f = torch.from_numpy(p.f).to("cuda:0")
                S = H.Solver(p, H.options_for(w, local_prec=32, keep_workspace=1))
                B = H.Batch([S], [1])
                for _ in range(warmup):
                    S.factor()
                    B.solve([f])
                st.synchronize()
                bar.wait()
                t0 = time.perf_counter()
                infos = []
                for _ in range(steps):
                    S.factor()
                    infos.append(B.solve([f])[1][0][0])
                st.synchronize()
                res[seed] = (time.perf_counter() - t0, infos)
                bar.wait()
                B.close()
                S.close()
        except Exception as e:      # reported below
            errs.append(repr(e))
            bar.abort()

    th = [threading.Thread(target=worker, args=(sd,)) for sd in range(n_flight)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    if errs or len(res) != n_flight:
        return {"error": errs[:1]}
    wall = max(v[0] for v in res.values())
    infos = [i for v in res.values() for i in v[1]]
    return {"in_flight": n_flight, "seeds": list(range(n_flight)), "steps_per_problem": steps,
            "steps_per_s": round(n_flight * steps / wall, 3),
            "converged": all(i["converged"] and i["relres_true"] <= 1e-8 for i in infos),
            "iters": [int(v[1][0]["iters"]) for _, v in sorted(res.items())]}


def run_cpu_baseline(w, p, sample: int):
    from oracle import fgmres, local, schwarz
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    opts = schwarz.Options(eig_mode=local.EIG_FIXED if w.eig_mode == 1 else local.EIG_THRESHOLD, nev=w.nev, tau=w.tau)
    t0 = time.perf_counter()
    iters = []
    x = None
    for _ in range(sample):
        M = schwarz.TwoLevelSchwarz(p, opts)
        x, info = fgmres.solve(p, M, restart=w.restart)
        iters.append(info["iters"])
    dt = time.perf_counter() - t0
    return dict(value=sample / dt, unit="solves/s", cores=int(threads), kind="oracle",
                sample=f"{sample} full solve(s) (setup + FGMRES) of {w.name} seed 0 on the host, "
                       f"{dt:.1f} s, {iters[0]} iterations", iters=iters[0], x=x)


def summary(r, steps):
    return {"steps_per_s": round(steps / r["total_s"], 3), "ms_per_step": round(1e3 * r["total_s"] / steps, 3),
            "iters": int(np.median(r["iters"])), "relres_max": max(r["relres"]),
            "factor_ms_p50": round(pct(r["fac_ms"], 50), 3), "solve_ms_p50": round(pct(r["sol_ms"], 50), 3),
            "solve_only_p50_ms": round(pct(r["lat"], 50), 3), "solve_only_p99_ms": round(pct(r["lat"], 99), 3),
            "rhs8_solves_per_s": round(8e3 / np.median(r["lat8"]), 1)}


def oracle_error(r, x):
    """relative error of a form's last solution against the float64 oracle's FGMRES solution"""
    if r is None or x is None or r.get("u") is None:
        return None
    return float(np.linalg.norm(r["u"] - x) / np.linalg.norm(x))


def run_next_rows(args, w):
    """The widened rows on the default workload, single-problem path, float64 local inverses:
    the nested decomposition (fine element blocks of half the coarse width, one fine overlap layer),
    GMRES on the left-preconditioned system in the D_k inner product, and the Delta-GenEO coarse
    space.  Per row: steps/s of (factor + solve), iterations, true residual, solve-only p50."""
    import torch
    from paper_2406_06283_amd import hkgeneo as H
    dev = torch.device("cuda:0")
    fine = 2 * w.s
    rows = {
        "nested": (w.problem(seed=0, fine=fine, fine_overlap=1), {},
                   f"nested decomposition: coarse {w.s}^{w.dim} subdomains (eigenproblems, B_0), fine pieces cut "
                   f"by {fine}^{w.dim} element blocks inside each and grown by 1 layer (local solves)"),
        "dk_gmres": (None, dict(krylov=H.HKG_KRYLOV_LEFT_DK),
                     "GMRES on M^-1 B u = M^-1 f in the D_k inner product, stopped on the preconditioned D_k norm"),
        "delta_geneo": (None, dict(coarse_op=H.HKG_COARSE_DELTA),
                        "Delta-GenEO coarse space (k = 0 eigenproblem, same tau), B_0 at the actual k"),
    }
    out = {}
    for name, (prob, kw, what) in rows.items():
        progress(f"next row {name}")
        p = prob if prob is not None else w.problem(seed=0)
        f = torch.from_numpy(p.f).to(dev)
        S = H.Solver(p, H.options_for(w, keep_workspace=1, **kw))

        def solve():
            u, info, _ = S.solve(f)
            return info[0], u
        r = timed_steps(S, solve, args.steps, args.warmup)
        r["lat"] = latency(lambda: S.solve(f), max(args.steps, args.lat_reps // 2))
        st = S.stats()
        own, nI, lam = S.fine()
        _, info, _ = S.solve(f)
        out[name] = {"what": what, "steps_per_s": round(args.steps / r["total_s"], 3),
                     "factor_ms_p50": round(pct(r["fac_ms"], 50), 3), "solve_ms_p50": round(pct(r["sol_ms"], 50), 3),
                     "solve_only_p50_ms": round(pct(r["lat"], 50), 3), "iters": int(np.median(r["iters"])),
                     "relres_true_max": max(r["relres"]), "relres_est": info[0]["relres_est"],
                     "converged": bool(info[0]["converged"]), "m0": int(st["m0"]),
                     "local_subdomains": int(len(nI)), "mean_local_dofs": round(float(np.mean(nI)), 1),
                     "lambda": int(lam), "device_mb": round(st["device_bytes"] / 2 ** 20, 1)}
        S.close()
    return out


def side_workload(args, name):
    """The mixed form of another named workload (steps/s, iterations, solve-only latency)."""
    import argparse as _ap
    from paper_2406_06283_amd.configs import WORKLOADS
    w = WORKLOADS[name]
    a = _ap.Namespace(**vars(args))
    a.forms = "mixed"
    r = run_default(a, w, w.problem(seed=0))["mixed"]
    out = summary(r, args.steps)
    out["profiled_steps_per_s"] = round(args.steps / r["profiled"]["total_s"], 3)
    out["m0"] = int(r["m0"])
    return out


def main_default(args):
    from paper_2406_06283_amd.configs import WORKLOADS
    w = WORKLOADS[args.workload]
    p = w.problem(seed=0)
    progress(f"{w.name}: forms {args.forms}")
    r = run_default(args, w, p)
    mx, f64, plain, pou = r["mixed"], r.get("fp64"), r.get("plain"), r.get("pou")
    rp = mx["profiled"]
    ref = plain or f64          # float64 iteration count the mixed form must stay within 2 of
    ok = all(x <= 1e-8 for x in rp["relres"]) and (
        ref is None or abs(int(np.median(rp["iters"])) - int(np.median(ref["iters"]))) <= 2)
    word = 4
    bpl = local_solve_bytes(mx["nI"], mx["m"], word)
    avg_s = rp["local_ms"] / max(rp["launches"], 1) / 1e3
    achieved = bpl / avg_s / 1e9
    iters = int(np.median(mx["iters"]))
    j_mean = (iters - 1) / 2.0 if iters <= w.restart else (w.restart - 1) / 2.0
    ibytes = iteration_bytes(p.n_dof, p.nnz, mx["nI"], mx["m"], int(mx["m0"]), word, j_mean)
    solve_s = pct(mx["lat"], 50) / 1e3
    it_achieved = ibytes * iters / solve_s / 1e9
    line = {
        "metric": METRIC,
        "value": round(args.steps / rp["total_s"], 3) if ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * rp["total_s"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (f32 local inverses)",
        "data": "synthetic",
        "config": {"workload": w.name, "n_dof": p.n_dof, "n_sub": p.n_sub, "k": w.k,
                   "eig": "tau=%g" % w.tau if w.eig_mode == 0 else "nev=%d" % w.nev, "m0": int(mx["m0"]), "nrhs": 1,
                   "restart": w.restart, "rtol": 1e-8,
                   "step": "numeric setup + FGMRES solve (batched engine, mixed precision), inputs resident"},
        "iters": int(np.median(rp["iters"])),
        "relres_max": max(rp["relres"]),
        "factor_ms_p50": round(pct(rp["fac_ms"], 50), 3),
        "solve_ms_p50": round(pct(rp["sol_ms"], 50), 3),
        "solve_only": {"p50_ms": round(pct(mx["lat"], 50), 3), "p99_ms": round(pct(mx["lat"], 99), 3),
                       "solves_per_s": round(1e3 / np.mean(mx["lat"]), 2)},
        "unprofiled_graph_replay": summary(mx, args.steps),
        "independent_problems_in_flight": run_in_flight(w, args.in_flight, args.steps, args.warmup)
        if args.in_flight > 1 else None,
        "fp64_batched": summary(f64, args.steps) if f64 else None,
        "fp64_plain": summary(plain, args.steps) if plain else None,
        "pou_mixed": summary(pou, args.steps) if pou else None,
        "roofline": {"kernel": "k_b_local<%d> (float32 inverses)" % rp["waves"], "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(w.name),
                     "bytes_per_launch": bpl,
                     "avg_launch_us": round(avg_s * 1e6, 3), "launches": int(rp["launches"])},
        "iteration_roofline": {"bound": "hbm", "achieved": round(it_achieved, 1), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": round(it_achieved / HBM_PEAK_GBS, 4),
                               "bytes_per_iteration": ibytes, "iterations": iters, "j_mean": j_mean,
                               "solve_only_p50_ms": round(solve_s * 1e3, 3)},
    }
    if not args.no_next_rows:
        line["next_rows"] = run_next_rows(args, w)
    for extra in [x for x in args.extra_workloads.split(",") if x and x != w.name]:
        progress(f"extra workload {extra}")
        line.setdefault("other_workloads", {})[extra] = side_workload(args, extra)
    if not args.no_cpu_baseline:
        progress("oracle on the host cores")
        cb = run_cpu_baseline(w, p, args.cpu_sample)
        line["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        x = cb["x"]
        line["vs_oracle"] = {
            "oracle_iters": cb["iters"],
            "rel_error": {tag: oracle_error(rr, x) for tag, rr in
                          (("mixed", mx), ("fp64_batched", f64), ("fp64_plain", plain), ("pou_mixed", pou))
                          if rr is not None},
            "iters": {tag: int(np.median(rr["iters"])) for tag, rr in
                      (("mixed", mx), ("fp64_batched", f64), ("fp64_plain", plain), ("pou_mixed", pou))
                      if rr is not None},
            "note": "relative 2-norm error of each form's solution against the float64 oracle's FGMRES "
                    "solution of the same problem (both stop at relative residual 1e-8)"}
    print(json.dumps(line), flush=True)


def main_mix(args):
    """64 independent problems (1-8 right-hand sides each) solved in one batch per step."""
    import torch
    from paper_2406_06283_amd import hkgeneo as H
    from paper_2406_06283_amd.configs import batch_mix, mix_options
    mix = batch_mix(64)
    t = time.perf_counter()
    probs = [m.problem() for m in mix]
    gen_s = time.perf_counter() - t
    progress(f"generated 64 problems in {gen_s:.1f} s")
    dev = torch.device("cuda:0")
    fs = [torch.from_numpy(np.ascontiguousarray(q.f)).to(dev) for q in probs]
    nrhs = sum(m.nrhs for m in mix)
    res = {}
    for tag, prec in (("mixed", 32), ("fp64", 64)):
        sync()
        t = time.perf_counter()
        Ss = [H.Solver(q, H.default_options(**mix_options(m, local_prec=prec))) for m, q in zip(mix, probs)]
        sync()
        setup_s = time.perf_counter() - t
        progress(f"{tag}: set up 64 problems in {setup_s:.1f} s")
        B = H.Batch(Ss, [m.nrhs for m in mix])
        for _ in range(args.warmup):
            B.solve(fs)
        sync()
        t = time.perf_counter()
        for _ in range(args.steps):
            _, infos, st = B.solve(fs)
        sync()
        total = time.perf_counter() - t
        its = [i["iters"] for pi in infos for i in pi]
        ok = all(i["converged"] and i["relres_true"] <= 1e-8 for pi in infos for i in pi)
        sync()
        t = time.perf_counter()
        for S, fq in zip(Ss, fs):
            S.solve(fq)
        sync()
        seq = time.perf_counter() - t
        progress(f"{tag}: {args.steps} batched steps in {total:.2f} s, sequential single-path pass {seq:.2f} s")
        res[tag] = dict(solves_per_s=nrhs * args.steps / total if ok else 0.0, ms_per_step=1e3 * total / args.steps,
                        setup_s=setup_s, iters_min=min(its), iters_med=statistics.median(its), iters_max=max(its),
                        converged=ok, waves=B.local_waves, sequential_plain_solves_per_s=nrhs / seq,
                        m0_range=[min(S.stats()["m0"] for S in Ss), max(S.stats()["m0"] for S in Ss)])
        B.close()
        for S in Ss:
            S.close()
    mx = res["mixed"]
    line = {"metric": METRIC, "value": round(mx["solves_per_s"], 2), "unit": "solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(mx["ms_per_step"], 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64 (f32 local inverses)",
            "data": "synthetic",
            "config": {"workload": "mix64_p1_h64-256_k0.3/h", "problems": 64, "rhs": nrhs,
                       "step": "one batched solve of every right-hand side of every problem (factors resident)",
                       "generation_s": round(gen_s, 1)},
            "mixed": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in mx.items()},
            "fp64": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in res["fp64"].items()}}
    print(json.dumps(line), flush=True)


def main_serve(args):
    """Poisson request stream through the continuous-batching server."""
    import torch
    from paper_2406_06283_amd import hkgeneo as H, problems as pb, serve
    from paper_2406_06283_amd.configs import serve_options, serve_problem, serve_stream
    dev = torch.device("cuda:0")
    n_req = args.requests
    problems = {}

    def payload(stream, tag0, rhs_offset=0):
        reqs = []
        for q, (arr, key, nrhs, rseed) in enumerate(stream):
            rseed += rhs_offset
            if key not in problems:
                problems[key] = serve_problem(key)
            pr = problems[key]
            g = np.random.Generator(np.random.PCG64(rseed)).standard_normal((nrhs, pr.coords.shape[0]))
            f = np.stack([pb.load_vector(pr.elem_vert, pr.vert_dof, pr.elem_M, g[r], pr.n_dof) for r in range(nrhs)])
            reqs.append(serve.Request(tag=tag0 + q, arrival=arr, key=key, f=torch.from_numpy(f).to(dev)))
        return reqs

    def make_solver(key, stream):
        return H.Solver(problems[key], H.default_options(**serve_options(key)), stream=stream)

    def estimate(key):      # an upper bound: no subdomain keeps more than max_eig_per_sub vectors
        o = serve_options(key)
        return serve.footprint_estimate(problems[key], o["local_prec"], o["max_eig_per_sub"])

    from paper_2406_06283_amd.configs import MIX_RESTART
    kw = dict(ctx_budget=96 << 30, workspace_budget=48 << 30, max_requests=64, max_nrhs=8, restart=MIX_RESTART)
    cache = serve.ContextCache(kw["ctx_budget"])
    out = {}
    t = time.perf_counter()
    # closed loop, cold cache: every request at t = 0 (setups included)
    cold = payload(serve_stream(n_req, 0.0, seed=1), 0)
    gen_s = time.perf_counter() - t
    progress(f"payload of {n_req} requests ({len(problems)} problems) in {gen_s:.1f} s")
    _, s_cold = serve.run_stream(cold, make_solver, estimate, cache=cache, **kw)
    out["closed_loop_cold"] = s_cold
    progress(f"closed loop, cold cache: {s_cold['wall_s']:.1f} s, {s_cold['setups']} setups")
    # closed loop, warm cache (the same keys, other right-hand sides): capacity
    warm = payload(serve_stream(n_req, 0.0, seed=1), 10 ** 6, rhs_offset=7919)
    _, s_warm = serve.run_stream(warm, make_solver, estimate, cache=cache, **kw)
    out["closed_loop_warm"] = s_warm
    progress(f"closed loop, warm cache: {s_warm['wall_s']:.1f} s, {s_warm['solves_per_s']:.1f} solves/s")
    cap_req = s_warm["requests"] / s_warm["wall_s"]
    for k, frac in enumerate((0.25, 0.5, 1.0, 2.0)):
        reqs = payload(serve_stream(n_req, frac * cap_req, seed=10 + k), (k + 2) * 10 ** 6)
        _, s = serve.run_stream(reqs, make_solver, estimate, cache=cache, **kw)
        out[f"rate_{frac:g}x"] = s
        progress(f"rate {frac:g}x capacity: p50 {s['p50_ms']:.1f} ms p99 {s['p99_ms']:.1f} ms")
    cache.close()
    rnd = lambda d: {k: (round(v, 3) if isinstance(v, float) else v) for k, v in d.items()}
    line = {"metric": METRIC, "value": round(s_warm["solves_per_s"], 2), "unit": "solves/s", "n_gpus": 1,
            "steps": n_req, "warmup": 0, "ms_per_step": round(1e3 * s_warm["wall_s"] / n_req, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64 (f32 local inverses)",
            "data": "synthetic",
            "config": {"workload": "serve_p1_h64-256_q1_h32", "requests_per_run": n_req,
                       "capacity_req_per_s": round(cap_req, 2), "payload_generation_s": round(gen_s, 1),
                       "step": "one request (1-8 right-hand sides)"},
            "p50_ms": round(s_warm["p50_ms"], 3), "p99_ms": round(s_warm["p99_ms"], 3),
            "runs": {k: rnd(v) for k, v in out.items()}}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="p1_h256_k80_16x16")
    ap.add_argument("--cpu-sample", type=int, default=1)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--lat-reps", type=int, default=20)
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip the nested / D_k GMRES / Delta-GenEO rows of the default workload")
    ap.add_argument("--extra-workloads", default="p1_h128_k40_8x8",
                    help="comma-separated named workloads whose mixed form is reported beside the line")
    ap.add_argument("--forms", default="plain,fp64,mixed,pou",
                    help="forms of the default workload to run (mixed is always run: it gives value)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="after the run, one elementwise copy of BYTES for hardware-counter calibration")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--in-flight", type=int, default=3,
                    help="independent problems stepped concurrently for the extra throughput field (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the path is a single-device kernel set; "
                                   "independent problems shard across GPUs without communication",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.workload == "mix64":
        main_mix(args)
    elif args.workload == "serve":
        main_serve(args)
    else:
        main_default(args)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)


if __name__ == "__main__":
    main()
