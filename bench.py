#!/usr/bin/env python3
"""Benchmark of the AA-PDHG hot path on one MI355X.

A step is one loop pass of the method (Alg 2 for AA-PDHG, Alg 3 for FAA-PDHG)
over the whole LP: the CSC pass
(K^T y and the primal update), the CSR pass (K x_bar, the dual update and the
float64 decisions) and, on Anderson steps, the mix pass; the KKT test runs
every 64 passes as in a solve.  The KKT tolerance is set to 0 inside the timed
region so that no pass is skipped by early termination.

Workloads (synthetic, seeded; see lpgen):
  powerlaw1m  (default) 1M x 2M LP, 20M nonzeros, power-law columns, Ruiz-scaled, FAA-PDHG,
              m_A = 10, float32 with float64 reductions and decisions: loop passes per
              second (value), the longest launch against the HBM roofline, SpMV GB/s, and
              the LP solved to relative KKT 1e-4; the line also carries the batch leg
              (batch256 below), a serving leg (Poisson stream at 200 requests/s), the
              cache-resident 20k x 50k LP, and the oracle on the host (cpu_baseline)
  mip20k      20k x 50k LP, 250k nonzeros, Zipf(1.8) rows, float32, m_A = 10: loop passes
              per second in the persistent kernel
  batch256    256 LPs of uneven sizes (rows log-uniform 1k..50k), m_A = 8: LPs solved per
              second to relative KKT 1e-4 in one batched float32 solve, beside float64
              single solves of a sample of the same LPs
  serve       Poisson stream of LP requests (200/s by default) through the continuous-
              batching server, float32, m_A = 10: LPs solved per second, p50/p99 latency
  serve_curve the serving mix at rising arrival rates: LPs/s and p50/p99 latency per rate
  compare     the 20k x 50k LP solved to relative KKT 1e-4 by PDHG, AA-PDHG, FAA-PDHG,
              AA-PDHG with primal weights and restarted PDHG: passes and seconds
  sweep       AA-PDHG hyperparameters (m_A, eta, Iter_AA / c) as members of one batch on
              the 20k x 50k LP: passes to relative KKT 1e-4 per configuration

Prints one JSON line (see the keys below).  --gpus N with N > 1 is refused:
this build measures one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def _bytes_model(n, m, Z, M, kkt_frac, dots=True):
    """Algorithmic bytes of one launch of each pass (float32 data, int32
    indices), with a full memory of M columns: the matrix once (value and
    index), the gathered vector once, and every vector the epilogue reads or
    writes once, and the new column pair is written.  With dots (the
    persistent kernel) the passes also read the M - 1 live history columns
    that are not being replaced, for the new Gram row; the three-launch
    passes leave that to the Gram launch, which on an Anderson step reads the
    M live columns and g ("gram")."""
    hist = (M - 1) * 4 if dots else 0
    primal = 8 * Z + 4 * (n + 1) + 4 * m + n * (7 * 4 + hist + 5 * 4)
    dual = 8 * Z + 4 * (m + 1) + 4 * n * (1 + kkt_frac) + m * (5 * 4 + 1 + hist + 4 * 4)
    mix = n * (5 * 4 + M * 4 + 4) + m * (3 * 4 + 1 + M * 4 + 4)
    gram = 0 if dots else (M + 1) * 4 * (n + m)
    spmv = 16 * Z + 8 * (n + m)
    return {"primal": primal, "dual": dual, "mix": mix, "gram": gram, "spmv": spmv}


def _src_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "aapdhg_internal.h"):
        with open(os.path.join(ROOT, "paper_2508_08062_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(workload, kernel, ppl):
    """HBM bytes per launch of `ppl` passes from the committed counter summary,
    if it was taken on the current kernel source (the summary stores bytes per
    pass: per dispatch for the three launches, per launch / passes for the
    persistent kernel)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != _src_hash():
        return None
    ks = t.get("kernels", {})
    k = ks.get(kernel)
    if k is None or "hbm_bytes_per_pass" not in k:
        return None
    b = k["hbm_bytes_per_pass"]
    if kernel == "dual":  # the dual launch's events bracket the panel kernel and the decisions too
        for extra in ("panel", "decide"):
            if extra in ks:
                b += ks[extra]["hbm_bytes_per_pass"]
    return b * ppl


def _workload(name):
    import lpgen
    if name == "mip20k":
        lp = lpgen.mip_like_lp(1)
        opts = dict(variant=1, precision=0, memory=10, kkt_every=64, ruiz_iters=10, dhat_mode=0)
        return [lp], opts, {"workload": "single LP 20000x50000, 250000 nnz, Zipf(1.8) rows (mip_like_lp seed 1)",
                            "variant": "AA-PDHG", "m_A": 10, "ruiz_iters": 10, "dhat_mode": 0}
    if name == "powerlaw1m":
        lp = lpgen.powerlaw_lp(2)
        opts = dict(variant=2, precision=0, memory=10, kkt_every=64, ruiz_iters=10, dhat_mode=0)
        return [lp], opts, {"workload": "single LP 1000000x2000000, 20000000 nnz, power-law columns "
                                        "(powerlaw_lp seed 2)", "variant": "FAA-PDHG", "m_A": 10,
                            "ruiz_iters": 10, "dhat_mode": 0}
    if name == "batch256":
        lps = lpgen.batch_lps(256, 3)
        opts = dict(variant=1, precision=0, memory=8, kkt_every=64, ruiz_iters=10, dhat_mode=0)
        return lps, opts, {"workload": "batch of 256 LPs, rows log-uniform 1k..50k, cols 2x rows, "
                                       "3..12 nnz/col (batch_lps seed 3)", "variant": "AA-PDHG", "m_A": 8,
                           "ruiz_iters": 10, "dhat_mode": 0}
    raise ValueError(name)


def _timed_passes(runner, stream, steps, warmup, ppl):
    """W untimed passes, then `steps` passes bracketed by events on the launch
    stream and device synchronisations; returns (passes, ms)."""
    import torch
    runner.iterate(1, stream)  # the init step
    for _ in range(max(1, warmup // ppl)):
        runner.iterate(ppl, stream)
    torch.cuda.synchronize()
    nlaunch = max(1, steps // ppl)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(nlaunch):
        runner.iterate(ppl, stream)
    end.record(stream)
    torch.cuda.synchronize()
    return nlaunch * ppl, start.elapsed_time(end)


def _launch_roofline(lps, opts, solvers, runner, stream, ppl, workload):
    """The launch that takes longest per pass, against the HBM roofline: its
    algorithmic bytes per launch over its average duration measured with HIP
    events on the launch stream (three timed repetitions), with the counter
    traffic of the committed summary when it was taken on the current kernel
    source."""
    n = sum(lp.n for lp in lps)
    m = sum(lp.m for lp in lps)
    Z = sum(lp.nnz for lp in lps)
    M = opts["memory"]
    def results():
        if runner in solvers:
            return [s.result() for s in solvers]
        return [runner.result(i) for i in range(len(solvers))]

    r0 = results()
    kt = [runner.iterate_timed(ppl, stream) for _ in range(3)]
    r1 = results()
    aa_frac = sum(b["aa_steps"] - a["aa_steps"] for a, b in zip(r0, r1)) / (3.0 * ppl * len(solvers))
    # the three-launch passes take the per-pass Gram dots unless every LP forms the Gram on demand
    dots = kt[0]["kernel"] == "persistent" or any(not r["gram_on_demand"] for r in r1)
    bm = _bytes_model(n, m, Z, M, 1.0 / opts["kkt_every"], dots=dots)
    if kt[0]["kernel"] == "persistent":
        launch_ms = sum(k["launch_ms"] for k in kt) / len(kt)
        per_pass = bm["primal"] + bm["dual"] + aa_frac * bm["mix"]
        dom, dom_bytes, dom_ms = "loop", per_pass * ppl, launch_ms
        ext = bool(opts.get("pw_period")) or opts.get("variant") == 3
        kernel_name = f"k_loop<float, {10 if M > 8 else 8}, {'true' if ext else 'false'}>"
        spmv_gbs = bm["spmv"] * ppl / (launch_ms * 1e-3) / 1e9
        launch = {"kernel": kernel_name, "passes_per_launch": ppl, "launch_ms": launch_ms,
                  "ms_per_pass": launch_ms / ppl, "aa_fraction": aa_frac}
        traffic = _traffic(workload, "loop", ppl)
    else:
        avg = {q: sum(k[q] for k in kt) / len(kt) for q in ("primal", "dual", "mix")}
        dom = max(avg, key=lambda q: avg[q])
        dom_bytes, dom_ms = bm[dom], avg[dom]
        kernel_name = {"primal": f"k_pass<float, {10 if M > 8 else 8}, 0>",
                       "dual": f"k_pass<float, {10 if M > 8 else 8}, 1>", "mix": "k_mix<float>"}[dom]
        # SpMV GB/s: the product pair's algorithmic bytes over the two SpMV launches
        spmv_gbs = bm["spmv"] / ((avg["primal"] + avg["dual"]) * 1e-3) / 1e9
        launch = {"kernel": "three launches per pass", **avg, "aa_fraction": aa_frac,
                  "per_launch": {q: {"algorithmic_bytes": bm[q], "ms": avg[q],
                                     "achieved_gbs": bm[q] / (avg[q] * 1e-3) / 1e9,
                                     "frac": bm[q] / (avg[q] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                     "traffic": _traffic(workload, q, 1)} for q in ("primal", "dual")}}
        traffic = _traffic(workload, dom, 1)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel_name,
            "algorithmic_bytes_per_launch": dom_bytes, "launch_ms": dom_ms}
    return roof, launch, {"spmv_gbps": spmv_gbs, "spmv_frac_of_peak": spmv_gbs / HBM_PEAK_GBS,
                          "bytes_per_pass": bm}


def _solve_leg(lp, opts, stream, seconds, tol=1e-4, precision=0):
    """One LP solved from its start point to relative KKT `tol` (time-limited):
    passes, seconds, KKT and the objective against the planted optimum."""
    import paper_2508_08062_amd as P
    s = P.Solver(lp, tol=tol, max_iter=10 ** 7, time_limit_s=seconds, **{**opts, "precision": precision})
    t0 = time.perf_counter()
    s.solve(stream)
    el = time.perf_counter() - t0
    r = s.result()
    s.close()
    out = {"status": r["status"], "iters": r["iters"], "seconds": el, "kkt": r["kkt"], "r_gap": r["r_gap"],
           "r_pri": r["r_pri"], "r_dual": r["r_dual"], "primal_obj": r["primal_obj"], "dual_obj": r["dual_obj"],
           "aa_steps": r["aa_steps"], "lps_per_s": (1.0 / el) if r["status"] == "converged" else 0.0,
           "tol": tol, "precision": "f64" if precision else "f32"}
    pstar = lp.planted.get("pstar") if lp.planted else None
    if pstar is not None:
        out["planted_pstar"] = pstar
        out["rel_obj_err_vs_planted"] = abs(r["primal_obj"] - pstar) / (1.0 + abs(pstar))
    return out


def _host_cpu():
    """The host the CPU baseline ran on: processor model and the cores this
    process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_cores_usable": len(os.sched_getaffinity(0))}


def _cpu_baseline(lps, opts, seconds):
    """The oracle on the host, one thread, on the first LP of the workload,
    for about `seconds` of loop passes; returns passes per second."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    lp = lps[0]
    with threadpool_limits(limits=1):
        print("# oracle set-up", file=sys.stderr, flush=True)
        P = oracle.Problem.from_lpdata(lp)
        if opts.get("ruiz_iters", 0):
            P, _, _ = oracle.ruiz(P, opts["ruiz_iters"])
            P = P.rounded_fp32()
        print("# oracle scaled", file=sys.stderr, flush=True)
        # the pass rate does not depend on the step size: a short power
        # iteration is enough for the large LP
        nrm = oracle.power_norm(P, iters=200 if lp.nnz < 2_000_000 else 10)
        o = oracle.Solver(P, oracle.Options(variant=opts["variant"], memory=opts["memory"],
                                            kkt_every=opts["kkt_every"], tol=0.0, tau=0.9 / nrm,
                                            sigma=0.9 / nrm, dhat_mode=opts.get("dhat_mode", 1)))
        o.start()
        print("# oracle started", file=sys.stderr, flush=True)
        for _ in range(3):
            o.step()
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < seconds:
            o.step()
            k += 1
        el = time.perf_counter() - t0
    return k / el, k, el


def _cpu_batch_baseline(lps, opts, seconds):
    """The oracle, one thread, solving members of the batch to relative KKT
    1e-4 one after the other (smallest first) for about `seconds`; the batch's
    LPs/s on one core follows from the time per nonzero-pass it shows."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    order = sorted(range(len(lps)), key=lambda i: lps[i].nnz)
    done, work, t_all = [], 0.0, 0.0
    with threadpool_limits(limits=1):
        for i in order:
            if t_all > seconds:
                break
            P = oracle.Problem.from_lpdata(lps[i])
            P, _, _ = oracle.ruiz(P, opts.get("ruiz_iters", 10))
            P = P.rounded_fp32()
            t0 = time.perf_counter()
            nrm = oracle.power_norm(P)
            o = oracle.Solver(P, oracle.Options(variant=opts["variant"], memory=opts["memory"], tol=1e-4,
                                                kkt_every=opts["kkt_every"], max_iter=20000, tau=0.9 / nrm,
                                                sigma=0.9 / nrm, dhat_mode=opts.get("dhat_mode", 1)))
            r = o.solve()
            el = time.perf_counter() - t0
            t_all += el
            done.append((i, r["status"], int(r["k"]), el))
            work += lps[i].nnz * r["k"]
    # seconds per nonzero-pass, applied to the batch's own passes would need its
    # iteration counts; report the sample and the LPs/s it reached
    n_conv = sum(1 for d in done if d[1] == "converged")
    return {"value": n_conv / max(t_all, 1e-9), "unit": "LPs/s", "cores": 1, "kind": "oracle", **_host_cpu(),
            "sample": f"{len(done)} smallest members solved one after the other by the float64 oracle "
                      f"({n_conv} converged, {t_all:.1f} s, one thread): " +
                      ", ".join(f"LP {i} {st} in {k} passes, {el:.1f} s" for i, st, k, el in done),
            "seconds_per_nnz_pass": t_all / max(work, 1.0)}


def _line(metric, value, unit, cfg, extra, higher=True, steps=0, warmup=0, ms=0.0, dtype="f32"):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": cfg, **extra}


def _batch_leg(args, stream, cpu_baseline=False):
    """256 LPs of uneven sizes: the aggregate batch iteration against the HBM
    roofline (all members running, three launches per pass), then the whole
    batch solved to relative KKT 1e-4 in float32, and a sample of the same LPs
    solved one at a time in float64 and in float32 (measured, not scaled)."""
    import numpy as np

    import paper_2508_08062_amd as P
    lps, opts, cfg = _workload("batch256")
    kw = dict(opts, tol=1e-4, max_iter=200000)
    # whole batch passes (64, far from any member's termination) with the
    # built-in or the autotuned work tables, launched directly or replayed
    # from a HIP graph, and with the Gram matrix formed on every pass (the
    # default for these LPs, which the persistent kernel can take alone) or
    # on demand (gram_mode 2); the batch is then solved in the fastest
    configs, params = {}, {}
    for tune, graph, gram in ((0, 0, 0), (0, 1, 0), (1, 0, 0), (1, 1, 0), (0, 0, 2), (0, 1, 2)):
        name = f"autotune{tune}_graph{graph}_gram{gram}"
        t0 = time.perf_counter()
        solvers = [P.Solver(lp, autotune=tune, graph=graph, gram_mode=gram, **kw) for lp in lps]
        t_create = time.perf_counter() - t0
        batch = P.Batch(solvers)
        _, ms = _timed_passes(batch, stream, 64, 8, 64)
        batch.close()
        for sv in solvers:
            sv.close()
        configs[name] = {"ms_per_batch_pass": ms / 64, "create_seconds": t_create}
        params[name] = dict(autotune=tune, graph=graph, gram_mode=gram)
        print(f"# autotune {tune} graph {graph} gram_mode {gram}: {ms / 64:.3f} ms per batch pass "
              f"(created in {t_create:.1f} s)", file=sys.stderr, flush=True)
    best_cfg = min(configs, key=lambda c: configs[c]["ms_per_batch_pass"])
    solvers = [P.Solver(lp, **params[best_cfg], **kw) for lp in lps]
    batch = P.Batch(solvers)
    batch.iterate(1, stream)
    batch.iterate(8, stream)
    roof, launch, spmv = _launch_roofline(lps, opts, solvers, batch, stream, 64, "batch256")
    batch.close()
    for sv in solvers:
        sv.reset(stream)
    batch = P.Batch(solvers)
    t0 = time.perf_counter()
    batch.solve(stream)
    el = time.perf_counter() - t0
    res = batch.results()
    iters = np.array([r["iters"] for r in res])
    done_s = np.array([r["solve_seconds"] for r in res])  # per LP: time until seen stopped
    conv = int(sum(r["status"] == "converged" for r in res))
    batch.close()
    for sv in solvers:
        sv.close()
    print(f"# batch solve {el:.2f} s, {conv} converged", file=sys.stderr, flush=True)
    # single solves of a sample, one after the other, float64 and float32
    rng = np.random.default_rng(5)
    sample = sorted(rng.choice(len(lps), size=min(args.fp64_sample, len(lps)), replace=False).tolist())
    single = {}
    for prec, key in ((1, "fp64_single"), (0, "fp32_single")):
        t, it, st = [], [], []
        for i in sample:
            sv = P.Solver(lps[i], **{**kw, "precision": prec})
            t1 = time.perf_counter()
            sv.solve(stream)
            t.append(time.perf_counter() - t1)
            r = sv.result()
            it.append(r["iters"])
            st.append(r["status"])
            sv.close()
        c = sum(x == "converged" for x in st)
        single[key] = {"sample": sample, "seconds": t, "iters": it, "status": st,
                       "lps_per_s": c / sum(t), "latency_p50_s": float(np.percentile(t, 50)),
                       "latency_p99_s": float(np.percentile(t, 99)),
                       "measured": "each sampled LP solved alone from create-time state to rel KKT 1e-4"}
    out = {"workload": cfg["workload"], "lps": len(lps), "nnz_total": sum(lp.nnz for lp in lps),
           "value": conv / el, "unit": "LPs/s", "batch_seconds": el, "converged": conv,
           "lps_stopped_per_s": len(lps) / el, "iters_median": float(np.median(iters)),
           "iters_max": int(iters.max()),
           "completion_p50_s": float(np.percentile(done_s, 50)),
           "completion_p99_s": float(np.percentile(done_s, 99)),
           "lps_done_by_p50_per_s": 0.5 * len(lps) / float(np.percentile(done_s, 50)),
           "batch_iteration": {"roofline": roof, "launch": launch, **spmv,
                               "ms_per_batch_iteration": launch.get("primal", 0) + launch.get("dual", 0)
                               + launch.get("aa_fraction", 0) * launch.get("mix", 0),
                               "configurations": configs, "solved_with": best_cfg,
                               "note": "launch durations (roofline) are timed with events per launch"},
           **single}
    if cpu_baseline:
        cb = _cpu_batch_baseline(lps, opts, args.cpu_seconds)
        # the whole batch on one core at the sample's time per nonzero-pass,
        # with the passes each LP took on the GPU
        est = cb["seconds_per_nnz_pass"] * float(sum(lps[i].nnz * r["iters"] for i, r in enumerate(res)))
        cb["sample_lps_per_s"] = cb["value"]
        cb["value"] = conv / est  # the batch on one core, scaled from the sample (converged LPs only)
        cb["sample"] += (f"; scaled to the batch: {est:.0f} s for its {len(lps)} LPs at the sample's seconds per "
                         "nonzero-pass and the passes each LP took on the GPU")
        out["cpu_baseline"] = cb
    return out


def _batch_solve(args):
    import torch
    stream = torch.cuda.Stream()
    out = _batch_leg(args, stream, cpu_baseline=not args.no_cpu_baseline)
    cfg = {"workload": out.pop("workload"), "variant": "AA-PDHG", "m_A": 8, "ruiz_iters": 10, "dhat_mode": 0,
           "lps": out["lps"], "nnz_total": out["nnz_total"]}
    value = out.pop("value")
    out.pop("unit")
    extra = {k: v for k, v in out.items() if k not in ("lps", "nnz_total")}
    print(json.dumps(_line("LPs solved/s at rel KKT 1e-4 (batched float32)", value, "LPs/s", cfg, extra,
                           ms=out["batch_seconds"] * 1e3)), flush=True)


def _compare(args):
    """The paper's comparison on one LP: vanilla PDHG, AA-PDHG, FAA-PDHG and
    fixed-frequency restarted PDHG solving the 20k x 50k LP to relative KKT
    1e-4 in float32, plus AA-PDHG in the configuration of Section 5.2
    (m_A = 5, primal-weight update every 3000 iterations with theta = 0.5,
    Iter_AA / 3 safeguard)."""
    import torch

    import paper_2508_08062_amd as P
    lps, opts, cfg = _workload("mip20k")
    stream = torch.cuda.Stream()
    methods = [
        ("PDHG", dict(variant=0)),
        ("AA-PDHG m_A=10", dict(variant=1)),
        ("FAA-PDHG m_A=10", dict(variant=2)),
        ("AA-PDHG m_A=5, primal weight U_P=3000, Iter_AA/3", dict(variant=1, memory=5, pw_period=3000,
                                                                 pw_theta=0.5, sg_div=3.0)),
        ("restarted PDHG R=75", dict(variant=3, restart_period=75)),
        ("restarted PDHG R=500", dict(variant=3, restart_period=500)),
        ("restarted PDHG R=3000", dict(variant=3, restart_period=3000)),
    ]
    out = []
    for name, m in methods:
        s = P.Solver(lps[0], tol=1e-4, max_iter=args.compare_max_iter, **{**opts, **m})
        t0 = time.perf_counter()
        s.solve(stream)
        el = time.perf_counter() - t0
        r = s.result()
        out.append({"method": name, "status": r["status"], "iters": r["iters"], "seconds": el, "kkt": r["kkt"],
                    "aa_steps": r["aa_steps"], "primal_obj": r["primal_obj"]})
        s.close()
        print(f"# {name}: {r['status']} after {r['iters']} passes, {el:.2f} s", file=sys.stderr, flush=True)
    best = min((o for o in out if o["status"] == "converged"), key=lambda o: o["seconds"], default=None)
    line = _line("LP solved to rel KKT 1e-4 (float32): passes and seconds by method",
                 best["seconds"] if best else None, "s", {**cfg, "max_iter": args.compare_max_iter},
                 {"methods": out, "fastest": best["method"] if best else None}, higher=False,
                 ms=(best["seconds"] * 1e3) if best else 0.0)
    print(json.dumps(line), flush=True)


def _sweep(args):
    """The supplement's tuning study on synthetic LPs: AA-PDHG with
    m_A in {3, 5, 7} x eta in {1e-6, 1e-8, 1e-10} x safeguard Iter_AA / c with
    c in {1, 3}, every configuration a member of one batched float32 solve of
    the same LP (relative KKT 1e-4)."""
    import itertools

    import numpy as np
    import torch

    import lpgen
    import paper_2508_08062_amd as P
    lp = lpgen.mip_like_lp(args.sweep_seed, m=args.sweep_m, n=int(2.5 * args.sweep_m), nnz=int(12.5 * args.sweep_m))
    grid = list(itertools.product((3, 5, 7), (1e-6, 1e-8, 1e-10), (1.0, 3.0)))
    base = dict(variant=1, precision=0, kkt_every=64, ruiz_iters=10, dhat_mode=0, tol=1e-4,
                max_iter=args.sweep_max_iter)
    solvers = [P.Solver(lp, memory=mA, eta=eta, sg_div=c, **base) for mA, eta, c in grid]
    batch = P.Batch(solvers)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.solve(stream)
    el = time.perf_counter() - t0
    res = batch.results()
    rows = [{"m_A": mA, "eta": eta, "sg_div": c, "status": r["status"], "iters": r["iters"],
             "aa_steps": r["aa_steps"], "kkt": r["kkt"], "seconds_to_stop": r["solve_seconds"]}
            for (mA, eta, c), r in zip(grid, res)]
    batch.close()
    for sv in solvers:
        sv.close()
    conv = [r for r in rows if r["status"] == "converged"]
    best = min(conv, key=lambda r: r["iters"], default=None)
    for r in rows:
        print(f"# m_A={r['m_A']} eta={r['eta']:.0e} c={r['sg_div']:.0f}: {r['status']} {r['iters']} passes",
              file=sys.stderr, flush=True)
    line = _line("AA-PDHG hyperparameter sweep: passes to rel KKT 1e-4 (batched float32)",
                 len(rows) / el, "configurations/s",
                 {"workload": f"one LP {lp.m}x{lp.n}, {lp.nnz} nnz (mip_like_lp seed {args.sweep_seed}), "
                              f"{len(rows)} configurations in one batch", "variant": "AA-PDHG"},
                 {"batch_seconds": el, "configurations": rows, "fewest_passes": best,
                  "median_passes": float(np.median([r["iters"] for r in rows]))}, ms=el * 1e3)
    print(json.dumps(line), flush=True)


def _dsweep(args):
    """The safeguard constant D (Alg 2's safeguard test; Section 5.1 shows the
    KKT history of AA-PDHG with m_A = 5 under several D): AA-PDHG with
    m_A = 5, eta = 1e-10, epsilon = 1 and D from 1e-2 to 1e6 on the sweep
    LP, float32, every value a member of one batch.  Every `dsweep_every`
    passes the relative KKT residual of each member is evaluated at its
    current iterate, until every member converged (1e-4) or reached the pass
    limit."""
    import numpy as np
    import torch

    import lpgen
    import paper_2508_08062_amd as P
    lp = lpgen.mip_like_lp(args.sweep_seed, m=args.sweep_m, n=int(2.5 * args.sweep_m), nnz=int(12.5 * args.sweep_m))
    Ds = [1e-2, 1e-1, 1.0, 10.0, 1e2, 1e4, 1e6]
    base = dict(variant=1, precision=0, memory=5, eta=1e-10, eps_sg=1.0, kkt_every=64, ruiz_iters=10, dhat_mode=0,
                tol=1e-4, max_iter=args.sweep_max_iter)
    solvers = [P.Solver(lp, D=D, **base) for D in Ds]
    batch = P.Batch(solvers)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    every = args.dsweep_every
    hist = [[] for _ in Ds]
    t0 = time.perf_counter()
    done = 0
    while done <= args.sweep_max_iter + every:  # members stop at the pass limit on their own
        batch.iterate(every, stream)
        done += every
        res = batch.results()
        for h, r in zip(hist, res):
            if r["status"] == "running" or not h or h[-1][0] < r["iters"]:
                h.append((r["iters"], r["kkt"]))
        if all(r["status"] != "running" for r in res):
            break
    el = time.perf_counter() - t0
    res = batch.results()
    rows = [{"D": D, "status": r["status"], "iters": r["iters"], "aa_steps": r["aa_steps"],
             "aa_fraction": r["aa_steps"] / max(1, r["iters"]), "kkt": r["kkt"],
             "kkt_history": [[int(k), float(v)] for k, v in h]}
            for D, r, h in zip(Ds, res, hist)]
    batch.close()
    for sv in solvers:
        sv.close()
    for r in rows:
        print(f"# D={r['D']:.0e}: {r['status']} {r['iters']} passes, {r['aa_steps']} Anderson steps, "
              f"KKT {r['kkt']:.2e}", file=sys.stderr, flush=True)
    line = _line("AA-PDHG safeguard constant sweep: passes to rel KKT 1e-4 (batched float32)",
                 len(rows) / el, "configurations/s",
                 {"workload": f"one LP {lp.m}x{lp.n}, {lp.nnz} nnz (mip_like_lp seed {args.sweep_seed}), "
                              f"{len(rows)} values of D in one batch", "variant": "AA-PDHG", "m_A": 5},
                 {"batch_seconds": el, "kkt_every_passes": every, "configurations": rows,
                  "median_passes": float(np.median([r["iters"] for r in rows]))}, ms=el * 1e3)
    print(json.dumps(line), flush=True)


def _serve_curve(args):
    """Latency against throughput of the server: Poisson streams at rising
    rates (each 10 s with up to 40 s of drain), the knee of the curve beside
    the overloaded 200/s point of the serve workload."""
    pts = []
    for rate in args.curve_rates:
        sv = _serve(args, rate=rate, seconds=args.serve_leg_seconds, pool_size=16, drain=args.serve_leg_drain,
                    emit=False)
        pts.append({"rate_per_s": rate, "lps_per_s": sv["value"], "finished": sv["finished"],
                    "unfinished": sv["unfinished"], "latency_p50_s": sv["latency_p50_s"],
                    "latency_p99_s": sv["latency_p99_s"]})
        print(f"# rate {rate}/s: {sv['value']:.2f} LPs/s, p50 {sv['latency_p50_s']}, p99 {sv['latency_p99_s']}",
              file=sys.stderr, flush=True)
    best = max(pts, key=lambda q: q["lps_per_s"])
    line = _line("LPs solved/s & p99 latency at rel KKT 1e-4 (served float32), by arrival rate",
                 best["lps_per_s"], "LPs/s",
                 {"workload": "Poisson streams of the serving mix (serving_requests seed 4), 16 distinct LPs cycled, "
                              f"{args.serve_leg_seconds} s each", "variant": "AA-PDHG", "m_A": 10},
                 {"curve": pts})
    print(json.dumps(line), flush=True)


def _serve(args, rate=None, seconds=None, pool_size=None, drain=None, emit=True):
    """A Poisson stream of LP requests through the server; LPs solved per
    second and latency from submission to completion."""
    import numpy as np
    import torch

    import lpgen
    import paper_2508_08062_amd as P
    rate = args.rate if rate is None else rate
    seconds = args.serve_seconds if seconds is None else seconds
    pool_size = args.pool if pool_size is None else pool_size
    drain = args.drain_seconds if drain is None else drain
    reqs = lpgen.serving_requests(rate=rate, duration=seconds, seed=4)
    pool = [lpgen.mip_like_lp(r[4], m=r[1], n=r[2], nnz=r[3]) for r in reqs[:pool_size]]
    opts = dict(variant=1, precision=0, memory=10, kkt_every=64, ruiz_iters=10, dhat_mode=0, tol=1e-4,
                max_iter=200000, epoch=64)
    torch.cuda.init()
    free, _ = torch.cuda.mem_get_info()
    srv = P.Server(hbm_budget_bytes=int(free * 0.8), max_slots=args.slots, **opts)
    print(f"# {len(reqs)} requests over {seconds} s, pool {len(pool)}", file=sys.stderr, flush=True)
    pending = {}
    lat = []
    t0 = time.perf_counter()
    i = 0
    last = 0.0
    while i < len(reqs) or pending:
        now = time.perf_counter() - t0
        if now - last >= 10.0:
            last = now
            print(f"# t={now:.0f} s submitted {i} finished {len(lat)} pending {len(pending)}", file=sys.stderr,
                  flush=True)
        while i < len(reqs) and reqs[i][0] <= now:
            pending[srv.submit(pool[i % len(pool)])] = reqs[i][0]
            i += 1
        for tk in list(pending):
            r = srv.poll(tk, want_solution=False)
            if r is not None:
                lat.append((r["t_done"], r["status"], pending.pop(tk)))
        if time.perf_counter() - t0 > seconds + drain:
            break  # requests still pending are reported as unfinished
        time.sleep(0.0005)
    el = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    d = np.array([x[0] for x in lat])
    # requests still pending at the end have waited at least this long
    ages = np.array([el - t_arr for t_arr in pending.values()])
    d_all = np.concatenate([d, ages])
    conv = sum(x[1] == "converged" for x in lat)
    line = _line("LPs solved/s & p99 latency at rel KKT 1e-4 (served float32)", conv / el, "LPs/s",
                 {"workload": f"Poisson stream {rate}/s for {seconds} s (serving_requests seed 4), "
                              f"columns lognormal(ln 20000, 1) in [1k, 500k], rows 0.4 x columns, 5 nnz/column; "
                              f"{len(pool)} distinct LPs cycled", "variant": "AA-PDHG", "m_A": 10},
                 {"requests": len(reqs), "finished": len(lat), "unfinished": len(pending), "converged": int(conv),
                  "seconds": el, "finished_per_s": len(lat) / el,
                  "latency_p50_s": float(np.percentile(d, 50)) if d.size else None,
                  "latency_p99_s": float(np.percentile(d, 99)) if d.size else None,
                  "latency_max_s": float(d.max()) if d.size else None,
                  "latency_p99_with_unfinished_lower_bound_s": float(np.percentile(d_all, 99)) if d_all.size else None,
                  "server": st})
    if emit:
        print(json.dumps(line), flush=True)
    return line


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="powerlaw1m", choices=["mip20k", "powerlaw1m", "batch256", "serve", "serve_curve", "compare", "sweep",
                                                                 "dsweep"])
    ap.add_argument("--compare-max-iter", type=int, default=300000, help="compare: pass limit per method")
    ap.add_argument("--sweep-m", type=int, default=20000, help="sweep: rows of the LP (columns 2.5x, 12.5 nnz/row)")
    ap.add_argument("--sweep-seed", type=int, default=1)
    ap.add_argument("--sweep-max-iter", type=int, default=100000)
    ap.add_argument("--dsweep-every", type=int, default=1000, help="dsweep: passes between KKT evaluations")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: requests per second")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="serve: length of the arrival stream")
    ap.add_argument("--pool", type=int, default=64, help="serve: distinct LPs cycled through the stream")
    ap.add_argument("--slots", type=int, default=64, help="serve: resident LPs at most")
    ap.add_argument("--drain-seconds", type=float, default=120.0, help="serve: wait after the last arrival")
    ap.add_argument("--fp64-sample", type=int, default=8, help="batch256: LPs solved singly in float64")
    ap.add_argument("--serve-rate", type=float, default=4.0,
                    help="mip20k: rate of the short serving leg (0 = none)")
    ap.add_argument("--serve-leg-seconds", type=float, default=5.0, help="length of the serving leg's stream")
    ap.add_argument("--serve-leg-drain", type=float, default=25.0, help="drain of the serving leg")
    ap.add_argument("--solve-seconds", type=float, default=150.0, help="time limit of the solve-to-1e-4 legs")
    ap.add_argument("--knee-rates", type=float, nargs="*", default=[2.0, 8.0],
                    help="powerlaw1m: arrival rates of the short streams that locate the serving knee")
    ap.add_argument("--no-legs", action="store_true",
                    help="powerlaw1m: only the headline passes (no batch, serving and 20k x 50k legs)")
    ap.add_argument("--curve-rates", type=float, nargs="+", default=[1.0, 2.0, 4.0, 8.0, 16.0],
                    help="serve_curve: arrival rates (requests per second)")
    ap.add_argument("--passes-per-launch", type=int, default=500,
                    help="loop passes per launch of the persistent loop kernel")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the solve-to-tolerance leg")
    ap.add_argument("--chunks-per-block", type=int, default=0, help="workgroup size in chunks (0 = automatic)")
    ap.add_argument("--pw-period", type=int, default=0,
                    help="primal-weight update every N iterations (Alg 7; 0 = off, as in the headline line)")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the timed loop passes (for rocprofv3 runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB between two device buffers 5 times (scale for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU; --gpus N with N > 1 is not supported by this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "copies": 5}), flush=True)
        return

    import paper_2508_08062_amd as P

    if args.workload == "serve":
        return _serve(args)
    if args.workload == "serve_curve":
        return _serve_curve(args)
    if args.workload == "batch256" and not args.profile_run:
        return _batch_solve(args)
    if args.workload == "compare":
        return _compare(args)
    if args.workload == "sweep":
        return _sweep(args)
    if args.workload == "dsweep":
        return _dsweep(args)
    lps, opts, cfg = _workload(args.workload)
    if args.chunks_per_block:
        opts["chunks_per_block"] = args.chunks_per_block
    if args.pw_period:
        opts["pw_period"] = args.pw_period
        cfg = {**cfg, "pw_period": args.pw_period}
    torch.cuda.init()
    stream = torch.cuda.Stream()
    solvers = [P.Solver(lp, tol=0.0, max_iter=10 ** 9, **opts) for lp in lps]
    runner = solvers[0] if len(solvers) == 1 else P.Batch(solvers)
    torch.cuda.synchronize()
    print(f"# created {len(solvers)} LP(s); warmup {args.warmup}", file=sys.stderr, flush=True)
    ppl = max(1, min(args.passes_per_launch, args.steps))
    steps, ms = _timed_passes(runner, stream, args.steps, args.warmup, ppl)
    print(f"# timed {steps} passes in {ms:.1f} ms", file=sys.stderr, flush=True)
    if args.profile_run:
        # every handle is destroyed, and the device idle, before the program ends
        if runner is not solvers[0]:
            runner.close()
        for sv in solvers:
            sv.close()
        torch.cuda.synchronize()
        return
    roof, launch, spmv = _launch_roofline(lps, opts, solvers, runner, stream, ppl, args.workload)
    if runner is not solvers[0]:
        runner.close()
    for sv in solvers:
        sv.close()
    n = sum(lp.n for lp in lps)
    m = sum(lp.m for lp in lps)
    Z = sum(lp.nnz for lp in lps)
    line = {
        "metric": "PDHG iters/s + SpMV HBM GB/s; LPs solved/s & p99 latency at rel KKT 1e-4",
        "value": steps / (ms * 1e-3),
        "unit": "iters/s" if len(lps) == 1 else "batch iters/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {**cfg, "m": m, "n": n, "nnz": Z},
        **spmv,
        "launch": launch,
        "roofline": roof,
    }
    if args.workload == "mip20k":
        ws = (16 * Z + 4 * (2 * opts["memory"] + 12) * (n + m)) / 1e6
        line["roofline"]["note"] = (f"working set about {ws:.0f} MB stays in L2/MALL: the pass is bound by "
                                    "latency, not HBM")

    if args.workload == "powerlaw1m" and not args.no_legs:
        # the same passes in float64 (the float32 path's gain where bandwidth decides)
        s64 = P.Solver(lps[0], tol=0.0, max_iter=10 ** 9, **{**opts, "precision": 1})
        st64, ms64 = _timed_passes(s64, stream, 500, 50, 500)
        kt64 = s64.iterate_timed(100, stream)
        s64.close()
        line["fp64_passes"] = {"value": st64 / (ms64 * 1e-3), "unit": "iters/s", "steps": st64,
                               "ms_per_step": ms64 / st64, "launch_ms": kt64,
                               "note": "same LP and method with float64 data and iterates"}
        print(f"# float64 passes: {st64 / (ms64 * 1e-3):.0f} iters/s", file=sys.stderr, flush=True)

    if not args.no_solve and len(lps) == 1:
        print("# solve to rel KKT 1e-4, float32", file=sys.stderr, flush=True)
        line["solve_fp32"] = _solve_leg(lps[0], opts, stream, args.solve_seconds)
        if args.workload == "mip20k":
            line["solve_fp64"] = _solve_leg(lps[0], opts, stream, args.solve_seconds, precision=1)

    if args.workload == "powerlaw1m" and not args.no_legs:
        print("# batch leg", file=sys.stderr, flush=True)
        line["batch"] = _batch_leg(args, stream)
        print("# serving leg", file=sys.stderr, flush=True)
        sv = _serve(args, rate=args.rate, seconds=args.serve_leg_seconds, pool_size=args.pool,
                    drain=args.serve_leg_drain, emit=False)
        line["serving"] = _serving_summary(sv)
        # where the latency-throughput curve bends: short streams below the 200/s overload
        knee = []
        for rate in args.knee_rates:
            sv = _serve(args, rate=rate, seconds=5.0, pool_size=16, drain=10.0, emit=False)
            knee.append({"rate_per_s": rate, "lps_per_s": sv["value"], "finished": sv["finished"],
                         "unfinished": sv["unfinished"], "latency_p50_s": sv["latency_p50_s"],
                         "latency_p99_s": sv["latency_p99_s"]})
            print(f"# knee: {rate}/s -> {sv['value']:.2f} LPs/s, p50 {sv['latency_p50_s']}", file=sys.stderr,
                  flush=True)
        line["serving"]["knee"] = knee
        print("# cache-resident leg", file=sys.stderr, flush=True)
        line["cache_resident"] = _c1_leg(args, stream)
    elif args.serve_rate > 0 and len(lps) == 1:
        sv = _serve(args, rate=args.serve_rate, seconds=args.serve_leg_seconds, pool_size=16,
                    drain=args.serve_leg_drain, emit=False)
        line["serving"] = _serving_summary(sv)

    if not args.no_cpu_baseline:
        print("# oracle on the host", file=sys.stderr, flush=True)
        rate, k, el = _cpu_baseline(lps, opts, args.cpu_seconds)
        line["cpu_baseline"] = {"value": rate, "unit": "iters/s", "cores": 1, "kind": "oracle", **_host_cpu(),
                                "sample": f"the first {k} loop passes (after 3 untimed) of the float64 oracle on "
                                          f"the same LP, Ruiz-scaled and float32-rounded ({el:.1f} s, one thread)"}
    print(json.dumps(line), flush=True)


def _serving_summary(sv):
    out = {k: sv[k] for k in ("value", "unit")}
    out.update({k: sv[k] for k in ("requests", "finished", "unfinished", "converged", "seconds", "finished_per_s",
                                   "latency_p50_s", "latency_p99_s", "latency_max_s",
                                   "latency_p99_with_unfinished_lower_bound_s", "server")})
    out["workload"] = sv["config"]["workload"]
    return out


def _c1_leg(args, stream):
    """The 20k x 50k LP (cache-resident): loop passes per second in the
    persistent kernel, and solves to relative KKT 1e-4 in float32 and float64."""
    import paper_2508_08062_amd as P
    lps, opts, cfg = _workload("mip20k")
    s = P.Solver(lps[0], tol=0.0, max_iter=10 ** 9, **opts)
    ppl = 500
    steps, ms = _timed_passes(s, stream, 2000, 500, ppl)
    roof, launch, spmv = _launch_roofline(lps, opts, [s], s, stream, ppl, "mip20k")
    s.close()
    roof["note"] = "working set about 13 MB stays in L2/MALL: the pass is bound by latency, not HBM"
    return {"workload": cfg["workload"], "variant": cfg["variant"], "m_A": cfg["m_A"], "value": steps / (ms * 1e-3),
            "unit": "iters/s", "steps": steps, "ms_per_step": ms / steps, **spmv, "launch": launch,
            "roofline": roof, "solve_fp32": _solve_leg(lps[0], opts, stream, 60.0),
            "solve_fp64": _solve_leg(lps[0], opts, stream, 60.0, precision=1)}


if __name__ == "__main__":
    main()
