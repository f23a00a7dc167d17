"""Benchmark: CP-APR MU on one MI355X, Phi(n) nonzeros per second.

Default workload: one step = one whole CP-APR MU job on the 3-way
200,000 x 150,000 x 20,000 tensor with 20M Zipf(1.1) nonzeros (duplicates
kept), counts 1+Poisson(3), rank 16: plan creation (per-mode device sort), the
fixed 5 outer x 10 inner schedule over all three modes (Phi, KKT, MU update,
normalisation), and the log-likelihood of the result. Inputs are resident in
HBM before timing.

value = Phi nonzero visits per second over the whole step (Phi evaluations
        the solve actually computed x nnz / step time).
roofline: the Phi kernel, timed by HIP events on its own stream around every
        7th Phi launch of the timed steps, against HBM peak. achieved = the compulsory traffic
        M_min of one launch / its average duration, M_min per mode n being
        nnz (4(N-1) + 8) (the other modes' coordinates and the value; i_n
        follows from the segment table) + S_n (2 R 8 + 8) (per nonempty row
        the B row read, the Phi row written and a segment entry) + sum over
        m != n of I_m R w (every row of the other factors once, w = 8 or 4
        bytes as stored). traffic: bytes past L2 per launch from committed
        counter runs / the same duration.
hbm_probe: a measured 1 GiB device copy, for reference beside the peak.
cpu_baseline: the FP64 CPU oracle pinned to one host core, Phi over every
        mode of the same tensor (zipf4: a sample of it), median of 5 runs,
        with the host's CPU model and core count.
serving: a short Poisson trace of solve requests through the continuous-
        batching server and through one-at-a-time solves (--no-serve skips it;
        --workload serve runs the long trace).

Other workloads: --workload zipf4 (4-way, 100M nonzeros, R = 32, solve to KKT
1e-4), batch (512 tensors, batched graph replays), serve (a Poisson stream of
solve requests), mttkrp (MTTKRP of every mode on the same engine, the kernel of
CP-ALS), plan (plan creation and the in-row orders), tune (the launch-policy
model against a search); --precision mixed; --method pqnr | pdnr.

Prints one JSON line. Only one GPU is supported.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROF_EVERY = 7  # Phi launches per timed one in the job benchmarks
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "phi_traffic.json")


def phi_min_bytes(N, R, nnz, dims, segs, mode, word=8):
    """Compulsory HBM bytes M_min of one Phi launch for `mode`: per nonzero the
    other modes' coordinates and the value, 4(N-1) + 8 bytes (the row i_n is
    implied by a segment table); per nonempty row of this mode the B row read,
    the Phi row written (FP64 in both precisions) and an 8-byte segment entry;
    every row of the other factors once, as stored (w = 8, or 4 for FP32
    copies)."""
    fac = sum(dims[m] for m in range(N) if m != mode) * R * word
    return nnz * (4 * (N - 1) + 8) + segs[mode] * (2 * R * 8 + 8) + fac


def phi_kernel_bytes(N, R, nnz, segs, mode, word=8):
    """What this kernel reads and writes at least: every nonzero's N
    coordinates and value once (4N + 8 bytes; the kernel reads the row index
    per nonzero), every *referenced* row of the other factors once (segments
    of mode m = distinct rows of mode m), and per nonempty row one B row read
    and one Phi row write."""
    per_nnz = 4 * N + 8
    fac = sum(segs[m] for m in range(N) if m != mode) * R * word
    return nnz * per_nnz + fac + segs[mode] * R * (8 + 8)


def hess_min_bytes(N, R, nnz, dims, segs, mode, word=8):
    """Compulsory HBM bytes of one PDNR Hessian pass for `mode`: M_min's reads,
    and per nonempty row one B row read and one row of R*R + R accumulated
    doubles (Hessian and Phi) written, plus the segment entry."""
    fac = sum(dims[m] for m in range(N) if m != mode) * R * word
    return nnz * (4 * (N - 1) + 8) + segs[mode] * (R * 8 + (R * R + R) * 8 + 8) + fac


def phi_issued_bytes(N, R, nnz, segs, mode, word=8):
    """Bytes the kernel issues with no reuse at all (every gathered factor row
    counted per nonzero): the fused-kernel model of the paper's Section 3.2
    applied to this kernel."""
    return nnz * (4 * N + 8 + (N - 1) * R * word) + segs[mode] * R * (8 + 8)


def kernel_source_hash():
    """Hash of the Phi kernel's source with comments and whitespace removed, so
    that counters stay attached to the code they were taken on and only to it."""
    import re
    h = hashlib.sha256()
    for f in ("phi.hip", "internal.hpp"):
        with open(os.path.join(ROOT, "paper_2307_03276_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """Bytes per Phi launch past L2 (FETCH_SIZE and WRITE_SIZE, scaled by the
    factors a 1 GiB device copy gives) from committed rocprofv3 counter runs,
    or None if they were taken on another kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(f"{workload}/{precision}")
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def progress(msg):
    """A progress line on stderr (the result stays the one JSON line on stdout)."""
    print(f"# {msg}", file=sys.stderr, flush=True)


def _counter_rows(path, counter):
    """(kernel name, value) per dispatch, in dispatch order, of one counter in a
    rocprofv3 --pmc csv (counter_collection.csv)."""
    import csv
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return [(k, v) for _, k, v in rows]


def record_traffic(fetch_csv, write_csv, workload, precision):
    """Bytes past L2 per Phi launch from two rocprofv3 counter runs of
    `bench.py --profile-phi` (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch),
    each scaled by what the same counter reads for the run's 1 GiB device copy;
    stored in the traffic file under the workload, precision and the kernel
    source's hash."""
    scaled = []
    factors = []
    names = set()
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        rows = _counter_rows(path, counter)
        copy = max((v for k, v in rows if "copyBuffer" in k or "copy" in k.lower()), default=0.0)
        if copy <= 0:
            raise SystemExit(f"{path}: no device copy to calibrate {counter}")
        factor = float(1 << 30) / (copy * 1024.0)
        phi = [v * 1024.0 * factor for k, v in rows if "phi_seg_kernel" in k]
        names.update(k for k, v in rows if "phi_seg_kernel" in k)
        scaled.append(phi)
        factors.append(factor)
    if len(scaled[0]) != len(scaled[1]) or not scaled[0]:
        raise SystemExit("the two runs hold different numbers of Phi dispatches")
    per_launch = [a + b for a, b in zip(*scaled)]
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        d = {}
    key = f"{workload}/{precision}"
    d[key] = {"bytes_per_launch": sum(per_launch) / len(per_launch), "per_launch_bytes": per_launch,
              "fetch_factor": factors[0], "write_factor": factors[1], "kernel": sorted(names)[0],
              "kernel_hash": kernel_source_hash()}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    print(json.dumps({key: d[key]}), flush=True)


def host_cpu():
    """The host's CPU model and core counts (what the CPU baseline ran on)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    allowed = sorted(os.sched_getaffinity(0))
    return {"cpu_model": model, "nproc": os.cpu_count(), "cores_allowed": len(allowed)}, allowed


def cpu_baseline(X, M, modes=None, max_nnz=None, runs=5, kind="phi"):
    """The FP64 oracle's Phi (or MTTKRP, kind="mttkrp") on the host: one thread
    pinned to one core, median of `runs` runs, each over `modes` modes of the
    first max_nnz nonzeros (nonzeros are drawn independently, so a prefix is a
    fair sample)."""
    import numpy as np

    import oracle
    from paper_2307_03276_amd import synth
    oracle.build(force=False)
    info, allowed = host_cpu()
    modes = X.nmodes if modes is None else modes
    if max_nnz is not None and X.nnz > max_nnz:
        X = synth.SparseTensor(X.dims, np.ascontiguousarray(X.idx[:, :max_nnz]), X.vals[:max_nnz].copy())
    Bs = [M.factors[n] * M.lam for n in range(modes)]
    core = allowed[-1]
    os.sched_setaffinity(0, {core})  # this thread only: the oracle call runs on it
    try:
        times = []
        for _ in range(runs):
            t0 = time.perf_counter()
            for n in range(modes):
                if kind == "mttkrp":
                    oracle.mttkrp(X, n, M.factors)
                else:
                    oracle.phi(X, n, Bs[n], M.factors)
            times.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, set(allowed))
    med = float(np.median(times))
    return dict({"value": modes * X.nnz / med, "unit": "nonzeros/s", "cores": 1, "kind": "oracle",
                 "pinned_core": core, "runs": runs, "run_s": times,
                 "sample": f"FP64 oracle {'MTTKRP' if kind == 'mttkrp' else 'Phi(n)'} over {modes} mode(s) of the "
                           f"first {X.nnz} nonzeros of the same "
                           f"tensor per run, single thread pinned to one core, median of {runs} runs "
                           f"({sum(times):.1f} s in all)"}, **info)


def hbm_probe(torch):
    """Device-to-device copy of 1 GiB (read + write), best of five, as a measured
    reference beside the 8 TB/s peak."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    gbs = 2 * src.numel() * 8 / (best / 1000.0) / 1e9
    del src, dst
    return {"copy_GBs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS, "bytes": 2 * (1 << 30)}


def batch_workload(args):
    """512 independent 3-way tensors (dims U{50..5000}, nnz LogUniform[1e3, 1e6],
    R in {8, 16, 32}): Phi of every tensor for one mode per graph replay, all
    three modes per step, against 512 one-at-a-time launches per mode."""
    import numpy as np
    import torch

    import oracle
    from paper_2307_03276_amd import cpapr, synth, tune

    prec = cpapr.CPAPR_MIXED if args.precision == "mixed" else cpapr.CPAPR_FP64
    pairs = synth.config_batch(seed=0, count=args.batch_count)
    dev = torch.device("cuda")
    stream = torch.cuda.Stream()
    total_nnz = sum(X.nnz for X, _ in pairs)
    with torch.cuda.stream(stream):
        items = []
        for X, M in pairs:
            P = cpapr.Plan.from_tensor(X, M.rank, precision=prec, stream=stream)
            A = [torch.from_numpy(a).to(dev) for a in M.factors]
            lam = torch.from_numpy(M.lam).to(dev)
            per_mode = []
            for n in range(3):
                B = (A[n] * lam).contiguous()
                Phi = torch.empty((X.dims[n], M.rank), dtype=torch.float64, device=dev)
                per_mode.append(dict(P=P, n=n, B=B, A=A, Phi=Phi))
            items.append(per_mode)
        tuner = tune.Autotuner(reps=2)
        choices = tuner.tune_items([it[0] for it in items])
        batches = []
        for n in range(3):
            tiles = sum(it[n]["P"].tiles() for it in items)
            b = cpapr.Batch(len(items), tiles + 1)
            for sl, it in enumerate(items):
                b.set(sl, it[n]["P"], n, it[n]["B"], it[n]["A"], it[n]["Phi"])
            b.commit(stream)
            b.run(use_graph=True, stream=stream)  # captures
            batches.append(b)
        torch.cuda.synchronize()

        def batched_step():
            for b in batches:
                b.run(use_graph=True, stream=stream)

        def single_step():
            for n in range(3):
                for it in items:
                    d = it[n]
                    d["P"].phi(n, d["B"], d["A"], out=d["Phi"], stream=stream)

        def timed(fn):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1000.0 / args.steps

        ms_batched = timed(batched_step)
        # one at a time, each plan on its standalone model shape (small tensors
        # take small tiles so that one launch fills the device), not on the
        # shape tuned for its batch class
        for it in items:
            it[0]["P"].set_shape(0, 0)
        ms_single = timed(single_step)
        # errors against the oracle on a sample of tensors (batched results)
        worst = 0.0
        for i in list(range(0, len(items), max(1, len(items) // 8)))[:8]:
            X, M = pairs[i]
            for n in range(3):
                ref = oracle.phi(X, n, M.factors[n] * M.lam, M.factors)
                got = items[i][n]["Phi"].cpu().numpy()
                mask = np.abs(ref) >= 1e-100
                worst = max(worst, float(np.max(np.abs(got[mask] - ref[mask]) / np.abs(ref[mask]))))
    out = {
        "metric": "batched Phi^(n) nonzeros/s",
        "value": 3 * total_nnz / (ms_batched / 1000.0),
        "unit": "nonzeros/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batched,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == cpapr.CPAPR_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": f"{len(items)} independent 3-way tensors, dims U[50,5000], nnz LogUniform[1e3,1e6], "
                               "R in {8,16,32}; one graph replay per mode over all tensors",
                   "tensors": len(items), "total_nnz": total_nnz, "precision": args.precision},
        "one_at_a_time": {"ms_per_step": ms_single, "nnz_per_s": 3 * total_nnz / (ms_single / 1000.0),
                          "launches_per_step": 3 * len(items)},
        "speedup_vs_one_at_a_time": ms_single / ms_batched,
        "max_rel_err_vs_oracle_sampled": worst,
        "autotuner": {k: {"group": v["group"], "chunk": v["chunk"], "ms": v["ms"],
                          "model": v.get("model"), "model_ms": v.get("model_ms"),
                          "model_vs_tuned": v.get("model_vs_tuned"), "fastest_candidates": v.get("candidates", [])[:6]}
                      for k, v in choices.items()},
    }
    print(json.dumps(out), flush=True)


def _max_rel(got, ref):
    """Normwise relative difference ||got - ref|| / ||ref||."""
    import numpy as np
    n = float(np.linalg.norm(ref))
    return float(np.linalg.norm(np.asarray(got) - ref) / n) if n > 0 else float(np.linalg.norm(got))


def _request_tensor(r):
    from paper_2307_03276_amd import synth
    return synth.request_tensor(r)


def generate_requests(count, seed=0, workers=1):
    """The serving trace's requests (tensors generated on the host). workers > 1
    forks a process pool: call it before the GPU is first used, so the children
    hold no GPU state."""
    from paper_2307_03276_amd import serve, synth
    trace = synth.serving_trace(seed=seed, count=count)
    t0 = time.perf_counter()
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            tensors = []
            for i, t in enumerate(pool.imap(_request_tensor, trace, chunksize=4)):
                tensors.append(t)
                if (i + 1) % 50 == 0:
                    progress(f"serving: {i + 1} of {len(trace)} requests generated")
    else:
        tensors = []
        for i, r in enumerate(trace):
            tensors.append(synth.request_tensor(r))
            if (i + 1) % 50 == 0:
                progress(f"serving: {i + 1} of {len(trace)} requests generated")
    reqs = [serve.Request(id=r["id"], X=X, M=M, arrival=r["arrival"]) for r, (X, M) in zip(trace, tensors)]
    progress(f"serving: {len(reqs)} requests generated in {time.perf_counter() - t0:.1f} s")
    return reqs, time.perf_counter() - t0


def run_serving(count, warmup, prec, fp64_checks=2, seed=0, policy="srpt", round_cap=32e6, round_cap_min=4e6,
                reqs=None):
    """Poisson arrivals at 200 requests/s of CP-APR MU solves (3- or 4-way, dims
    U[1e3, 1e5], nnz LogUniform[1e4, 2e7], Zipf(1.1), R in {10, 16, 32}, KKT
    tolerance 1e-4, k_max 20), admitted by a 200 GB HBM budget; against the
    same trace served one request at a time. Accuracy: every served result
    against the same request solved alone (same precision), and `fp64_checks`
    requests of the trace against an FP64 solve of the same request."""
    import numpy as np
    import torch

    from paper_2307_03276_amd import cpapr, serve, synth

    if reqs is None:
        reqs, t_gen = generate_requests(count + warmup, seed=seed)
    else:
        t_gen = None
    kw = dict(kmax=20, lmax=10, tol=1e-4, precision=prec)
    warm, meas = reqs[:warmup], reqs[warmup:]
    t_first = meas[0].arrival
    for r in meas:
        r.arrival -= t_first
    for r in warm:
        r.arrival = 0.0
    serve.Server(budget_bytes=200e9, max_slots=64, **kw).run_trace(warm)
    torch.cuda.synchronize()
    # every active request in every round (the plain continuous batching)
    srv_all = serve.Server(budget_bytes=200e9, max_slots=64, **kw)
    done_all = srv_all.run_trace([serve.Request(id=r.id, X=r.X, M=r.M, arrival=r.arrival) for r in meas])
    summary_all = serve.latency_summary(done_all)
    del done_all  # frees the results' device memory
    torch.cuda.synchronize()
    progress(f"serving: every request every round done ({summary_all.get('solves_per_s', 0):.1f} solves/s)")
    srv = serve.Server(budget_bytes=200e9, max_slots=64, policy=policy, round_cap=round_cap,
                       round_cap_min=round_cap_min, **kw)
    done = srv.run_trace(meas)
    summary = serve.latency_summary(done)
    serve.results_to_host(done)  # after the timed trace
    by_id = {r.id: r for r in done}
    progress(f"serving: {policy} done ({summary.get('solves_per_s', 0):.1f} solves/s); one request at a time next")
    # the plain path on the same trace: one request at a time, in arrival order
    clock = 0.0
    ttc, busy = [], 0.0
    err_lam, err_fac = 0.0, 0.0
    fac_errs = {}
    stream = torch.cuda.Stream()
    for r in sorted(meas, key=lambda q: q.arrival):
        start = max(clock, r.arrival)
        t0 = time.perf_counter()
        lam1, facs1, _ = serve.solve_one(serve.Request(id=r.id, X=r.X, M=r.M, arrival=r.arrival), stream=stream, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        lam1, facs1 = lam1.cpu().numpy(), [a.cpu().numpy() for a in facs1]  # outside the timed solve
        busy += dt
        clock = start + dt
        ttc.append(clock - r.arrival)
        s = by_id.get(r.id)
        if s is not None and s.result_lam is not None:
            err_lam = max(err_lam, _max_rel(s.result_lam, lam1))
            fac_errs[r.id] = max(_max_rel(a, b) for a, b in zip(s.result_factors, facs1))
            err_fac = max(err_fac, fac_errs[r.id])
    # served results (this precision) against FP64 solves of the same requests:
    # the smallest and the largest request, and the one whose served and
    # one-at-a-time results differ most
    fp64 = []
    pick = sorted(meas, key=lambda q: q.X.nnz)
    checks = [pick[(i * (len(pick) - 1)) // max(1, fp64_checks - 1)] for i in range(fp64_checks)] if pick else []
    if fac_errs:
        worst = max(fac_errs, key=fac_errs.get)
        if all(r.id != worst for r in checks):
            checks.append(next(r for r in meas if r.id == worst))
    for r in checks:
        s = by_id[r.id]
        lam64, facs64, st64 = serve.solve_one(serve.Request(id=r.id, X=r.X, M=r.M), stream=stream,
                                              **dict(kw, precision=cpapr.CPAPR_FP64))
        lam64, facs64 = lam64.cpu().numpy(), [a.cpu().numpy() for a in facs64]
        fp64.append({"id": r.id, "nnz": r.X.nnz, "rank": r.M.rank, "lambda_rel": _max_rel(s.result_lam, lam64),
                     "factors_rel": max(_max_rel(a, b) for a, b in zip(s.result_factors, facs64)),
                     "loglik_rel": abs(s.stats.get("loglik", float("nan")) - st64["loglik"]) / abs(st64["loglik"]),
                     "outer_iters": [s.stats.get("outer_iters"), st64["outer_iters"]]})
    ttc = np.array(ttc)
    nnz = np.array([r.X.nnz for r in meas])
    span = float(max(r.arrival for r in meas)) if meas else 0.0
    return {
        "requests": len(meas), "warmup_requests": len(warm), "total_nnz": int(nnz.sum()),
        "mean_nnz": float(nnz.mean()), "arrival_span_s": span,
        "offered_req_per_s": (len(meas) - 1) / span if span > 0 else None,
        "served": dict(summary, policy=policy, round_cap_nnz=[round_cap_min, round_cap], peak_active=srv.peak_active,
                       peak_hbm_bytes=srv.peak_used, ticks=srv.ticks,
                       host_phase_s={k: round(v, 4) for k, v in srv.phase_s.items()},
                       converged=int(sum(1 for r in done if r.stats.get("converged"))),
                       mean_outer_iters=float(np.mean([r.stats["outer_iters"] for r in done]))),
        "served_all_each_round": dict(summary_all, ticks=srv_all.ticks,
                                      host_phase_s={k: round(v, 4) for k, v in srv_all.phase_s.items()}),
        "one_at_a_time": {"p50_from_arrival_s": float(np.percentile(ttc, 50)),
                          "p99_from_arrival_s": float(np.percentile(ttc, 99)),
                          "solves_per_s": len(meas) / clock, "busy_s": busy},
        "accuracy": {"served_vs_alone_lambda_rel_max": err_lam, "served_vs_alone_factors_rel_max": err_fac,
                     "served_vs_alone_factors_rel_median": float(np.median(list(fac_errs.values()))) if fac_errs else None,
                     "vs_fp64_solve": fp64},
        "generation_s": t_gen,
    }


def serve_workload(args, reqs=None):
    """The long served trace as its own JSON line."""
    from paper_2307_03276_amd import cpapr

    prec = cpapr.CPAPR_MIXED if args.precision == "mixed" else cpapr.CPAPR_FP64
    res = run_serving(args.serve_count, args.serve_warmup, prec, round_cap=args.round_cap,
                      round_cap_min=args.round_cap_min, reqs=reqs)
    out = {
        "metric": "served solves/s",
        "value": res["served"]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": args.serve_warmup, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == cpapr.CPAPR_MIXED else "f64", "data": "synthetic",
        "config": {"workload": "Poisson 200 req/s CP-APR MU solves, 3/4-way, dims U[1e3,1e5], nnz LogUniform[1e4,2e7], "
                               "Zipf(1.1), R in {10,16,32}, tol 1e-4, kmax 20, HBM budget 200 GB",
                   "precision": args.precision},
    }
    out.update(res)
    print(json.dumps(out), flush=True)


def tune_workload(args):
    """The launch-policy model against a measured search: for every mode of
    tensors from 1e4 to 1e8 nonzeros (uniform and Zipf, R = 8..32, N = 3 and 4,
    both precisions) Phi is timed at every (lanes, chunk) candidate and at the
    model's shape; model_vs_tuned = model time / fastest time."""
    import numpy as np
    import torch

    from paper_2307_03276_amd import cpapr, synth, tune

    cases = []
    rng = np.random.default_rng(5)
    for i, (N, nnz, R) in enumerate([(3, 10_000, 8), (3, 50_000, 16), (3, 100_000, 32), (3, 200_000, 16),
                                     (3, 400_000, 16), (3, 400_000, 32), (3, 700_000, 32), (3, 1_000_000, 8),
                                     (3, 1_000_000, 16), (3, 1_000_000, 32), (4, 400_000, 16), (4, 400_000, 32)]):
        dims = tuple(int(d) for d in rng.integers(100, 5000, size=N))
        cases.append((f"uniform {N}-way {dims}, {nnz} nnz, R={R}", lambda d=dims, z=nnz, r=R, s=900 + i: (
            synth.random_tensor(s, d, z), synth.random_model(s, d, r))))
    cases.append(("Zipf 3-way 20000x15000x2000, 2M nnz, R=16", lambda: (
        synth.random_tensor(950, (20000, 15000, 2000), 2_000_000, zipf=(1.1, 1.1, 1.1), mu=3.0),
        synth.random_model(950, (20000, 15000, 2000), 16))))
    cases.append(("zipf3: 3-way 200000x150000x20000, 20M nnz, R=16", lambda: synth.config_zipf3()[:2]))
    cases.append(("zipf4: 4-way 1000000x200000x10000x500, 100M nnz, R=32", lambda: synth.config_zipf4()[:2]))
    rows = []
    dev = torch.device("cuda")
    for name, make in cases:
        X, M = make()
        idx = torch.from_numpy(X.idx).to(dev)
        vals = torch.from_numpy(X.vals).to(dev)
        A = [torch.from_numpy(a).to(dev) for a in M.factors]
        lam = torch.from_numpy(M.lam).to(dev)
        for prec in (cpapr.CPAPR_FP64, cpapr.CPAPR_MIXED):
            P = cpapr.Plan(X.dims, idx, vals, M.rank, precision=prec)
            res = tune.tune_plan(P, lambda n: ((A[n] * lam).contiguous(), A))
            for r in res:
                r.update(tensor=name, precision="fp64" if prec == cpapr.CPAPR_FP64 else "mixed", nnz=X.nnz,
                         rank=M.rank, segments=P.segments(r["mode"]))
                print(f"# {name} {r['precision']} mode {r['mode']}: model {tuple(r['model'])} {r['model_ms']:.4f} ms, "
                      f"best {tuple(r['best'])} {r['best_ms']:.4f} ms, ratio {r['model_vs_tuned']:.3f}", flush=True)
                rows.append(r)
            P.close()
        del idx, vals, A, lam
        torch.cuda.empty_cache()
    worst = max(r["model_vs_tuned"] for r in rows)
    out = {"metric": "launch-policy model time / fastest measured shape (Phi per mode)", "value": worst,
           "unit": "ratio", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64 and f32+f64", "data": "synthetic",
           "config": {"workload": f"per-mode launch-shape search over {len(cases)} tensors x 2 precisions"},
           "within_5pct": sum(r["model_vs_tuned"] <= 1.05 for r in rows), "modes_timed": len(rows),
           "cases": [{k: r[k] for k in ("tensor", "precision", "mode", "nnz", "rank", "segments", "model", "model_ms",
                                          "best", "best_ms", "model_vs_tuned", "finalists", "candidates")}
                     for r in rows]}
    print(json.dumps(out), flush=True)


def mttkrp_min_bytes(N, R, nnz, dims, segs, mode):
    """Compulsory HBM bytes of one MTTKRP launch for `mode` (Eqs. 10-12): per
    nonzero the other modes' coordinates and the value, 4(N-1) + 8 bytes; per
    nonempty row of this mode the output row written and an 8-byte segment
    entry; every row of the other factors once (FP64). Phi's M_min without the
    B row reads."""
    fac = sum(dims[m] for m in range(N) if m != mode) * R * 8
    return nnz * (4 * (N - 1) + 8) + segs[mode] * (R * 8 + 8) + fac


def mttkrp_workload(args):
    """MTTKRP, the kernel of CP-ALS (Eqs. 10-12: M(n) = X_(n) times the
    Khatri-Rao product of the other factors), on the same plan and tile code
    as Phi: one step = one MTTKRP per mode of the zipf3 (or, with --tensor
    zipf4, the zipf4) tensor, FP64, with the plan built beforehand (an ALS
    solver builds it once and calls MTTKRP every sweep)."""
    import math

    import torch

    from paper_2307_03276_amd import cpapr, synth

    if args.tensor == "zipf4":
        X, M, _ = synth.config_zipf4()
        wl_name = "mttkrp-zipf4-100M-R32"
        wl_desc = ("mttkrp 4-way 1000000x200000x10000x500, 100M nnz (Zipf(1.2) modes 1-2, uniform 3-4), R=32, "
                   "one MTTKRP per mode per step, plan prebuilt")
    else:
        X, M, _ = synth.config_zipf3(nnz=args.nnz)
        wl_name = "mttkrp-zipf3-20M-R16"
        wl_desc = ("mttkrp 3-way 200000x150000x20000, 20M Zipf(1.1) nnz, R=16, one MTTKRP per mode per step, "
                   "plan prebuilt")
    N, R = X.nmodes, M.rank
    dev = torch.device("cuda")
    progress(f"{wl_name}: building the plan")
    P = cpapr.Plan.from_tensor(X, R)
    A = [torch.from_numpy(a).to(dev) for a in M.factors]
    outs = [torch.empty((X.dims[n], R), dtype=torch.float64, device=dev) for n in range(N)]
    segs = [P.segments(n) for n in range(N)]
    if args.profile_phi:
        progress("MTTKRP twice per mode, then a 1 GiB device copy")
        for n in range(N):
            for _ in range(2):
                P.mttkrp(n, A, out=outs[n])
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        P.close()
        print("profile-mttkrp done", flush=True)
        return

    def step():
        for n in range(N):
            P.mttkrp(n, A, out=outs[n])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # every `every`-th launch bracketed by events; every is coprime to N so
    # that all modes are sampled
    every = next(k for k in range(2, 10) if math.gcd(k, N) == 1)
    cap = N * args.steps // every + 16
    cpapr.cpapr_prof_enable_sampled(cap, every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    recs = cpapr.cpapr_prof_read(cap)
    cpapr.cpapr_prof_disable()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = N * X.nnz / (ms_per_step / 1000.0)
    tot_bytes = sum(mttkrp_min_bytes(N, R, X.nnz, list(X.dims), segs, m) for m, _ in recs)
    tot_ms = sum(ms for _, ms in recs)
    avg_ms = tot_ms / max(1, len(recs))
    achieved = tot_bytes / (tot_ms / 1000.0) / 1e9
    per_mode_ms = [sum(ms for m, ms in recs if m == n) / max(1, sum(1 for m, _ in recs if m == n)) for n in range(N)]
    traffic_bytes = measured_traffic(wl_name, "fp64")
    traffic = None if traffic_bytes is None else traffic_bytes / (avg_ms / 1000.0) / 1e9
    out = {"metric": "MTTKRP nonzeros/s", "value": value, "unit": "nonzeros/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": wl_desc, "nnz": X.nnz, "rank": R},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
           "mttkrp_kernel": {"kernel": "phi_seg_kernel (MTTKRP)", "launches": len(recs), "sampled_every": every,
                             "avg_ms": avg_ms, "avg_ms_per_mode": per_mode_ms,
                             "min_bytes_per_launch": tot_bytes / max(1, len(recs)),
                             "measured_bytes_per_launch": traffic_bytes, "segments": segs}}
    if not args.no_cpu_baseline:
        progress("CPU baseline (the oracle's MTTKRP on the host)")
        out["cpu_baseline"] = cpu_baseline(X, M, modes=1 if N > 3 else None,
                                           max_nnz=10_000_000 if N > 3 else None, kind="mttkrp")
    P.close()
    print(json.dumps(out), flush=True)


def plan_workload(args):
    """Plan creation against the in-row order it buys: for the zipf3 and zipf4
    tensors (FP64) and both sort orders, the plan's creation time (host clock
    around the call, median of 3) and Phi per mode (library-recorded kernel
    time, median of 7 launches), and the largest difference between the two
    orders' Phi (the order only changes rounding)."""
    import time

    import torch

    from paper_2307_03276_amd import cpapr, synth

    dev = torch.device("cuda")
    cases = []
    for name, make in (("zipf3-20M-R16", lambda: synth.config_zipf3()[:2]),
                       ("zipf4-100M-R32", lambda: synth.config_zipf4()[:2])):
        progress(f"generating the {name} tensor on the host")
        X, M = make()
        R = M.rank
        idx = torch.from_numpy(X.idx).to(dev)
        vals = torch.from_numpy(X.vals).to(dev)
        A = [torch.from_numpy(a).to(dev) for a in M.factors]
        lam = torch.from_numpy(M.lam).to(dev)
        phis = {}
        for sort, sname in ((cpapr.CPAPR_SORT_ROW_COL, "row_col"), (cpapr.CPAPR_SORT_ROW, "row")):
            ts = []
            for rep in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                P = cpapr.Plan(X.dims, idx, vals, R, sort=sort)
                torch.cuda.synchronize()
                ts.append(1e3 * (time.perf_counter() - t0))
                if rep < 2:
                    P.close()
            per_mode, outs = [], []
            for n in range(X.nmodes):
                B = (A[n] * lam).contiguous()
                out = torch.empty((X.dims[n], R), dtype=torch.float64, device=dev)
                P.phi(n, B, A, out=out)
                torch.cuda.synchronize()
                cpapr.cpapr_prof_enable(7)
                for _ in range(7):
                    P.phi(n, B, A, out=out)
                torch.cuda.synchronize()
                recs = cpapr.cpapr_prof_read(7)
                cpapr.cpapr_prof_disable()
                per_mode.append(sorted(t for _, t in recs)[3])
                outs.append(out.cpu())
            phis[sname] = outs
            cases.append({"tensor": name, "sort": sname, "plan_ms": sorted(ts)[1], "plan_ms_reps": ts,
                          "phi_ms_per_mode": per_mode, "phi_ms_sum": sum(per_mode)})
            progress(f"{name} {sname}: plan {sorted(ts)[1]:.2f} ms, Phi summed over modes {sum(per_mode):.4f} ms")
            P.close()
            torch.cuda.empty_cache()
        cases[-1]["phi_max_rel_diff_between_orders"] = max(
            float((a - b).abs().max() / a.abs().max()) for a, b in zip(phis["row_col"], phis["row"]))
        del idx, vals, A, lam
        torch.cuda.empty_cache()
    out = {"metric": "plan creation time (ROW_COL order, zipf3)", "value": cases[0]["plan_ms"], "unit": "ms",
           "n_gpus": 1, "steps": 3, "warmup": 0, "ms_per_step": cases[0]["plan_ms"], "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "plan creation and Phi per mode, both in-row orders, zipf3 and zipf4"},
           "cases": cases}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--method", choices=["mu", "pqnr", "pdnr"], default="mu",
                    help="inner solver of the zipf3 / zipf4 jobs: MU (Algorithm 1), PQNR or PDNR row solves")
    ap.add_argument("--nnz", type=int, default=20_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["zipf3", "zipf4", "batch", "serve", "tune", "plan", "mttkrp"],
                    default="zipf3",
                    help="zipf3: the 20M-nonzero 3-way CP-APR MU job (default); zipf4: the 100M-nonzero 4-way "
                         "solve to KKT 1e-4; batch: 512 uneven tensors; serve: a Poisson stream of solve requests; "
                         "tune: the launch-policy model against a search; plan: plan creation and the in-row orders; "
                         "mttkrp: MTTKRP per mode on the zipf3 (or --tensor zipf4) tensor")
    ap.add_argument("--tensor", choices=["zipf3", "zipf4"], default="zipf3", help="tensor of --workload mttkrp")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--serve-count", type=int, default=60)
    ap.add_argument("--round-cap", type=float, default=32e6,
                    help="serving: most nonzeros per round of the shortest-remaining-work policy")
    ap.add_argument("--round-cap-min", type=float, default=4e6,
                    help="serving: the round cap's floor (the cap is an eighth of the pending nonzeros, clamped)")
    ap.add_argument("--serve-warmup", type=int, default=6)
    ap.add_argument("--no-serve", action="store_true", help="skip the short served trace of the default run")
    ap.add_argument("--short-serve-count", type=int, default=16)
    ap.add_argument("--short-serve-warmup", type=int, default=4)
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="store bytes past L2 per Phi launch from two rocprofv3 counter runs of --profile-phi "
                         "(FETCH_SIZE, WRITE_SIZE) for --workload / --precision, then exit")
    ap.add_argument("--profile-phi", action="store_true",
                    help="counter-collection driver: two Phi launches per mode on the benchmark tensor (MTTKRP "
                         "launches with --workload mttkrp), then a 1 GiB device copy that calibrates the byte "
                         "counters; prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.record_traffic:
        names = {"zipf3": "zipf3-20M-R16", "zipf4": "zipf4-100M-R32"}
        wl = names.get(args.workload)
        if args.workload == "mttkrp":
            wl = "mttkrp-" + names[args.tensor]
        if wl is None:
            raise SystemExit("--record-traffic takes --workload zipf3, zipf4 or mttkrp")
        record_traffic(args.record_traffic[0], args.record_traffic[1], wl, args.precision)
        return

    serve_reqs = None
    if args.workload == "serve":
        # generated in forked workers before the GPU is first used
        serve_reqs, _ = generate_requests(args.serve_count + args.serve_warmup, workers=8)

    import numpy as np
    import torch

    from paper_2307_03276_amd import cpapr, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "batch":
        batch_workload(args)
        return
    if args.workload == "tune":
        tune_workload(args)
        return
    if args.workload == "plan":
        plan_workload(args)
        return
    if args.workload == "mttkrp":
        mttkrp_workload(args)
        return
    if args.workload == "serve":
        if args.precision == "fp64" and "--precision" not in sys.argv:
            args.precision = "mixed"  # the served configuration stores factors in FP32
        serve_workload(args, serve_reqs)
        return
    progress(f"generating the {args.workload} tensor on the host")
    if args.workload == "zipf4":
        X, M, sched = synth.config_zipf4()
        wl_name, wl_desc = "zipf4-100M-R32", ("cpapr-mu 4-way 1000000x200000x10000x500, 100M nnz (Zipf(1.2) modes 1-2, "
                                              "uniform 3-4), R=32, solve to KKT 1e-4 or 20 outer x 10 inner, "
                                              "plan + solve + loglik per step")
    else:
        X, M, sched = synth.config_zipf3(nnz=args.nnz)
        wl_name, wl_desc = "zipf3-20M-R16", ("cpapr-mu 3-way 200000x150000x20000, 20M Zipf(1.1) nnz, R=16, "
                                              "5 outer x 10 inner, plan + solve + loglik per step")
    N, R = X.nmodes, M.rank
    prec = cpapr.CPAPR_MIXED if args.precision == "mixed" else cpapr.CPAPR_FP64
    method = {"mu": cpapr.CPAPR_METHOD_MU, "pqnr": cpapr.CPAPR_METHOD_PQNR,
              "pdnr": cpapr.CPAPR_METHOD_PDNR}[args.method]
    if method != cpapr.CPAPR_METHOD_MU:
        wl_desc = wl_desc.replace("cpapr-mu", "cpapr-" + args.method)
    params = cpapr.cpapr_params_default(kmax=sched["kmax"], lmax=sched["lmax"], tol=sched["tau"],
                                        eps=sched["eps"], precision=prec, method=method)
    dev = torch.device("cuda")
    idx = torch.from_numpy(X.idx).to(dev)
    vals = torch.from_numpy(X.vals).to(dev)
    lam0 = torch.from_numpy(M.lam).to(dev)
    A0 = [torch.from_numpy(a).to(dev) for a in M.factors]
    lam = lam0.clone()
    A = [a.clone() for a in A0]
    coo = cpapr.make_coo(X.dims, idx, vals)
    ws = torch.empty(cpapr.cpapr_plan_workspace_size(coo, R, params), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    if args.profile_phi:
        progress("Phi twice per mode, then a 1 GiB device copy")
        h = cpapr.cpapr_plan_create(coo, R, params, ws, stream)
        phi = torch.empty((max(X.dims), R), dtype=torch.float64, device=dev)
        for n in range(N):
            B = (A0[n] * lam0).contiguous()
            for _ in range(2):
                cpapr.cpapr_phi(h, n, B, A0, sched["eps"], phi, stream)
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        cpapr.cpapr_plan_destroy(h)
        print("profile-phi done", flush=True)
        return

    def step():
        h = cpapr.cpapr_plan_create(coo, R, params, ws, stream)
        lam.copy_(lam0)
        for a, a0 in zip(A, A0):
            a.copy_(a0)
        st = cpapr.cpapr_solve(h, lam, A, stream)
        segs = [cpapr.cpapr_plan_segments(h, n) for n in range(N)]
        cpapr.cpapr_plan_destroy(h)
        return st, segs

    progress(f"{wl_name} {args.precision}: plan inputs on the device; {args.warmup} warm-up steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    progress(f"{args.steps} timed steps")
    launches_per_step = sched["kmax"] * N * sched["lmax"]
    # Every 7th Phi launch of the timed steps is bracketed by HIP events (7 is
    # coprime to the 10 inner iterations and 3 modes, so every mode and inner
    # position is sampled); an event pair holds the stream for about 5 us on
    # either side of its kernel, so timing all launches would cost the job 3 %.
    cpapr.cpapr_prof_enable_sampled(launches_per_step * args.steps // PROF_EVERY + 16, PROF_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, segs = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    recs = cpapr.cpapr_prof_read(launches_per_step * args.steps // PROF_EVERY + 16)
    cpapr.cpapr_prof_disable()

    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    # passes over the nonzeros actually computed in one step: Phi passes, plus
    # the line-search passes of PQNR
    visits = (st["phi_evals"] + st["trial_evals"]) * X.nnz
    value = visits / (ms_per_step / 1000.0)
    # launches enqueued after an inner loop stopped exit at once; time only real ones
    med = sorted(ms for _, ms in recs)[len(recs) // 2] if recs else 0.0
    recs = [(m, ms) for m, ms in recs if ms > 0.2 * med]
    word = 4 if prec == cpapr.CPAPR_MIXED else 8
    dims = list(X.dims)
    pdnr = method == cpapr.CPAPR_METHOD_PDNR
    # the timed launches: Phi (MU, PQNR) or the Hessian pass (PDNR)
    minb = hess_min_bytes if pdnr else phi_min_bytes
    tot_bytes = sum(minb(N, R, X.nnz, dims, segs, m, word) for m, _ in recs)
    kern_bytes = sum(phi_kernel_bytes(N, R, X.nnz, segs, m, word) for m, _ in recs)
    issued = sum(phi_issued_bytes(N, R, X.nnz, segs, m, word) for m, _ in recs)
    tot_ms = sum(ms for _, ms in recs)
    achieved = tot_bytes / (tot_ms / 1000.0) / 1e9
    avg_ms = tot_ms / max(1, len(recs))
    per_mode_ms = [sum(ms for m, ms in recs if m == n) / max(1, sum(1 for m, _ in recs if m == n)) for n in range(N)]
    traffic_bytes = measured_traffic(wl_name, args.precision) if not pdnr else None
    traffic = None if traffic_bytes is None else traffic_bytes / (avg_ms / 1000.0) / 1e9
    out = {
        "metric": "Phi^(n) nonzeros/s" if args.method == "mu" else "nonzero passes/s (Phi + line search)",
        "value": value,
        "unit": "nonzeros/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == cpapr.CPAPR_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl_desc, "nnz": X.nnz, "rank": R, "outer": sched["kmax"], "inner": sched["lmax"],
                   "tol": sched["tau"], "precision": args.precision},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "phi_kernel": {"kernel": "pdnr_hess_kernel" if pdnr else "phi_seg_kernel",
                       "launches": len(recs), "avg_ms": avg_ms, "avg_ms_per_mode": per_mode_ms,
                       "nnz_per_s": X.nnz / (avg_ms / 1000.0),
                       "min_bytes_per_launch": tot_bytes / max(1, len(recs)),
                       "kernel_bytes_per_launch": kern_bytes / max(1, len(recs)),
                       "kernel_bytes_frac": kern_bytes / (tot_ms / 1000.0) / 1e9 / HBM_PEAK_GBS,
                       "issued_bytes_per_launch": issued / max(1, len(recs)),
                       "issued_GBs": issued / (tot_ms / 1000.0) / 1e9,
                       "measured_bytes_per_launch": traffic_bytes,
                       "segments": segs, "sampled_every": PROF_EVERY,
                       # the sampled launches stand for PROF_EVERY launches each
                       "share_of_step": PROF_EVERY * tot_ms / (ms_per_step * args.steps)},
        "solve": {"method": args.method, "outer": st["outer_iters"], "inner_updates": st["inner_iters"],
                  "phi_evals": st["phi_evals"], "trial_evals": st["trial_evals"], "row_steps": st["row_steps"],
                  "converged": bool(st["converged"]), "kkt": st["kkt_violation"], "loglik": st["loglik"]},
    }
    out["hbm_probe"] = hbm_probe(torch)
    del idx, vals, ws, A, A0, lam, lam0
    torch.cuda.empty_cache()
    progress(f"timed steps done: {ms_per_step:.1f} ms per step")
    if not args.no_serve and args.workload == "zipf3" and args.method == "mu":
        progress("short served trace")
        try:
            out["serving"] = run_serving(args.short_serve_count, args.short_serve_warmup, cpapr.CPAPR_MIXED,
                                         fp64_checks=1)
            out["serving"]["config"] = ("Poisson 200 req/s CP-APR MU solves, 3/4-way, dims U[1e3,1e5], nnz "
                                        "LogUniform[1e4,2e7], Zipf(1.1), R in {10,16,32}, tol 1e-4, kmax 20, "
                                        "HBM budget 200 GB, FP32-stored factors; a short trace")
        except Exception as e:  # the Phi line above stays valid
            out["serving"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        progress("CPU baseline (the oracle on the host)")
        if args.workload == "zipf4":
            out["cpu_baseline"] = cpu_baseline(X, M, modes=1, max_nnz=10_000_000)
        else:
            out["cpu_baseline"] = cpu_baseline(X, M)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
