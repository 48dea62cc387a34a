"""Throughput of the SPIDER hot path on one MI355X.

One step = minibatch selection, travel-time network forward and source
gradient, residuals, exact whitening, per-event reduction, priors and the
pSGLD update with Philox noise, for every chain (all rows of the hot path).
Metric: double-difference observation likelihood-gradient evaluations per
second = chains x batch x steps / wall time, with the catalog resident in HBM.

Prints one JSON line.  The default workload is the 200k-event clustered
catalog (~200M observations, 6->256x6->1 network, batch 2^20, 8 chains).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2500.0, "fp32": 157.3}       # TFLOP/s, MI355X dense
HBM_PEAK = 8000.0                             # GB/s

# HBM bytes per launch of the BF16 network kernel on the 200k-event workload
# (16,777,216 rows), from rocprofv3 FETCH_SIZE and WRITE_SIZE passes over the
# same command, each scaled by what the counter reads for a 1 GiB device copy
# (FETCH x2.0, WRITE x1.0); profiles/network_bf16_clustered200k_traffic.md.
# Valid only for the kernel built from the template sources with this digest
# and the same variant; otherwise the bench reports traffic as null.
NETWORK_TRAFFIC = {
    "kernel_sources": ["paper_2508_12117_amd/csrc/mlp_mfma.h", "paper_2508_12117_amd/csrc/mlp_pp.h",
                       "paper_2508_12117_amd/csrc/net_rows.h"],
    "sha256": "f6d4994416d9a8bbedd13597551fbd8d90bbf36d0d08403b8ccf5b4d3c01070e",
    "variant": {"waves": 8, "row_tiles": 4, "schedule": 2},
    "rows": 16777216,
    "fetch_bytes": 229268608,
    "write_bytes": 268435456,
}


SCHEDULES = {0: "barrier per layer", 1: "row-half ping-pong",
             2: "row-half ping-pong, 1.5-layer weight ring"}


def network_traffic(rows, variant):
    """Measured HBM bytes per network launch, or None if the kernel changed."""
    import hashlib
    h = hashlib.sha256()
    for f in NETWORK_TRAFFIC["kernel_sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if (h.hexdigest() != NETWORK_TRAFFIC["sha256"] or variant != NETWORK_TRAFFIC["variant"]
            or rows != NETWORK_TRAFFIC["rows"]):
        return None
    return NETWORK_TRAFFIC["fetch_bytes"] + NETWORK_TRAFFIC["write_bytes"]


def flops_per_eval(H, D):
    """Matrix flops of one travel-time evaluation, forward + source gradient:
    first layer 12H, D-1 hidden layers 2H^2 each way, output 2H, input
    gradient 6H + 2H."""
    return 4 * (D - 1) * H * H + 22 * H


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered200k")
    ap.add_argument("--precision", default="auto", choices=["auto", "bf16", "fp32", "both"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-batch", type=int, default=1 << 20)
    ap.add_argument("--seed", type=int, default=20250817)
    ap.add_argument("--moments-steps", type=int, default=300, metavar="K",
                    help="also run K sampler steps per precision (second half recorded, thin "
                         "10) and compare the BF16 and FP32 posterior moments (0: skip)")
    ap.add_argument("--no-graph-compare", action="store_true",
                    help="skip the graph-against-stream rates of the tiny catalog")
    ap.add_argument("--configs", action="store_true",
                    help="instead of the bench line: rates and errors of the tiny and "
                         "faults10k workloads on the GPU (FP32, BF16) and in the oracle")
    ap.add_argument("--stream-only", action="store_true",
                    help="launch every step on the stream, graphs off, and time only that pass "
                         "(per-kernel profiles: no graph branch overlaps one step's kernels "
                         "with the next step's)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="first copy BYTES between two device buffers (one device-to-device "
                         "copy of known size, to calibrate HBM byte counters in a profile)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_precision(ctx, spider, base_sets, step_size, prec, steps, warmup, seed, graphs=True):
    """base_sets: (cat_id, net_id, chains, batch) per catalog; several catalogs
    advance together in the library's fused steps.  Two timed passes of
    `steps` steps from the same warmed-up start: the step as the library runs
    it (one eager step, then replays of a HIP graph of one step) for the
    throughput, then with the network launches bracketed by HIP events on the
    library's stream (profiling launches every step on the stream) for the
    network kernel's time.  Returns (graph wall s, stream wall s, network ms,
    launches, rows).  With graphs off the first pass is skipped and its wall
    time is that of the second."""
    import torch
    sets = [(cid, nid, C, n, prec) for cid, nid, C, n in base_sets]

    def fresh():
        for cid, _, C, _ in base_sets:
            ctx.reset_chains(cid, C)
        ctx.sgld_steps(sets, warmup, step=step_size, seed=seed)
        ctx.sync()
        torch.cuda.synchronize()

    ctx.set_graphs(graphs)
    wall_graph = None
    if graphs:
        fresh()
        t0 = time.perf_counter()
        ctx.sgld_steps(sets, steps, step=step_size, seed=seed)
        ctx.sync()
        torch.cuda.synchronize()
        wall_graph = time.perf_counter() - t0
    fresh()
    ctx.profile(True)
    t0 = time.perf_counter()
    ctx.sgld_steps(sets, steps, step=step_size, seed=seed)
    ctx.sync()
    torch.cuda.synchronize()
    wall_stream = time.perf_counter() - t0
    ms, launches, rows = ctx.profile_read()
    ctx.profile(False)
    ctx.set_graphs(True)
    return wall_graph if graphs else wall_stream, wall_stream, ms, launches, rows


def small_catalog_rates(spider, seed, steps=2000):
    """Steps per second of the tiny catalog (200 events, 32,000 observations,
    one chain, minibatch 1,024, FP32 network), where the step is launch-bound:
    HIP-graph replay against launching every kernel of every step."""
    import torch

    from paper_2508_12117_amd import synth
    cat = synth.make_catalog("tiny")
    out = {}
    with spider.Context(0) as ctx:
        cid = ctx.load_catalog(cat, whiten=spider.WHITEN_EXACT)
        nid = ctx.load_net(synth.net_for(cat))
        sets = [(cid, nid, 1, cat.wl.batch, spider.FP32)]
        for name, graphs in (("graph", True), ("stream", False)):
            ctx.set_graphs(graphs)
            ctx.reset_chains(cid, 1)
            ctx.sgld_steps(sets, 50, seed=seed)
            ctx.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.sgld_steps(sets, steps, seed=seed)
            ctx.sync()
            torch.cuda.synchronize()
            out[name] = steps / (time.perf_counter() - t0)
    return {"workload": "tiny", "steps": steps, "steps_per_s_graph": out["graph"],
            "steps_per_s_stream": out["stream"],
            "dd_obs_per_s_graph": out["graph"] * cat.wl.batch}


def sample_error(ctx, spider, cat, net, nid, prec, rows=4096, seed=5):
    """Travel time and gradient error against the oracle on sampled batch rows."""
    import numpy as np
    import torch

    from oracle import travel_time as ott
    rng = np.random.default_rng(seed)
    obs = rng.integers(0, cat.N, rows)
    pr = cat.obs_pair[obs]
    ev = np.where(rng.random(rows) < 0.5, cat.pair_i[pr], cat.pair_j[pr])
    x = cat.hypo0[ev, 0:3]
    s = cat.stations[cat.obs_sta[obs]]
    T = torch.empty(rows, dtype=torch.float64, device="cuda")
    g = torch.empty(rows, 3, dtype=torch.float64, device="cuda")
    ctx.travel_time(nid, torch.tensor(x, device="cuda"), torch.tensor(s, device="cuda"), T, g,
                    precision=prec)
    Tw, gw = ott.travel_time(net, x, s)
    T, g = T.cpu().numpy(), g.cpu().numpy()
    return {"T_rel_max": float(np.max(np.abs(T - Tw) / Tw)),
            "gradT_rel_max": float(np.max(np.linalg.norm(g - gw, axis=1)
                                          / np.linalg.norm(gw, axis=1))),
            "rows": rows}


def posterior_moments(ctx, spider, cats, base_sets, step_size, steps, seed):
    """Pooled per-event posterior moments of both paths after the same number
    of steps from the same start with the same batch and noise streams (all
    catalogs of the workload, advanced together)."""
    import numpy as np
    import torch
    out = {}
    for name, code in (("bf16", spider.BF16), ("fp32", spider.FP32)):
        sets = [(cid, nid, C, n, code) for cid, nid, C, n in base_sets]
        for cid, _, C, _ in base_sets:
            ctx.reset_chains(cid, C)
        t = time.perf_counter()
        done = 0
        while done < steps:  # in chunks (a split run equals an uninterrupted one)
            k = min(100, steps - done)
            ctx.sgld_steps(sets, k, step=step_size, seed=seed, burn_in=steps // 2, thin=10)
            ctx.sync()
            done += k
            log(f"moments {name}: {done}/{steps} steps ({time.perf_counter() - t:.1f}s)")
        means, covs, counts = [], [], []
        for c, (cid, _, _, _) in zip(cats, base_sets):
            mean = torch.empty(c.M, 4, dtype=torch.float64, device="cuda")
            cov = torch.empty(c.M, 10, dtype=torch.float64, device="cuda")
            counts.append(ctx.moments(cid, -1, mean, cov))
            means.append(mean.cpu().numpy())
            covs.append(cov.cpu().numpy())
        out[name] = (np.concatenate(means), np.concatenate(covs), counts)
        log(f"moments {name}: {steps} steps in {time.perf_counter() - t:.1f}s, {counts[0]} samples")
    mb, cb, n = out["bf16"]
    mf, cf, _ = out["fp32"]
    diag = [0, 4, 7, 9]  # xx, yy, zz, tt in the packed upper triangle
    sdb, sdf = np.sqrt(cb[:, diag]), np.sqrt(cf[:, diag])
    z = np.abs(mb - mf) / sdf
    ratio = sdb / sdf
    true = np.concatenate([c.hypo_true[:, 0:3] for c in cats])
    err_b = np.sqrt(np.mean((mb[:, 0:3] - true) ** 2))
    err_f = np.sqrt(np.mean((mf[:, 0:3] - true) ** 2))
    q = lambda a, p: float(np.percentile(a, p))
    # the coordinates where the paths differ most, with the number of
    # observations of their event (the best-constrained events have the
    # smallest posterior s.d., so a smooth BF16 travel-time bias is the most
    # standard deviations there)
    nobs = np.concatenate([np.bincount(c.pair_i[c.obs_pair], minlength=c.M)
                           + np.bincount(c.pair_j[c.obs_pair], minlength=c.M) for c in cats])
    flat = np.argsort(z, axis=None)[::-1][:5]
    worst = []
    for f in flat:
        ev, comp = np.unravel_index(f, z.shape)
        worst.append({"event": int(ev), "component": "xyzt"[comp], "observations": int(nobs[ev]),
                      "sd_fp32": float(sdf[ev, comp]), "abs_mean_diff": float(abs(mb - mf)[ev, comp]),
                      "diff_over_sd": float(z[ev, comp])})
    dec = np.argsort(nobs)
    top = dec[-max(1, len(dec) // 10):]
    low = dec[:max(1, len(dec) // 10)]
    return {"steps": steps, "burn_in": steps // 2, "thin": 10,
            "worst": worst,
            "median_diff_over_sd_by_observations": {
                "fewest_10pct": float(np.median(z[low])), "most_10pct": float(np.median(z[top]))},
            "samples": int(n[0]) if len(n) == 1 else [int(k) for k in n],
            "events": int(mb.shape[0]),
            "mean_diff_over_sd": {"median": q(z, 50), "p99": q(z, 99), "max": float(z.max())},
            "sd_ratio_bf16_fp32": {"p1": q(ratio, 1), "median": q(ratio, 50), "p99": q(ratio, 99)},
            "location_rms_error_km": {"bf16": float(err_b), "fp32": float(err_f)},
            "note": "pooled over all chains; same batch and noise streams for both paths"}


def host_description():
    """CPU model, logical CPUs and the BLAS library numpy calls."""
    from threadpoolctl import threadpool_info
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = [f"{i.get('internal_api')} {i.get('version')} ({i.get('threading_layer', '')})"
            for i in threadpool_info() if i.get("user_api") == "blas"]
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable,
            "blas": "; ".join(blas) or "none"}


def cpu_baseline(cat, net, n, seed):
    """The FP64 oracle, as it stands, on one chain step with a batch of n."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import likelihood as lk
    from oracle import sampler
    prob = lk.load(cat)
    cfg = sampler.SamplerConfig(step=cat.wl.step_size, seed=seed)
    ch = sampler.new_chain(prob)
    sampler.step(prob, net, ch, cfg, 0, 0, n)          # first call warms caches
    t0 = time.perf_counter()
    sampler.step(prob, net, ch, cfg, 0, 0, n)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    n1 = max(n // 16, 1)  # one core: a smaller batch of the same stream
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        sampler.step(prob, net, ch, cfg, 0, 1, n1)
        dt1 = time.perf_counter() - t0
    return {"value": n / dt, "unit": "dd-obs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one pSGLD step of 1 chain, batch {n} of the {cat.M}-event catalog and its "
                      f"network, "
                      f"exact whitening, FP64 numpy ({dt:.1f} s)",
            "host": host_description(),
            "single_core": {"value": n1 / dt1, "unit": "dd-obs/s", "cores": 1,
                            "sample": f"one pSGLD step of 1 chain, batch {n1} ({dt1:.1f} s)"}}


def config_table(spider, seed=23, steps=200, burn=100):
    """The small workloads, each one chain from the initial locations with the
    batch and noise streams of `seed`, `steps` pSGLD steps, moments over the
    states after steps burn .. steps-1: tiny (200 events, 32,000 observations,
    minibatch 1,024, 6-32x3-1) and faults10k (10,000 events, 5,000,000
    observations, minibatch 65,536, 6-128x4-1).  Per precision: the GPU rate
    (graph replay, dd-obs/s), travel-time errors on 4,096 sampled rows, and
    the posterior-moment errors against the FP64 oracle's run of the same
    streams (tiny: run here, whole; faults10k: the stored 200-step run of
    tests/golden for its 500 sampled events).  The oracle rate is timed on
    the whole tiny run and on a 3-step prefix of faults10k."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_info

    from oracle import likelihood as lk
    from oracle import sampler
    from paper_2508_12117_amd import synth
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    golden = os.path.join(ROOT, "tests", "golden", "trajectory_faults10k.txt")
    diag = [0, 4, 7, 9]
    out = {"host": host_description()}
    for name, stream, oracle_steps in (("tiny", 3, steps), ("faults10k", 5, 3)):
        cat = synth.make_catalog(name)
        net = synth.net_for(cat)
        prob = lk.load(cat)
        n = cat.wl.batch
        cfg = sampler.SamplerConfig(step=cat.wl.step_size, beta2=cat.wl.beta2, eps_p=cat.wl.eps_p,
                                    seed=seed, burn_in=burn, thin=1)
        log(f"{name}: oracle, {oracle_steps} steps")
        t0 = time.perf_counter()
        ch, _ = sampler.run(prob, net, cfg, n, oracle_steps, stream=stream, chain_id=0)
        t_or = time.perf_counter() - t0
        if oracle_steps == steps:
            ev = np.arange(cat.M)
            mean_o, cov_o = ch.mom.mean, sampler.covariance(ch.mom)
        else:
            ref = np.loadtxt(golden)
            ev = ref[:, 0].astype(np.int64)
            mean_o, cov_o = ref[:, 1:5], ref[:, 5:15]
        sd = np.sqrt(cov_o[:, diag])
        row = {"events": cat.M, "observations": cat.N, "batch": n, "steps": steps,
               "net": f"6-{net.H}x{net.D}-1",
               "oracle": {"dd_obs_per_s": n * oracle_steps / t_or, "steps_timed": oracle_steps,
                          "cores": int(threads)},
               "moment_events": int(len(ev))}
        with spider.Context(0) as ctx:
            cid = ctx.load_catalog(cat, whiten=spider.WHITEN_EXACT, stream_id=stream)
            nid = ctx.load_net(net)
            for pname, prec in (("fp32", spider.FP32), ("bf16", spider.BF16)):
                sets = [(cid, nid, 1, n, prec)]
                walls = []
                for _ in range(2):  # the second run is timed (the first tunes and warms)
                    ctx.reset_chains(cid, 1)
                    ctx.sync()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ctx.sgld_steps(sets, steps, step=cat.wl.step_size, beta2=cat.wl.beta2,
                                   eps_p=cat.wl.eps_p, seed=seed, burn_in=burn, thin=1)
                    ctx.sync()
                    torch.cuda.synchronize()
                    walls.append(time.perf_counter() - t0)
                mean = torch.empty(cat.M, 4, dtype=torch.float64, device="cuda")
                cov = torch.empty(cat.M, 10, dtype=torch.float64, device="cuda")
                ctx.moments(cid, 0, mean, cov)
                mean, cov = mean.cpu().numpy()[ev], cov.cpu().numpy()[ev]
                em = np.abs(mean - mean_o) / sd
                ec = np.linalg.norm(cov - cov_o, axis=1) / np.linalg.norm(cov_o, axis=1)
                row[pname] = {
                    "dd_obs_per_s": n * steps / walls[-1], "ms_per_step": 1e3 * walls[-1] / steps,
                    "T1_T2": sample_error(ctx, spider, cat, net, nid, prec),
                    "T6_mean_diff_over_sd": {"median": float(np.median(em)),
                                             "p99": float(np.percentile(em, 99)),
                                             "max": float(em.max())},
                    "T7_cov_rel": {"median": float(np.median(ec)), "max": float(ec.max())}}
                log(f"{name} {pname}: {row[pname]['dd_obs_per_s']:.3e} dd-obs/s")
        out[name] = row
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the "
              "multi-GPU path exists only as a sharding design, not as code).", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2508_12117_amd import spider, synth
    if args.configs:
        config_table(spider)
        return
    if args.copy_probe > 0:
        a = torch.ones(args.copy_probe, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log(f"copied {args.copy_probe} bytes device to device")
    t = time.perf_counter()
    if args.workload in synth.MULTI:
        cats, net = synth.make_multi(
            args.workload, progress=lambda k, c: log(f"  catalog {k}: M={c.M} N={c.N} "
                                                     f"({time.perf_counter() - t:.1f}s)"))
    else:
        cats = [synth.make_catalog(args.workload)]
        net = synth.net_for(cats[0])
    cat, wl = cats[0], cats[0].wl
    log(f"generated {args.workload}: {len(cats)} catalog(s), M={sum(c.M for c in cats)} "
        f"N={sum(c.N for c in cats)} in {time.perf_counter() - t:.1f}s")
    ctx = spider.Context(0)
    t = time.perf_counter()
    cids = [ctx.load_catalog(c, whiten=spider.WHITEN_EXACT, stream_id=k) for k, c in enumerate(cats)]
    nid = ctx.load_net(net)
    base_sets = [(cid_k, nid, c.wl.chains, c.wl.batch) for cid_k, c in zip(cids, cats)]
    dd_per_step = sum(C * n for _, _, C, n in base_sets)
    log(f"loaded in {time.perf_counter() - t:.1f}s")

    bf16_ok = spider.lib() is not None and _bf16_supported(ctx, nid)
    if args.precision == "auto":
        precs = ["bf16", "fp32"] if bf16_ok else ["fp32"]
    elif args.precision == "both":
        precs = ["bf16", "fp32"]
    else:
        precs = [args.precision]
    res = {}
    for p in precs:
        code = spider.BF16 if p == "bf16" else spider.FP32
        wall, wall_stream, ms, launches, rows = run_precision(ctx, spider, base_sets, wl.step_size,
                                                              code, args.steps, args.warmup,
                                                              args.seed, not args.stream_only)
        dd = dd_per_step * args.steps
        fl = flops_per_eval(wl.H, wl.D)
        avg_ms = ms / max(launches, 1)
        achieved = rows / max(launches, 1) * fl / (avg_ms * 1e-3) / 1e12
        waves, tiles = ctx.network_variant(nid, code)
        sched = ctx.network_schedule(nid, code)
        traffic = network_traffic(rows // max(launches, 1),
                                  {"waves": waves, "row_tiles": tiles, "schedule": sched})
        res[p] = dict(value=dd / wall, ms_per_step=wall * 1e3 / args.steps,
                      ms_per_step_stream=wall_stream * 1e3 / args.steps, net_ms=ms,
                      net_launches=launches, net_avg_ms=avg_ms, achieved=achieved, traffic=traffic,
                      variant={"waves_per_workgroup": waves, "rows_per_workgroup": 16 * tiles,
                               "schedule": SCHEDULES.get(sched, str(sched))},
                      error=sample_error(ctx, spider, cat, net, nid, code))
        log(f"{p}: {dd / wall:.4g} dd-obs/s, {wall * 1e3 / args.steps:.2f} ms/step, network "
            f"{avg_ms:.3f} ms/launch = {achieved:.2f} TFLOP/s, tiles {waves} waves x {16 * tiles} rows")
    head = precs[0]
    r = res[head]
    line = {
        "metric": "dd-obs likelihood-gradient evals/s, BF16-MFMA vs FP32 path, at stated error",
        "value": r["value"], "unit": "dd-obs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head, "data": "synthetic",
        "config": ({"workload": args.workload, "events": cat.M, "stations": cat.L,
                    "observations": cat.N, "batch": wl.batch, "chains": wl.chains,
                    "net": f"6-{wl.H}x{wl.D}-1 tanh", "whiten": "exact", "sampler": "pSGLD",
                    "state": "fp64"} if len(cats) == 1 else
                   {"workload": args.workload, "catalogs": len(cats),
                    "events": sum(c.M for c in cats), "observations": sum(c.N for c in cats),
                    "chains": sum(c.wl.chains for c in cats), "obs_per_step": dd_per_step,
                    "per_catalog": [[c.M, c.L, c.N, c.wl.batch, c.wl.chains] for c in cats],
                    "net": f"6-{wl.H}x{wl.D}-1 tanh", "whiten": "exact", "sampler": "pSGLD",
                    "state": "fp64", "launch": "all catalogs' network rows in one launch per step"}),
        "roofline": {"bound": "mfma", "kernel": "travel-time network (forward + source "
                     "gradient)", "achieved": r["achieved"], "peak": PEAK[head],
                     "unit": "TFLOP/s", "frac": r["achieved"] / PEAK[head],
                     "traffic": r["traffic"]},
        "paths": {p: {"value": v["value"], "ms_per_step": v["ms_per_step"],
                      "ms_per_step_stream_launches": v["ms_per_step_stream"],
                      "network_ms_per_launch": v["net_avg_ms"],
                      "network_tflops": v["achieved"], "network_tiles": v["variant"],
                      "error_vs_oracle": v["error"]}
                  for p, v in res.items()},
    }
    if "bf16" in res and "fp32" in res:
        line["bf16_over_fp32"] = res["bf16"]["value"] / res["fp32"]["value"]
    if args.moments_steps > 0 and bf16_ok:
        line["posterior_moments"] = posterior_moments(ctx, spider, cats, base_sets, wl.step_size,
                                                      args.moments_steps, args.seed)
    if not args.no_graph_compare:
        line["small_catalog"] = small_catalog_rates(spider, args.seed)
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        # several catalogs: the oracle on the one nearest 200k events
        cb = min(cats, key=lambda c: abs(c.M - 200_000)) if len(cats) > 1 else cat
        line["cpu_baseline"] = cpu_baseline(cb, net, min(args.cpu_batch, cb.N), args.seed)
        log(f"cpu baseline in {time.perf_counter() - t:.1f}s")
    ctx.close()
    print(json.dumps(line), flush=True)


def _bf16_supported(ctx, nid):
    import torch

    from paper_2508_12117_amd import spider
    x = torch.zeros(1, 3, dtype=torch.float64, device="cuda")
    s = torch.ones(1, 3, dtype=torch.float64, device="cuda")
    T = torch.empty(1, dtype=torch.float64, device="cuda")
    try:
        ctx.travel_time(nid, x, s, T, precision=spider.BF16)
        return True
    except spider.SpiderError as e:
        if e.code == spider.E_UNSUPPORTED:
            return False
        raise


if __name__ == "__main__":
    main()
