"""Throughput and latency of lib_linmin on the orbital-cube workload.

Workload: N = 36 spectra (32 synthetic minerals + 4 extra continuum spectra),
L = 240 channels, P = 128 x 4,096 = 524,288 pixels, float32 cube resident in
HBM, per-pixel sigma.  One step = one ``linmin_unmix`` over the whole cube:
projections (MFMA), interior-point solve with the finishing step, and the
full FP64 covariance.  Prints one JSON line.  Beside it: the mixed form, the
precision cube (N = 64, L = 438, P = 640 x 480) in both forms, the many-cube
batch, the serving loop and the CPU oracle (all host threads, then one).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import math
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12          # MI355X FP64, dense matrix cores and vector units alike, FLOP/s
PEAK_HBM = 8.0e12            # bytes/s
PROFILE = os.path.join(ROOT, "profiles", "orbital_N36_L240_kernels.md")
IPM_KERNEL = "lm::ipm_tile_kernel<9, 0, 0, false>"
IPM_SOURCES = ("paper_1402_2518_amd/csrc/ipm_tile.hip", "paper_1402_2518_amd/csrc/ipm_body.h",
               "paper_1402_2518_amd/csrc/common.h", "paper_1402_2518_amd/csrc/kernels.h")


def profiled_traffic():
    """HBM bytes per launch of the interior-point kernel from the committed
    rocprofv3 counter summary, or None when the kernel's sources have changed
    since the counters were taken."""
    import hashlib
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in IPM_SOURCES)).hexdigest()
    for line in text.splitlines():
        if line.startswith("traffic " + IPM_KERNEL + " "):
            kv = dict(t.split("=", 1) for t in line.split() if "=" in t)
            if kv.get("src_sha256") == h:
                return float(kv["read_bytes"]) + float(kv["write_bytes"])
    return None


def ipm_flops_per_iteration(n: int) -> float:
    """Algorithmic FP64 flops of one interior-point iteration for a library of
    n spectra: L D L^T of the n x n Newton matrix (n^3 / 3) and the O(n^2)
    work of two solves, the bordered elimination and the product with the
    Gram matrix (8 n^2)."""
    return n ** 3 / 3.0 + 8.0 * n ** 2


IPM_KERNELS = {36: "lm::ipm_tile_kernel<9, 0, 0, false>", 64: "lm::ipm_tile_kernel<16, 0, 0, true>"}


def workload_leg(name, args, dev, stream, steps, warmup, latency_calls, variants=0, keep_host=False):
    """One synthetic cube unmixed whole, FP64 and mixed, full covariance:
    throughput, stage times, single-cube latency, the interior-point
    kernel's roofline, and a sampled check of both forms against the oracle."""
    import torch
    import oracle
    from paper_1402_2518_amd import linmin, synth

    w = synth.WORKLOADS[name]
    S = synth.make_library(w)
    t_gen = time.perf_counter()
    X, s = synth.make_cube(w, S)
    t_gen = time.perf_counter() - t_gen
    Xd = torch.from_numpy(X).to(dev)
    sd = torch.from_numpy(s).to(dev)
    P, N = w.P, w.N
    lib = linmin.Library(S)
    out_a = torch.empty((P, N), dtype=torch.float64, device=dev)
    out_cov = torch.empty((P, N, N), dtype=torch.float64, device=dev)
    status = torch.empty(P, dtype=torch.uint8, device=dev)
    iters = torch.empty(P, dtype=torch.int32, device=dev)
    obj = torch.empty(P, dtype=torch.float64, device=dev)

    def run(precision, steps, warmup, a_out, cov="full", npix=P):
        X_, s_ = Xd[:npix], sd[:npix]
        a_, st_, it_, ob_ = a_out[:npix], status[:npix], iters[:npix], obj[:npix]
        c_ = out_cov[:npix] if cov == "full" else (out_cov.view(-1)[:npix * N].view(npix, N) if cov == "diag" else None)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                lib.unmix_into(X_, s_, a_, c_, st_, it_, ob_, precision=precision, cov=cov, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(steps):
                lib.unmix_into(X_, s_, a_, c_, st_, it_, ob_, precision=precision, cov=cov, stream=stream,
                               events=evs[k])
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        stage = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3]),
                           e[0].elapsed_time(e[3])] for e in evs])  # ms
        return wall, stage

    print(f"# {name}: generated cube in {t_gen:.1f}s; P={P} N={N} L={w.L}", file=sys.stderr, flush=True)
    res, a_keep, F_keep, st_keep = {}, {}, {}, {}
    for prec in ("fp64", "mixed"):
        buf = out_a if prec == "fp64" else torch.empty_like(out_a)
        wall, st = run(prec, steps, warmup, buf)
        it = iters.cpu().numpy()
        stat = status.cpu().numpy()
        a_keep[prec], F_keep[prec], st_keep[prec] = buf, obj.clone(), stat
        res[prec] = {"value": P * steps / wall, "ms_per_step": wall / steps * 1e3,
                     "stages_ms": {"projection": float(np.mean(st[:, 0])), "ipm": float(np.mean(st[:, 1])),
                                   "covariance": float(np.mean(st[:, 2]))},
                     "mean_iters": float(it.mean()),
                     "status_counts": {str(k): int(v) for k, v in zip(*np.unique(stat, return_counts=True))}}
        if prec == "fp64":
            ipm_ms = float(np.mean(st[:, 1]))
            flops = float(it.astype(np.float64).sum()) * ipm_flops_per_iteration(N)
            achieved = flops / (ipm_ms * 1e-3)
            kname = IPM_KERNELS.get(N, "interior point")
            roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_FP64, "traffic": profiled_traffic() if N == 36 else None,
                    "kernel": kname + " (FP64, 4x4x4 matrix-core tiles)", "kernel_ms": ipm_ms,
                    "flops_per_launch": flops, "mean_iters": float(it.mean()),
                    "flops_per_iteration": ipm_flops_per_iteration(N)}
        fam = {v: k for k, v in linmin.KERNELS.items()}
        stages = [("fp64", linmin.STAGE_FP64)] if prec == "fp64" else [("fp32", linmin.STAGE_FP32),
                                                                         ("fp64", linmin.STAGE_FP64)]
        res[prec]["kernels"] = {}
        for sname, stg in stages:
            f_, l_ = linmin.get_kernel_lanes(N, stg)
            res[prec]["kernels"][sname] = fam[f_] + (f"/{l_}" if l_ else "")
        print(f"# {name} {prec}: {wall / steps * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
        if latency_calls > 0:
            _, stl = run(prec, latency_calls, 1, buf)
            res[prec]["latency_ms"] = {"p50": float(np.percentile(stl[:, 3], 50)),
                                       "p99": float(np.percentile(stl[:, 3], 99)), "calls": int(latency_calls)}
        else:
            res[prec]["latency_ms"] = {"p50": float(np.percentile(st[:, 3], 50)),
                                       "p99": float(np.percentile(st[:, 3], 99)), "calls": int(len(st))}
    res["mixed"]["max_abs_coeff_diff_vs_fp64"] = float((a_keep["mixed"] - a_keep["fp64"]).abs().max().item())
    res["mixed"]["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]

    # both forms against the FP64 oracle on a prefix of the cube
    n_or = min(P, args.oracle_pixels)
    r = oracle.unmix(S, X[:n_or], s[:n_or], cov=False)
    samp = {"pixels": n_or}
    for prec in ("fp64", "mixed"):
        a = a_keep[prec][:n_or].cpu().numpy()
        F = F_keep[prec][:n_or].cpu().numpy()
        both = (st_keep[prec][:n_or] == 0) & (r["status"] == 0)
        samp[prec] = {"max_abs_coeff_err": float(np.abs(a - r["a"]).max()),
                      "max_rel_objective_err": float(np.abs(F[both] / r["F"][both] - 1).max()),
                      "status_agreement": float((st_keep[prec][:n_or] == r["status"]).mean())}
    samp["oracle_mean_iters"] = float(r["iters"].mean())

    var = {}
    if variants > 0:
        for prec in ("fp64", "mixed"):
            buf = a_keep[prec]
            for cov in ("diag", "none"):
                wv, _ = run(prec, variants, 1, buf, cov=cov)
                var[f"{prec}_cov_{cov}"] = {"pixels_per_s": P * variants / wv, "ms_per_call": wv / variants * 1e3}
        shard = P // 8
        for prec in ("fp64", "mixed"):
            wv, _ = run(prec, variants, 1, a_keep[prec], npix=shard)
            var[f"{prec}_cov_full_P{shard}"] = {"pixels_per_s": shard * variants / wv,
                                                "ms_per_call": wv / variants * 1e3}
        print(f"# {name} variants: {var}", file=sys.stderr, flush=True)
    out = {"workload": f"{name} cube: N={N} ({w.n_minerals} minerals + {w.n_extra} extras), L={w.L}, P={P}, "
                       "fp32 reflectance, sigma~U[0.002,0.01], full covariance",
           "fp64": res["fp64"], "mixed": res["mixed"], "roofline": roof, "oracle_sample": samp, "variants": var}
    if keep_host:
        out["_host"] = (S, X, s, a_keep["fp64"].cpu().numpy())
    lib.close()
    del out_a, out_cov, a_keep, F_keep, Xd, sd
    return out


def batch_leg(args, dev, stream):
    """Many cubes, each with its own library, in one planned batch: fused
    launches against the same cubes unmixed by sequential single calls."""
    import torch
    import oracle
    from paper_1402_2518_amd import linmin, synth

    ws = synth.batch_workloads(args.batch_cubes)
    t0 = time.perf_counter()
    libs, items, S_host = [], [], []
    for w in ws:
        S = synth.make_library(w)
        lib = linmin.Library(S)
        X, s = synth.make_cube_device(w, S, dev)
        libs.append(lib)
        items.append((lib, X, s))
        S_host.append(S)
    torch.cuda.synchronize()
    P_tot = sum(w.P for w in ws)
    print(f"# batch: {len(ws)} cubes, {P_tot} pixels, built in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    out = {"cubes": len(ws), "pixels": P_tot, "cov_layout": "diag", "runs": args.batch_runs,
           "workload": "200 cubes, N in {16,24,36,48,64,96} and L in {128,240,438} per cube, P log-uniform "
                       "in [1e3, 2e5], 4 extras, 1-4 active minerals, sigma~U[0.002,0.01]",
           "pixels_by_N": {str(n): sum(w.P for w in ws if w.N == n) for n in synth.BATCH_N}}
    for prec in ("fp64", "mixed"):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        b = linmin.Batch(items, precision=prec, cov="diag", events=evs)

        def sequential():
            for (lib, X, s), r in zip(items, b.results):
                lib.unmix_into(X, s, r["a"], r["cov"], r["status"], r["iters"], r["objective"],
                               precision=prec, cov="diag", stream=stream)

        with torch.cuda.stream(stream):
            b.run(stream)
            torch.cuda.synchronize()
            ref = [(r["a"].clone(), r["cov"].clone(), r["status"].clone()) for r in b.results]
            t1 = time.perf_counter()
            for _ in range(args.batch_runs):
                b.run(stream)
            torch.cuda.synchronize()
            wall_b = (time.perf_counter() - t1) / args.batch_runs
            stages = [evs[0].elapsed_time(evs[1]), evs[1].elapsed_time(evs[2]), evs[2].elapsed_time(evs[3])]
            sequential()
            torch.cuda.synchronize()
            same = all(torch.equal(r["a"], a) and torch.equal(r["cov"].nan_to_num(3.5), c.nan_to_num(3.5))
                       and torch.equal(r["status"], st) for r, (a, c, st) in zip(b.results, ref))
            t1 = time.perf_counter()
            for _ in range(args.batch_runs):
                sequential()
            torch.cuda.synchronize()
            wall_s = (time.perf_counter() - t1) / args.batch_runs
        # oracle on the first pixels of one cube of every library size
        err = 0.0
        for n in synth.BATCH_N:
            i = next(k for k, w in enumerate(ws) if w.N == n)
            X8, s8 = items[i][1][:8].cpu().numpy(), items[i][2][:8].cpu().numpy()
            r = oracle.unmix(S_host[i], X8, s8, cov=False)
            err = max(err, float(np.abs(ref[i][0][:8].cpu().numpy() - r["a"]).max()))
        stat = torch.cat([st for _, _, st in ref]).cpu().numpy()
        by_n = {}
        for wk, (_, _, st) in zip(ws, ref):
            d = by_n.setdefault(str(wk.N), {})
            for k, v in zip(*np.unique(st.cpu().numpy(), return_counts=True)):
                d[str(int(k))] = d.get(str(int(k)), 0) + int(v)
        out[prec] = {"pixels_per_s": P_tot / wall_b, "ms_per_run": wall_b * 1e3,
                     "stages_ms": {"projection": stages[0], "ipm": stages[1], "covariance": stages[2]},
                     "sequential_pixels_per_s": P_tot / wall_s, "sequential_ms_per_run": wall_s * 1e3,
                     "speedup_vs_sequential": wall_s / wall_b, "identical_to_single_calls": bool(same),
                     "max_abs_coeff_err_vs_oracle_sample": err,
                     "status_counts": {str(k): int(v) for k, v in zip(*np.unique(stat, return_counts=True))},
                     "status_counts_by_N": by_n,
                     "device_bytes": b.device_bytes()}
        print(f"# batch {prec}: {out[prec]}", file=sys.stderr, flush=True)
        b.close()
    for lib in libs:
        lib.close()
    return out


def serve_leg(args, dev, rate=None, seconds=None, host_inputs=False):
    """Poisson arrivals of cubes of 8 resident libraries through the request
    loop: latency under load, and sampled requests checked against the same
    request served alone and against the oracle.  host_inputs: the arriving
    cubes sit in pinned host memory and each request includes its
    host-to-device copy."""
    import torch
    import oracle
    from paper_1402_2518_amd import linmin, serve, synth

    rng = np.random.default_rng(5150)
    P_POOL = 200_000
    libs, pools, host = {}, {}, {}
    for k in range(8):
        N, L = int(rng.choice(synth.BATCH_N)), int(rng.choice(synth.BATCH_L))
        w = synth.custom_workload(N, L, P_POOL, seed=40_000 + k)
        S = synth.make_library(w)
        libs[k] = linmin.Library(S)
        pools[k] = synth.make_cube_device(w, S, dev)
        host[k] = S
        libs[k].unmix(pools[k][0][:64], pools[k][1][:64], cov="full")  # loads the kernels
        if host_inputs:
            pools[k] = tuple(t.cpu().pin_memory() for t in pools[k])
    torch.cuda.synchronize()
    rate = args.serve_rate if rate is None else rate
    seconds = args.serve_seconds if seconds is None else seconds
    t = serve.poisson_arrivals(rate, seconds, rng)
    sample = set(rng.choice(len(t), size=min(12, len(t)), replace=False).tolist())
    reqs = []
    for rid, ta in enumerate(t):
        k = int(rng.integers(0, 8))
        P = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
        off = int(rng.integers(0, P_POOL - P + 1))
        X, s = pools[k]
        r = serve.Request(rid, k, X[off:off + P], s[off:off + P], float(ta), keep=rid in sample)
        reqs.append(r)
    srv = serve.Server(libs, streams=4, slots=8, hbm_budget=96 << 30, precision="fp64", cov="full")
    print(f"# serving: {len(reqs)} requests over {seconds:.0f}s", file=sys.stderr, flush=True)
    done = srv.run(reqs)
    torch.cuda.synchronize()
    out = serve.latency_summary(done)
    out.update({"offered_rate_per_s": rate, "seconds": seconds, "libraries": 8,
                "libraries_NL": [[libs[k].N, libs[k].L] for k in range(8)], "cov_layout": "full",
                "precision": "fp64", "slots": srv.slots, "streams": len(srv.streams),
                "hbm_budget_bytes": srv.budget, "max_running": srv.stats["max_running"],
                "max_bytes_in_use": srv.stats["max_bytes"],
                "inputs": ("pinned host cube pools (200,000 pixels per library), requests are row ranges copied to "
                           "the device on a copy stream inside each request's latency") if host_inputs else
                          "device-resident cube pools (200,000 pixels per library), requests are row ranges"})
    same, err = True, 0.0
    for r in done:
        if not r.keep:
            continue
        alone = libs[r.lib].unmix(r.cube.to(dev), r.sigma.to(dev), precision="fp64", cov="full")
        torch.cuda.synchronize()
        same &= all(torch.equal(r.out[k].nan_to_num(3.5), alone[k].nan_to_num(3.5)) for k in ("a", "cov", "status"))
        X8 = r.cube[:4].cpu().numpy()
        s8 = r.sigma[:4].cpu().numpy()
        ro = oracle.unmix(host[r.lib], X8, s8, cov=False)
        err = max(err, float(np.abs(r.out["a"][:4].cpu().numpy() - ro["a"]).max()))
        r.out = None
    out["sampled_requests"] = len(sample)
    out["identical_alone_and_in_mix"] = bool(same)
    out["max_abs_coeff_err_vs_oracle_sample"] = err
    print(f"# serving: {out}", file=sys.stderr, flush=True)
    for lib in libs.values():
        lib.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-seconds-1core", type=float, default=4.0)
    ap.add_argument("--oracle-pixels", type=int, default=8192,
                    help="cube prefix checked against the oracle in each workload leg")
    ap.add_argument("--precision-steps", type=int, default=10,
                    help="timed whole-cube calls of the precision cube (N=64, L=438; 0 = skip)")
    ap.add_argument("--precision-latency-calls", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--latency-calls", type=int, default=200,
                    help="sequential whole-cube calls behind the p50/p99 latency")
    ap.add_argument("--variants", type=int, default=5,
                    help="timed calls for each covariance layout / shard-size variant (0 = skip)")
    ap.add_argument("--batch-cubes", type=int, default=200,
                    help="cubes in the many-cube batch leg (0 = skip)")
    ap.add_argument("--batch-runs", type=int, default=2, help="timed runs of the batch leg")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson arrival stream of the serving leg (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=50.0, help="cubes per second arriving")
    ap.add_argument("--serve-light-rate", type=float, default=25.0,
                    help="a second, lighter stream (20 s) to show latency below saturation (0 = skip)")
    ap.add_argument("--serve-host-seconds", type=float, default=20.0,
                    help="a third stream at the configured rate whose cubes arrive in host memory (0 = skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "lib_linmin runs on one GPU: pixels are independent and this build "
                                   "measures one MI355X; run with --gpus 1"}))
        sys.exit(2)

    import torch
    import oracle
    from paper_1402_2518_amd import synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()

    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src_t = torch.empty(nb, dtype=torch.uint8, device=dev).fill_(1)
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        print(f"# copy calibration: {nb} bytes read, {nb} bytes written", file=sys.stderr, flush=True)
        del src_t, dst_t

    orb = workload_leg("orbital", args, dev, stream, args.steps, args.warmup, args.latency_calls,
                       variants=args.variants, keep_host=not args.no_cpu)
    w = synth.WORKLOADS["orbital"]
    P, N = w.P, w.N
    result = {
        "metric": "pixels unmixed/sec (N=36,L=240) plain FP64 vs mixed; p50/p99 cube latency",
        "value": orb["fp64"]["value"],
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": orb["fp64"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "orbital cube: N=36 (32 minerals + 4 extras), L=240, P=128x4096=524288, "
                               "fp32 reflectance, sigma~U[0.002,0.01], FP64 solve, full covariance",
                   "global_batch": P, "seq_len": w.L, "parallelism": "single GPU"},
        "latency_ms": orb["fp64"]["latency_ms"],
        "stages_ms": orb["fp64"]["stages_ms"],
        "mixed": orb["mixed"],
        "variants": orb["variants"],
        "status_counts": orb["fp64"]["status_counts"],
        "oracle_sample": orb["oracle_sample"],
        "roofline": orb["roofline"],
    }
    host = orb.pop("_host", None)
    torch.cuda.empty_cache()
    if args.precision_steps > 0:
        pc = workload_leg("precision", args, dev, stream, args.precision_steps, 2, args.precision_latency_calls)
        pc.pop("_host", None)
        result["precision_cube"] = pc
        torch.cuda.empty_cache()

    if args.batch_cubes > 0:
        torch.cuda.empty_cache()
        result["batch"] = batch_leg(args, dev, stream)

    if args.serve_seconds > 0:
        torch.cuda.empty_cache()
        result["serving"] = serve_leg(args, dev)
        if args.serve_light_rate > 0:
            torch.cuda.empty_cache()
            result["serving_light"] = serve_leg(args, dev, rate=args.serve_light_rate, seconds=20.0)
        if args.serve_host_seconds > 0:
            torch.cuda.empty_cache()
            result["serving_host_inputs"] = serve_leg(args, dev, seconds=args.serve_host_seconds, host_inputs=True)

    if not args.no_cpu:
        S, X, s, a64h = host
        oracle.build(force=False)
        done, cpu_time, p0, chunk = 0, 0.0, 0, 16384
        max_err = 0.0
        while cpu_time < args.cpu_seconds and p0 < P:
            p1 = min(P, p0 + chunk)
            t1 = time.perf_counter()
            r = oracle.unmix(S, X[p0:p1], s[p0:p1], cov=True)
            cpu_time += time.perf_counter() - t1
            max_err = max(max_err, float(np.abs(r["a"] - a64h[p0:p1]).max()))
            done += p1 - p0
            p0 = p1
        cores = oracle.max_threads()
        # the same oracle on one thread, over a smaller prefix (this leaves the
        # oracle's thread count at one, so it runs last)
        done1, cpu1, p0 = 0, 0.0, 0
        while cpu1 < args.cpu_seconds_1core and p0 < P:
            p1 = min(P, p0 + 1024)
            t1 = time.perf_counter()
            oracle.unmix(S, X[p0:p1], s[p0:p1], cov=True, threads=1)
            cpu1 += time.perf_counter() - t1
            done1 += p1 - p0
            p0 = p1
        result["cpu_baseline"] = {"value": done / cpu_time, "unit": "pixels/s", "cores": cores,
                                  "kind": "oracle",
                                  "sample": f"first {done} pixels of the same cube, FP64 with full covariance",
                                  "value_1core": done1 / cpu1, "cores_1core": 1,
                                  "sample_1core": f"first {done1} pixels of the same cube, one thread"}
        result["parity_sample"] = {"pixels": done, "max_abs_coeff_err_fp64_vs_oracle": max_err}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
