"""Benchmark: half-space spectral Ewald summation on one MI355X.

One step = one full evaluation of the half-space stokeslet sum (binning,
real-space sum, spreading, zero-padded 3D transforms with the fused scaling,
inverse transforms, quadrature and FP64 combination) for N = 100,000 sources
= targets uniform in [0,1)^2 x (0,1], forces N(0,1), FP64 at tol 1e-10, with
xi and r_c chosen for about 30 neighbours per point.  Inputs are resident in
device memory before the timed region; the truncated-kernel precompute is done
during warm-up (it depends only on the grid size and is excluded, as in the
paper's timings).

Prints one JSON line.  Extra fields: the FP32 path on the same workload at
tol 1e-5, the same FP64 problem at the runtime-optimal (xi, r_c) that the
tuning procedure of the paper's results section finds (`tuned`), the relative
RMS error of all three against the FP64 oracle on a sample of targets,
per-stage times, the roofline of the dominant kernel and the oracle's own
throughput on the host cores (cpu_baseline).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFS = 78.6


def _stage_bytes(rep, ncin, esz):
    """Algorithmic HBM bytes of each transform pass per evaluation (inputs read
    once, outputs written once; the multiplier octants read once)."""
    Mt = rep.Mt
    c = 2 * esz
    real = Mt * Mt * 2 * Mt * esz
    a = (Mt + 1) * 2 * Mt * Mt * c
    z = (Mt + 1) * 4 * Mt * Mt * c
    kinds = 1 if rep.family == 2 else 2
    nout = 4 if esz == 8 else 6  # output grids: T1 and phi (FP64) or T1 and grad phi (FP32)
    oct_bytes = (Mt + 1) * (Mt + 1) * (2 * Mt + 1) * (8 if esz == 8 else 4) * kinds
    # the inverse side produces only the x3 nodes from x3_first up (the ones
    # the quadrature at the targets reads); the correction grids (components
    # from nca on, spread at the images) are read only below x3_corr_end
    keep = (2 * Mt - rep.x3_first) / (2 * Mt)
    nca = 6 if rep.family == 1 else 3
    nin = nca + (ncin - nca) * rep.x3_corr_end / (2 * Mt)
    return {
        "fwd_x": nin * (real + a),
        "fwd_y": nin * (a + z),
        "z_scale": nin * z + nout * z * keep + oct_bytes,
        "inv_y": nout * (z + a) * keep,
        "inv_x": nout * (a + real) * keep,
    }


# kernels whose sources determine the fused x3 pass (a change voids the traffic counters)
_Z_SOURCES = ["paper_1802_07844_amd/csrc/fft.hip", "paper_1802_07844_amd/csrc/common.h",
              "paper_1802_07844_amd/csrc/kernels.h"]


def _sources_sha():
    import hashlib

    h = hashlib.sha256()
    for p in _Z_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _measured_traffic(name):
    """HBM bytes per launch from a committed rocprofv3 counter summary (a line
    'traffic-json: {...}' in profiles/<name>), if it was taken on the current
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-json:"):
            d = json.loads(line.split(":", 1)[1])
            if d.get("sources_sha") == _sources_sha():
                return d
    return None


def _measured_valu(name):
    """FP64 flops per launch of the fused x3 pass from a committed rocprofv3
    counter summary (a line 'valu-json: {...}' in profiles/<name>), if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("valu-json:"):
            d = json.loads(line.split(":", 1)[1])
            if d.get("sources_sha") == _sources_sha():
                return d
    return None


def _ncin(rep):
    """Input grids of the plan: the kernel grid and either the correction
    density (FP64 D-grid plans) or the separate correction grids."""
    nca = 6 if rep.family == 1 else 3
    ncb = {0: 4, 1: 7, 2: 2}[rep.family]
    return nca + (1 if rep.dgrid else ncb)


def _roofline(rep, stage_ms, ncin, esz, traffic_file=None, valu_file=None):
    sb = _stage_bytes(rep, ncin, esz)
    dom = max(sb.keys(), key=lambda k: stage_ms[k])
    launches = 1
    if dom in ("fwd_y", "z_scale", "inv_y"):
        launches = (rep.Mt + rep.zslab) // rep.zslab  # one launch per group of k1 slabs
    per_launch = sb[dom] / launches
    ms_launch = stage_ms[dom] / launches
    achieved = per_launch / (ms_launch * 1e-3) / 1e9
    traffic = None
    if traffic_file and dom == "z_scale":
        t = _measured_traffic(traffic_file)
        if t is not None:
            traffic = t["bytes_per_launch"] * (per_launch / t["algorithmic_bytes_per_launch"])
    # the vector FP64 rate of the same launches (flops from the committed
    # counter summary, time from this run)
    valu = None
    if valu_file and dom == "z_scale" and esz == 8:
        v = _measured_valu(valu_file)
        if v is not None:
            tf = v["fp64_flops_per_launch"] / (ms_launch * 1e-3) / 1e12
            valu = {"achieved": tf, "peak": FP64_VALU_PEAK_TFS, "unit": "TFLOP/s", "frac": tf / FP64_VALU_PEAK_TFS}
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "bytes_per_launch": per_launch,
            "launches_per_step": launches, "ms_per_launch": ms_launch, "valu_fp64": valu}


def _serve_rc(kernel, n, tol):
    """Fixed cutoff rule of the serving stream: about 600 neighbours per point
    at FP64 (balances the real-space and Fourier work on this device), 300 at
    FP32 with a lower bound on r_c per kernel so that xi L stays where the
    planner's FP32 rounding estimate admits FP32 at tol 1e-5 (stokeslet
    xi L <~ 45, stresslet <~ 30; the rotlet's rounding does not grow)."""
    nb = 600.0 if tol < 1e-6 else 300.0
    rc = (nb * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
    if tol >= 1e-6:
        rc = max(rc, {"stokeslet": 0.08, "stresslet": 0.15, "rotlet": 0.0}[kernel])
    return min(rc, 0.45)


def serve_bench(args, ehs, workloads, torch, np):
    """Serving stream: Poisson arrivals of mixed requests through one ehs.Server."""
    import queue
    import threading

    npool = args.serve_pool
    seed = workloads.SEED_BASE + 5
    y, f, gq, v = workloads.serving_pool(npool, seed)
    dev = torch.device("cuda:0")
    yd = torch.from_numpy(y).to(dev)
    sd = {"stokeslet": torch.from_numpy(f).to(dev), "stresslet": torch.from_numpy(gq).to(dev),
          "rotlet": torch.from_numpy(v).to(dev)}
    sh = {"stokeslet": f, "stresslet": gq, "rotlet": v}
    torch.cuda.synchronize()

    def prep(d):
        n = min(d["n"], npool)
        off = d["seed"] % (npool - n + 1)
        rc = _serve_rc(d["kernel"], n, d["tol"])
        xi = ehs.xi_for_cutoff(d["kernel"], rc, d["tol"] / 2)
        prec = 0  # auto: FP32 at tol 1e-5 where its rounding estimate allows, else FP64
        return n, off, rc, xi, prec

    def submit(srv, d):
        n, off, rc, xi, prec = prep(d)
        ys = yd[off:off + n]
        return srv.submit(d["kernel"], ys, sd[d["kernel"]][off:off + n], ys, xi, rc, d["tol"], precision=prec)

    free = torch.cuda.mem_get_info()[0]
    arena = int(min(args.serve_arena_gb * 2**30, 0.8 * free))
    srv = ehs.Server(0, arena_bytes=arena, nslots=args.serve_slots)
    # capacity from a closed-loop calibration batch of the same distribution
    cal = workloads.serving_stream(args.serve_calib, seed + 1)
    t0 = time.perf_counter()
    for t in [submit(srv, d) for d in cal]:
        srv.wait(t)
    cal_wall = time.perf_counter() - t0
    mu = len(cal) / cal_wall
    lam = args.serve_util * mu
    stream = workloads.serving_stream(args.serve_requests, seed)
    q = queue.Queue()
    tstart = time.perf_counter() + 0.05
    deadline = tstart + args.serve_max_seconds

    def feeder():
        for i, d in enumerate(stream):
            ts = tstart + d["arrival"] / lam
            if ts > deadline:
                break
            now = time.perf_counter()
            if ts > now:
                time.sleep(ts - now)
            tcall = time.perf_counter()
            q.put((i, submit(srv, d), ts, tcall))
        q.put(None)

    th = threading.Thread(target=feeder, daemon=True)
    th.start()
    lat, que, svc, pts, rows = [], [], [], 0, []
    t_end = tstart
    while True:
        item = q.get()
        if item is None:
            break
        i, tk, ts, tcall = item
        u, st = srv.wait(tk)
        lag = tcall - ts
        lat.append((st["t_done_ms"] - st["t_submit_ms"]) + lag * 1e3)
        que.append((st["t_admit_ms"] - st["t_submit_ms"]) + lag * 1e3)
        svc.append(st["t_done_ms"] - st["t_admit_ms"])
        pts += stream[i]["n"]
        t_end = max(t_end, time.perf_counter())
        rows.append((i, u, st))
    th.join()
    stats = srv.stats()
    # rel-RMS against the oracle on sampled targets of a few requests
    errs = {1: [], 2: []}
    checked = []
    if not args.no_cpu_baseline and rows:
        import oracle

        g = workloads.rng(seed + 2)
        pick = rows[:: max(1, len(rows) // args.serve_checks)][: args.serve_checks]
        for i, u, st in pick:
            d = stream[i]
            n, off, rc, xi, prec = prep(d)
            idx = np.sort(g.choice(n, size=min(n, 256), replace=False))
            ref = oracle.halfspace(d["kernel"], y[off:off + n], sh[d["kernel"]][off:off + n], y[off:off + n][idx])
            err = oracle.rel_rms(ref, u.cpu().numpy()[idx])
            ran = st["report"]["precision"]
            errs[ran].append(err)
            checked.append({"kernel": d["kernel"], "N": n, "tol": d["tol"], "precision": ran, "xi": round(xi, 3),
                            "r_c": round(rc, 5), "Mt": st["report"]["Mt"], "rel_rms": err})
    srv.close()
    pc = lambda a, p: float(np.percentile(np.array(a), p)) if a else None
    return {
        "requests": len(lat), "requests_planned": args.serve_requests, "lambda_per_s": lam,
        "capacity_per_s": mu, "utilization_target": args.serve_util,
        "p50_ms": pc(lat, 50), "p99_ms": pc(lat, 99), "queue_p50_ms": pc(que, 50), "queue_p99_ms": pc(que, 99),
        "service_p50_ms": pc(svc, 50), "service_p99_ms": pc(svc, 99),
        "points_per_s": pts / max(t_end - tstart, 1e-9), "nslots": args.serve_slots, "arena_gb": arena / 2**30,
        "arena_peak_gb": stats["arena_peak"] / 2**30, "cache_hits": stats["cache_hits"],
        "cache_misses": stats["cache_misses"], "evictions": stats["evictions"], "failed": stats["failed"],
        "rel_rms_fp64_max": max(errs[1]) if errs[1] else None, "rel_rms_fp32_max": max(errs[2]) if errs[2] else None,
        "rel_rms_checked": len(errs[1]) + len(errs[2]), "checked": checked,
        "workload": "Poisson arrivals; N log-uniform in [1e3, 1e6]; kernel uniform over stokeslet/stresslet/rotlet; "
                    "tol uniform over {1e-5 FP32, 1e-10 FP64}; uniform unit-cube positions (slices of a seeded pool); "
                    "r_c for ~600 (FP64) / ~300 (FP32; r_c >= 0.08 stokeslet, >= 0.15 stresslet) neighbours, "
                    "xi from the real-space estimate, auto precision",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--neighbours", type=float, default=30.0)
    ap.add_argument("--fp32-neighbours", type=float, default=300.0,
                    help="neighbours per point for the FP32 variant (its rounding error grows with xi L)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target duration of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-tune", action="store_true", help="skip the runtime-optimal (xi, r_c) search")
    ap.add_argument("--tune-evals", type=int, default=12, help="candidates the (xi, r_c) search may time")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-util", type=float, default=0.7, help="arrival rate as a fraction of measured capacity")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-arena-gb", type=float, default=200.0)
    ap.add_argument("--serve-calib", type=int, default=48, help="closed-loop calibration requests")
    ap.add_argument("--serve-max-seconds", type=float, default=120.0, help="stop admitting arrivals after this")
    ap.add_argument("--serve-pool", type=int, default=1_000_000)
    ap.add_argument("--serve-checks", type=int, default=12, help="requests checked against the oracle (256 targets each)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB device-to-device copy first (calibrates profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1802_07844_amd as ehs
    from paper_1802_07844_amd import workloads

    n = args.n
    seed = workloads.SEED_BASE + 1
    y, f = workloads.uniform_stokeslet(n, seed)
    dev = torch.device("cuda:0")
    yd = torch.from_numpy(y).to(dev)
    fd = torch.from_numpy(f).to(dev)
    out = torch.empty((n, 3), dtype=torch.float64, device=dev)
    # r_c for ~30 neighbours in the unit box, xi from the real-space estimate
    rc = (args.neighbours * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
    tol = 1e-10
    # the real-space estimate takes a quarter of the budget (xi_for_cutoff gives estimate = tol'/2)
    xi = ehs.xi_for_cutoff("stokeslet", rc, tol / 2)

    if args.copy_probe:
        src = torch.ones(2**27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = ehs.Context(0)
    ctx.set_option(ehs.OPT_PRECISION, 1)
    ctx.set_option(ehs.OPT_TIMING, 1)

    def step(o, t):
        return ctx.stokeslet(yd, fd, yd, xi, rc, t, out=o, report=True)[1]

    for _ in range(args.warmup):
        step(out, tol)
    torch.cuda.synchronize()
    stage_sum = np.zeros(ehs.NSTAGES)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rep = step(out, tol)
        stage_sum += np.array(list(rep.ms_stage))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = n * args.steps / dt
    stage_ms = dict(zip(ehs.STAGES, (stage_sum / args.steps).tolist()))
    u64 = out.cpu().numpy()

    # dominant kernel and its roofline: algorithmic bytes per launch / average
    # launch duration (HIP events on the evaluation's stream)
    roofline = _roofline(rep, stage_ms, _ncin(rep), 8, "z_scale_stokeslet_N100k_fp64_counters.md",
                         "valu_stokeslet_N100k_fp64_counters.md")

    result = {
        "metric": "points/sec at rel-RMS 1e-10 (FP64)",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"half-space stokeslet, N={n} sources=targets uniform in [0,1)^2x(0,1], "
                               f"forces N(0,1), FP64 tol 1e-10, ~{args.neighbours:g} neighbours",
                   "N": n, "xi": xi, "r_c": rc, "tol": tol, "M": rep.M, "P": rep.P, "Mt": rep.Mt,
                   "eta": rep.eta, "zslab": rep.zslab, "Ps": rep.Ps, "Pg": rep.Pg, "dgrid": rep.dgrid,
                   "x3_first": rep.x3_first, "x3_corr_end": rep.x3_corr_end,
                   "seed": seed},
        "stage_ms": stage_ms,
        "roofline": roofline,
    }

    # the same problem at the runtime-optimal (xi, r_c) of the tuning procedure
    # (both truncation errors held, xi perturbed), timed like the main line
    def tuned(xi0, rc0, t, dtype):
        tres = ctx.tune("stokeslet", yd, fd, yd, xi0, rc0, t, max_evals=args.tune_evals)
        xit, rct = tres["xi"], tres["r_c"]
        outt = torch.empty_like(out)
        for _ in range(args.warmup):
            rt = ctx.stokeslet(yd, fd, yd, xit, rct, t, out=outt, report=True)[1]
        torch.cuda.synchronize()
        stt = np.zeros(ehs.NSTAGES)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rt = ctx.stokeslet(yd, fd, yd, xit, rct, t, out=outt, report=True)[1]
            stt += np.array(list(rt.ms_stage))
        torch.cuda.synchronize()
        dtt = time.perf_counter() - t0
        res = {"value": n * args.steps / dtt, "unit": "points/s", "ms_per_step": dtt / args.steps * 1e3,
               "dtype": dtype, "tol": t, "xi": xit, "r_c": rct,
               "neighbours": 4.0 / 3.0 * math.pi * rct**3 * n, "M": rt.M, "P": rt.P, "Mt": rt.Mt,
               "stage_ms": dict(zip(ehs.STAGES, (stt / args.steps).tolist())),
               "search": [{"xi": a, "r_c": b, "ms": c} for a, b, c in tres["trace"]],
               "note": "same points and forces; xi perturbed with both truncation estimates held"}
        return res, outt.cpu().numpy()

    ut = None
    if not args.no_tune:
        result["tuned"], ut = tuned(xi, rc, tol, "f64")

    # FP32 path on the same workload at tol 1e-5
    u32 = ut32 = None
    if not args.no_fp32:
        tol32 = 1e-5
        ctx.set_option(ehs.OPT_PRECISION, 2)
        rc32 = (args.fp32_neighbours * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
        xi32 = ehs.xi_for_cutoff("stokeslet", rc32, tol32 / 2)
        out32 = torch.empty_like(out)

        def step32():
            return ctx.stokeslet(yd, fd, yd, xi32, rc32, tol32, out=out32, report=True)[1]

        for _ in range(args.warmup):
            step32()
        torch.cuda.synchronize()
        st32 = np.zeros(ehs.NSTAGES)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r32 = step32()
            st32 += np.array(list(r32.ms_stage))
        torch.cuda.synchronize()
        dt32 = time.perf_counter() - t0
        u32 = out32.cpu().numpy()
        sm32 = dict(zip(ehs.STAGES, (st32 / args.steps).tolist()))
        result["fp32"] = {"value": n * args.steps / dt32, "unit": "points/s", "ms_per_step": dt32 / args.steps * 1e3,
                          "dtype": "f32", "tol": tol32, "xi": xi32, "r_c": rc32, "neighbours": args.fp32_neighbours,
                          "M": r32.M, "P": r32.P, "Mt": r32.Mt, "stage_ms": sm32,
                          "roofline": _roofline(r32, sm32, _ncin(r32), 4)}
        if not args.no_tune:
            result["fp32"]["tuned"], ut32 = tuned(xi32, rc32, tol32, "f32")

    # oracle on the host cores: a bounded sample of targets against all sources
    if not args.no_cpu_baseline:
        import oracle

        cores = oracle.max_threads()
        # size the sample from two short probes (the first also absorbs thread start-up)
        S = 64
        for target_s in (0.5, args.cpu_seconds):
            t0 = time.perf_counter()
            oracle.halfspace("stokeslet", y, f, y[:S])
            tp = time.perf_counter() - t0
            if target_s == args.cpu_seconds:
                break
            S = int(max(64, min(n, S * target_s / max(tp, 1e-6))))
        S = int(max(64, min(n, S * args.cpu_seconds / max(tp, 1e-6))))
        g = workloads.rng(seed + 1000)
        idx = np.sort(g.choice(n, size=S, replace=False))
        t0 = time.perf_counter()
        ref = oracle.halfspace("stokeslet", y, f, y[idx])
        tc = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": S / tc, "unit": "points/s", "cores": cores, "kind": "oracle",
                                  "sample": f"{S} of {n} targets against all {n} sources, FP64 direct sum, "
                                            f"{tc:.1f} s"}
        result["rel_rms_fp64"] = oracle.rel_rms(ref, u64[idx])
        if u32 is not None:
            result["fp32"]["rel_rms"] = oracle.rel_rms(ref, u32[idx])
        if ut is not None:
            result["tuned"]["rel_rms"] = oracle.rel_rms(ref, ut[idx])
        if ut32 is not None:
            result["fp32"]["tuned"]["rel_rms"] = oracle.rel_rms(ref, ut32[idx])
    if not args.no_serve:
        del out
        if u32 is not None:
            del out32
        ctx.close()
        torch.cuda.empty_cache()
        result["serving"] = serve_bench(args, ehs, workloads, torch, np)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
