"""Benchmark: half-space spectral Ewald summation on one MI355X.

One step = one full evaluation of the half-space sum: bounding box and plan,
cell binning, real-space sum, spreading, zero-padded 3D transforms with the
fused scaling, inverse transforms, quadrature and FP64 combination.  Inputs
are resident in device memory before the timed region; the truncated-kernel
precompute happens during warm-up (it depends on the grid size only and is
left out, as in the paper's timings).

Headline (`value`): the N = 4,000,000 stokeslet clustered at the wall
(x1, x2 uniform in [0,1), x3 ~ Exp(mean 0.05) clipped to (0,1]), forces
N(0,1), sources = targets, FP64 at tol 1e-10 -- the largest single-GPU
workload of the benchmark set.  Beside it, each with its relative RMS error
against the FP64 oracle on a sample of targets, its stage times and its
roofline:

  fp32      the same clustered set in FP32 at tol 1e-5;
  c3        N = 1,000,000 uniform stresslet (unit orientations) and rotlet,
            FP64 at tol 1e-10 and FP32 at tol 1e-5;
  c2        N = 100,000 uniform stokeslet, FP64 at tol 1e-10 (~30
            neighbours) and FP32 at tol 1e-5 (~300 neighbours);
  tuned     the N = 100,000 FP64 problem at the (xi, r_c) of the runtime
            parameter search (the tuning procedure of the paper's results);
  serving   a Poisson stream of mixed requests through one server;
  cpu_baseline  the FP64 oracle on the host cores, on a bounded sample of the
            headline workload's targets against all its sources.

The roofline of every leg is the per-stage model in stage_model(): closed-
form algorithmic bytes (inputs read once, outputs written once) and flops
(transforms counted as 5 n log2 n per complex line of length n, less one
radix-2 stage where half the input or output is zero; spreading, quadrature
and real-space pairs counted from their formulas), each stage bound by the
larger of bytes / 8 TB/s and flops / vector peak.  Prints one JSON line.
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
VALU_PEAK_TFS = {8: 78.6, 4: 157.3}  # vector FP64 / FP32, MI355X

# flops per in-range pair of the real-space sum, counted from the kernels'
# formulas (direct_term / image_term) with the transcendental parts costed as
# their instruction sequences: exp 22, sqrt 8, division 8 (reciprocal and
# Newton steps), erfc from the exponential 39 (division, degree-14 Horner,
# one product); the per-pair distance 8
PAIR_FLOPS = {
    "direct": {0: 112, 1: 131, 2: 99},
    "image": {0: 171, 1: 246, 2: 158},
}


def _fft(n, pruned=True):
    """Flops of one complex line transform of length n (one radix-2 stage
    fewer when half its input or output is zero)."""
    return 5.0 * n * (math.log2(n) - (1.0 if pruned else 0.0))


def stage_model(rep, N, T, esz):
    """Closed-form algorithmic bytes and flops of each stage of one evaluation
    under the plan in `rep` (an ehs.Report): {stage: (bytes, flops)}."""
    Mt = rep.Mt
    e = esz
    fam = rep.family
    free = bool(rep.free_space)                  # free space: sources only, kernel grids only
    nca = 6 if fam == 1 else 3                   # kernel-grid components
    ncb = {0: 4, 1: 7, 2: 2}[fam]                # separate correction grids
    nin = nca + (0 if free else 1 if rep.dgrid else ncb)  # spread / forward grids
    nout = 3 if free else 4 if e == 8 else 6     # inverse grids
    ns = 6 if fam == 1 else 3                    # strength values per source
    keep = (2 * Mt - rep.x3_first) / (2 * Mt)    # inverse side: rows the quadrature reads
    czf = rep.x3_corr_end / (2 * Mt)             # correction grids: rows below the images' support top
    nin_eff = nin * czf if free else nca + (nin - nca) * czf
    V_R = Mt * Mt * 2 * Mt
    V_A = (Mt + 1) * 2 * Mt * Mt
    V_Z = (Mt + 1) * 4 * Mt * Mt
    kinds = 1 if (fam == 2 or free) else 2
    oct_bytes = (Mt + 1) ** 2 * (2 * Mt + 1) * (8 if e == 8 else 4) * kinds
    n2, n4 = 2 * Mt, 4 * Mt
    Ps3, Pg3 = rep.Ps ** 3, rep.Pg ** 3
    m = {}
    m["realspace"] = (N * (3 + ns) * 8 + T * 9 * 8,
                      rep.pairs_direct * PAIR_FLOPS["direct"][fam] + rep.pairs_image * PAIR_FLOPS["image"][fam])
    # sources carry the kernel grid, images the kernel grid and the corrections
    m["spread"] = (nin * V_R * e + N * (3 + ns) * 8,
                   N * Ps3 * (1 + 2 * nca) + (0 if free else N * Ps3 * (1 + 2 * nin)))
    # x1: real lines of padded length 2 Mt (two per complex transform)
    m["fwd_x"] = (nin_eff * (V_R * e + V_A * 2 * e), nin_eff * Mt * n2 * 0.5 * _fft(n2))
    # x2: A (x1 half spectrum, x2 nodes) to the x2 spectrum over the padded length
    m["fwd_y"] = (nin_eff * (V_A + V_Z) * 2 * e, nin_eff * (Mt + 1) * n2 * _fft(n2))
    # x3 pass: forward (input half zero) and inverse (output kept from x3_first)
    # of length 4 Mt per (k1, k2) line, and the scaling (about 8 flops per
    # input component and k); the k-space grid is never stored
    m["z_scale"] = (nin_eff * V_Z * 2 * e + nout * V_Z * 2 * e * keep + oct_bytes,
                    (Mt + 1) * n2 * ((nin + nout) * _fft(n4) + 8.0 * nin * n4))
    m["inv_y"] = (nout * (V_Z + V_A) * keep * 2 * e, nout * (Mt + 1) * n2 * keep * _fft(n2))
    m["inv_x"] = (nout * (V_A * 2 * e + V_R * e) * keep, nout * Mt * n2 * keep * 0.5 * _fft(n2))
    m["gather"] = (nout * V_R * keep * e + T * 9 * 8, T * Pg3 * (1 + 2 * nout))
    return m


def roofline(rep, stage_ms, N, T, esz, ms_step):
    """Per stage: floor = max(bytes / HBM peak, flops / vector peak) and the
    bound it names; for the dominant stage (largest measured time) the
    achieved rate against that bound's peak; for the whole step the sum of
    the floors against the measured time."""
    model = stage_model(rep, N, T, esz)
    vpk = VALU_PEAK_TFS[esz]
    stages = {}
    floor_sum = 0.0
    for k, (b, f) in model.items():
        t_h = b / (HBM_PEAK_GBS * 1e9) * 1e3
        t_v = f / (vpk * 1e12) * 1e3
        fl = max(t_h, t_v)
        floor_sum += fl
        ms = stage_ms.get(k, 0.0)
        stages[k] = {"ms": ms, "bytes": b, "flops": f, "floor_ms": fl, "bound": "hbm" if t_h >= t_v else "alu",
                     "frac": fl / ms if ms > 0 else None}
    dom = max(stages, key=lambda k: stages[k]["ms"])
    d = stages[dom]
    launches = 1
    if dom in ("fwd_y", "z_scale", "inv_y"):
        launches = (rep.Mt + rep.zslab) // rep.zslab  # one launch per group of k1 slabs
    ms_launch = d["ms"] / launches
    gbs = d["bytes"] / launches / (ms_launch * 1e-3) / 1e9
    tfs = d["flops"] / launches / (ms_launch * 1e-3) / 1e12
    if d["bound"] == "hbm":
        achieved, peak, unit = gbs, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, unit = tfs, vpk, "TFLOP/s"
    # the method's own minimum over the whole step: the spread grids read once,
    # the output grids written once, the octants and the point data (the
    # transform intermediates not materialised), against all its flops
    Mt, e = rep.Mt, esz
    free = bool(rep.free_space)
    nin = (6 if rep.family == 1 else 3) + (0 if free else 1 if rep.dgrid else {0: 4, 1: 7, 2: 2}[rep.family])
    nout = 3 if free else 4 if e == 8 else 6
    keep = (2 * Mt - rep.x3_first) / (2 * Mt)
    V_R = Mt * Mt * 2 * Mt
    oct_bytes = (Mt + 1) ** 2 * (2 * Mt + 1) * (8 if e == 8 else 4) * (1 if (rep.family == 2 or free) else 2)
    mb = (nin + nout * keep) * V_R * e + oct_bytes + model["realspace"][0]
    mf = sum(f for _, f in model.values())
    m_floor = max(mb / (HBM_PEAK_GBS * 1e9), mf / (vpk * 1e12)) * 1e3
    method = {"bytes": mb, "flops": mf, "floor_ms": m_floor,
              "bound": "hbm" if mb / (HBM_PEAK_GBS * 1e9) >= mf / (vpk * 1e12) else "alu",
              "hbm_frac": mb / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
              "valu_frac": mf / (ms_step * 1e-3) / 1e12 / vpk}
    return {"bound": d["bound"], "kernel": dom, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": None,
            "hbm": {"achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS},
            "valu": {"achieved_tfs": tfs, "frac": tfs / vpk, "precision": "fp64" if esz == 8 else "fp32"},
            "bytes_per_launch": d["bytes"] / launches, "flops_per_launch": d["flops"] / launches,
            "launches_per_step": launches, "ms_per_launch": ms_launch,
            "step": {"floor_ms": floor_sum, "ms": ms_step, "frac": floor_sum / ms_step},
            "method": method, "stages": stages}


def _measured_traffic(name, kernel):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary (a line 'traffic-json: {...}' in profiles/<name>) taken on the
    current library sources; else None."""
    import hashlib

    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1802_07844_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    sha = h.hexdigest()[:16]
    for line in open(path):
        if line.startswith("traffic-json:"):
            d = json.loads(line.split(":", 1)[1])
            if d.get("kernel") == kernel and d.get("sources_sha") == sha:
                return d
    return None


def _rc(nb, n):
    return (nb * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)


# the legs: (family, layout, N, precision, tol, r_c rule)
WORKLOADS = {
    # (r_c, xi): the runtime-optimal pair that ehs_tune's search finds from
    # (0.035, xi for it) in FP64 and (0.03, xi for it) in FP32 on these points
    "c4_fp64": ("stokeslet", "clustered", 4_000_000, 1, 1e-10, (0.04170, 117.15)),
    "c4_fp32": ("stokeslet", "clustered", 4_000_000, 2, 1e-5, (0.02746, 126.89)),
    "c3_stresslet_fp64": ("stresslet", "uniform", 1_000_000, 1, 1e-10, ("nb", 2000)),
    "c3_rotlet_fp64": ("rotlet", "uniform", 1_000_000, 1, 1e-10, ("nb", 2000)),
    "c3_stresslet_fp32": ("stresslet", "uniform", 1_000_000, 2, 1e-5, ("nb", 2000)),
    "c3_rotlet_fp32": ("rotlet", "uniform", 1_000_000, 2, 1e-5, ("nb", 2000)),
    "c2_fp64": ("stokeslet", "uniform", 100_000, 1, 1e-10, ("nb", 30)),
    "c2_fp32": ("stokeslet", "uniform", 100_000, 2, 1e-5, ("nb", 300)),
    # half space and free space side by side (the same points and parameters)
    "c2_stresslet_fp64": ("stresslet", "uniform", 100_000, 1, 1e-10, ("nb", 300)),
    "c2_rotlet_fp64": ("rotlet", "uniform", 100_000, 1, 1e-10, ("nb", 300)),
    "free_stokeslet_fp64": ("stokeslet", "uniform", 100_000, 1, 1e-10, ("nb", 30), True),
    "free_stresslet_fp64": ("stresslet", "uniform", 100_000, 1, 1e-10, ("nb", 300), True),
    "free_rotlet_fp64": ("rotlet", "uniform", 100_000, 1, 1e-10, ("nb", 300), True),
}
SEEDS = {"c2": 1, "c3": 2, "c4": 3}


def _free(name):
    return len(WORKLOADS[name]) > 6 and WORKLOADS[name][6]


def describe(name):
    fam, layout, n, prec, tol, rcr = WORKLOADS[name][:6]
    where = ("x1, x2 uniform in [0,1), x3 ~ Exp(mean 0.05) clipped to (0,1]" if layout == "clustered"
             else "uniform in [0,1)^2 x (0,1]")
    strengths = {"stokeslet": "forces N(0,1)", "stresslet": "strengths N(0,1)^3, orientations uniform on S^2",
                 "rotlet": "torques N(0,1)^3"}[fam]
    if not isinstance(rcr, tuple):
        cut = f"r_c = {rcr}"
    elif rcr[0] == "nb":
        cut = f"r_c for ~{rcr[1]} neighbours"
    else:
        cut = f"r_c = {rcr[0]}, xi = {rcr[1]} (runtime-optimal pair of the parameter search)"
    return (f"{'free-space' if _free(name) else 'half-space'} {fam}, N={n} sources=targets {where}, {strengths}, "
            f"{'FP64' if prec == 1 else 'FP32'} tol {tol:g}, {cut}")


class Runner:
    def __init__(self, args, ehs, workloads, torch, np):
        self.args, self.ehs, self.wl, self.torch, self.np = args, ehs, workloads, torch, np
        self.ctx = ehs.Context(0)
        self.ctx.set_option(ehs.OPT_TIMING, 1)
        self.serial = bool(getattr(args, "serial", False))
        self.ctx.set_option(ehs.OPT_OVERLAP, 0 if self.serial else 1)
        self.data = {}

    def inputs(self, name):
        fam, layout, n, prec, tol, rcr = WORKLOADS[name][:6]
        key = (fam, layout, n)
        if key not in self.data:
            seed = self.wl.SEED_BASE + SEEDS[name[:2]]
            y, s = self.wl.make(fam, n, seed, layout=layout)
            dev = self.torch.device("cuda:0")
            self.data = {k: v for k, v in self.data.items() if k[2] <= 1_000_000}  # keep device memory modest
            self.data[key] = (y, s, self.torch.from_numpy(y).to(dev), self.torch.from_numpy(s).to(dev), seed)
        return self.data[key]

    def params(self, name):
        fam, layout, n, prec, tol, rcr = WORKLOADS[name][:6]
        if isinstance(rcr, tuple) and rcr[0] != "nb":
            rc, xi = rcr  # a searched (r_c, xi) pair
            return fam, n, prec, tol, rc, xi
        rc = _rc(rcr[1], n) if isinstance(rcr, tuple) else rcr
        # the real-space estimate takes a quarter of the budget
        xi = self.ehs.xi_for_cutoff(fam, rc, tol / 2)
        return fam, n, prec, tol, rc, xi

    def run(self, name, steps, warmup, xi=None, rc=None):
        np, torch = self.np, self.torch
        fam, n, prec, tol, rc0, xi0 = self.params(name)
        xi = xi0 if xi is None else xi
        rc = rc0 if rc is None else rc
        y, s, yd, sd, seed = self.inputs(name)
        self.ctx.set_option(self.ehs.OPT_PRECISION, prec)
        out = torch.empty((n, 3), dtype=torch.float64, device="cuda:0")
        fs = _free(name)
        for _ in range(warmup):
            self.ctx.evaluate(fam, yd, sd, yd, xi, rc, tol, out=out, report=True, free_space=fs)
        torch.cuda.synchronize()
        st = np.zeros(self.ehs.NSTAGES)
        t0 = time.perf_counter()
        for _ in range(steps):
            rep = self.ctx.evaluate(fam, yd, sd, yd, xi, rc, tol, out=out, report=True, free_space=fs)[1]
            st += np.array(list(rep.ms_stage))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms = dt / steps * 1e3
        stage_ovl = dict(zip(self.ehs.STAGES, (st / steps).tolist()))
        # The timed steps run the real-space sum beside the grid stages
        # (EHS_OPT_OVERLAP), where a stage's events also count the time its
        # kernels wait for the other stream's blocks; the per-stage times of
        # the roofline come from a few steps in serial order right after.
        nser = 0 if self.serial else min(3, steps)
        self.ctx.set_option(self.ehs.OPT_OVERLAP, 0)
        st = np.zeros(self.ehs.NSTAGES)
        for _ in range(nser):
            rep = self.ctx.evaluate(fam, yd, sd, yd, xi, rc, tol, out=out, report=True, free_space=fs)[1]
            st += np.array(list(rep.ms_stage))
        self.ctx.set_option(self.ehs.OPT_OVERLAP, 0 if self.serial else 1)
        stage_ms = dict(zip(self.ehs.STAGES, (st / nser).tolist())) if nser else stage_ovl
        esz = 8 if rep.precision == 1 else 4
        nin = (6 if rep.family == 1 else 3) + (0 if fs else 1 if rep.dgrid else {0: 4, 1: 7, 2: 2}[rep.family])
        res = {"value": n * steps / dt, "unit": "points/s", "ms_per_step": ms, "steps": steps, "warmup": warmup,
               "transforms": {"forward": nin, "inverse": 3 if fs else (4 if esz == 8 else 6)},
               "dtype": "f64" if esz == 8 else "f32", "tol": tol, "xi": xi, "r_c": rc,
               "plan": {"M": rep.M, "P": rep.P, "Mt": rep.Mt, "eta": rep.eta, "Ps": rep.Ps, "Pg": rep.Pg,
                        "zslab": rep.zslab, "dgrid": rep.dgrid, "x3_first": rep.x3_first,
                        "x3_corr_end": rep.x3_corr_end, "cell_reach": rep.cell_reach,
                        "occupancy": rep.occupancy, "precision": rep.precision, "warnings": rep.warnings,
                        "est_real": rep.est_real, "est_fourier": rep.est_fourier, "est_fp32": rep.est_fp32},
               "pairs": {"direct": rep.pairs_direct, "image": rep.pairs_image,
                         "per_target": (rep.pairs_direct + rep.pairs_image) / n},
               "stage_ms": stage_ms, "stage_ms_overlapped": stage_ovl,
               "stage_note": ("stage_ms: the timed steps, in serial order (--serial)" if self.serial else
                              f"stage_ms: {nser} steps in serial order after the timed region; "
                              "stage_ms_overlapped: the timed steps, real-space sum beside the grid stages"),
               "roofline": roofline(rep, stage_ms, n, n, esz, ms)}
        u = out.cpu().numpy()
        del out
        return res, u

    def check(self, name, u, nsample):
        """rel-RMS and the worst target's error against the oracle on a seeded sample."""
        import oracle

        fam, n, prec, tol, rc, xi = self.params(name)
        y, s, yd, sd, seed = self.inputs(name)
        idx = self.np.sort(self.wl.rng(seed + 1000).choice(n, size=min(n, nsample), replace=False))
        ref = (oracle.freespace if _free(name) else oracle.halfspace)(fam, y, s, y[idx])
        err = oracle.rel_rms(ref, u[idx])
        vrms = self.np.sqrt(self.np.mean(self.np.sum(ref * ref, axis=1)))
        worst = float(self.np.max(self.np.linalg.norm(u[idx] - ref, axis=1)) / vrms)
        return {"rel_rms": err, "worst_target_rel": worst, "sample": len(idx)}


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


_T0 = time.perf_counter()


def progress(msg):
    """One line per finished step of the run, on stderr (the JSON line stays
    alone on stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


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
    srv.set_option(ehs.OPT_ADMISSION, args.serve_admission)
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
        if len(rows) % 250 == 0:
            progress(f"serving: {len(rows)} requests done")
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
    sizes = np.array([stream[i]["n"] for i, _, _ in rows]) if rows else np.array([])
    pc = lambda a, p: float(np.percentile(np.array(a), p)) if len(a) else None
    by_size = {}
    for lo, hi, lab in ((1e3, 1e4, "N<1e4"), (1e4, 1e5, "1e4<=N<1e5"), (1e5, 1e6 + 1, "N>=1e5")):
        ks = [k for k in range(len(lat)) if lo <= sizes[k] < hi]
        sel, sq, ss = [lat[k] for k in ks], [que[k] for k in ks], [svc[k] for k in ks]
        by_size[lab] = {"requests": len(sel), "p50_ms": pc(sel, 50), "p99_ms": pc(sel, 99),
                        "queue_p99_ms": pc(sq, 99), "service_p50_ms": pc(ss, 50), "service_p99_ms": pc(ss, 99)}
    return {
        "requests": len(lat), "requests_planned": args.serve_requests, "lambda_per_s": lam,
        "capacity_per_s": mu, "utilization_target": args.serve_util,
        "p50_ms": pc(lat, 50), "p99_ms": pc(lat, 99), "queue_p50_ms": pc(que, 50), "queue_p99_ms": pc(que, 99),
        "service_p50_ms": pc(svc, 50), "service_p99_ms": pc(svc, 99), "by_size": by_size,
        "points_per_s": pts / max(t_end - tstart, 1e-9), "nslots": args.serve_slots, "arena_gb": arena / 2**30,
        "admission": "smallest-first, one slot kept for <= 65,536 points" if args.serve_admission else "first-come",
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
    ap.add_argument("--leg-steps", type=int, default=10, help="timed steps of each leg beside the headline")
    ap.add_argument("--workload", default="c4_fp64", choices=sorted(WORKLOADS), help="headline workload")
    ap.add_argument("--legs", default="fp32,c3,c2,free,tuned",
                    help="comma list of extra legs (fp32, c3, c2, free, tuned) or 'none'")
    ap.add_argument("--oracle-sample", type=int, default=512, help="targets checked against the oracle per leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target duration of the oracle timing sample")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing and every oracle check")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--tune-evals", type=int, default=12, help="candidates the (xi, r_c) search may time")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-util", type=float, default=0.7, help="arrival rate as a fraction of measured capacity")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-admission", type=int, default=1, choices=[0, 1],
                    help="1: smallest request first with one slot kept for small ones; 0: first come first served")
    ap.add_argument("--serve-arena-gb", type=float, default=200.0)
    ap.add_argument("--serve-calib", type=int, default=48, help="closed-loop calibration requests")
    ap.add_argument("--serve-max-seconds", type=float, default=120.0, help="stop admitting arrivals after this")
    ap.add_argument("--serve-pool", type=int, default=1_000_000)
    ap.add_argument("--serve-checks", type=int, default=12, help="requests checked against the oracle (256 targets each)")
    ap.add_argument("--serial", action="store_true",
                    help="run the real-space sum on the caller's stream, in order with the grid stages "
                         "(profiling runs: every kernel's trace is then its own time)")
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

    if args.copy_probe:
        src = torch.ones(2**27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    R = Runner(args, ehs, workloads, torch, np)
    legs = [] if args.legs == "none" else [x for x in args.legs.split(",") if x]
    head = args.workload
    fam, layout, n, prec, tol, rcr = WORKLOADS[head]
    res, u = R.run(head, args.steps, args.warmup)
    progress(f"{head}: {res['ms_per_step']:.1f} ms per step")
    rec = {"metric": "points/sec at rel-RMS 1e-10 (FP64)" if prec == 1 else "points/sec at rel-RMS 1e-5 (FP32)",
           "value": res["value"], "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": res["dtype"], "data": "synthetic",
           "config": {"workload": describe(head), "N": n, "xi": res["xi"], "r_c": res["r_c"], "tol": tol,
                      "seed": workloads.SEED_BASE + SEEDS[head[:2]], **res["plan"]},
           "pairs": res["pairs"], "stage_ms": res["stage_ms"], "stage_ms_overlapped": res["stage_ms_overlapped"],
           "stage_note": res["stage_note"], "roofline": res["roofline"]}
    tr = _measured_traffic(f"{res['roofline']['kernel']}_{head}_counters.md", res["roofline"]["kernel"])
    if tr is not None:
        rec["roofline"]["traffic"] = tr["bytes_per_launch"]
    checks = []  # (record, leg name, u)
    checks.append((rec, head, u))
    extra = {}

    def leg(name, steps=args.leg_steps):
        r, uu = R.run(name, steps, min(args.warmup, 2))
        r["workload"] = describe(name)
        checks.append((r, name, uu))
        progress(f"{name}: {r['ms_per_step']:.1f} ms per step")
        return r

    if "fp32" in legs and head == "c4_fp64":
        rec["fp32"] = leg("c4_fp32")
    if "c3" in legs:
        extra["c3"] = {k: leg(f"c3_{k}") for k in ("stresslet_fp64", "rotlet_fp64", "stresslet_fp32", "rotlet_fp32")}
    if "c2" in legs:
        extra["c2"] = {"fp64": leg("c2_fp64"), "fp32": leg("c2_fp32")}
    if "free" in legs:
        # the free-space sum of the same kernels on the same points and
        # parameters (no images, no corrections): the step-time ratio
        # half space / free space and the transformed grids of each
        half = {"stokeslet": extra["c2"]["fp64"] if "c2" in extra else leg("c2_fp64"),
                "stresslet": leg("c2_stresslet_fp64"), "rotlet": leg("c2_rotlet_fp64")}
        fr = {k: leg(f"free_{k}_fp64") for k in ("stokeslet", "stresslet", "rotlet")}
        extra["free"] = {k: {"free": fr[k], "half": half[k] if k != "stokeslet" else None,
                             "ratio_half_over_free": half[k]["ms_per_step"] / fr[k]["ms_per_step"],
                             "transforms_half": half[k]["transforms"], "transforms_free": fr[k]["transforms"]}
                         for k in fr}
    if "tuned" in legs:
        # the N = 1e5 FP64 problem at the runtime-optimal (xi, r_c) of the
        # tuning procedure (both truncation errors held, xi perturbed)
        _, nn, _, t64, rc64, xi64 = R.params("c2_fp64")
        y, s, yd, sd, _ = R.inputs("c2_fp64")
        R.ctx.set_option(ehs.OPT_PRECISION, 1)
        tres = R.ctx.tune("stokeslet", yd, sd, yd, xi64, rc64, t64, max_evals=args.tune_evals)
        r, uu = R.run("c2_fp64", args.leg_steps, min(args.warmup, 2), xi=tres["xi"], rc=tres["r_c"])
        r["workload"] = describe("c2_fp64") + " at the (xi, r_c) of the runtime parameter search"
        r["search"] = [{"xi": a, "r_c": b, "ms": c} for a, b, c in tres["trace"]]
        progress(f"tuned: {r['ms_per_step']:.1f} ms per step after {len(tres['trace'])} candidates")
        r["neighbours"] = 4.0 / 3.0 * math.pi * tres["r_c"] ** 3 * nn
        checks.append((r, "c2_fp64", uu))
        extra["tuned"] = r
    rec.update(extra)

    if not args.no_cpu_baseline:
        import oracle

        # the oracle's own throughput on the host cores: a bounded sample of
        # the headline workload's targets against all its sources
        y, s, yd, sd, seed = R.inputs(head)
        cores = oracle.max_threads()
        # double a seeded sample of targets until one call takes at least
        # half the requested time (a call also pays a fixed pass over all N
        # sources, so the time is not proportional to the sample at first);
        # the last call is the measurement
        oracle.halfspace(fam, y, s, y[:8])  # thread pool start-up
        order = workloads.rng(seed + 2000).permutation(n)
        S = 32
        while True:
            idx = np.sort(order[:S])
            t0 = time.perf_counter()
            oracle.halfspace(fam, y, s, y[idx])
            tc = time.perf_counter() - t0
            progress(f"oracle timing: {S} targets in {tc:.1f} s")
            if tc >= 0.5 * args.cpu_seconds or S >= min(n, 1 << 20):
                break
            S = min(n, 1 << 20, 2 * S if tc > 0.25 * args.cpu_seconds else 4 * S)
        rec["cpu_baseline"] = {"value": S / tc, "unit": "points/s", "cores": cores, "kind": "oracle",
                               "sample": f"{S} of {n} targets against all {n} sources ({describe(head)}), "
                                         f"FP64 direct sum, {tc:.1f} s"}
        progress(f"oracle timing sample: {S} targets, {tc:.1f} s")
        for r, name, uu in checks:
            r["oracle"] = R.check(name, uu, args.oracle_sample)
            progress(f"{name}: oracle rel-RMS {r['oracle']['rel_rms']:.2e}")
        rec["rel_rms"] = rec["oracle"]["rel_rms"]
    if not args.no_serve:
        R.ctx.close()
        R.data.clear()
        checks.clear()
        torch.cuda.empty_cache()
        progress("serving stream")
        rec["serving"] = serve_bench(args, ehs, workloads, torch, np)
        progress("serving done")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
