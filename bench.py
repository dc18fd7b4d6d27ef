"""Throughput of the two-component lattice Boltzmann hot path on one MI355X.

Workload: the 128^3 droplet box (R = 16, FP32 populations) driven through its
ghost nodes by a seeded Ornstein-Uhlenbeck velocity-gradient history (synthetic
stand-in for the turbulence-simulation gradients of Sec. 3).  One benchmark
"step" is one sample period of 50 lattice steps — 50 fused stream-collide
launches — followed by the droplet inertia-tensor moments of that sample (FP64
reduction into a device time series).  --steps 400 (default) times the full
20000-step run.

Prints one JSON line with MLUPS (one update = both components at one node),
the roofline of the step kernel (algorithmic bytes per launch over its average
launch duration, from HIP events on the library's stream) and the FP64 CPU
oracle timed on a bounded sample of the same box on the host cores.

The same line carries the surrogate comparison ("surrogate"): the ensemble of
64 boxes of 64^3 (R = 10, FP32, one OU drive each, 20000 lattice steps through
the captured step loop, droplet moments every 50 steps) gives the lattice
Boltzmann rate of shape samples and the training windows; the network is
trained on 56 trajectories by the library's kernels and evaluated on the 8
held out, and one 8192-window inference batch is timed with HIP events.  Surrogate
samples/s count the lattice Boltzmann replays of windows whose predicted D
exceeds 0.5.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STRIDE = 50


def step_kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("step_kernel.hpp", "lattice.hpp"):
        with open(os.path.join(ROOT, "paper_2112_09972_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per step-kernel launch (FETCH_SIZE + WRITE_SIZE, each scaled by
    the same counter's reading for a plain copy of known size) from the committed
    rocprofv3 summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "k_step_%s_traffic.txt" % workload)
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                d[k.strip()] = v.strip()
    if d.get("source_hash") != step_kernel_source_hash():
        return None
    return int(d["hbm_bytes_per_launch"])


def cpu_baseline(case):
    """The FP64 oracle (plain C, OpenMP over z) timed on the host cores: the 32^3
    shear box, one 64^3 ensemble box and the benchmark's 128^3 box with their own
    drives, on one core and on all cores (the 128^3 box only on all: one step
    there takes seconds on one core).  Each case: one warm-up step, then the median
    MLUPS of 5 repetitions of k steps, k chosen from the warm-up so that a
    repetition takes about 0.3 s.  `value` is the 128^3 box on all cores."""
    import oracle
    all_threads = oracle.num_threads()
    c1, c4 = wl.case_c1(), wl.case_c4(nsteps=400, nbox=1)
    boxes = [(c1, (1, all_threads)), (c4, (1, all_threads)), (case, (all_threads,))]
    cases = []
    t_start = time.perf_counter()
    for cs, thread_counts in boxes:
        tab = cs.tables[0]
        for th in thread_counts:
            oracle.set_num_threads(th)
            o = oracle.Oracle(cs.n, cs.n, cs.n, periodic=False, tau=(cs.tau, cs.tau), g=wl.G_AB, rho_b=cs.rho_b)
            o.init_droplet(o.xc, cs.radius, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tab[0])
            t0 = time.perf_counter()
            o.step(tab[0])  # warm-up (page-in, thread start)
            k = max(1, int(round(0.3 / (time.perf_counter() - t0))))
            rates = []
            step = 1
            for _ in range(5):
                t0 = time.perf_counter()
                for _ in range(k):
                    o.step(tab[step])
                    step += 1
                rates.append(cs.n ** 3 * k / (time.perf_counter() - t0) / 1e6)
            med = float(np.median(rates))
            cases.append({"box": cs.n, "workload": cs.name, "threads": th, "steps_per_rep": k, "reps": 5,
                          "mlups": round(med, 3), "mlups_per_core": round(med / th, 3)})
            del o
    oracle.set_num_threads(all_threads)
    big = cases[-1]
    return {"value": big["mlups"], "unit": "MLUPS", "cores": big["threads"], "kind": "oracle",
            "sample": "FP64 oracle on the %d^3 droplet box (same OU drive), median of 5 repetitions of %d steps on "
                      "%d threads; 32^3 and 64^3 boxes on 1 and %d threads in `cases`; %.1f s in all"
                      % (case.n, big["steps_per_rep"], big["threads"], all_threads, time.perf_counter() - t_start),
            "host_cpus": os.cpu_count(), "cases": cases}


def c1_against_oracle(sc, nsteps: int = 1000):
    """The 32^3 droplet box in steady simple shear at Ca = 0.1 (tau = 1) in every
    storage format against the FP64 oracle after `nsteps` steps: the largest
    per-node relative density error, the mass drift per component and the
    deformation D of the sheared droplet (Sec. 2 Eq. 4) next to the oracle's."""
    import oracle
    case = wl.case_c1()
    tab = case.tables[0][:nsteps]
    rho_b = case.rho_b
    o = oracle.Oracle(case.n, case.n, case.n, periodic=False, tau=(case.tau, case.tau), g=wl.G_AB, rho_b=rho_b)
    o.init_droplet(o.xc, case.radius, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tab[0])
    om0, _ = o.totals()
    o.run(nsteps, tab)
    om, _ = o.totals()
    oa, ob, _ = o.fields()
    od = oracle.droplet_stats(oa, ob, o.xc)["deformation"]
    out = {"workload": case.name, "lattice_steps": nsteps, "oracle": {"mass_drift_rel": [float(v) for v in (om - om0) / om0],
                                                                      "deformation": float(od)}, "results": {}}
    for prec in ("f64", "f32", "f32d", "f16dev", "bf16dev"):
        lat = sc.Lattice(case.n, case.n, case.n, bc="ghost", prec=prec, table_len=nsteps, g_ab=wl.G_AB, rho_b=rho_b,
                         mach_max=0.25)
        lat.init_droplet(lat.xc, case.radius, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tab[0])
        lat.set_gradient_table(tab, 0)
        m0, _ = lat.totals()
        lat.step(nsteps)
        m1, _ = lat.totals(check=False)
        ra, rb = (t.cpu().numpy() for t in lat.fields(velocity=False))
        err = max(float(np.max(np.abs(ra - oa) / oa)), float(np.max(np.abs(rb - ob) / ob)))
        d = lat.droplet()["deformation"]
        out["results"][prec] = {"max_rel_density_err": err, "mass_drift_rel": [float(v) for v in (m1 - m0) / m0],
                                "deformation": float(d), "deformation_abs_err": float(abs(d - od))}
        lat.close()
    print(json.dumps({"c1_against_oracle": out}), flush=True)
    return out


def precision_study(sc, nsteps: int):
    """The 256^3 droplet box (R = 32, OU drive seed 3) in every storage format:
    MLUPS, algorithmic bytes per update, mass drift and semi-axis / deformation
    error against the FP64 GPU run, from the droplet moments every 50 steps."""
    import torch
    case = wl.case_c3(prec="f64", nsteps=nsteps + 1)
    tab = case.tables[0]
    nodes = case.n ** 3
    bpl = {"f64": 608, "f32": 304, "f16dev": 160, "bf16dev": 160}
    series = {}
    out = {"workload": "c3_256cube_ou", "box": case.n, "radius": case.radius, "lattice_steps": nsteps,
           "results": {}}
    for prec in ("f64", "f32", "f16dev", "bf16dev"):
        lat = sc.Lattice(case.n, case.n, case.n, bc="ghost", prec=prec, table_len=nsteps, g_ab=wl.G_AB,
                         rho_b=case.rho_b, mach_max=wl.MACH_MAX)
        lat.init_droplet(lat.xc, case.radius, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tab[0])
        lat.set_gradient_table(tab[:nsteps], 0)
        m0, _ = lat.totals()
        ns = nsteps // STRIDE
        mom = torch.zeros((ns, 10), dtype=torch.float64, device=lat.device)
        lat.synchronize()
        t0 = time.perf_counter()
        for k in range(ns):
            lat.step(STRIDE)
            lat.droplet_moments(mom[k])
        lat.synchronize()
        el = time.perf_counter() - t0
        m1, _ = lat.totals(check=False)
        mm = mom.cpu().numpy()
        st = [sc.sclbm_droplet_from_moments(mm[i], lat.xc) for i in range(ns)]
        series[prec] = (np.array([x["semi_axes"] for x in st]), np.array([x["deformation"] for x in st]))
        ty, zc, wx = lat.get_launch()
        r = {"mlups": round(nodes * STRIDE * ns / el / 1e6, 1), "bytes_per_update": bpl[prec],
             "launch": {"tile_rows": ty, "zchunk": zc, "tile_waves": wx},
             "mass_drift_rel": [float(v) for v in (m1 - m0) / m0]}
        if prec != "f64":
            a64, d64 = series["f64"]
            a, d = series[prec]
            r["semi_axes_rel_err_max"] = float(np.max(np.abs(a - a64) / a64))
            r["deformation_abs_err_max"] = float(np.max(np.abs(d - d64)))
        out["results"][prec] = r
        print(json.dumps({prec: r}), flush=True)
        lat.close()
        del lat, mom
        torch.cuda.empty_cache()
    a64, d64 = series["f64"]
    out["f64_deformation_range"] = [float(d64.min()), float(d64.max())]
    out["c1_against_oracle"] = c1_against_oracle(sc)
    print(json.dumps(out))


MFMA_BF16_PEAK_TFLOPS = 2500.0


def surrogate_study(train_steps: int = 10000, nsamp: int = 400, log=None):
    """Ensemble data, training, held-out errors against the sphere and the
    Maffettone-Minale model, inference throughput against the boxes' own."""
    from paper_2112_09972_amd import surrogate as S
    log = log or (lambda *a: None)
    case = wl.case_c4(nsteps=(nsamp - 1) * STRIDE + 1)
    run = S.generate(case, nsamp)
    log("ensemble: %d boxes of %d^3, %d lattice steps, %.0f MLUPS" % (case.nbox, case.n, (nsamp - 1) * STRIDE,
                                                                     run.mlups))
    ws = S.make_windows(run)
    tr, va = S.split_by_box(ws)
    res = S.train(tr, steps=train_steps)
    log("trained %d steps in %.1f s" % (res.steps, res.seconds))
    val = S.predict_with_fallback(res.net, va.windows, radius=case.radius, n=case.n)
    allw = S.predict_with_fallback(res.net, ws.windows, radius=case.radius, n=case.n)
    mm = S.mm_shapes(run)
    t_inf = S.inference_seconds(res.net, windows=np.resize(va.windows, (8192, va.windows.shape[1])))
    lbm_rate = run.lattice_updates / run.seconds
    f = float(allw.fallback.mean())
    replay_lups = (S.WINDOW - 1) * STRIDE * case.n ** 3
    per_sample = t_inf / 8192 + f * replay_lups / lbm_rate
    flops = 2.0 * 8192 * (576 * 512 + 2 * 512 * 512 + 512 * 3)
    achieved = flops / t_inf / 1e12
    e = S.errors(val.axes, va.targets)
    out = {
        "workload": case.name, "boxes": case.nbox, "box": case.n, "radius": case.radius,
        "lattice_steps": (nsamp - 1) * STRIDE, "ensemble_mlups": round(run.mlups, 1),
        "ensemble_hbm_frac": round(run.mlups * 1e6 * 304 / (HBM_PEAK_GBS * 1e9), 4),
        "ensemble_launch": {"tile_rows": run.launch[0], "zchunk": run.launch[1], "tile_waves": run.launch[2]},
        "windows": {"train": int(len(tr.targets)), "held_out": int(len(va.targets)), "samples": 64, "stride": STRIDE},
        "train": {"steps": res.steps, "batch": 256, "seconds": round(res.seconds, 2), "augment": "48 cubic maps"},
        "lbm_samples_per_s": round(run.lbm_samples_per_s, 1),
        "inference_batch": 8192, "inference_ms": round(t_inf * 1e3, 4),
        "fallback_threshold_D": 0.5, "fallback_fraction": f,
        "samples_per_s": round(1.0 / per_sample, 1),
        "speedup_vs_lbm": round(1.0 / per_sample / run.lbm_samples_per_s, 1),
        "semi_axis_rel_err": {k: round(v, 5) for k, v in e.items()},
        "within_5pct": bool(e["max"] <= 0.05),
        "baselines": {"sphere": {k: round(v, 5) for k, v in S.errors(np.ones_like(va.targets), va.targets).items()},
                      "maffettone_minale": {k: round(v, 5) for k, v in S.errors(mm[va.box, va.k], va.targets).items()}},
        "roofline": {"bound": "mfma", "kernel": "inference batch (k_forward: the four layers in one launch)",
                     "achieved": round(achieved, 1), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 4), "flops_per_batch": flops},
    }
    res.net.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400, help="timed samples of 50 lattice steps")
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", type=str, default="", help="tile_rows,zchunk[,tile_waves]")
    ap.add_argument("--workload", choices=["c2", "c3"], default="c2",
                    help="c2: the headline 128^3 FP32 box (default); c3: the 256^3 precision study")
    ap.add_argument("--c3-steps", type=int, default=10000)
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate comparison")
    ap.add_argument("--surrogate-train-steps", type=int, default=10000)
    ap.add_argument("--copy-reference", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (HBM counter calibration)")
    ap.add_argument("--format-steps", type=int, default=0,
                    help="only run this many steps of the droplet box in each of --formats, default launch "
                         "(for per-kernel counter runs)")
    ap.add_argument("--format-box", type=int, default=128, help="box of --format-steps: 128 (OU seed 2) or 256 "
                    "(OU seed 3)")
    ap.add_argument("--formats", type=str, default="f32,f64", help="storage formats of --format-steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the hot path on a single MI355X "
              "(sharding over several GPUs is designed but not built); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_reference:
        n = 1 << 28  # 2^28 FP32 = 1 GiB
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes_read": 4 * n, "copy_reference_bytes_written": 4 * n, "launches": 5}))
        return
    import paper_2112_09972_amd as sc
    global wl
    from paper_2112_09972_amd import workloads as wl
    if args.workload == "c3":
        precision_study(sc, args.c3_steps)
        return
    if args.format_steps > 0:
        if args.format_box == 256:
            case = wl.case_c3(nsteps=args.format_steps + 1)
        else:
            case = wl.case_c2(nsteps=args.format_steps + 1)
        tab = case.tables[0]
        for prec in args.formats.split(","):
            lat = sc.Lattice(case.n, case.n, case.n, bc="ghost", prec=prec, table_len=args.format_steps,
                             g_ab=wl.G_AB, rho_b=case.rho_b, mach_max=wl.MACH_MAX)
            lat.init_droplet(lat.xc, case.radius, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tab[0])
            lat.set_gradient_table(tab[:args.format_steps], 0)
            lat.step(args.format_steps)
            lat.synchronize()
            print(json.dumps({"format": prec, "steps": args.format_steps, "launch": lat.get_launch()}), flush=True)
            lat.close()
        return

    K, W = args.steps, args.warmup
    total_steps = (K + W) * STRIDE
    case = wl.case_c2(nsteps=total_steps + 1)
    tab = case.tables[0]
    lat = sc.Lattice(case.n, case.n, case.n, bc="ghost", prec=case.prec, table_len=total_steps, tau=(1.0, 1.0),
                     g_ab=wl.G_AB, rho_b=case.rho_b, mach_max=wl.MACH_MAX)
    if args.launch:
        lat.set_launch(*(int(v) for v in args.launch.split(",")))
    lat.init_droplet(lat.xc, case.radius, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tab[0])
    lat.set_gradient_table(tab[:total_steps], 0)
    m0, _ = lat.totals()
    moments = torch.zeros((K + W, 10), dtype=torch.float64, device=lat.device)

    for k in range(W):
        lat.step(STRIDE)
        lat.droplet_moments(moments[k])
    lat.synchronize()
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    t0 = time.perf_counter()
    for k in range(K):
        ev[k][0].record(lat.stream)
        lat.step(STRIDE)
        ev[k][1].record(lat.stream)
        lat.droplet_moments(moments[W + k])
    lat.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    step_ms = sum(a.elapsed_time(b) for a, b in ev) / (K * STRIDE)
    m1, _ = lat.totals()
    mom = moments.cpu().numpy()
    axes = np.array([sc.sclbm_droplet_from_moments(mom[i], lat.xc)["semi_axes"] for i in range(K + W)])
    ca = np.array([wl.capillary(tab[i * STRIDE], case.radius) for i in range(K + W)])

    nodes = case.n ** 3
    lups = nodes * STRIDE * K
    mlups = lups / elapsed / 1e6
    bytes_per_lup = 2 * 19 * 2 * 4  # both components, 19 populations, read + write, FP32
    achieved = bytes_per_lup * nodes / (step_ms * 1e-3) / 1e9
    ty, zc, wx = lat.get_launch()
    out = {
        "metric": "MLUPS & % HBM peak (2-comp LBM); surrogate vs LBM samples/sec at <=5% err",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(elapsed * 1e3 / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "box": case.n, "radius": case.radius, "lattice_steps_per_step": STRIDE,
                   "lattice_steps_timed": STRIDE * K, "tau": case.tau, "g_ab": wl.G_AB,
                   "storage": "fp32 row-blocked SoA, 2x19 populations", "arithmetic": "fp32 (fp64 totals and moments)", "launch": {"tile_rows": ty, "zchunk": zc, "tile_waves": wx},
                   "ca_max": round(float(ca.max()), 4), "ca_mean": round(float(ca.mean()), 4),
                   "mass_drift_rel": [float(v) for v in ((m1 - m0) / m0)],
                   "semi_axes_last": [round(float(v), 4) for v in axes[-1]]},
        "roofline": {"bound": "hbm", "kernel": "k_step<fp32 storage>", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(case.name),
                     "bytes_per_launch": bytes_per_lup * nodes, "avg_launch_ms": round(step_ms, 5)},
    }
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    log("timed %d x %d lattice steps: %.1f MLUPS" % (K, STRIDE, mlups))
    lat.close()
    del lat, moments
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
        log("cpu baseline: %s" % out["cpu_baseline"]["value"])
    if not args.no_surrogate:
        out["surrogate"] = surrogate_study(args.surrogate_train_steps, log=log)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
