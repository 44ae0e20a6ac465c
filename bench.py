#!/usr/bin/env python3
"""Benchmark of the Chebyshev hot path on one MI355X.

One step = one full pass of the plain FP64 path over the paper-scale sheet:
periodic graphene of 2828 x 1414 sites (3,998,792 rows; 0.5 % vacancies,
Anderson disorder W = 0.1 eV), one random-phase vector,
  * DOS moments: 3000 Chebyshev moments,
  * VAC: 20 time steps (21 time points) of U(-dt) with 40 Bessel terms on two
    states plus 3000 moments per time point,
  * MSD: 20 time steps of the coupled [X, U(dt)] recursion and U(dt) with 40
    Bessel terms plus 3000 moments per time point,
dt = hbar/|t|.  Inputs are resident in HBM before the timed region.

Prints one JSON line: whole-step throughput in Gsite-updates/s, the roofline
of the dominant kernel (the fused moment step) from HIP events recorded by
the library on its stream, and the oracle's CPU rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import kpm_inputs as ki  # noqa: E402
from profile_run import (float_onsite, joint_shape, measured_traffic, moment_kernel_name,  # noqa: E402
                         multi_step, re_launch)

HBM_PEAK_GBS = 8000.0
# VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 vector
# instruction per SIMD every 4 cycles (16 lanes per cycle; the FP64 FMA at this
# rate is the published 78.6 TFLOP/s)
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4
SQ_FILE = os.path.join(ROOT, "profiles", "moment_multistep_fp64_paper_sq.json")
SQ_FILE_R64 = os.path.join(ROOT, "profiles", "moment_multistep_fp32_r64_paper_sq.json")
TRAFFIC_FILE_R64 = os.path.join(ROOT, "profiles", "moment_multistep_fp32_r64_paper_traffic.json")
SQ_FILE_R64A = os.path.join(ROOT, "profiles", "moment_multistep_fp32a_r64_paper_sq.json")
TRAFFIC_FILE_R64A = os.path.join(ROOT, "profiles", "moment_multistep_fp32a_r64_paper_traffic.json")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "moment_step_fp64_paper_traffic.json")
TRAFFIC_FILE_DBL = os.path.join(ROOT, "profiles", "moment_step_doubled_fp64_paper_traffic.json")
TRAFFIC_FILE2 = os.path.join(ROOT, "profiles", "moment_multistep_fp64_paper_traffic.json")
TRAFFIC_FILE2_DBL = os.path.join(ROOT, "profiles", "moment_multistep_doubled_fp64_paper_traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def achieved_gbs(st) -> float:
    """Algorithmic GB/s of the timed moment-step launches: their bytes over
    their summed event time."""
    return st["step_bytes_total"] / max(st["step_ms"], 1e-9) / 1e6


def host_cores() -> int:
    """Host threads this process may use: the CPU affinity set, capped by
    OMP_NUM_THREADS when that is set (the share of the host given to one GPU)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(env))) if env.isdigit() else max(1, n)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, lat_args, n_moments: int):
    """The oracle's moment recursion on a bounded sample of the same sheet, on
    one core and on all the host cores this process may use (the oracle's row
    loops split over threads; its inner products stay serial)."""
    import oracle
    c_ons, c_act = lat_args
    lat = oracle.graphene(p["nx"], p["ny"], "sheet", p["t"], c_ons, c_act)
    phi = ki.random_phase(lat.n, 1, 3000, c_act)[:, 0]
    ups = (n_moments - 1) * lat.n
    rates = {}
    cores = host_cores()
    for th in (1, cores):
        oracle.set_threads(th)
        t0 = time.perf_counter()
        oracle.moments(lat, p["e_scale"], phi, phi, n_moments)
        rates[th] = (ups / (time.perf_counter() - t0) / 1e9, time.perf_counter() - t0)
    sample = (f"{n_moments} Chebyshev moments (phi_2 = 2H~phi_1 - phi_0 plus the inner product) "
              f"on the full {lat.n}-site sheet, one vector, complex128 C oracle")
    return {"value": round(rates[cores][0], 5), "unit": "Gsite-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{sample}, row loops on {cores} threads, {rates[cores][1]:.1f} s",
            "all_cores": {"value": round(rates[cores][0], 5), "cores": cores},
            "one_core": {"value": round(rates[1][0], 5), "cores": 1,
                         "seconds": round(rates[1][1], 1)},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def copy_ceiling_gbs(gib: float = 1.0, reps: int = 10) -> float:
    """Device-to-device copy rate of two buffers beyond every cache (read +
    write bytes per second, best of 3 rounds): the streaming rate this box
    reaches in practice, below the 8 TB/s of the data sheet."""
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = 0.0
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = max(best, 2 * 8 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return round(best, 1)


def valu_record(path: str, step_rows: int, launch: dict, kernel: str):
    """Vector instructions per launch of the dominant kernel from a committed
    SQ-counter record (same kernel source, size, shape and name), or None."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    from profile_run import kernel_sha
    sha = kernel_sha(launch)
    for r in t.get("records", [t]):
        if r.get("kernel_sha") == sha and r.get("step_rows") == step_rows \
                and dict({"steps": 1}, **r.get("launch_shape", {})) == dict({"steps": 1}, **launch) \
                and r.get("kernel", "").split(" ")[0] == kernel:
            return r
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-moments", type=int, default=400,
                    help="moments in the oracle's CPU-baseline sample (0 skips it)")
    ap.add_argument("--workload", default="paper",
                    choices=["paper", "batched", "ragged", "doubled", "ballistic", "learned",
                             "ftm"],
                    help="paper: plain FP64, one vector (default); batched: 64 vectors, "
                         "FP32 states vs FP64; ragged: 32 samples of 1e4..1e6 sites in one "
                         "launch per step; doubled: DOS and MSD moments in the doubling "
                         "form vs the direct form, as moments/s; ballistic: G(E) of a "
                         "pristine 65536x16 ZGNR from the exact trace over one cell; learned: "
                         "moment-to-spectrum network trained on 2000 generated sheets; ftm: "
                         "DOS by KPM vs the Fourier-transform method at equal resolution")
    ap.add_argument("--samples", type=int, default=2000,
                    help="learned workload: generated samples (the last 10 %% are held out)")
    ap.add_argument("--label-vectors", type=int, default=16,
                    help="learned workload: random-phase vectors per sample (the labels' "
                         "stochastic error falls as one over the square root of this)")
    ap.add_argument("--graph-steps", type=int, default=5,
                    help="paper workload: further steps with every moment set replayed from a "
                         "captured hipGraph, reported as their median step time (0 skips them)")
    ap.add_argument("--onsite", default="f64", choices=["f64", "f32"],
                    help="paper workload: the generator's disorder draw (f64, default), or the "
                         "same draw rounded to float32 (f32: the library then stores the on-site "
                         "terms in 4 bytes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1307_0288_amd as kp
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "batched":
        return batched(args)
    if args.workload == "ragged":
        return ragged(args)
    if args.workload == "doubled":
        return doubled(args)
    if args.workload == "ballistic":
        return ballistic(args)
    if args.workload == "learned":
        return learned(args)
    if args.workload == "ftm":
        return ftm(args)

    p = ki.sheet_config("paper")
    n = p["nx"] * p["ny"]
    log(f"inputs: {p['nx']}x{p['ny']} sheet, {n} sites")
    act = ki.vacancy_mask(n, p["vac"], 2000)
    ons = ki.anderson_onsite(n, p["w"], 1000)
    if args.onsite == "f32":
        ons = ons.astype(np.float32).astype(np.float64)
    onsf = float_onsite(ons)
    phi_h = ki.random_phase(n, 1, 3000, act)
    sysg = kp.graphene_system(p["nx"], p["ny"], "sheet", p["t"], ons, act, p["e_scale"], "fp64")
    phi = sysg.upload(phi_h)
    nm, ns, nb, dt = p["n_moments"], p["n_steps"], p["n_bessel"], p["dt_fs"]
    # 200 recursion steps per candidate and round (25 eight-step passes): shapes
    # of the same wavefront count differ by about 2 %, within shorter rounds' noise
    launch = kp.kpm_autotune(sysg, phi, 200)
    log(f"autotuned launch shape: {launch}")

    def step():
        # DOS, VAC and MSD in one call: the DOS set beside the VAC set of t_0,
        # the VAC and MSD sets of each later time step together, every set as
        # two vector planes of one launch sequence
        kp.kpm_dos_vac_msd(sysg, phi, ns, dt, nb, nm)

    for w in range(args.warmup):
        step()
        log(f"warmup {w + 1}/{args.warmup} done")
    kp.kpm_reset_stats(sysg)
    kp.kpm_set_timing(sysg, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = kp.kpm_get_stats(sysg)
    kp.kpm_set_timing(sysg, False)

    value = st["site_updates"] / elapsed / 1e9
    # the dominant kernel: the moment sets run as two vector planes of one
    # launch sequence (the DOS set with the VAC set of t_0, the VAC and MSD
    # sets of each later time step), with half the one-vector grid per plane;
    # they are the widest launches of the step, timed on their own (HIP
    # events around their runs)
    wide = st["wide_rows"] == st["step_rows"] and st["wide_launches"] > 0
    launch_ms = (st["wide_ms"] / st["wide_launches"] if wide
                 else st["step_ms"] / max(st["step_launches"], 1))
    bytes_launch = st["step_bytes"]
    two = multi_step(launch)
    # the two-plane passes' shape (ten steps per pass where the one-vector
    # shape takes eight)
    shape2 = joint_shape(launch, torch.cuda.get_device_properties(0).multi_processor_count)
    bpu = bytes_launch / st["step_rows"] / ((shape2 if wide else launch)["steps"] if two else 1)
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9 if wide else achieved_gbs(st)
    # the VAC and MSD moment sets keep only real parts
    kname = moment_kernel_name("double2", shape2 if wide else launch, False, real=True,
                               onsf=onsf)
    tfile = TRAFFIC_FILE2 if two else TRAFFIC_FILE
    traffic = measured_traffic(tfile, st["step_rows"], shape2, kname if two else "")
    sq = valu_record(SQ_FILE, st["step_rows"], shape2, kname)
    launch_s = launch_ms * 1e-3
    hbm = (traffic if traffic is not None else bytes_launch) / launch_s / 1e9
    roofs = {"hbm": round(hbm / HBM_PEAK_GBS, 4)}
    valu = None
    if sq is not None:
        valu = sq["valu_insts_per_launch"] / launch_s / 1e9
        roofs["alu"] = round(valu / VALU_PEAK_GINST, 4)
    bound = max(roofs, key=roofs.get)
    log("copy ceiling")
    ceiling = copy_ceiling_gbs()

    # the same step with every moment set replayed from its captured graph
    # (captured in the first, untimed step); median step time
    graph = None
    if args.graph_steps > 0:
        kp.kpm_set_graphs(sysg, True)
        step()
        times = []
        for k in range(args.graph_steps):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            log(f"graph-replay step {k + 1}/{args.graph_steps} done")
        kp.kpm_set_graphs(sysg, False)
        med = float(np.median(times))
        graph = {"steps": args.graph_steps, "median_ms_per_step": round(med * 1e3, 3),
                 "gsu": round(st["site_updates"] / args.steps / med / 1e9, 4)}

    cpu = None
    if args.cpu_moments > 0:
        log(f"cpu baseline: oracle, {args.cpu_moments} moments, 1 core and all cores")
        cpu = cpu_baseline(p, (ons, act), args.cpu_moments)

    out = {
        "metric": "Gsite-updates/s (plain FP64 Chebyshev hot path: DOS + VAC + MSD)",
        "value": round(value, 4),
        "unit": "Gsite-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "graphene sheet 2828x1414 sites (3998792), 0.5% vacancies, "
                               "W=0.1 eV" + (" (on-site draw rounded to float32)"
                                             if args.onsite == "f32" else "") +
                               ", 1 random-phase vector, 3000 moments, VAC+MSD 20 steps "
                               "x 40 Bessel terms, dt=hbar/|t|",
                   "n_sites": n, "n_vec": 1, "n_moments": nm, "n_steps": ns,
                   "n_bessel": nb, "onsite_bytes": 4 if onsf else 8,
                   "site_updates_per_step": st["site_updates"] // args.steps},
        "roofline": {"kernel": kname, "bound": bound,
                     **({"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4)} if bound == "hbm" else
                        {"achieved": round(valu, 1), "peak": VALU_PEAK_GINST,
                         "unit": "G VALU wave-instructions/s",
                         "frac": round(valu / VALU_PEAK_GINST, 4),
                         "hbm_algorithmic_gbs": round(achieved, 1)}),
                     "traffic": traffic,
                     "traffic_source": (f"lookup: {os.path.relpath(tfile, ROOT)} (rocprofv3 "
                                        "FETCH_SIZE + WRITE_SIZE, calibrated, same kernel "
                                        "source, size and shape; not measured in this run)")
                                       if traffic is not None else None,
                     "bound_by": {"roof": bound, "frac_of_peak": roofs,
                                  "hbm_gbs": round(hbm, 1),
                                  "hbm_basis": "measured traffic" if traffic is not None
                                               else "algorithmic bytes",
                                  "valu_ginst_per_s": None if valu is None else round(valu, 1),
                                  "valu_peak_ginst_per_s": VALU_PEAK_GINST,
                                  "valu_source": (f"lookup: {os.path.relpath(SQ_FILE, ROOT)} "
                                                  "(rocprofv3 SQ_INSTS_VALU)") if sq else None},
                     "copy_ceiling_gbs": ceiling,
                     "frac_of_copy_ceiling": round(hbm / ceiling, 4),
                     "bytes_per_site_update": round(bpu, 3),
                     "avg_launch_us": round(launch_ms * 1e3, 3),
                     "timing": "HIP events around each run of launches on the library's stream "
                               "(mean over the two-plane launches of the timed steps; direct "
                               "launches, no graph replay)",
                     "launches": st["wide_launches"] if wide else st["step_launches"],
                     "all_moment_launches": {"launches": st["step_launches"],
                                             "avg_launch_us": round(st["step_ms"] * 1e3 / max(
                                                 st["step_launches"], 1), 3),
                                             "algorithmic_gbs": round(achieved_gbs(st), 1)},
                     "launch_shape": launch,
                     "two_plane_shape": shape2},
        "graph_replay": graph,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def doubled(args):
    """Moment doubling for phi_L = phi_R on the paper-scale sheet (FP64, one
    vector): 3000 DOS moments and the 20-step MSD, each in the direct form of
    Alg. 5 and in the doubling form.  Reported as moments/s (moments of one
    vector over the whole sheet per second), separately from the headline."""
    import torch
    import paper_1307_0288_amd as kp
    p = ki.sheet_config("paper")
    n = p["nx"] * p["ny"]
    act = ki.vacancy_mask(n, p["vac"], 2000)
    ons = ki.anderson_onsite(n, p["w"], 1000)
    sysg = kp.graphene_system(p["nx"], p["ny"], "sheet", p["t"], ons, act, p["e_scale"], "fp64")
    phi = sysg.upload(ki.random_phase(n, 1, 3000, act))
    nm, ns, nb, dt = p["n_moments"], p["n_steps"], p["n_bessel"], p["dt_fs"]
    launch = kp.kpm_autotune(sysg, phi, 50)
    launch_dbl = kp.kpm_get_launch_doubled(sysg, 1)
    log(f"autotuned launch shapes: direct {launch}, doubling {launch_dbl}")
    calls = {
        "dos_direct": lambda: kp.kpm_moments(sysg, phi, phi, nm),
        "dos_doubled": lambda: kp.kpm_moments_doubled(sysg, phi, nm),
        "msd_direct": lambda: kp.kpm_msd(sysg, phi, ns, dt, nb, nm),
        "msd_doubled": lambda: kp.kpm_msd_doubled(sysg, phi, ns, dt, nb, nm),
    }
    res, outs = {}, {}
    for name, fn in calls.items():
        for _ in range(args.warmup):
            fn()
        kp.kpm_reset_stats(sysg)
        kp.kpm_set_timing(sysg, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            outs[name] = fn()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / args.steps
        st = kp.kpm_get_stats(sysg)
        kp.kpm_set_timing(sysg, False)
        launch_ms = st["step_ms"] / max(st["step_launches"], 1)
        n_mom = nm * (ns if name.startswith("msd") else 1)
        res[name] = {"ms": round(el * 1e3, 3), "moments_per_s": round(n_mom / el, 1),
                     "step_launch_us": round(launch_ms * 1e3, 3),
                     "step_bytes": st["step_bytes"],
                     "step_gbs": round(achieved_gbs(st), 1)}
        log(f"{name}: {res[name]}")
    n_act = float(np.count_nonzero(act))
    err_dos = float(np.max(np.abs(outs["dos_doubled"] - outs["dos_direct"])) / n_act)
    m_ref = outs["msd_direct"]
    err_msd = float(np.max(np.abs(outs["msd_doubled"] - m_ref)) / np.max(np.abs(m_ref)))
    dd = res["dos_doubled"]
    out = {
        "metric": "moments/s (DOS moments of one vector over the 4M-site sheet, doubling form)",
        "value": dd["moments_per_s"],
        "unit": "moments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dd["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "graphene sheet 2828x1414 sites (3998792), 0.5% vacancies, "
                               "W=0.1 eV, 1 random-phase vector, 3000 moments; MSD 20 steps x "
                               "40 Bessel terms, dt=hbar/|t|",
                   "n_sites": n, "n_moments": nm, "launch_shape": launch,
                   "launch_shape_doubling": launch_dbl},
        "roofline": {"kernel": moment_kernel_name("double2", launch_dbl, True), "bound": "hbm",
                     "achieved": dd["step_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dd["step_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(TRAFFIC_FILE2_DBL if multi_step(launch_dbl)
                                                 else TRAFFIC_FILE_DBL, n, launch_dbl),
                     "bytes_per_launch": dd["step_bytes"],
                     "avg_launch_us": dd["step_launch_us"]},
        "forms": res,
        "max_rel_diff_vs_direct": {"dos": err_dos, "msd": err_msd},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def ballistic(args):
    """Ballistic conductance of the paper's pristine ZGNR (Sec. 5.1): 65536 x 16
    sites (1,048,576), periodic along x.  The trace over all sites is exact
    from the 32 unit vectors of one translation cell (2 sites along x times 16
    chains) times the 32768 cells, so one batch of 32 vectors per Chebyshev
    step gives rho(E) and Delta X^2(E, t) without stochastic error.  One step:
    DOS and MSD moments (doubling form, 1000 moments, 20 time steps of 2 fs,
    45 Bessel terms), then G(E) = (W/L) sigma_E1 (Eq. 51) on 64 energies.
    Reports Gsite-updates/s and the deviation of G from 2 e^2/h on the first
    plateau (0.2 eV <= |E| <= 0.55 eV; the second subband of this 16-chain
    ribbon opens near 0.7 eV)."""
    import torch
    import paper_1307_0288_amd as kp
    nx, ny, nm, ns, dt, nb = 65536, 16, 1000, 20, 2.0, 45
    es = 1.01 * 3 * 2.7
    n = nx * ny
    n_vec = 2 * ny
    sites = np.array([j * nx + i for j in range(ny) for i in (0, 1)], dtype=np.int64)
    phi_h = np.zeros((n, n_vec), dtype=np.complex128)
    phi_h[sites, np.arange(n_vec)] = 1.0
    cells = nx // 2
    sysg = kp.graphene_system(nx, ny, "zgnr", -2.7, None, None, es, "fp64")
    phi = sysg.upload(phi_h)
    del phi_h
    launch = kp.kpm_autotune(sysg, phi, 20)
    log(f"autotuned launch shape (32 vectors): {launch}")
    lx = np.sqrt(3.0) * nx * 0.142 / 2.0
    width = 3.0 * ny * 0.142 / 2.0
    area = lx * width
    en = np.linspace(-3.0, 3.0, 64)

    def step():
        mu = kp.kpm_moments_doubled(sysg, phi, nm).real.sum(axis=0) * cells
        ms = kp.kpm_msd_doubled(sysg, phi, ns, dt, nb, nm).sum(axis=0) * cells
        rho = kp.kpm_kpm_sum(mu, en, es, area)
        rm = kp.kpm_kpm_sum(ms, en, es, area)
        return kp.kpm_conductance(kp.kpm_sigma_e1(rm, dt), kp.kpm_length(rm, rho), width)

    for _ in range(args.warmup):
        step()
    kp.kpm_reset_stats(sysg)
    kp.kpm_set_timing(sysg, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        g = step()
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = kp.kpm_get_stats(sysg)
    kp.kpm_set_timing(sysg, False)
    launch_ms = st["step_ms"] / max(st["step_launches"], 1)
    achieved = achieved_gbs(st)
    plateau = (np.abs(en) >= 0.2) & (np.abs(en) <= 0.55)
    k_mid = ns // 2
    dev = float(np.max(np.abs(g[k_mid:-1, plateau] - 2.0)))
    out = {
        "metric": "Gsite-updates/s (ballistic G(E) pipeline, exact cell trace, 32 vectors)",
        "value": round(st["site_updates"] / elapsed / 1e9, 4),
        "unit": "Gsite-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "pristine ZGNR 65536x16 sites (1048576), periodic along x, exact "
                               "trace from 32 cell unit vectors, 1000 moments (doubling form), "
                               "MSD 20 steps x 2 fs x 45 Bessel terms, G(E) on 64 energies",
                   "n_sites": n, "n_vec": n_vec, "launch_shape": launch},
        "roofline": {"kernel": moment_kernel_name("double2", launch, True, n_vec), "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "avg_launch_us": round(launch_ms * 1e3, 3)},
        "first_plateau_max_abs_dev_from_2": dev,
        "g_at_t_mid": {f"{e:.3f}": round(float(v), 5) for e, v in zip(en, g[k_mid])},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def learned(args):
    """Learned moment-to-spectrum reconstruction (not the paper's method).

    Data: `--samples` periodic sheets of 632 x 316 sites (199,712), vacancy
    fraction in [0, 2 %), Anderson W in [0, 2) eV, `--label-vectors` random-phase
    vectors each (16 by default),
    FP32 states, E_s = 1.01 (3|t| + 1 eV) for all; per sample 4000 DOS moments
    and 4000 MSD moments at t* = 10 fs (10 steps of 1 fs, 40 Bessel terms), both
    in the doubling form, in ragged batches of 20 samples.  Targets: Jackson KPM
    sums of all 4000 moments (DOS and sigma_E2(t*), 1024 energies in
    [-7.5, 7.5] eV); features: the first 256 moments of each.  The network
    (513 -> 1024 -> 1024 -> 2048, tanh) trains with Adam on 90 % of the samples;
    on the held-out 10 % its spectra are compared with plain 4000-moment KPM,
    and plain KPM is kept wherever the learned error exceeds 1e-3.  Reported
    side by side, in the same norm against the 4000-moment spectra: the
    learned error, the error of plain Jackson KPM from the same 256 moments
    the network reads (Eq. 29-31, 35), and the labels' own stochastic error."""
    import torch
    import paper_1307_0288_amd as kp
    nx, ny = 632, 316
    n = nx * ny
    r_vec, nm, n_in, nc, dt, nb = args.label_vectors, 4000, 256, 10, 1.0, 40
    if r_vec < 2 or r_vec & (r_vec - 1) or r_vec > 64:
        raise SystemExit("--label-vectors must be a power of two in 2 .. 64")
    es = 1.01 * (3 * 2.7 + 1.0)
    t_star = nc * dt
    en = np.linspace(-7.5, 7.5, 1024)
    per_batch = 20
    specs = ki.learned_sample_specs(args.samples, 100000)
    mus, cs = [], []
    t_gen = 0.0

    def inputs(sp):
        act = ki.vacancy_mask(n, sp["vac"], sp["vac_seed"])
        ons = ki.anderson_onsite(n, sp["w"], sp["onsite_seed"])
        return (dict(nx=nx, ny=ny, geometry="sheet", onsite=ons, active=act, e_scale=es),
                ki.random_phase(n, r_vec, sp["vec_seed"], act))

    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(max(1, host_cores()))

    def submit(b0):          # the host inputs of one batch, drawn on every core
        return [pool.submit(inputs, sp) for sp in specs[b0:b0 + per_batch]]

    nxt = submit(0)
    for b0 in range(0, len(specs), per_batch):
        group = [f.result() for f in nxt]
        nxt = submit(b0 + per_batch)              # one batch ahead, while this one runs
        samples = [g[0] for g in group]
        phis = [g[1] for g in group]
        del group
        sysg = kp.graphene_batch(samples, "fp32")
        d = sysg.upload(np.concatenate(phis))
        del phis
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu = kp.kpm_moments_doubled(sysg, d, nm).real
        y_state = kp.kpm_xu_state(sysg, d, nc, dt, nb)
        cm = kp.kpm_moments_doubled(sysg, y_state, nm).real
        torch.cuda.synchronize()
        t_gen += time.perf_counter() - t0
        mus.append(mu)
        cs.append(cm)
        sysg.close()
        del d, y_state
        log(f"generated {min(b0 + per_batch, len(specs))}/{len(specs)} samples "
            f"({t_gen:.1f} s GPU)")
    pool.shutdown()
    mu = np.concatenate(mus)
    cm = np.concatenate(cs)
    lx = np.sqrt(3.0) * nx * 0.142 / 2.0
    area = lx * 3.0 * ny * 0.142 / 2.0
    x = kp.kpm_learned_features(mu, cm, n_in)
    y = kp.kpm_learned_targets(mu, cm, en, es, area, t_star)
    n_train = int(0.9 * len(specs))
    sizes = [x.shape[1], 1024, 1024, y.shape[1]]
    batch = 100
    net = kp.MLP(sizes, max_batch=max(batch, len(specs) - n_train))
    net.set_params(np.concatenate([np.concatenate([w.ravel(), b.ravel()])
                                   for w, b in ki.mlp_init(sizes, 77)]).astype(np.float32))
    xt = torch.from_numpy(x[:n_train]).cuda()
    yt = torch.from_numpy(y[:n_train]).cuda()
    order = np.arange(n_train)
    rng = np.random.default_rng(0)
    epochs = 300
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    loss = float("nan")
    for ep in range(epochs):
        rng.shuffle(order)
        lr = 1e-3 * (0.5 * (1 + np.cos(np.pi * ep / epochs)))
        last = (n_train - batch) // batch * batch
        for q in range(0, n_train - batch + 1, batch):
            idx = torch.from_numpy(order[q:q + batch]).cuda()
            out_loss = net.train_step(xt[idx].contiguous(), yt[idx].contiguous(), float(lr),
                                      want_loss=(q == last))
            loss = out_loss if out_loss is not None else loss
            steps += 1
        if ep % 50 == 0 or ep == epochs - 1:
            log(f"epoch {ep}: loss {loss:.3e}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    xh = torch.from_numpy(x[n_train:]).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = net.forward(xh)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    pred = pred.cpu().numpy()
    yh = y[n_train:]
    k = en.size
    e_dos = np.max(np.abs(pred[:, :k] - yh[:, :k]), axis=1) / np.max(np.abs(yh[:, :k]), axis=1)
    e_sig = np.max(np.abs(pred[:, k:] - yh[:, k:]), axis=1) / np.max(np.abs(yh[:, k:]), axis=1)
    accept = (e_dos <= 1e-3) & (e_sig <= 1e-3)
    # stochastic spread of plain KPM itself on the same samples: the targets of
    # the two disjoint halves of the vectors differ by about twice the error of
    # the target from all of them
    h = r_vec // 2
    ya = kp.kpm_learned_targets(mu[n_train:, :h], cm[n_train:, :h], en, es, area, t_star)
    yb = kp.kpm_learned_targets(mu[n_train:, h:], cm[n_train:, h:], en, es, area, t_star)
    s_dos = 0.5 * np.max(np.abs(ya[:, :k] - yb[:, :k]), axis=1) / np.max(np.abs(yh[:, :k]), axis=1)
    s_sig = 0.5 * np.max(np.abs(ya[:, k:] - yb[:, k:]), axis=1) / np.max(np.abs(yh[:, k:]), axis=1)
    # what the network replaces: plain Jackson KPM from the same 256 moments
    y256 = kp.kpm_learned_targets(mu[n_train:, :, :n_in], cm[n_train:, :, :n_in], en, es, area,
                                  t_star)
    k_dos = np.max(np.abs(y256[:, :k] - yh[:, :k]), axis=1) / np.max(np.abs(yh[:, :k]), axis=1)
    k_sig = np.max(np.abs(y256[:, k:] - yh[:, k:]), axis=1) / np.max(np.abs(yh[:, k:]), axis=1)

    def stats(e):
        return {"median": float(np.median(e)), "p90": float(np.quantile(e, 0.9)),
                "max": float(np.max(e))}
    # cost per sample: the learned path needs the first 256 moments of each set,
    # plain KPM all 4000; both need the [X, U(t*)] state
    flops_step = 6.0 * batch * sum(sizes[l] * sizes[l + 1] for l in range(len(sizes) - 1))
    gen_per_sample = t_gen / len(specs)
    su_state = 2 * (nb - 1) * nc + (nb - 1) * (nc - 1)            # coupled steps count twice
    frac_learned = (2 * (n_in // 2) + su_state) / (2 * (nm // 2) + su_state)
    out = {
        "metric": "samples/s (learned sigma(E)/DOS reconstruction from 256 moments with plain "
                  "4000-moment KPM as fallback above 1e-3 error) and the learned error",
        # the path as deployed: learned inputs for every sample, plus plain KPM for
        # every held-out sample whose learned error exceeds the bar
        "value": round(1.0 / (gen_per_sample * (frac_learned + float(np.mean(~accept)))), 3),
        "unit": "samples/s",
        "n_gpus": 1, "steps": epochs, "warmup": 0,
        "ms_per_step": round(t_train / steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(specs)} sheets 632x316 (199712 sites), vacancies 0-2%, "
                               f"W 0-2 eV, {r_vec} vectors, FP32 states; 4000 DOS + 4000 MSD(t*=10 fs) "
                               "moments; MLP 513-1024-1024-2048 on 256 moments, 1024 energies",
                   "train": n_train, "held_out": len(specs) - n_train},
        "plain_kpm_samples_per_s": round(1.0 / gen_per_sample, 3),
        "learned_only_samples_per_s": round(1.0 / (gen_per_sample * frac_learned), 3),
        "error_vs_4000_moment_kpm": {
            "norm": "per held-out sample max|dy| / max|y| over the 1024 energies",
            "learned": {"dos": stats(e_dos), "sigma_e2": stats(e_sig)},
            "plain_kpm_256_moments": {"dos": stats(k_dos), "sigma_e2": stats(k_sig)},
            "label_noise": {"dos": stats(s_dos), "sigma_e2": stats(s_sig),
                            "estimate": f"half the difference of the targets of vectors "
                                        f"0..{h - 1} and {h}..{r_vec - 1}, same norm"}},
        "learned_beats_kpm_256": {
            "dos_fraction": float(np.mean(e_dos < k_dos)),
            "sigma_fraction": float(np.mean(e_sig < k_sig)),
            "dos_median_ratio": float(np.median(e_dos / k_dos)),
            "sigma_median_ratio": float(np.median(e_sig / k_sig))},
        "label_vectors": r_vec,
        "gate_1e-3_reachable": bool(np.median(s_dos) <= 1e-3),
        "label_vectors_for_1e-3_dos": int(np.ceil(r_vec * (np.median(s_dos) / 1e-3) ** 2)),
        "accepted_at_1e-3": int(accept.sum()), "fallback_to_kpm": int((~accept).sum()),
        "train_seconds": round(t_train, 2), "train_steps": steps,
        "train_tflops": round(flops_step * steps / t_train / 1e12, 3),
        "inference_ms_held_out": round(t_inf * 1e3, 3),
        "roofline": {"kernel": "k_gemm (training step, all layers)", "bound": "mfma",
                     "achieved": round(flops_step * steps / t_train / 1e12, 3),
                     "peak": 157.3, "unit": "TFLOP/s",
                     "frac": round(flops_step * steps / t_train / 1e12 / 157.3, 5),
                     "traffic": None},
        "final_train_loss": loss,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def ftm(args):
    """DOS of the paper-scale sheet by KPM and by the FTM at the same energy
    resolution (Sec. 4.2): KPM with N_m = 3000 moments (resolution
    pi Delta E / N_m) against the FTM with 2 N_f + 1 = 955 Fourier moments
    (resolution Delta E / (2 N_f + 1)) at dtau = pi hbar / E_s, 20 Bessel terms
    per step; KPM also in the doubling form.  FP64, one vector.  Reports both
    times, their ratio (the paper estimates 20 / pi = 6.4 in Chebyshev steps)
    and the difference of the two DOS curves."""
    import torch
    import paper_1307_0288_amd as kp
    p = ki.sheet_config("paper")
    n = p["nx"] * p["ny"]
    act = ki.vacancy_mask(n, p["vac"], 2000)
    ons = ki.anderson_onsite(n, p["w"], 1000)
    sysg = kp.graphene_system(p["nx"], p["ny"], "sheet", p["t"], ons, act, p["e_scale"], "fp64")
    phi = sysg.upload(ki.random_phase(n, 1, 3000, act))
    kp.kpm_autotune(sysg, phi, 50)
    es, nm = p["e_scale"], p["n_moments"]
    nf = int(round((nm / np.pi - 1) / 2))
    hbar = 0.6582119569
    dtau, npb = np.pi * hbar / es, 20
    en = np.linspace(-0.9 * es, 0.9 * es, 2001)
    calls = {
        "kpm": lambda: kp.kpm_moments(sysg, phi, phi, nm),
        "kpm_doubled": lambda: kp.kpm_moments_doubled(sysg, phi, nm),
        "ftm": lambda: kp.kpm_fourier_moments(sysg, phi, phi, nf, dtau, npb),
    }
    times, outs = {}, {}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(args.steps, 1)):
            t0 = time.perf_counter()
            outs[name] = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        times[name] = min(ts)
        log(f"{name}: {times[name] * 1e3:.1f} ms")
    rho_kpm = kp.kpm_kpm_sum(outs["kpm"][0].real, en, es, sysg.area_nm2)
    rho_ftm = kp.kpm_ftm_sum(outs["ftm"][0], en, dtau, sysg.area_nm2)
    diff = float(np.sqrt(np.mean((rho_ftm - rho_kpm) ** 2)) / np.sqrt(np.mean(rho_kpm ** 2)))
    out = {
        "metric": "DOS time at equal energy resolution: FTM / KPM (Sec. 4.2)",
        "value": round(times["ftm"] / times["kpm"], 3),
        "unit": "ratio",
        "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(times["kpm"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "graphene sheet 2828x1414 sites (3998792), 0.5% vacancies, W=0.1 eV, "
                               f"1 vector; KPM 3000 moments vs FTM {2 * nf + 1} Fourier moments, "
                               "dtau = pi hbar / E_s, 20 Bessel terms",
                   "kpm_resolution_ev": round(np.pi * 2 * es / nm, 5),
                   "ftm_resolution_ev": round(2 * es / (2 * nf + 1), 5)},
        "times_ms": {k: round(v * 1e3, 3) for k, v in times.items()},
        "paper_estimate": round(20 / np.pi, 2),
        "ftm_over_doubled_kpm": round(times["ftm"] / times["kpm_doubled"], 3),
        "dos_rel_rms_difference": diff,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def _golden_vector(seed, ons, act, phi):
    """The oracle's stored moments of the paper-scale sheet's vector of this
    seed (tests/golden/paper_sheet_oracle.npz for seed 3000,
    paper_sheet_oracle_seed<S>.npz for others; written by a script that calls
    only the oracle), when they are stored for these inputs; else None."""
    import hashlib
    name = "paper_sheet_oracle.npz" if seed == 3000 else f"paper_sheet_oracle_seed{seed}.npz"
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    if not {"dos_re", "vac", "msd"} <= set(z.files):
        return None
    meta = json.loads(bytes(z["meta"]).decode())
    h = hashlib.sha256()
    for a in (ons, act, phi):
        h.update(np.ascontiguousarray(a).tobytes())
    if meta.get("input_sha256") != h.hexdigest():
        return None
    return dict(dos=z["dos_re"], vac=z["vac"], msd=z["msd"])


def _spectra(kp, dos, vac, msd, en, es, area, dt):
    """DOS (Eq. 29) and sigma_GK / sigma_E1 / sigma_E2 (Eq. 6, 9, 11) at the
    energies en and every time point, from moments [3000], [21][3000] x 2,
    through the library's sums."""
    rho_v = kp.kpm_kpm_sum(vac, en, es, area)
    rho_m = kp.kpm_kpm_sum(msd, en, es, area)
    return dict(dos=kp.kpm_kpm_sum(dos[None, :], en, es, area),
                gk=kp.kpm_sigma_gk(rho_v, dt), e1=kp.kpm_sigma_e1(rho_m, dt),
                e2=kp.kpm_sigma_e2(rho_m, dt))


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def batched(args):
    """64 random-phase vectors on the paper-scale sheet, the whole hot path per
    step (DOS moments, VAC and MSD over 20 time steps, 3000 moments each), with
    FP32 states (FP64 arithmetic, inner products and moments) and with FP64
    states, next to plain FP64 with one vector on the same GPU.

    sigma(E) error per result, max over the 2048 energies and 21 times of
    |d sigma| / max |sigma_ref|: the DOS (Eq. 29), sigma_GK (Eq. 6), sigma_E1
    (Eq. 9) and sigma_E2 (Eq. 11) of the FP32 run against the FP64 run (both
    averaged over the 64 vectors), and of vector 0 of each run (seed 3000)
    against the oracle's stored moments of that vector, all through the same
    sums (Eq. 29-31, Jackson kernel).
    """
    import torch
    import paper_1307_0288_amd as kp
    p = ki.sheet_config("paper")
    n = p["nx"] * p["ny"]
    r = 64
    log(f"batched inputs: {n} sites x {r} vectors")
    act = ki.vacancy_mask(n, p["vac"], 2000)
    ons = ki.anderson_onsite(n, p["w"], 1000)
    phi_h = ki.random_phase(n, r, 3000, act)
    nm, ns, nb, dt, es = p["n_moments"], p["n_steps"], p["n_bessel"], p["dt_fs"], p["e_scale"]
    # vectors 0 .. 3 whose oracle moments are stored
    golds = {q: g for q in range(4)
             if (g := _golden_vector(3000 + q, ons, act, phi_h[:, q])) is not None}
    en = np.linspace(-0.95 * es, 0.95 * es, 2048)
    steps = max(1, args.steps)
    res, spec, spec0 = {}, {}, {}
    for prec in ("fp64", "fp32", "fp32_arith"):
        sysg = kp.graphene_system(p["nx"], p["ny"], "sheet", p["t"], ons, act, es, prec)
        area = sysg.area_nm2
        phi = sysg.upload(phi_h)
        launch = kp.kpm_autotune(sysg, phi, 8)
        log(f"{prec} autotuned launch shape: {launch}")
        kp.kpm_moments(sysg, phi, phi, 64)                      # warm-up
        kp.kpm_vac(sysg, phi, 1, dt, nb, 64)
        kp.kpm_reset_stats(sysg)
        kp.kpm_set_timing(sysg, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            dos = kp.kpm_moments(sysg, phi, phi, nm)
            vac = kp.kpm_vac(sysg, phi, ns, dt, nb, nm)
            msd = kp.kpm_msd(sysg, phi, ns, dt, nb, nm)
            log(f"{prec} step {k + 1}/{steps} done")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        st = kp.kpm_get_stats(sysg)
        kp.kpm_set_timing(sysg, False)
        launch_ms = st["step_ms"] / max(st["step_launches"], 1)
        res[prec] = dict(gsu=st["site_updates"] / elapsed / 1e9, ms=elapsed / steps * 1e3,
                         launch=launch, launch_us=launch_ms * 1e3,
                         bytes_launch=st["step_bytes"], rows=st["step_rows"],
                         site_updates=st["site_updates"] // steps)
        log(f"{prec}: {res[prec]['gsu']:.1f} Gsite-updates/s")
        spec[prec] = _spectra(kp, dos.real.mean(axis=0), vac.mean(axis=0), msd.mean(axis=0),
                              en, es, area, dt)
        spec0[prec] = {q: _spectra(kp, dos[q].real, vac[q], msd[q], en, es, area, dt)
                       for q in golds}
        sysg.close()
        del phi
        torch.cuda.empty_cache()
    # plain FP64, one vector, on the same GPU (the default workload's step)
    sysg = kp.graphene_system(p["nx"], p["ny"], "sheet", p["t"], ons, act, es, "fp64")
    phi1 = sysg.upload(phi_h[:, :1])
    kp.kpm_autotune(sysg, phi1, 50)
    kp.kpm_moments(sysg, phi1, phi1, 64)
    kp.kpm_reset_stats(sysg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kp.kpm_dos_vac_msd(sysg, phi1, ns, dt, nb, nm)
    torch.cuda.synchronize()
    plain = kp.kpm_get_stats(sysg)["site_updates"] / (time.perf_counter() - t0) / 1e9
    sysg.close()
    log(f"plain fp64, one vector: {plain:.1f} Gsite-updates/s")

    f32s = ("fp32", "fp32_arith")
    err32 = {q: {k: _rel(spec[q][k], spec["fp64"][k]) for k in spec["fp64"]} for q in f32s}
    err_or = None
    if golds:
        refs = {q: _spectra(kp, g["dos"], g["vac"], g["msd"], en, es, area, dt)
                for q, g in golds.items()}
        # per result, the worst of the checked vectors
        err_or = {prec: {k: max(_rel(spec0[prec][q][k], refs[q][k]) for q in refs)
                         for k in next(iter(refs.values()))} for prec in spec0}
    worst = {q: max(list(err32[q].values()) +
                    ([] if err_or is None else list(err_or[q].values()))) for q in f32s}
    # the reported FP32 form: the faster one whose sigma(E) error is within the bar
    ok = [q for q in f32s if worst[q] <= 1e-3]
    best = max(ok or list(f32s), key=lambda q: res[q]["gsu"])
    f32 = res[best]
    kname = moment_kernel_name("float2", re_launch(f32["launch"], best, r), False, real=True,
                               onsf=False, n_vec=r, arith32=best == "fp32_arith")
    tfile, sfile = ((TRAFFIC_FILE_R64, SQ_FILE_R64) if best == "fp32" else
                    (TRAFFIC_FILE_R64A, SQ_FILE_R64A))
    achieved = f32["bytes_launch"] / (f32["launch_us"] * 1e-6) / 1e9
    launch_s = f32["launch_us"] * 1e-6
    traffic = measured_traffic(tfile, f32["rows"], f32["launch"], kname)
    sq = valu_record(sfile, f32["rows"], f32["launch"], kname)
    hbm = (traffic if traffic is not None else f32["bytes_launch"]) / launch_s / 1e9
    valu = None if sq is None else sq["valu_insts_per_launch"] / launch_s / 1e9
    # the roof closer to its peak: HBM (measured traffic when known) or VALU issue
    bound = "alu" if valu is not None and valu / VALU_PEAK_GINST > hbm / HBM_PEAK_GBS else "hbm"
    out = {
        "metric": "Gsite-updates/s (batched Chebyshev hot path: DOS + VAC + MSD, 64 vectors, "
                  "FP32 states)",
        "fp32_form": best,
        "value": round(f32["gsu"], 3), "unit": "Gsite-updates/s", "n_gpus": 1,
        "steps": steps, "warmup": 0, "ms_per_step": round(f32["ms"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ("f32-states-and-strip-arithmetic/f64-dots" if best == "fp32_arith"
                  else "f32-states/f64-arithmetic-and-dots"), "data": "synthetic",
        "config": {"workload": "graphene sheet 2828x1414 sites (3998792), 0.5% vacancies, "
                               "W=0.1 eV, 64 random-phase vectors (seeds 3000..3063), 3000 "
                               "moments, VAC+MSD 20 steps x 40 Bessel terms, dt=hbar/|t|",
                   "n_sites": n, "n_vec": r, "site_updates_per_step": f32["site_updates"]},
        "fp64_batched_gsu": round(res["fp64"]["gsu"], 3),
        "fp32_states_gsu": round(res["fp32"]["gsu"], 3),
        "fp32_arith_gsu": round(res["fp32_arith"]["gsu"], 3),
        "plain_fp64_one_vector_gsu": round(plain, 3),
        "moment_launch_us": {q: round(v["launch_us"], 2) for q, v in res.items()},
        "speedup_fp32_batched_vs_plain_fp64": round(f32["gsu"] / plain, 3),
        "speedup_fp32_vs_fp64_batched": round(f32["gsu"] / res["fp64"]["gsu"], 3),
        "sigma_rel_err_fp32_vs_fp64": err32,
        "sigma_rel_err_vs_oracle": err_or,
        "sigma_error_norm": "max over 2048 energies in [-0.95 E_s, 0.95 E_s] and 21 times of "
                            "|d sigma| / max |sigma_ref|; vs_oracle: each of the vectors in "
                            "oracle_vectors against the oracle's stored moments of that vector "
                            "(the worst of them)",
        "oracle_vectors": sorted(golds),
        "sigma_bar": 1e-3, "sigma_within_bar": {q: bool(worst[q] <= 1e-3) for q in f32s},
        "roofline": {"kernel": kname, "bound": bound,
                     **({"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4)} if bound == "hbm" else
                        {"achieved": round(valu, 1), "peak": VALU_PEAK_GINST,
                         "unit": "G VALU wave-instructions/s",
                         "frac": round(valu / VALU_PEAK_GINST, 4),
                         "hbm_algorithmic_gbs": round(achieved, 1)}),
                     "traffic": traffic,
                     "traffic_source": (f"lookup: {os.path.relpath(tfile, ROOT)} "
                                        "(rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated, same "
                                        "kernel source, size and shape; not measured in this run)")
                                       if traffic is not None else None,
                     "bound_by": {"hbm_gbs": round(hbm, 1),
                                  "hbm_basis": "measured traffic" if traffic is not None
                                               else "algorithmic bytes",
                                  "frac_of_peak": {"hbm": round(hbm / HBM_PEAK_GBS, 4),
                                                   **({} if valu is None else
                                                      {"alu": round(valu / VALU_PEAK_GINST, 4)})},
                                  "valu_ginst_per_s": None if valu is None else round(valu, 1),
                                  "valu_source": (f"lookup: {os.path.relpath(sfile, ROOT)}"
                                                  " (rocprofv3 SQ_INSTS_VALU)") if sq else None},
                     "bytes_per_launch": f32["bytes_launch"],
                     "avg_launch_us": round(f32["launch_us"], 2),
                     "launch_shape": f32["launch"]},
        "launch_shapes": {k: v["launch"] for k, v in res.items()},
    }
    print(json.dumps(out), flush=True)


def ragged(args):
    """32 independent samples (AGNR, ZGNR, sheets of 1e4..1e6 sites, Anderson W in
    {0.5, 1, 2} eV), 8 random vectors each, 1000 moments per sample, all samples
    advanced together by every launch (eight recursion steps per launch in the
    marching strips when the autotuner keeps them); direct launches vs hipGraph
    replay, FP64 states, FP32 states and FP32 strip arithmetic."""
    import torch
    import paper_1307_0288_amd as kp
    cfg = ki.sheet_config("ragged")
    specs = ki.ragged_specs(cfg["count"], cfg["seed"], cfg["n_min"], cfg["n_max"],
                            cfg["w_min"], cfg["w_max"])
    r, nm = cfg["n_vec"], cfg["n_moments"]
    samples, phis = [], []
    for s, sp in enumerate(specs):
        n = sp["nx"] * sp["ny"]
        ons = ki.anderson_onsite(n, sp["w"], 1000 + s)
        samples.append(dict(nx=sp["nx"], ny=sp["ny"], geometry=sp["geometry"], onsite=ons,
                            e_scale=1.01 * (3 * 2.7 + sp["w"] / 2)))
        phis.append(ki.random_phase(n, r, 3000 + 100 * s))
    phi_h = np.concatenate(phis)
    total = phi_h.shape[0]
    log(f"ragged inputs: {len(specs)} samples, {total} sites, {r} vectors")
    res, rates = {}, {}
    for prec in ("fp64", "fp32", "fp32_arith"):
        sysg = kp.graphene_batch(samples, prec)
        phi = sysg.upload(phi_h)
        launch = kp.kpm_autotune(sysg, phi, 20)
        log(f"{prec} autotuned launch shape: {launch}")
        # per-launch rate of the moment passes (HIP events, direct launches)
        kp.kpm_moments(sysg, phi, phi, nm)
        kp.kpm_reset_stats(sysg)
        kp.kpm_set_timing(sysg, True)
        kp.kpm_moments(sysg, phi, phi, nm)
        st = kp.kpm_get_stats(sysg)
        kp.kpm_set_timing(sysg, False)
        us = st["step_ms"] / max(st["step_launches"], 1) * 1e3
        rates[prec] = {"avg_launch_us": round(us, 3), "launches": st["step_launches"],
                       "bytes_per_launch": st["step_bytes"],
                       "algorithmic_gbs": round(achieved_gbs(st), 1),
                       "frac_of_8tbs": round(achieved_gbs(st) / HBM_PEAK_GBS, 4)}
        for graphs in (False, True):
            kp.kpm_set_graphs(sysg, graphs)
            kp.kpm_moments(sysg, phi, phi, nm)                # warm-up (and capture)
            torch.cuda.synchronize()
            times = []
            for k in range(max(args.steps, 1)):
                t0 = time.perf_counter()
                kp.kpm_moments(sysg, phi, phi, nm)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            ups = (nm - 1) * total * r
            res[f"{prec}_{'graph' if graphs else 'direct'}"] = dict(
                seconds=min(times), gsu=ups / min(times) / 1e9, launch=launch)
            log(f"{prec} graphs={graphs}: {min(times) * 1e3:.1f} ms, "
                f"{ups / min(times) / 1e9:.1f} Gsite-updates/s")
        sysg.close()
        del phi
        torch.cuda.empty_cache()
    best = res["fp64_graph"]
    out = {
        "metric": "Gsite-updates/s (ragged batch of 32 samples, Chebyshev moments, FP64)",
        "value": round(best["gsu"], 3), "unit": "Gsite-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(best["seconds"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "32 samples: AGNR/ZGNR/sheets of 1e4..1e6 sites, widths 20-400 "
                               "cells, W in {0.5,1,2} eV, 8 vectors each, 1000 moments",
                   "n_sites": int(total), "n_vec": r, "samples": len(specs)},
        "runs": {k: {"ms": round(v["seconds"] * 1e3, 3), "gsu": round(v["gsu"], 3),
                     "launch_shape": v["launch"]} for k, v in res.items()},
        "moment_launches": rates,
        "fp32_arith_over_fp64": round(res["fp32_arith_graph"]["gsu"] / best["gsu"], 3),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
