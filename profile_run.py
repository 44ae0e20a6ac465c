"""Short, fixed workload for hardware-counter collection with rocprofv3, and
the summary of its counter readings.

Collect (one counter per run):

    rocprofv3 --pmc FETCH_SIZE -d OUT/fetch -o c --output-format csv -- \
        python3 profile_run.py --moments 40 --copy-mib 512 \
        --meta OUT/meta.json
    rocprofv3 --pmc WRITE_SIZE -d OUT/write -o c --output-format csv -- \
        python3 profile_run.py --moments 40 --copy-mib 512

Summarise:

    python3 profile_run.py --summarize OUT/fetch OUT/write \
        --meta OUT/meta.json --out profiles/<name>.json
    python3 profile_run.py --trace-table OUT/bench_kernel_stats.csv

The run does one Chebyshev-moment call on the paper-scale sheet (2828 x 1414
sites, 0.5 % vacancies, W = 0.1 eV; n_moments - 2 launches of the fused moment
step, or about n_moments / 2 in the doubling form) in the precision and vector
count asked for, followed by plain device-to-device copies of a known size.
FETCH_SIZE and WRITE_SIZE count in KiB per dispatch; the copies, which read
and write exactly copy-mib MiB each, give the factor that turns each counter
into bytes.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

KERNEL_SRC = os.path.join(ROOT, "paper_1307_0288_amd", "csrc", "kpm_kernels.hip")
DEVICE_SRC = os.path.join(ROOT, "paper_1307_0288_amd", "csrc", "kpm_device.h")
MARCH32_SRC = os.path.join(ROOT, "paper_1307_0288_amd", "csrc", "kpm_march32.hip")
MARCH_H = os.path.join(ROOT, "paper_1307_0288_amd", "csrc", "kpm_march.h")
MARCH_LONG_SRC = os.path.join(ROOT, "paper_1307_0288_amd", "csrc", "kpm_march_long.hip")


def _read(path: str) -> str:
    with open(path) as f:
        return f.read()


def multi_step(launch: dict, n_vec: int = 1) -> bool:
    """Whether moment sets take the multi-step sweeps under this launch shape
    (compact form; one vector, or several kept vector-major, which take the
    strips; the sample must be a chain lattice)."""
    planar = n_vec > 1 and launch.get("vectors_per_wave", 0) == 1 and launch.get("tiled", 0) >= 3
    return launch.get("steps", 1) >= 2 and (n_vec == 1 or planar) and bool(launch["compact"])


def float_onsite(onsite) -> bool:
    """Whether the library stores these on-site energies as floats (it does
    when every value is exactly a float)."""
    import numpy as np
    if onsite is None:
        return True
    a = np.asarray(onsite, dtype=np.float64)
    return bool(np.array_equal(a.astype(np.float32).astype(np.float64), a))


def joint_shape(launch: dict, cus: int, fp64: bool = True) -> dict:
    """Launch shape of the joint VAC / MSD moment sets (two vector planes)
    under the one-vector shape `launch` on a GPU of `cus` compute units: the
    one-vector grid's wavefronts (groups per CU times CUs, a multiple of the 8
    XCDs, times the wavefronts per group) shared between the two planes in
    groups of 256 threads; with FP64 states the eight-step strips take ten
    steps per pass (both sets keep only real parts)."""
    nwg = max(8, cus * launch["groups_per_cu"] // 8 * 8)
    waves = nwg * launch.get("group_size", 256) // 64
    shape = {k: v for k, v in launch.items() if k != "group_size"}
    if fp64 and shape.get("steps") == 8 and shape.get("tiled", 0) >= 3:
        shape["steps"] = 10
    return dict(shape, vectors_per_wave=1, plane_groups=max(8, waves // 4 // 2 // 8 * 8))


def re_launch(launch: dict, precision: str, n_vec: int) -> dict:
    """The shape the library's real-part moment sets (VAC, MSD) of n_vec
    vectors kept vector-major actually run under `launch`: with FP64 states the
    eight-step strips take ten steps per pass (in groups of 256 threads or
    more); the FP32 forms keep eight."""
    if (n_vec > 1 and precision == "fp64" and launch.get("steps") == 8
            and launch.get("tiled", 0) >= 3 and launch.get("vectors_per_wave", 0) == 1
            and launch.get("group_size", 0) in (0, 256, 512)):
        return dict(launch, steps=10)
    return launch


def moment_kernel_name(v: str, launch: dict, dbl: bool, n_vec: int = 1,
                       real: bool = False, onsf: bool = True, arith32: bool = False) -> str:
    """Instantiation of the moment step for a graphene system from the builder
    (width 3, uniform hopping, at least 24 chains) under a launch shape; onsf:
    on-site terms stored as floats (float_onsite) or doubles; real: the moment
    sets whose callers keep only the real parts (VAC and MSD), which the
    marching strips accumulate alone."""
    nt, db = ("true" if launch["streaming"] else "false"), ("true" if dbl else "false")
    of = "true" if onsf else "false"
    if multi_step(launch, n_vec):
        k, tiled = launch["steps"], launch["tiled"]
        if arith32 and tiled >= 3:          # FP32 recursion arithmetic in the strips
            if real and not dbl:
                return f"k_moment_march_re_f32<{of},{k}>"
            return f"k_moment_march_f32<{of},{db},{k}>"
        if k == 2 and tiled == 0:
            return f"k_moment_step2<{v},{nt},{of},{db},16>"
        if tiled >= 3 and real and not dbl:
            return f"k_moment_march_re<{v},{of},{k}>"
        if tiled >= 3:
            return f"k_moment_march<{v},{of},{db},{k}>"
        return f"k_moment_stepk<{v},{of},{db},{4 if tiled == 2 else 8},{k}>"
    form = ("kFormC3F" if onsf else "kFormC3D") if launch["compact"] else \
        ("kFormL3F" if onsf else "kFormL3D")
    return f"k_moment_step<{v},{launch['ilp']},{nt},{form},{db}>"


def kernel_sha(launch: dict | None = None) -> str:
    """Hash of the source the moment step under `launch` is compiled from (the
    single-step kernel by default): the kernel file up to the first kernel
    after the moment step, plus the multi-step kernels for a multi-step shape,
    plus the launchers (edits elsewhere in the file change neither); the
    marching strips live in kpm_march.h, kpm_march_long.hip and
    kpm_march32.hip."""
    with open(KERNEL_SRC) as f:
        t = f.read()
    with open(DEVICE_SRC) as f:          # the helpers every kernel file shares
        t = f.read() + t
    head = t[:t.index("// Loads and stores of the propagator kernels")]
    if launch is not None and multi_step(launch):
        # LDS tiles | register tiles (and the helpers the marching form uses) |
        # marching strips: each form hashes its own section(s)
        lds = t.index("// ---------------------------------------------------------------- multi-step sweeps")
        reg = t.index("// Register-tiled sweep of K = 2, 3 or 4")
        march = t.index("// Marching form of the register-tiled K-step sweep")
        end = t.index("// ---------------------------------------------------------------- launchers")
        c = t.index("template <typename V>\nbool launch_moment_multi(")
        d = t.index("#define KPM_INSTANTIATE(V)")
        k, tiled = launch["steps"], launch["tiled"]
        strips = _read(MARCH_H) + _read(MARCH_LONG_SRC) + _read(MARCH32_SRC)
        body = (t[lds:reg] if (k == 2 and tiled == 0) else
                t[reg:end] + strips if tiled >= 3 else t[reg:march])
        return hashlib.sha256((head + body + t[c:d]).encode()).hexdigest()[:16]
    a = t.index("template <typename V, int ILP, bool NT, bool DBL>\nstatic void launch_step_shape(")
    b = t.index("template <typename V>\nvoid launch_evolve_step(")
    return hashlib.sha256((head + t[a:b]).encode()).hexdigest()[:16]


def measured_traffic(path: str, step_rows: int, launch: dict, kernel: str = ""):
    """HBM bytes per moment-step launch from a committed counter summary (one
    record, or {"records": [...]} for several launch shapes), or None when
    no record matches this kernel version, size and launch shape (and, when
    given, kernel name)."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    sha = kernel_sha(launch)
    for r in t.get("records", [t]):
        stored = dict({"steps": 1}, **r.get("launch_shape", {}))
        if r.get("kernel_sha") == sha and r.get("step_rows") == step_rows \
                and stored == dict({"steps": 1}, **launch) \
                and (not kernel or r.get("kernel", "").split(" ")[0] == kernel):
            return r.get("bytes_per_launch")
    return None


def _read_counter(d: str):
    rows = []
    for root, _, files in os.walk(d):
        for fn in files:
            if fn.endswith("counter_collection.csv"):
                with open(os.path.join(root, fn)) as f:
                    rows.extend(csv.DictReader(f))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return rows


def _dispatch_sums(rows):
    """Counter value per dispatch (summed over the rows of its instances)."""
    out = {}
    for r in rows:
        out[r["Dispatch_Id"]] = out.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return out


def _mean(vals):
    vals = list(vals)
    if not vals:
        raise SystemExit("no matching dispatches")
    return sum(vals) / len(vals)


def summarize(fetch_dir: str, write_dir: str, meta_path: str, out_path: str):
    with open(meta_path) as f:
        meta = json.load(f)
    # dispatches of the kernel instantiation named in the meta
    want = meta["kernel"].split(" ")[0]
    res = {}
    for key, d in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _read_counter(d)
        # the calibration copies: the largest device copies of the run (a
        # workload's own state copies, of one state each, are far smaller)
        copies = _dispatch_sums(r for r in rows if r["Kernel_Name"] == "__amd_rocclr_copyBuffer")
        big = max(copies.values())
        copy_kib = _mean(v for v in copies.values() if v >= 0.5 * big)
        step = _mean(float(r["Counter_Value"]) for r in rows if _is_kernel(r["Kernel_Name"], want))
        res[key] = (step, meta["copy_mib"] * 1024.0 / copy_kib)
    fetch_kib, fs = res["fetch"]
    write_kib, ws = res["write"]
    out = {
        "kernel": meta["kernel"],
        "kernel_sha": meta["kernel_sha"],
        "step_rows": meta["step_rows"],
        "launch_shape": meta["launch_shape"],
        "fetch_kib_per_launch": round(fetch_kib, 3),
        "write_kib_per_launch": round(write_kib, 3),
        "fetch_scale": round(fs, 4),
        "write_scale": round(ws, 4),
        "bytes_per_launch": int(round((fetch_kib * fs + write_kib * ws) * 1024)),
        "algorithmic_bytes_per_launch": meta["step_bytes"],
        "command": meta["command"],
    }
    out["traffic_over_algorithmic"] = round(out["bytes_per_launch"] / meta["step_bytes"], 4)
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


SQ_KEYS = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
           "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_LDS", "SQ_INSTS_VALU",
           "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
           "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_SCA")


def summarize_sq(dirs, meta_path: str, out_path: str):
    """Per-launch averages of the SQ counters of the kernel named in the meta
    (one or more --pmc runs, one directory each), as one record: the VALU
    instructions per launch are what bench.py reads for its VALU roof."""
    with open(meta_path) as f:
        meta = json.load(f)
    want = meta["kernel"].split(" ")[0]
    vals = {}
    for d in dirs:
        rows = [r for r in _read_counter(d) if _is_kernel(r["Kernel_Name"], want)]
        per = {}
        for r in rows:
            key = (r["Counter_Name"], r["Dispatch_Id"])
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        for name in {k[0] for k in per}:
            vals[name] = round(_mean(v for (c, _), v in per.items() if c == name), 1)
    out = {
        "kernel": meta["kernel"],
        "kernel_sha": meta["kernel_sha"],
        "step_rows": meta["step_rows"],
        "launch_shape": meta["launch_shape"],
        "counters_per_launch": {k: vals[k] for k in SQ_KEYS if k in vals},
        "valu_insts_per_launch": vals.get("SQ_INSTS_VALU"),
        "command": meta["command"].replace("--pmc FETCH_SIZE (then WRITE_SIZE)",
                                           "--pmc <SQ counter set>"),
    }
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def _short_kernel_name(name: str) -> str:
    name = name.replace("HIP_vector_type<double, 2u>", "double2")
    name = name.replace("HIP_vector_type<float, 2u>", "float2")
    name = name.replace("(anonymous namespace)::", "")
    name = name.removeprefix("void ")
    return name.split("(")[0] if "(" in name else name


def _is_kernel(name: str, want: str) -> bool:
    """Whether a profiler's kernel name is the instantiation `want` (written
    as moment_kernel_name writes it: no namespace, no spaces)."""
    return _short_kernel_name(name).removeprefix("kpm::").replace(" ", "") == want


def trace_table(stats_csv: str, top: int, only: str = "") -> str:
    """Markdown table of the `top` kernels of a rocprofv3 --stats kernel summary
    (only those whose short name matches the regular expression `only`, if given)."""
    import re
    with open(stats_csv) as f:
        rows = list(csv.DictReader(f))
    if only:
        rows = [r for r in rows if re.search(only, _short_kernel_name(r["Name"]))]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg (us) | min (us) | max (us) | share of GPU time |",
           "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{_short_kernel_name(r['Name'])}` | {r['Calls']} | "
                   f"{float(r['AverageNs']) / 1e3:.3f} | {float(r['MinNs']) / 1e3:.3f} | "
                   f"{float(r['MaxNs']) / 1e3:.3f} | {float(r['Percentage']):.2f} % |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--moments", type=int, default=40)
    ap.add_argument("--n-vec", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "fp32_arith"])
    ap.add_argument("--doubled", action="store_true", help="doubling form (kpm_moments_doubled)")
    ap.add_argument("--real", action="store_true",
                    help="a real-part moment set as the VAC takes them (kpm_vac, no time steps: "
                         "the moments of V phi)")
    ap.add_argument("--joint", type=int, default=0, metavar="STEPS",
                    help="the joint VAC / MSD call (kpm_vac_msd) over this many time steps: "
                         "its moment sets of t_1 .. t_STEPS run as two vector planes, the "
                         "kernel summarised (one vector; --launch gives the one-vector shape)")
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--copies", type=int, default=3)
    ap.add_argument("--launch", default="",
                    help="groups_per_cu,ilp,streaming,compact[,tiled[,steps[,vectors_per_wave"
                         "[,plane_groups]]]] (default: the library's)")
    ap.add_argument("--autotune", type=int, default=0,
                    help="run kpm_autotune with this many repetitions first (the benchmark's "
                         "choice of shape)")
    ap.add_argument("--meta", default="", help="write the run's launch shape, sizes and "
                                               "algorithmic bytes here")
    ap.add_argument("--summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-sq", nargs="+", metavar="PMC_DIR",
                    help="per-launch SQ counter averages of the meta's kernel")
    ap.add_argument("--out", default="")
    ap.add_argument("--trace-table", metavar="KERNEL_STATS_CSV",
                    help="print a markdown table of a --stats kernel summary")
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--only", default="", help="--trace-table: kernels whose name matches this "
                                               "regular expression")
    args = ap.parse_args()
    if args.trace_table:
        print(trace_table(args.trace_table, args.top, args.only))
        return
    if args.summarize:
        return summarize(args.summarize[0], args.summarize[1], args.meta, args.out)
    if args.summarize_sq:
        return summarize_sq(args.summarize_sq, args.meta, args.out)

    import torch
    import kpm_inputs as ki
    import paper_1307_0288_amd as kp

    torch.cuda.set_device(0)
    p = ki.sheet_config("paper")
    n = p["nx"] * p["ny"]
    act = ki.vacancy_mask(n, p["vac"], 2000)
    ons = ki.anderson_onsite(n, p["w"], 1000)
    onsf = float_onsite(ons)
    sysg = kp.graphene_system(p["nx"], p["ny"], "sheet", p["t"], ons, act, p["e_scale"],
                              args.precision)
    phi = sysg.upload(ki.random_phase(n, args.n_vec, 3000, act))
    if args.launch:
        kp.kpm_set_launch(sysg, args.n_vec, *(int(x) for x in args.launch.split(",")))
    if args.autotune:
        kp.kpm_autotune(sysg, phi, args.autotune)
    launch = kp.kpm_get_launch(sysg, args.n_vec)
    print(f"launch shape: {launch}", flush=True)
    kp.kpm_reset_stats(sysg)
    if args.joint:
        if args.n_vec != 1:
            raise SystemExit("--joint runs one vector")
        vac, _ = kp.kpm_vac_msd(sysg, phi, args.joint, p["dt_fs"], p["n_bessel"], args.moments)
        mu = vac[:, 0, :]
    elif args.doubled:
        mu = kp.kpm_moments_doubled(sysg, phi, args.moments)
    elif args.real:
        mu = kp.kpm_vac(sysg, phi, 0, p["dt_fs"], p["n_bessel"], args.moments)[:, 0, :]
    else:
        mu = kp.kpm_moments(sysg, phi, phi, args.moments)
    st = kp.kpm_get_stats(sysg)
    print(f"moments: n={n} n_vec={args.n_vec} {args.precision} doubled={args.doubled} "
          f"C_0={mu[0, 0].real:.1f}", flush=True)
    src = torch.ones(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.copies):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copies: {args.copies} x {args.copy_mib} MiB", flush=True)
    if args.meta:
        v = "double2" if args.precision == "fp64" else "float2"
        cmd = ["python3 profile_run.py", f"--moments {args.moments}",
               f"--n-vec {args.n_vec}", f"--precision {args.precision}",
               f"--copy-mib {args.copy_mib}"]
        if args.doubled:
            cmd.append("--doubled")
        if args.real:
            cmd.append("--real")
        if args.joint:
            cmd.append(f"--joint {args.joint}")
        if args.launch:
            cmd.append(f"--launch {args.launch}")
        if args.autotune:
            cmd.append(f"--autotune {args.autotune}")
        if args.joint:          # the two-plane passes: real parts, two vectors
            launch = joint_shape(launch, torch.cuda.get_device_properties(0).multi_processor_count,
                                 args.precision == "fp64")
            kname = moment_kernel_name(v, launch, False, 2, True, onsf)
        else:
            kl = re_launch(launch, args.precision, args.n_vec) if args.real else launch
            kname = moment_kernel_name(v, kl, args.doubled, args.n_vec, args.real, onsf,
                                       args.precision == "fp32_arith")
        meta = {
            "kernel": f"{kname} ({args.precision}, {2 if args.joint else args.n_vec} vector(s))",
            "kernel_sha": kernel_sha(launch),
            "step_rows": st["step_rows"],
            "step_bytes": st["step_bytes"],
            "launch_shape": launch,
            "copy_mib": args.copy_mib,
            "command": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -d OUT -o c "
                       "--output-format csv -- " + " ".join(cmd),
        }
        with open(args.meta, "w") as f:
            json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
