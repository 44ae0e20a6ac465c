"""Short, fixed workload for hardware-counter collection with rocprofv3.

    rocprofv3 --pmc FETCH_SIZE -d OUT -o fetch --output-format csv -- \
        python3 -m paper_1307_0288_amd.profile_run --moments 40 --copy-mib 512

Runs one Chebyshev-moment call on the paper-scale sheet (2828 x 1414 sites,
0.5 % vacancies, W = 0.1 eV; n_moments - 2 launches of the fused moment step)
in the precision and vector count asked for, followed by plain device-to-device
copies of a known size, whose counter readings calibrate FETCH_SIZE and
WRITE_SIZE to bytes.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--moments", type=int, default=40)
    ap.add_argument("--n-vec", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--copies", type=int, default=3)
    ap.add_argument("--launch", default="",
                    help="groups_per_cu,ilp,streaming,compact (default: the library's)")
    args = ap.parse_args()

    import torch
    import kpm_inputs as ki
    import paper_1307_0288_amd as kp

    torch.cuda.set_device(0)
    p = ki.sheet_config("paper")
    n = p["nx"] * p["ny"]
    act = ki.vacancy_mask(n, p["vac"], 2000)
    ons = ki.anderson_onsite(n, p["w"], 1000)
    sysg = kp.graphene_system(p["nx"], p["ny"], "sheet", p["t"], ons, act, p["e_scale"],
                              args.precision)
    phi = sysg.upload(ki.random_phase(n, args.n_vec, 3000, act))
    if args.launch:
        g, ilp, nt, cp = (int(x) for x in args.launch.split(","))
        kp.kpm_set_launch(sysg, args.n_vec, g, ilp, nt, cp)
    print(f"launch shape: {kp.kpm_get_launch(sysg, args.n_vec)}", flush=True)
    mu = kp.kpm_moments(sysg, phi, phi, args.moments)
    print(f"moments: n={n} n_vec={args.n_vec} {args.precision} C_0={mu[0, 0].real:.1f}",
          flush=True)
    src = torch.ones(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.copies):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copies: {args.copies} x {args.copy_mib} MiB", flush=True)


if __name__ == "__main__":
    main()
