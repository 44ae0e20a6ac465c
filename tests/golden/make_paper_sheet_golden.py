"""Oracle values for the paper-scale sheet, written once and stored.

    python tests/golden/make_paper_sheet_golden.py [--threads T] [--vector-seed S] [--out PATH]

The sample is the plain-method workload at paper scale: a periodic graphene
sheet of 2828 x 1414 sites (1414 x 1414 two-atom cells, 3,998,792 sites),
t = -2.7 eV, 0.5 % vacancies (seed 2000), Anderson disorder W = 0.1 eV (seed
1000), E_s = 1.01 (3 |t| + W/2), and the random-phase vector of seed 3000
(paper_sheet_oracle.npz) or of another seed S (paper_sheet_oracle_seedS.npz;
seeds 3001 .. 3003 are vectors 1 .. 3 of the 64-vector workload).
Stored (float64, numpy .npz without pickled objects):

  * dos_re, dos_im  [3000]     C_m = <phi|T_m(H~)|phi> (Eq. 46, Alg. 5)
  * vac             [21][3000] Re <V U^dag(t_k) phi|T_m|U^dag(t_k) V phi>,
                               t_k = k dt, k = 0 .. 20 (Alg. 2, Eq. 42-43)
  * msd             [21][3000] Re <[X,U(t_k)] phi|T_m|[X,U(t_k)] phi> (Alg. 3, Eq. 44)

with dt = hbar/|t| and 40 Bessel terms per time step (Eq. 36-41).  Only the
oracle and the shared input generator are called: every stored value is the
oracle's.  The three loops take about 5e11 site-updates; the oracle's row
loops run on T threads (its results do not depend on T), and the parts can be
computed in separate runs (--parts), each stored as soon as it is done.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import kpm_inputs as ki  # noqa: E402
import oracle  # noqa: E402

VECTOR_SEED = 3000


def golden_path(seed: int = VECTOR_SEED) -> str:
    """Where the values for the vector of this seed are stored."""
    name = "paper_sheet_oracle.npz" if seed == VECTOR_SEED else f"paper_sheet_oracle_seed{seed}.npz"
    return os.path.join(HERE, name)


OUT = golden_path()


def inputs(seed: int = VECTOR_SEED):
    """The paper-scale sheet's inputs (lattice arguments, vector of the given
    seed) from the shared generator, and the parameters of the run."""
    p = ki.sheet_config("paper")
    n = p["nx"] * p["ny"]
    act = ki.vacancy_mask(n, p["vac"], 2000)
    ons = ki.anderson_onsite(n, p["w"], 1000)
    phi = ki.random_phase(n, 1, seed, act)[:, 0]
    return p, ons, act, phi


def input_digest(ons, act, phi) -> str:
    """SHA-256 of the input arrays, so a reader can check that the stored
    values belong to the inputs the generator gives today."""
    h = hashlib.sha256()
    for a in (ons, act, phi):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _load_parts(path, digest):
    """Parts already stored for the same inputs (a run may be split)."""
    if not os.path.exists(path):
        return {}
    z = np.load(path, allow_pickle=False)
    meta = json.loads(bytes(z["meta"]).decode())
    if meta.get("input_sha256") != digest:
        return {}
    return {k: z[k] for k in z.files if k != "meta"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0, help="oracle threads (0: its default)")
    ap.add_argument("--vector-seed", type=int, default=VECTOR_SEED)
    ap.add_argument("--out", default="", help="default: the seed's file beside this script")
    ap.add_argument("--parts", default="dos,vac,msd",
                    help="parts to compute now (the others are kept from an earlier run)")
    args = ap.parse_args()
    os.environ["ORC_PROGRESS"] = "1"
    th = oracle.set_threads(args.threads)
    args.out = args.out or golden_path(args.vector_seed)
    p, ons, act, phi = inputs(args.vector_seed)
    digest = input_digest(ons, act, phi)
    parts = _load_parts(args.out, digest)
    lat = oracle.graphene(p["nx"], p["ny"], "sheet", p["t"], ons, act)
    es, nm, ns, nb, dt = p["e_scale"], p["n_moments"], p["n_steps"], p["n_bessel"], p["dt_fs"]
    print(f"[golden] {lat.n} sites, {th} oracle threads, stored parts {sorted(parts)}", flush=True)
    meta = dict(nx=p["nx"], ny=p["ny"], t_ev=p["t"], w_ev=p["w"], vacancies=p["vac"],
                e_scale=es, n_moments=nm, n_steps=ns, n_bessel=nb, dt_fs=dt,
                onsite_seed=1000, vacancy_seed=2000, vector_seed=args.vector_seed,
                input_sha256=digest)

    def save():
        tmp = args.out + ".tmp.npz"
        np.savez(tmp, meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8), **parts)
        os.replace(tmp, args.out)

    t0 = time.time()
    for part in args.parts.split(","):
        if part == "dos":
            dos = oracle.moments(lat, es, phi, phi, nm)
            parts.update(dos_re=dos.real, dos_im=dos.imag)
        elif part == "vac":
            parts["vac"] = oracle.vac(lat, es, phi, ns, dt, nb, nm)
        elif part == "msd":
            parts["msd"] = oracle.msd(lat, es, phi, ns, dt, nb, nm)
        else:
            raise SystemExit(f"unknown part {part}")
        save()
        print(f"[golden] {part} done and stored ({time.time() - t0:.0f} s)", flush=True)
    print(f"[golden] {args.out}: parts {sorted(parts)}", flush=True)


if __name__ == "__main__":
    main()
