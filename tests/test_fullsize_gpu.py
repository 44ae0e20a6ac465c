"""Parity at full size, in the launch configurations bench.py times, on
sampled outputs the oracle can compute one by one.

* Batched precision: the 3,998,792-site sheet with 64 random-phase vectors,
  FP32 states, autotuned launch shape: the first 24 moments of vectors 0 and
  63 against the oracle (FP32 states: max|dC| / |phi|^2 <= 1e-5), and
  properties of all 64 x 300 moments (C_0 = N_active to FP32 rounding,
  |C_m| <= C_0).
* Ragged batch: the 32-sample batch (8.0 M sites, 8 vectors, 1000 moments),
  autotuned, FP64: every moment of the three smallest samples against the
  oracle run on each alone (1e-10), and C_0 of every sample and vector.
"""
import numpy as np
import pytest

import kpm_inputs as ki
import oracle
from cases import rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _log(msg):
    print(msg, flush=True)


def test_paper_scale_64_vectors_fp32():
    _need_gpu()
    p = ki.sheet_config("paper")
    n = p["nx"] * p["ny"]
    act = ki.vacancy_mask(n, p["vac"], 2000)
    ons = ki.anderson_onsite(n, p["w"], 1000)
    phi = ki.random_phase(n, 64, 3000, act)
    _log("batched 64 vectors fp32: build + autotune")
    sysg = kp.graphene_system(p["nx"], p["ny"], "sheet", p["t"], ons, act, p["e_scale"], "fp32")
    d = sysg.upload(phi)
    kp.kpm_autotune(sysg, d, 3)
    got = kp.kpm_moments(sysg, d, d, 300)
    n_act = float(np.count_nonzero(act))
    assert np.max(np.abs(got[:, 0].real - n_act)) < 1e-6 * n_act
    assert np.all(np.abs(got.real) <= n_act * (1 + 1e-6))
    del d
    sysg.close()
    torch.cuda.empty_cache()
    _log("oracle: 24 moments of vectors 0 and 63")
    lat = oracle.graphene(p["nx"], p["ny"], "sheet", p["t"], ons, act)
    for r in (0, 63):
        ref = oracle.moments(lat, p["e_scale"], phi[:, r], phi[:, r], 24)
        assert rel_err(got[r, :24], ref, n_act) < 1e-5, r


def test_ragged_batch_full_size():
    _need_gpu()
    cfg = ki.sheet_config("ragged")
    specs = ki.ragged_specs(cfg["count"], cfg["seed"], cfg["n_min"], cfg["n_max"],
                            cfg["w_min"], cfg["w_max"])
    r, nm = cfg["n_vec"], cfg["n_moments"]
    samples, phis, cases = [], [], []
    for s, sp in enumerate(specs):
        n = sp["nx"] * sp["ny"]
        ons = ki.anderson_onsite(n, sp["w"], 1000 + s)
        es = 1.01 * (3 * 2.7 + sp["w"] / 2)
        samples.append(dict(nx=sp["nx"], ny=sp["ny"], geometry=sp["geometry"], onsite=ons,
                            e_scale=es))
        phis.append(ki.random_phase(n, r, 3000 + 100 * s))
        cases.append((sp, ons, es))
    _log(f"ragged batch: {sum(p.shape[0] for p in phis)} sites")
    sysg = kp.graphene_batch(samples, "fp64")
    d = sysg.upload(np.concatenate(phis))
    kp.kpm_autotune(sysg, d, 3)
    got = kp.kpm_moments(sysg, d, d, nm)
    sizes = [p.shape[0] for p in phis]
    for s in range(len(specs)):
        assert np.max(np.abs(got[s, :, 0].real - sizes[s])) < 1e-9 * sizes[s], s
    for s in np.argsort(sizes)[:3]:
        sp, ons, es = cases[s]
        _log(f"oracle: sample {s} ({sizes[s]} sites)")
        lat = oracle.graphene(sp["nx"], sp["ny"], sp["geometry"], -2.7, ons)
        for v in (0, r - 1):
            ref = oracle.moments(lat, es, phis[s][:, v], phis[s][:, v], nm)
            assert rel_err(got[s, v], ref, sizes[s]) < 1e-10, (s, v)
