"""Parity on the paper-scale sheet, end to end, in the launch configuration
bench.py times (autotuned on the same vector).

The sample: 2828 x 1414 periodic sheet (3,998,792 sites), 0.5 % vacancies,
W = 0.1 eV, the random-phase vector of seed 3000; 3000 moments, 20 time steps
of dt = hbar/|t| with 40 Bessel terms.  Reference values: the oracle's, stored
by tests/golden/make_paper_sheet_golden.py (DOS moments, and the VAC and MSD
moments at all 21 time points).  Bars: moments max|dC| / (|phi_L| |phi_R|) <=
1e-10 (DOS), max|dC| / max|C| <= 1e-10 (VAC, MSD), sigma_GK / sigma_E1 /
sigma_E2 and the DOS on 2048 energies max|d| / max|ref| <= 1e-8.
"""
import json
import os

import numpy as np
import pytest

import kpm_inputs as ki
import oracle
from cases import rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "paper_sheet_oracle.npz")


def _log(msg):
    print(msg, flush=True)


def _golden_module():
    import sys
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_paper_sheet_golden as mk
    return mk


def load_golden():
    """The stored oracle values, checked against today's inputs."""
    mk = _golden_module()
    z = np.load(GOLDEN, allow_pickle=False)
    meta = json.loads(bytes(z["meta"]).decode())
    p, ons, act, phi = mk.inputs()
    assert meta["input_sha256"] == mk.input_digest(ons, act, phi), \
        "stored oracle values belong to other inputs: rerun make_paper_sheet_golden.py"
    return p, ons, act, phi, dict(dos=z["dos_re"] + 1j * z["dos_im"], vac=z["vac"], msd=z["msd"])


def load_golden_seed(seed, ons, act, phi):
    """The stored oracle values for the vector of another seed (phi), or None
    when none are stored; checked against today's inputs."""
    mk = _golden_module()
    path = mk.golden_path(seed)
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    if not {"dos_re", "vac", "msd"} <= set(z.files):
        return None
    meta = json.loads(bytes(z["meta"]).decode())
    assert meta["input_sha256"] == mk.input_digest(ons, act, phi), \
        f"stored oracle values of seed {seed} belong to other inputs"
    return dict(dos=z["dos_re"], vac=z["vac"], msd=z["msd"])


@pytest.fixture(scope="module")
def paper():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p, ons, act, phi, gold = load_golden()
    _log("paper-scale sheet (3998792 sites): system, autotune")
    sysg = kp.graphene_system(p["nx"], p["ny"], "sheet", p["t"], ons, act, p["e_scale"], "fp64")
    d = sysg.upload(phi[:, None])
    launch = kp.kpm_autotune(sysg, d, 50)
    _log(f"autotuned shape {launch}")
    return p, act, phi, gold, sysg, d


def test_dos_moments_all_3000(paper):
    p, act, phi, gold, sysg, d = paper
    _log("paper-scale DOS moments (3000)")
    got = kp.kpm_moments(sysg, d, d, p["n_moments"])[0]
    n_act = float(np.count_nonzero(act))
    assert abs(got[0] - n_act) < 1e-6
    assert rel_err(got, gold["dos"], n_act) < 1e-10


def test_dos_moments_doubled_all_3000(paper):
    p, act, phi, gold, sysg, d = paper
    _log("paper-scale DOS moments, doubling form (3000)")
    got = kp.kpm_moments_doubled(sysg, d, p["n_moments"])[0]
    assert rel_err(got, gold["dos"], float(np.count_nonzero(act))) < 1e-10


@pytest.fixture(scope="module")
def loops(paper):
    p, act, phi, gold, sysg, d = paper
    args = (p["n_steps"], p["dt_fs"], p["n_bessel"], p["n_moments"])
    _log("paper-scale VAC and MSD (20 steps x 3000 moments)")
    return kp.kpm_vac(sysg, d, *args)[0], kp.kpm_msd(sysg, d, *args)[0]


def test_vac_all_time_points(paper, loops):
    gold = paper[3]
    gv, _ = loops
    assert gv.shape == gold["vac"].shape == (21, 3000)
    assert rel_err(gv, gold["vac"]) < 1e-10
    for k in (0, 10, 20):
        assert rel_err(gv[k], gold["vac"][k]) < 1e-10, k


def test_msd_all_time_points(paper, loops):
    gold = paper[3]
    _, gm = loops
    assert np.all(gm[0] == 0)
    assert rel_err(gm, gold["msd"]) < 1e-10
    for k in (1, 10, 20):
        assert rel_err(gm[k], gold["msd"][k]) < 1e-10, k


def test_joint_vac_msd_all_time_points(paper):
    """kpm_vac_msd (both loops, their moment sets as two planes of one launch
    sequence) against the stored oracle values."""
    p, act, phi, gold, sysg, d = paper
    _log("paper-scale VAC and MSD in one call")
    gv, gm = kp.kpm_vac_msd(sysg, d, p["n_steps"], p["dt_fs"], p["n_bessel"], p["n_moments"])
    assert rel_err(gv[0], gold["vac"]) < 1e-10
    assert rel_err(gm[0], gold["msd"]) < 1e-10


def test_dos_vac_msd_all_moments(paper):
    """kpm_dos_vac_msd (the DOS set as the second plane of the VAC set of t_0,
    every set a two-plane launch sequence) against the stored oracle values:
    all 3000 DOS moments and the 21 x 3000 VAC and MSD moments."""
    p, act, phi, gold, sysg, d = paper
    _log("paper-scale DOS, VAC and MSD in one call")
    gd, gv, gm = kp.kpm_dos_vac_msd(sysg, d, p["n_steps"], p["dt_fs"], p["n_bessel"],
                                    p["n_moments"])
    n_act = float(np.count_nonzero(act))
    assert abs(gd[0][0] - n_act) < 1e-6
    assert rel_err(gd[0], gold["dos"].real, n_act) < 1e-10
    assert rel_err(gv[0], gold["vac"]) < 1e-10
    assert rel_err(gm[0], gold["msd"]) < 1e-10
    assert np.all(gm[0][0] == 0)


def test_msd_doubled_all_time_points(paper):
    p, act, phi, gold, sysg, d = paper
    _log("paper-scale MSD, doubling form")
    gm = kp.kpm_msd_doubled(sysg, d, p["n_steps"], p["dt_fs"], p["n_bessel"], p["n_moments"])[0]
    assert rel_err(gm, gold["msd"]) < 1e-10


def test_sigma_on_2048_energies(paper, loops):
    """DOS, sigma_GK (Eq. 6), sigma_E1 (Eq. 9) and sigma_E2 (Eq. 11) from the
    GPU moments through the library's sums, against the oracle's
    reconstruction of the stored moments."""
    p, act, phi, gold, sysg, d = paper
    gv, gm = loops
    es, dt = p["e_scale"], p["dt_fs"]
    area = sysg.area_nm2
    # the oracle side's area: L_x L_y of its lattice (Sec. 2)
    o_area = (np.sqrt(3.0) * p["nx"] * oracle.BOND_NM / 2.0) * (3.0 * p["ny"] * oracle.BOND_NM / 2.0)
    en = oracle.energies_grid(2048, es)
    g_dos = kp.kpm_kpm_sum(kp.kpm_moments(sysg, d, d, p["n_moments"])[0].real, en, es, area)
    r_dos = oracle.dos(gold["dos"].real, en, es, o_area)
    assert rel_err(g_dos, r_dos) < 1e-8
    r_v = oracle.kpm_sum(gold["vac"], en, es, o_area)
    r_m = oracle.kpm_sum(gold["msd"], en, es, o_area)
    g_v, g_m = kp.kpm_kpm_sum(gv, en, es, area), kp.kpm_kpm_sum(gm, en, es, area)
    pairs = ((kp.kpm_sigma_gk(g_v, dt), oracle.sigma_gk(r_v, dt)),
             (kp.kpm_sigma_e1(g_m, dt), oracle.sigma_e1(r_m, dt)),
             (kp.kpm_sigma_e2(g_m, dt), oracle.sigma_e2(r_m, dt)))
    for name, (g, r) in zip(("gk", "e1", "e2"), pairs):
        assert g.shape == r.shape == (21, 2048)
        assert rel_err(g, r) < 1e-8, name


def test_evolve_norm_and_inverse(paper):
    p, act, phi, gold, sysg, d = paper
    e = sysg.upload(ki.random_phase(phi.shape[0], 1, 3005, act))
    ref = e.cpu().numpy()
    n0 = float(torch.vdot(e[:, 0], e[:, 0]).real)
    kp.kpm_evolve(sysg, e, p["dt_fs"], 1, p["n_bessel"])
    n1 = float(torch.vdot(e[:, 0], e[:, 0]).real)
    assert abs(n1 - n0) < 1e-10 * n0
    kp.kpm_evolve(sysg, e, p["dt_fs"], -1, p["n_bessel"])
    assert np.max(np.abs(e.cpu().numpy() - ref)) < 1e-11


def _oracle_spectra(dos, vac, msd, en, es, area, dt):
    rho_v = oracle.kpm_sum(vac, en, es, area)
    rho_m = oracle.kpm_sum(msd, en, es, area)
    return dict(dos=oracle.dos(dos, en, es, area), gk=oracle.sigma_gk(rho_v, dt),
                e1=oracle.sigma_e1(rho_m, dt), e2=oracle.sigma_e2(rho_m, dt))


def test_fp32_states_eight_vectors_sigma(paper):
    """Eight vectors (seeds 3000 .. 3007) with FP32 states (FP64 arithmetic,
    inner products and moments; and with the strips' recursion arithmetic in
    FP32 as well) through the whole hot path: the DOS (Eq. 29)
    and sigma_GK / sigma_E1 / sigma_E2 (Eq. 6, 9, 11) at 2048 energies and all
    21 times are within 1e-3 of the FP64 states' (mean over the vectors), and
    vectors 0 .. 3 (those whose oracle values are stored) within 1e-3 of the
    oracle's; the FP64 states' vectors match the oracle to 1e-8."""
    p, act, phi, gold, sysg, d = paper
    n = p["nx"] * p["ny"]
    es, dt, nm = p["e_scale"], p["dt_fs"], p["n_moments"]
    ons = ki.anderson_onsite(n, p["w"], 1000)
    phi8 = ki.random_phase(n, 8, 3000, act)
    assert np.array_equal(phi8[:, 0], phi)
    args = (p["n_steps"], dt, p["n_bessel"], nm)
    o_area = (np.sqrt(3.0) * p["nx"] * oracle.BOND_NM / 2.0) * (3.0 * p["ny"] * oracle.BOND_NM / 2.0)
    en = oracle.energies_grid(2048, es)
    runs = {}
    for prec in ("fp32", "fp32_arith", "fp64"):
        _log(f"paper-scale, 8 vectors, {prec} states: DOS, VAC, MSD")
        s8 = kp.graphene_system(p["nx"], p["ny"], "sheet", p["t"], ons, act, es, prec)
        _log(f"launch shape {kp.kpm_get_launch(s8, 8)}")
        d8 = s8.upload(phi8)
        runs[prec] = (kp.kpm_moments(s8, d8, d8, nm).real, kp.kpm_vac(s8, d8, *args),
                      kp.kpm_msd(s8, d8, *args))
        s8.close()
        del d8
    mean = {k: _oracle_spectra(v[0].mean(axis=0), v[1].mean(axis=0), v[2].mean(axis=0), en, es,
                               o_area, dt) for k, v in runs.items()}
    for key in ("dos", "gk", "e1", "e2"):
        for p32 in ("fp32", "fp32_arith"):
            e32 = rel_err(mean[p32][key], mean["fp64"][key])
            _log(f"sigma {key}: {p32} vs fp64 {e32:.2e}")
            assert e32 <= 1e-3, (key, p32)
    # vectors 0 .. 3 against the oracle's stored moments of each (vector 0
    # always; 1 .. 3 where their values are stored)
    golds = {0: gold}
    for r in (1, 2, 3):
        g = load_golden_seed(3000 + r, ons, act, phi8[:, r])
        if g is not None:
            golds[r] = g
    _log(f"vectors checked against the oracle: {sorted(golds)}")
    for r, g in golds.items():
        ref = _oracle_spectra(g["dos"].real, g["vac"], g["msd"], en, es, o_area, dt)
        got = {k: _oracle_spectra(v[0][r], v[1][r], v[2][r], en, es, o_area, dt)
               for k, v in runs.items()}
        for key in ("dos", "gk", "e1", "e2"):
            for p32 in ("fp32", "fp32_arith"):
                o32 = rel_err(got[p32][key], ref[key])
                _log(f"vector {r} sigma {key}: {p32} vs oracle {o32:.2e}")
                assert o32 <= 1e-3, (r, key, p32)
            o64 = rel_err(got["fp64"][key], ref[key])
            _log(f"vector {r} sigma {key}: fp64 vs oracle {o64:.2e}")
            assert o64 <= 1e-8, (r, key)
