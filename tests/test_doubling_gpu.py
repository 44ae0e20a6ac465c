"""Moments in the doubling form (kpm_moments_doubled, kpm_msd_doubled) against
the oracle's direct Chebyshev moments (Alg. 5).

For phi_L = phi_R = phi the product identities T_{2n} = 2 T_n^2 - T_0 and
T_{2n+1} = 2 T_{n+1} T_n - T_1 give every moment from about half the
recursion steps.  The values equal the direct ones up to rounding, so the bars
are those of the direct path: max|dC| / |phi|^2 <= 1e-10 (FP64), MSD moments
max|dC| / max|C| <= 1e-10, FP32 states sigma error <= 1e-3.
"""
import numpy as np
import pytest

import kpm_inputs as ki
import oracle
from cases import gpu_system, oracle_lattice, phases, recipe, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")

SMALL = ki.sheet_config("small")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def small():
    _need_gpu()
    c = recipe("sheet", SMALL["nx"], SMALL["ny"], w=SMALL["w"], e_scale=SMALL["e_scale"])
    return c, oracle_lattice(c), gpu_system(c)


# 1, 2: no recursion step; 3: one step whose second sum is dropped;
# 257 / 513: the partial ring (256 slots) fills mid-set, odd counts.
@pytest.mark.parametrize("nm", [1, 2, 3, 4, 257, 500, 513])
def test_doubled_moments_small_config(small, nm):
    c, lat, sysg = small
    _log(f"doubled moments small nm={nm}")
    phi = phases(c)
    ref = oracle.moments(lat, c["e_scale"], phi[:, 0], phi[:, 0], max(nm, 2))[:nm]
    got = kp.kpm_moments_doubled(sysg, sysg.upload(phi), nm)[0]
    assert got.shape == (nm,)
    assert rel_err(got, ref, np.vdot(phi, phi).real) < 1e-10


@pytest.mark.parametrize("geometry,nx,ny,w,vac,nm,n_vec", [
    ("sheet", 64, 32, 1.0, 0.02, 300, 1),   # vacancies
    ("agnr", 7, 6, 2.0, 0.0, 51, 2),        # 42 rows: one ragged block
    ("zgnr", 10, 13, 0.5, 0.05, 64, 8),     # 130 rows
    ("sheet", 100, 50, 0.1, 0.005, 201, 64),
])
def test_doubled_moments_geometries(geometry, nx, ny, w, vac, nm, n_vec):
    _need_gpu()
    _log(f"doubled moments {geometry} {nx}x{ny} nm={nm} n_vec={n_vec}")
    c = recipe(geometry, nx, ny, w=w, vac=vac, seed=17)
    lat = oracle_lattice(c)
    sysg = gpu_system(c)
    phi = phases(c, n_vec, 3000)
    got = kp.kpm_moments_doubled(sysg, sysg.upload(phi), nm)
    for r in range(n_vec):
        ref = oracle.moments(lat, c["e_scale"], phi[:, r], phi[:, r], nm)
        assert rel_err(got[r], ref, np.vdot(phi[:, r], phi[:, r]).real) < 1e-10, r


@pytest.mark.parametrize("n_vec,precision", [(1, "fp64"), (8, "fp32"), (64, "fp64")])
def test_doubled_launch_shapes(n_vec, precision):
    """Every ILP, streaming and neighbour form gives bit-identical doubled
    moments at a fixed grid; they agree with the direct form."""
    _need_gpu()
    c = recipe("sheet", 100, 50, w=1.0, vac=0.01, seed=2)
    sysg = gpu_system(c, precision)
    phi = sysg.upload(phases(c, n_vec, 3000))
    ref = None
    for ilp in (1, 2, 4):
        for nt in (0, 1):
            for cp in (0, 1):
                kp.kpm_set_launch(sysg, n_vec, 4, ilp, nt, cp)
                mu = kp.kpm_moments_doubled(sysg, phi, 41)
                ref = mu if ref is None else ref
                assert np.array_equal(mu, ref), (ilp, nt, cp)
    direct = kp.kpm_moments(sysg, phi, phi, 41)
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert rel_err(ref, direct, float(np.abs(direct[:, 0]).max())) < tol


def test_doubled_msd_small_config(small):
    c, lat, sysg = small
    phi = phases(c, 1, 3000)
    args = (SMALL["n_steps"], SMALL["dt_fs"], SMALL["n_bessel"], SMALL["n_moments"])
    _log("doubled msd small")
    ref = oracle.msd(lat, c["e_scale"], phi[:, 0], *args)
    got = kp.kpm_msd_doubled(sysg, sysg.upload(phi), *args)[0]
    assert np.all(got[0] == 0)
    assert rel_err(got, ref) < 1e-10


def test_doubled_fp32_sigma_within_1e3(small):
    c, lat, _ = small
    sys32 = gpu_system(c, "fp32")
    phi = phases(c, 1, 3000)
    args = (SMALL["n_steps"], SMALL["dt_fs"], SMALL["n_bessel"], SMALL["n_moments"])
    _log("doubled fp32 msd small")
    rm = oracle.msd(lat, c["e_scale"], phi[:, 0], *args)
    gm = kp.kpm_msd_doubled(sys32, sys32.upload(phi), *args)[0]
    es, area, dt = c["e_scale"], lat.area_nm2, SMALL["dt_fs"]
    en = oracle.energies_grid(257, es)
    r = oracle.sigma_e1(oracle.kpm_sum(rm, en, es, area), dt)
    g = kp.kpm_sigma_e1(kp.kpm_kpm_sum(gm, en, es, area), dt)
    assert rel_err(g, r) < 1e-3


def test_doubled_batch_per_sample_and_graphs():
    """Ragged batch: each sample's doubled moments against the oracle on that
    sample alone; graph replays equal eager launches bit for bit."""
    _need_gpu()
    specs = [("sheet", 24, 12, 1.0, 0.02), ("zgnr", 30, 7, 0.5, 0.0),
             ("agnr", 9, 40, 2.0, 0.01), ("sheet", 8, 4, 0.0, 0.0)]
    cases = [recipe(g, nx, ny, w=w, vac=vac, seed=40 + s)
             for s, (g, nx, ny, w, vac) in enumerate(specs)]
    sysg = kp.graphene_batch([dict(nx=c["nx"], ny=c["ny"], geometry=c["geometry"],
                                   onsite=c["onsite"], active=c["active"],
                                   e_scale=c["e_scale"]) for c in cases])
    phis = [ki.random_phase(c["nx"] * c["ny"], 2, 3000 + 100 * s, c["active"])
            for s, c in enumerate(cases)]
    d = sysg.upload(np.concatenate(phis))
    nm = 301
    got = kp.kpm_moments_doubled(sysg, d, nm)
    assert got.shape == (len(cases), 2, nm)
    for s, c in enumerate(cases):
        lat = oracle_lattice(c)
        for r in range(2):
            ref = oracle.moments(lat, c["e_scale"], phis[s][:, r], phis[s][:, r], nm)
            scale = max(np.vdot(phis[s][:, r], phis[s][:, r]).real, 1.0)
            assert rel_err(got[s, r], ref, scale) < 1e-10, (s, r)
    kp.kpm_set_graphs(sysg, True)
    for rep in range(3):
        assert np.array_equal(kp.kpm_moments_doubled(sysg, d, nm), got), rep
        e = d.clone()
        kp.kpm_evolve(sysg, e, 0.2, 1, 12)
        torch.cuda.synchronize()
    kp.kpm_set_graphs(sysg, False)


def test_doubled_stats_count_half_the_steps(small):
    c, lat, sysg = small
    d = sysg.upload(phases(c))
    kp.kpm_reset_stats(sysg)
    kp.kpm_moments_doubled(sysg, d, 500)
    st = kp.kpm_get_stats(sysg)
    assert st["site_updates"] == 250 * lat.n
    assert st["step_rows"] == lat.n
