"""Parity of the gfx950 library (through its C ABI) with the CPU oracle.

Tolerances (FP64): moments max|dC| / (|phi_L| |phi_R|) <= 1e-10; VAC/MSD
moments max|dC| / max|C| <= 1e-10; sigma(E) max|d sigma| / max|sigma| <= 1e-8.
FP32 states (FP64 arithmetic and dots): sigma error <= 1e-3.
"""
import numpy as np
import pytest

import kpm_inputs as ki
import oracle
from cases import gpu_system, oracle_lattice, phases, recipe, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")

HBAR = oracle.HBAR_EV_FS
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


# ------------------------------------------------------------------ moments
def test_moments_small_config(small):
    c, lat, sysg = small
    _log("moments small 2048 sites 500 moments")
    phi = phases(c)
    ref = oracle.moments(lat, c["e_scale"], phi[:, 0], phi[:, 0], SMALL["n_moments"])
    d = sysg.upload(phi)
    got = kp.kpm_moments(sysg, d, d, SMALL["n_moments"])[0]
    scale = np.vdot(phi, phi).real
    assert rel_err(got, ref, scale) < 1e-10
    assert abs(got[0] - lat.n) < 1e-9


@pytest.mark.parametrize("geometry,nx,ny,w,vac,nm", [
    ("sheet", 64, 32, 1.0, 0.02, 300),    # vacancies
    ("agnr", 7, 6, 2.0, 0.0, 50),         # 42 rows: one ragged block
    ("zgnr", 10, 13, 0.5, 0.05, 64),      # 130 rows
    ("sheet", 100, 50, 0.1, 0.005, 200),  # 5000 rows: several blocks and a ragged tail
    ("sheet", 8, 4, 1.0, 0.0, 1),         # only C_0
    ("sheet", 8, 4, 1.0, 0.0, 2),         # C_0 and C_1
    ("sheet", 8, 4, 1.0, 0.0, 3),
])
def test_moments_left_right_ragged(geometry, nx, ny, w, vac, nm):
    _need_gpu()
    _log(f"moments {geometry} {nx}x{ny} nm={nm}")
    c = recipe(geometry, nx, ny, w=w, vac=vac, seed=11)
    lat = oracle_lattice(c)
    sysg = gpu_system(c)
    pl = phases(c, 1, 3000)
    pr = phases(c, 1, 3500)
    ref = oracle.moments(lat, c["e_scale"], pl[:, 0], pr[:, 0], nm)
    got = kp.kpm_moments(sysg, sysg.upload(pl), sysg.upload(pr), nm)[0]
    scale = np.linalg.norm(pl) * np.linalg.norm(pr)
    assert rel_err(got, ref, scale) < 1e-10


@pytest.mark.parametrize("n_vec", [2, 8, 64])
def test_moments_batched_vectors(n_vec):
    _need_gpu()
    _log(f"moments batched n_vec={n_vec}")
    c = recipe("sheet", 48, 20, w=1.0, vac=0.01, seed=5)
    lat = oracle_lattice(c)
    sysg = gpu_system(c)
    phi = phases(c, n_vec, 3000)
    got = kp.kpm_moments(sysg, sysg.upload(phi), sysg.upload(phi), 100)
    for r in range(n_vec):
        ref = oracle.moments(lat, c["e_scale"], phi[:, r], phi[:, r], 100)
        assert rel_err(got[r], ref, np.vdot(phi[:, r], phi[:, r]).real) < 1e-10


def test_moments_all_sites_removed():
    _need_gpu()
    c = recipe("sheet", 8, 4)
    c["active"] = np.zeros(32, np.uint8)
    sysg = gpu_system(c)
    z = sysg.new_state(1)
    got = kp.kpm_moments(sysg, z, z, 10)
    assert np.all(got == 0)


def test_moments_deterministic(small):
    c, lat, sysg = small
    d = sysg.upload(phases(c, 1, 3001))
    a = kp.kpm_moments(sysg, d, d, 200)
    b = kp.kpm_moments(sysg, d, d, 200)
    assert np.array_equal(a, b)


# ------------------------------------------------------------------ propagators
@pytest.mark.parametrize("sign,nb,dt", [(1, 30, SMALL["dt_fs"]), (-1, 30, SMALL["dt_fs"]),
                                        (1, 2, 0.05), (1, 40, 1.0)])
def test_evolve(small, sign, nb, dt):
    c, lat, sysg = small
    _log(f"evolve sign={sign} nb={nb} dt={dt}")
    phi = phases(c, 1, 3002)
    ref = oracle.evolve(lat, c["e_scale"], phi[:, 0], dt, sign, nb)
    d = sysg.upload(phi)
    kp.kpm_evolve(sysg, d, dt, sign, nb)
    got = d.cpu().numpy()[:, 0]
    assert rel_err(got, ref) < 1e-12


def test_evolve_zero_time_is_identity(small):
    c, lat, sysg = small
    phi = phases(c, 1, 3003)
    d = sysg.upload(phi)
    kp.kpm_evolve(sysg, d, 0.0, 1, 10)
    assert np.array_equal(d.cpu().numpy(), phi)


@pytest.mark.parametrize("geometry,nx,ny", [("sheet", 64, 32), ("zgnr", 10, 13), ("agnr", 9, 8)])
def test_evolve_x(geometry, nx, ny):
    _need_gpu()
    _log(f"evolve_x {geometry}")
    c = recipe(geometry, nx, ny, w=1.0, vac=0.02, seed=7)
    lat = oracle_lattice(c)
    sysg = gpu_system(c)
    phi = phases(c, 1, 3004)
    rx, ru = oracle.evolve_x(lat, c["e_scale"], phi[:, 0], SMALL["dt_fs"], 30)
    d = sysg.upload(phi)
    ox, ou = sysg.new_state(1), sysg.new_state(1)
    kp.kpm_evolve_x(sysg, d, ox, ou, SMALL["dt_fs"], 30)
    assert rel_err(ox.cpu().numpy()[:, 0], rx) < 1e-12
    assert rel_err(ou.cpu().numpy()[:, 0], ru) < 1e-12


# ------------------------------------------------------------------ VAC / MSD / sigma
@pytest.fixture(scope="module")
def loops(small):
    c, lat, sysg = small
    phi = phases(c, 1, 3000)
    args = (SMALL["n_steps"], SMALL["dt_fs"], SMALL["n_bessel"], SMALL["n_moments"])
    _log("vac/msd oracle small")
    rv = oracle.vac(lat, c["e_scale"], phi[:, 0], *args)
    rm = oracle.msd(lat, c["e_scale"], phi[:, 0], *args)
    _log("vac/msd gpu small")
    d = sysg.upload(phi)
    gv = kp.kpm_vac(sysg, d, *args)[0]
    gm = kp.kpm_msd(sysg, d, *args)[0]
    return c, lat, rv, rm, gv, gm


def test_vac_small_config(loops):
    c, lat, rv, rm, gv, gm = loops
    assert rel_err(gv, rv) < 1e-10


def test_msd_small_config(loops):
    c, lat, rv, rm, gv, gm = loops
    assert np.all(gm[0] == 0)
    assert rel_err(gm, rm) < 1e-10


def test_sigma_small_config(loops):
    """DOS, sigma_GK, sigma_E1, sigma_E2 on an energy grid: device KPM sum +
    library conductivities vs the oracle's reconstruction."""
    c, lat, rv, rm, gv, gm = loops
    es, area, dt = c["e_scale"], lat.area_nm2, SMALL["dt_fs"]
    en = oracle.energies_grid(257, es)
    r_gk = oracle.sigma_gk(oracle.kpm_sum(rv, en, es, area), dt)
    r_e1 = oracle.sigma_e1(oracle.kpm_sum(rm, en, es, area), dt)
    r_e2 = oracle.sigma_e2(oracle.kpm_sum(rm, en, es, area), dt)
    g_gk = kp.kpm_sigma_gk(kp.kpm_kpm_sum(gv, en, es, area), dt)
    g_e1 = kp.kpm_sigma_e1(kp.kpm_kpm_sum(gm, en, es, area), dt)
    g_e2 = kp.kpm_sigma_e2(kp.kpm_kpm_sum(gm, en, es, area), dt)
    for g, r in ((g_gk, r_gk), (g_e1, r_e1), (g_e2, r_e2)):
        assert rel_err(g, r) < 1e-8


def test_dos_device_sum(small):
    c, lat, sysg = small
    phi = phases(c, 1, 3000)
    mu = oracle.moments(lat, c["e_scale"], phi[:, 0], phi[:, 0], 500).real
    en = oracle.energies_grid(1001, c["e_scale"])
    ref = oracle.dos(mu, en, c["e_scale"], lat.area_nm2)
    got = kp.kpm_kpm_sum(mu, en, c["e_scale"], lat.area_nm2)
    assert rel_err(got, ref) < 1e-12


def test_fp32_states_sigma_within_1e3(small):
    c, lat, sys64 = small
    _log("fp32 states small loops")
    sys32 = gpu_system(c, "fp32")
    phi = phases(c, 1, 3000)
    args = (SMALL["n_steps"], SMALL["dt_fs"], SMALL["n_bessel"], SMALL["n_moments"])
    rv = oracle.vac(lat, c["e_scale"], phi[:, 0], *args)
    d = sys32.upload(phi)
    gv = kp.kpm_vac(sys32, d, *args)[0]
    es, area, dt = c["e_scale"], lat.area_nm2, SMALL["dt_fs"]
    en = oracle.energies_grid(257, es)
    r = oracle.sigma_gk(oracle.kpm_sum(rv, en, es, area), dt)
    g = kp.kpm_sigma_gk(kp.kpm_kpm_sum(gv, en, es, area), dt)
    assert rel_err(g, r) < 1e-3


def test_invalid_calls_raise(small):
    c, lat, sysg = small
    d = sysg.upload(phases(c, 1, 3000))
    with pytest.raises(kp.KpmError):
        kp.kpm_evolve(sysg, d, 0.1, 0, 10)          # sign must be +-1
    with pytest.raises(kp.KpmError):
        kp.kpm_evolve(sysg, d, 0.1, 1, 1)           # n_bessel >= 2
    with pytest.raises(kp.KpmError):
        kp.kpm_moments(sysg, d, d, 0)               # n_moments >= 1
    bad = torch.zeros((sysg.n_sites, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(kp.KpmError):
        kp.kpm_moments(sysg, bad, bad, 4)           # n_vec not a power of two


# ------------------------------------------------------------------ launch shapes
@pytest.mark.parametrize("n_vec,precision", [(1, "fp64"), (8, "fp32"), (64, "fp64")])
def test_launch_shapes(n_vec, precision):
    """At a fixed grid every ILP visits each work-group's elements in the same
    order with the same explicit FMAs, so the moments are bit-identical; another
    grid size partitions the inner-product sums differently (rounding only).
    The autotuner keeps one of the candidate shapes."""
    _need_gpu()
    c = recipe("sheet", 100, 50, w=1.0, vac=0.01, seed=2)
    sysg = gpu_system(c, precision)
    default = kp.kpm_get_launch(sysg, n_vec)
    phi = sysg.upload(phases(c, n_vec, 3000))
    first = None
    for g in (2, 16):
        ref = None
        for ilp in (1, 2, 4):
            for nt in (0, 1):
                for cp in (0, 1):
                    kp.kpm_set_launch(sysg, n_vec, g, ilp, nt, cp)
                    mu = kp.kpm_moments(sysg, phi, phi, 40)
                    ref = mu if ref is None else ref
                    assert np.array_equal(mu, ref), (g, ilp, nt, cp)
        first = ref if first is None else first
        assert rel_err(ref, first, float(np.abs(first[:, 0]).max())) < 1e-13
    best = kp.kpm_autotune(sysg, phi, 3)
    if best["steps"] >= 2 and n_vec == 1:       # multi-step candidates of one vector
        assert best["groups_per_cu"] in (1, 2, 3, 4, 6, 8) and best["compact"] == 1
    elif best["steps"] >= 2:                    # several vectors: vector-major strips
        assert best["vectors_per_wave"] == 1 and best["tiled"] == 5 and best["compact"] == 1
        assert best["plane_groups"] in (0, 16, 32, 64, 128) or best == default
    else:
        assert best["steps"] == 1 and best["groups_per_cu"] in (4, 8, 16)
        assert best["tiled"] in (0, 1, 2, 3)
    assert best["ilp"] in (1, 2, 4)
    assert best["streaming"] in (0, 1) and best["compact"] in (0, 1)
    assert kp.kpm_get_launch(sysg, n_vec) == best


@pytest.mark.parametrize("nx,ny,n_vec,precision,tiled", [
    (300, 30, 8, "fp64", 1), (300, 30, 64, "fp32", 1), (600, 16, 1, "fp64", 1),
    (300, 30, 64, "fp64", 1), (1100, 8, 64, "fp32", 2), (1100, 8, 64, "fp64", 3),
    (300, 30, 8, "fp64", 3)])         # chains shorter than two 256-row tiles: row order
def test_tiled_traversal(nx, ny, n_vec, precision, tiled):
    """Strip-by-strip traversal (chains of nx rows, tiles of 64 rows for 8+
    vectors and 256 rows for one; nx is not a multiple of the tile, so the last
    strip is padded): moments, evolution and the VAC agree with row order up to
    the order of the partial sums, and with the oracle; every ILP, streaming
    and neighbour form is bit-identical under the tiled traversal."""
    _need_gpu()
    _log(f"tiled traversal {nx}x{ny} n_vec={n_vec} {precision} tiled={tiled}")
    c = recipe("sheet", nx, ny, w=1.0, vac=0.01, seed=21)
    sysg = gpu_system(c, precision)
    phi = phases(c, n_vec, 3000)
    d = sysg.upload(phi)
    kp.kpm_set_launch(sysg, n_vec, 8, 1, 1, 1, 0)
    row = kp.kpm_moments(sysg, d, d, 60)
    e_row = d.clone()
    kp.kpm_evolve(sysg, e_row, 0.5, 1, 20)
    ref = None
    for ilp in (1, 2, 4):
        for nt in (0, 1):
            for cp in (0, 1):
                kp.kpm_set_launch(sysg, n_vec, 8, ilp, nt, cp, tiled)
                mu = kp.kpm_moments(sysg, d, d, 60)
                ref = mu if ref is None else ref
                assert np.array_equal(mu, ref), (ilp, nt, cp)
    norm = float(np.abs(row[:, 0]).max())
    tol = 1e-13 if precision == "fp64" else 1e-6
    assert rel_err(ref, row, norm) < tol
    e_t = d.clone()
    kp.kpm_evolve(sysg, e_t, 0.5, 1, 20)
    assert rel_err(e_t.cpu().numpy(), e_row.cpu().numpy()) < (1e-13 if precision == "fp64" else 1e-6)
    if precision == "fp64":
        lat = oracle_lattice(c)
        for r in (0, n_vec - 1):
            mo = oracle.moments(lat, c["e_scale"], phi[:, r], phi[:, r], 60)
            assert rel_err(ref[r], mo, np.vdot(phi[:, r], phi[:, r]).real) < 1e-10
        if n_vec <= 8:
            gv = kp.kpm_vac(sysg, d, 2, 0.4, 16, 32)
            rv = oracle.vac(lat, c["e_scale"], phi[:, 0], 2, 0.4, 16, 32)
            assert rel_err(gv[0], rv) < 1e-10


# ------------------------------------------------------------------ Fourier moments (FTM)
@pytest.mark.parametrize("geometry,nx,ny,vac,n_vec", [("sheet", 64, 32, 0.02, 1),
                                                       ("zgnr", 30, 7, 0.0, 2)])
def test_fourier_moments(geometry, nx, ny, vac, n_vec):
    _need_gpu()
    c = recipe(geometry, nx, ny, w=1.0, vac=vac, seed=13)
    lat = oracle_lattice(c)
    sysg = gpu_system(c)
    pl = phases(c, n_vec, 3000)
    pr = phases(c, n_vec, 3500)
    nm, dtau = 24, np.pi * HBAR / c["e_scale"]
    got = kp.kpm_fourier_moments(sysg, sysg.upload(pl), sysg.upload(pr), nm, dtau, 25)
    for r in range(n_vec):
        ref = oracle.fourier_moments(lat, c["e_scale"], pl[:, r], pr[:, r], nm, dtau, 25)
        assert rel_err(got[r], ref, np.linalg.norm(pl[:, r]) * np.linalg.norm(pr[:, r])) < 1e-10


def test_ftm_dos_device_sum(small):
    c, lat, sysg = small
    phi = phases(c, 1, 3000)
    nm, dtau = 60, np.pi * HBAR / c["e_scale"]
    f = oracle.fourier_moments(lat, c["e_scale"], phi[:, 0], phi[:, 0], nm, dtau, 25)
    en = oracle.energies_grid(777, c["e_scale"])
    ref = oracle.ftm_sum(f, en, dtau, lat.area_nm2)
    got = kp.kpm_ftm_sum(f, en, dtau, lat.area_nm2)
    assert rel_err(got, ref) < 1e-12
