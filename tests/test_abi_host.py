"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-only entry points (lattice builder, descriptor validation,
running conductivities) agree with the oracle.  No GPU compute here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import kpm_inputs as ki
import oracle
import paper_1307_0288_amd as kp
from paper_1307_0288_amd import kpm as kb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "kpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"\b(kpm_[a-z0-9_]+)\s*\(", src))


def test_library_exports_every_declared_symbol():
    lib = kp.lib()
    declared = _declared()
    assert declared == set(kp.ABI_SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.kpm_version()


@pytest.mark.parametrize("geometry,nx,ny,vac", [("sheet", 8, 4, 0.0), ("sheet", 24, 12, 0.05),
                                                ("zgnr", 10, 7, 0.0), ("agnr", 9, 8, 0.03)])
def test_graphene_builder_matches_oracle_lattice(geometry, nx, ny, vac):
    n = nx * ny
    act = ki.vacancy_mask(n, vac, 2000) if vac else None
    nbr, dx = kp.kpm_build_graphene(nx, ny, geometry, act)
    lat = oracle.graphene(nx, ny, geometry, -2.7, None, act)
    h = np.zeros((n, n))
    d = np.zeros((n, n))
    for k in range(3):
        for s in range(n):
            m = nbr[k, s]
            if m >= 0:
                h[s, m] += -2.7
                d[s, m] += dx[k, s]
    assert np.array_equal(h, oracle.dense_h(lat))
    dref = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(lat.row_ptr))
    dref[rows, lat.col] = lat.dx
    assert np.allclose(d, dref, atol=1e-15)


def test_builder_rejects_bad_sizes():
    with pytest.raises(kp.KpmError):
        kp.kpm_build_graphene(7, 4, "sheet")          # odd periodic x
    with pytest.raises(kp.KpmError):
        kp.kpm_build_graphene(8, 3, "agnr")           # odd periodic y


def _desc(nbr, e_scale, onsite=None):
    keep = [nbr]
    d = kb._Desc(nbr.shape[1], nbr.shape[0], nbr.ctypes.data_as(C.POINTER(C.c_int32)), None,
                 -2.7, None if onsite is None else kb._dp(onsite), None, None, e_scale)
    return d, keep


@pytest.mark.parametrize("case", ["asymmetric", "out_of_range", "gershgorin", "width",
                                  "too_many_sites", "no_sites", "nan_scale", "null_nbr",
                                  "nan_onsite"])
def test_create_validates_before_touching_a_device(case):
    nbr, _ = kp.kpm_build_graphene(8, 4)
    nbr = nbr.copy()
    es = 8.2
    if case == "asymmetric":
        nbr[2, 5] = -1
    elif case == "out_of_range":
        nbr[0, 3] = 10_000
    elif case == "gershgorin":
        es = 8.0                                      # 3 * 2.7 = 8.1 > 8.0
    elif case == "nan_scale":
        es = float("nan")
    ons = None
    if case == "nan_onsite":
        ons = np.zeros(32)
        ons[7] = np.nan
    d, keep = _desc(nbr, es, ons)
    if case == "width":
        d.width = 9
    elif case == "too_many_sites":
        d.n_sites = 2 ** 31                           # rejected before the arrays are read
    elif case == "no_sites":
        d.n_sites = 0
    elif case == "null_nbr":
        d.nbr = None
    h = C.c_void_p()
    st = kp.lib().kpm_system_create(C.byref(d), 0, 0, None, C.byref(h))
    assert st == 1, kp.lib().kpm_last_error()
    msg = kp.lib().kpm_last_error()
    assert msg
    # the host-only check applies the same rules and reports the same message
    bound = C.c_double(-1.0)
    assert kp.lib().kpm_validate(C.byref(d), C.byref(bound)) == 1
    assert kp.lib().kpm_last_error() == msg


@pytest.mark.parametrize("geometry", ["sheet", "zgnr", "agnr"])
def test_validate_reports_gershgorin_bound(geometry):
    """Full coordination in a periodic sheet: 3|t| + max|H_nn|; ribbon edges and
    vacancies lower some rows but a bulk row still has three bonds."""
    n = 12 * 10
    ons = ki.anderson_onsite(n, 1.2, 3)
    act = ki.vacancy_mask(n, 0.03, 4)
    nbr, dx = kp.kpm_build_graphene(12, 10, geometry, act)
    bound = kp.kpm_validate(nbr, dx=dx, onsite=ons, active=act)
    rows = [abs(ons[s]) * act[s] + 2.7 * np.sum(nbr[:, s] >= 0) for s in range(n)]
    assert bound == pytest.approx(max(rows), rel=1e-15)
    assert kp.kpm_validate(nbr, e_scale=bound, dx=dx, onsite=ons, active=act) == bound
    with pytest.raises(kp.KpmError):
        kp.kpm_validate(nbr, e_scale=0.999 * bound, dx=dx, onsite=ons, active=act)


def test_running_conductivities_match_oracle():
    rng = np.random.default_rng(0)
    rows = rng.standard_normal((17, 5))
    dt = 0.24
    assert np.allclose(kp.kpm_sigma_gk(rows, dt), oracle.sigma_gk(rows, dt), rtol=1e-13, atol=1e-14)
    assert np.allclose(kp.kpm_sigma_e1(rows, dt), oracle.sigma_e1(rows, dt), rtol=1e-13, atol=1e-14)
    assert np.allclose(kp.kpm_sigma_e2(rows, dt), oracle.sigma_e2(rows, dt), rtol=1e-13, atol=1e-14)


def _same(a, b, rtol=1e-13, atol=1e-14):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape
    assert np.array_equal(np.isnan(a), np.isnan(b))
    m = ~np.isnan(a)
    assert np.allclose(a[m], b[m], rtol=rtol, atol=atol)


def test_transport_quantities_match_oracle():
    """Host transport functions of the library (Eq. 50-55, 60) against the
    oracle on random data, NaN pattern included (rho = 0 and a negative MSD
    give NaN lengths)."""
    from oracle import transport as tr
    rng = np.random.default_rng(1)
    nt, ne, dt, w = 13, 7, 0.3, 2.5
    rho = rng.uniform(0.01, 0.1, ne)
    rho[3] = 0.0
    rm = rng.uniform(0.0, 5.0, (nt, ne)) * rho
    rm[0] = 0.0
    rm[5, 1] = -0.2
    sig = rng.standard_normal((nt, ne))
    lg_lib, lg_orc = kp.kpm_length(rm, rho), tr.length(rm, rho)
    _same(lg_lib, lg_orc)
    _same(kp.kpm_conductance(sig, lg_orc, w), tr.conductance(sig, lg_orc, w))
    _same(kp.kpm_ballistic_conductance(rm, rho, dt, w), tr.ballistic_conductance(rm, rho, dt, w))
    _same(kp.kpm_sigma_sc_max(sig), tr.sigma_sc_max(sig))
    _same(kp.kpm_sigma_sc_average(sig, 2, 9), tr.sigma_sc_average(sig, 2, 9))
    g = rng.uniform(0.01, 3.0, (6, ne))
    _same(kp.kpm_typical_conductance(g), tr.typical_conductance(g))


@pytest.mark.parametrize("m,n,sweeps", [(2, 2, 8), (2, 2, 0), (3, 1, 4), (1, 0, 0)])
def test_pade_matches_oracle(m, n, sweeps):
    from oracle import transport as tr
    rng = np.random.default_rng(2)
    t = np.linspace(50.0, 3000.0, 120)
    y = 300.0 * t ** 2 / (2e5 + t ** 2) * (1 + 1e-3 * rng.standard_normal(t.shape))
    a_l, b_l = kp.kpm_pade_fit(t, y, m, n, sweeps)
    a_o, b_o = tr.pade_fit(t, y, m, n, sweeps)
    v_l, d_l = kp.kpm_pade_eval(a_l, b_l, t)
    v_o, d_o = tr.pade_eval(a_o, b_o, t)
    # two independent least-squares solvers: agreement to the conditioning of the fit
    assert np.allclose(v_l, v_o, rtol=1e-8, atol=1e-10 * np.abs(v_o).max())
    assert np.allclose(d_l, d_o, rtol=1e-6, atol=1e-8 * np.abs(d_o).max())
    # evaluation alone, same coefficients
    v2, d2 = kp.kpm_pade_eval(a_o, b_o, t)
    assert np.allclose(v2, v_o, rtol=1e-13) and np.allclose(d2, d_o, rtol=1e-12, atol=1e-15)


def test_transport_rejects_bad_arguments():
    with pytest.raises(kp.KpmError):
        kp.kpm_sigma_sc_average(np.zeros((5, 2)), 3, 3)
    with pytest.raises(kp.KpmError):
        kp.kpm_sigma_sc_max(np.zeros((1, 2)))
    with pytest.raises(kp.KpmError):
        kp.kpm_pade_fit(np.arange(3.0), np.arange(3.0), 2, 2)      # too few points
    with pytest.raises(kp.KpmError):
        kp.kpm_typical_conductance(np.array([[1.0, -1.0]]))
    with pytest.raises(kp.KpmError):
        kp.kpm_conductance(np.ones((2, 2)), np.ones((2, 2)), 0.0)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(kb, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(kb, "_lib", None)
    with pytest.raises(ImportError):
        kb.lib()


def test_learned_features_match_oracle():
    from oracle import learned as ln
    rng = np.random.default_rng(4)
    mu = rng.uniform(-1, 1, (3, 2, 40))
    mu[:, :, 0] = rng.uniform(50, 60, (3, 2))
    c = rng.uniform(-1, 1, (3, 2, 40))
    c[:, :, 0] = rng.uniform(500, 600, (3, 2))
    x = kp.kpm_learned_features(mu, c, 16)
    ref = ln.features(mu, c, 16)
    assert x.dtype == np.float32 and x.shape == (3, 33)
    assert np.allclose(x, ref, rtol=2e-7, atol=1e-7)
    with pytest.raises(kp.KpmError):
        kp.kpm_learned_features(mu, c, 41)


ENV_KEYS = ("KPM_GROUPS_PER_CU", "KPM_ILP", "KPM_STREAMING", "KPM_COMPACT_LAUNCH", "KPM_TILED",
            "KPM_STEPS")


def _valid_shape(l):
    """The shapes kernels exist for (kpm_set_launch accepts exactly these)."""
    return (1 <= l["groups_per_cu"] <= 32 and l["ilp"] in (1, 2, 4) and l["streaming"] in (0, 1)
            and l["compact"] in (0, 1) and 0 <= l["tiled"] <= (5 if l["steps"] > 1 else 3)
            and 1 <= l["steps"] <= (8 if l["tiled"] >= 3 else 4))


@pytest.mark.parametrize("tiled", [None, "0", "1", "2", "3", "4", "5", "9", "-1"])
@pytest.mark.parametrize("steps", [None, "1", "2", "3", "4", "5", "8", "12"])
def test_environment_overrides_give_valid_shapes(monkeypatch, tiled, steps):
    """Every combination of KPM_TILED and KPM_STEPS (with the other overrides
    set too) yields a shape the multi-step kernels exist for: a traversal
    below the strips never keeps more than 4 steps."""
    for k in ENV_KEYS:
        monkeypatch.delenv(k, raising=False)
    if tiled is not None:
        monkeypatch.setenv("KPM_TILED", tiled)
    if steps is not None:
        monkeypatch.setenv("KPM_STEPS", steps)
    monkeypatch.setenv("KPM_GROUPS_PER_CU", "3")
    for n_vec in (1, 2, 8, 64):
        for prec in ("fp64", "fp32"):
            l = kp.kpm_default_launch(n_vec, prec)
            assert _valid_shape(l), (n_vec, prec, l)
            assert l["groups_per_cu"] == 3
            if steps is not None:
                want = max(1, min(8, int(steps)))
                if tiled is not None and int(tiled) < 3 and 4 < want:
                    assert l["steps"] == want and l["tiled"] == 5    # steps select the strips
                elif want <= 4 or l["tiled"] >= 3:
                    assert l["steps"] == want
            if tiled is not None and steps is None and int(tiled) < 3:
                assert l["tiled"] == max(0, int(tiled)) and l["steps"] <= 4


def test_default_shapes_without_overrides(monkeypatch):
    for k in ENV_KEYS:
        monkeypatch.delenv(k, raising=False)
    one = kp.kpm_default_launch(1)
    assert one == dict(groups_per_cu=2, ilp=1, streaming=0, compact=1, tiled=5, steps=8)
    assert kp.kpm_default_launch(64, "fp32")["steps"] == 1
    with pytest.raises(kp.KpmError):
        kp.kpm_default_launch(3)
