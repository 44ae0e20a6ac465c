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


@pytest.mark.parametrize("case", ["asymmetric", "out_of_range", "gershgorin", "width"])
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
    d, keep = _desc(nbr, es)
    if case == "width":
        d.width = 9
    h = C.c_void_p()
    st = kp.lib().kpm_system_create(C.byref(d), 0, 0, None, C.byref(h))
    assert st == 1, kp.lib().kpm_last_error()
    assert kp.lib().kpm_last_error()


def test_running_conductivities_match_oracle():
    rng = np.random.default_rng(0)
    rows = rng.standard_normal((17, 5))
    dt = 0.24
    assert np.allclose(kp.kpm_sigma_gk(rows, dt), oracle.sigma_gk(rows, dt), rtol=1e-13, atol=1e-14)
    assert np.allclose(kp.kpm_sigma_e1(rows, dt), oracle.sigma_e1(rows, dt), rtol=1e-13, atol=1e-14)
    assert np.allclose(kp.kpm_sigma_e2(rows, dt), oracle.sigma_e2(rows, dt), rtol=1e-13, atol=1e-14)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(kb, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(kb, "_lib", None)
    with pytest.raises(ImportError):
        kb.lib()
