"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes from
an independent source -- the paper's printed numbers (tests/golden), the
analytic graphene band structure, dense exact diagonalisation and matrix
exponentials (numpy/scipy), scipy's Bessel routine, the Daleckii-Krein
formula for derivatives of matrix functions, and exact-trace identities.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.special as sps

import kpm_inputs as ki
import oracle
from oracle import HBAR_EV_FS as HBAR

A = oracle.BOND_NM


def _lat(nx, ny, geometry="sheet", w=0.0, vac=0.0, seed=0):
    n = nx * ny
    act = ki.vacancy_mask(n, vac, 2000 + seed) if vac else None
    ons = ki.anderson_onsite(n, w, 1000 + seed)
    return oracle.graphene(nx, ny, geometry, -2.7, ons, act)


def _escale(lat):
    return 1.01 * (3 * 2.7 + np.max(np.abs(lat.onsite)))


def _active_eig(lat, e_scale):
    """Eigenpairs of H~ restricted to the active sites (vacancies removed)."""
    idx = np.flatnonzero(lat.active)
    h = oracle.dense_h(lat)[np.ix_(idx, idx)] / e_scale
    ev, q = np.linalg.eigh(h)
    return idx, ev, q


# --------------------------------------------------------------------------- lattice

@pytest.mark.parametrize("geometry,nx,ny", [("sheet", 8, 4), ("sheet", 12, 6),
                                            ("zgnr", 8, 5), ("agnr", 7, 6)])
def test_lattice_structure(geometry, nx, ny):
    lat = _lat(nx, ny, geometry)
    n = nx * ny
    h = oracle.dense_h(lat)
    assert np.array_equal(h, h.T)
    deg = np.diff(lat.row_ptr)
    if geometry == "sheet":
        assert np.all(deg == 3)
        assert len(lat.col) == 3 * n            # 3N/2 bonds
    else:
        assert set(np.unique(deg)) <= {2, 3}
        # open boundary across the ribbon: one bond lost per edge pair
        lost = nx // 2 if geometry == "zgnr" else ny
        if geometry == "zgnr":
            lost = sum(1 for i in range(nx) if (i + ny - 1) % 2 == 1)
        assert len(lat.col) == 3 * n - 2 * lost
    # bipartite: every bond joins opposite (i + j) parities
    rows = np.repeat(np.arange(n), deg)
    par = lambda s: (s % nx + s // nx) % 2
    assert np.all(par(rows) != par(lat.col))
    assert np.all(lat.hop == -2.7)


def _positions(nx, ny):
    i = np.arange(nx * ny) % nx
    j = np.arange(nx * ny) // nx
    x = i * np.sqrt(3) * A / 2
    y = j * 1.5 * A + np.where((i + j) % 2 == 1, A / 2, 0.0)
    return x, y


@pytest.mark.parametrize("geometry,nx,ny", [("sheet", 8, 4), ("zgnr", 8, 5), ("agnr", 7, 6)])
def test_bond_vectors_are_minimum_image_displacements(geometry, nx, ny):
    lat = _lat(nx, ny, geometry)
    x, y = _positions(nx, ny)
    pos, period = (y, 1.5 * A * ny) if geometry == "agnr" else (x, np.sqrt(3) * A * nx / 2)
    rows = np.repeat(np.arange(lat.n), np.diff(lat.row_ptr))
    d = pos[rows] - pos[lat.col]
    d = (d + period / 2) % period - period / 2           # minimum image
    assert np.allclose(lat.dx, d, atol=1e-14)
    # every bond has length a
    full = np.hypot(*(((u[rows] - u[lat.col]) + p / 2) % p - p / 2
                      for u, p in ((x, np.sqrt(3) * A * nx / 2), (y, 1.5 * A * ny))))
    assert np.allclose(full, A, atol=1e-14)


def test_lengths_match_paper(golden_rows):
    for geometry, nx, ny, what, val, tol in golden_rows("lattice_lengths.txt"):
        lat = oracle.Lattice(int(nx), int(ny), geometry, -2.7, *([None] * 6))
        got = lat.lx_nm if what == "lx" else lat.width_nm
        assert abs(got - float(val)) <= float(tol), (geometry, nx, ny, got)


@pytest.mark.parametrize("nx,ny", [(8, 4), (12, 6), (16, 8)])
def test_pristine_spectrum_is_graphene_band_structure(nx, ny):
    """Periodic sheet: eigenvalues are +-|t| |1 + e^{ik.u} + e^{ik.v}| on the
    k-grid compatible with the supercell (nearest-neighbour graphene bands)."""
    lat = _lat(nx, ny)
    ev = np.linalg.eigvalsh(oracle.dense_h(lat))
    lx, ly = np.sqrt(3) * A * nx / 2, 1.5 * A * ny
    u = np.array([np.sqrt(3) * A / 2, 1.5 * A])
    v = np.array([-np.sqrt(3) * A / 2, 1.5 * A])
    bands = []
    for p in range(nx // 2):
        for q in range(ny):
            k = np.array([2 * np.pi * p / lx, 2 * np.pi * q / ly])
            f = abs(1 + np.exp(1j * k @ u) + np.exp(1j * k @ v))
            bands += [2.7 * f, -2.7 * f]
    assert np.allclose(np.sort(ev), np.sort(bands), atol=1e-12)


def test_vacancies_exact_count_and_removed():
    n = 24 * 12
    act = ki.vacancy_mask(n, 0.05, 7)
    assert int((act == 0).sum()) == round(0.05 * n)
    lat = oracle.graphene(24, 12, "sheet", -2.7, None, act)
    dead = np.flatnonzero(act == 0)
    assert np.all(np.diff(lat.row_ptr)[dead] == 0)
    assert not np.isin(lat.col, dead).any()


# --------------------------------------------------------------------------- moments

@pytest.mark.parametrize("geometry,nx,ny,w,vac", [("sheet", 8, 4, 1.0, 0.0),
                                                  ("sheet", 12, 6, 2.0, 0.1),
                                                  ("zgnr", 8, 5, 0.5, 0.0),
                                                  ("agnr", 7, 6, 1.0, 0.05)])
def test_moments_match_eigendecomposition(geometry, nx, ny, w, vac):
    """C_n = sum_a conj(<a|L>) <a|R> T_n(e_a) with T_n(e) = cos(n arccos e)."""
    lat = _lat(nx, ny, geometry, w, vac, seed=3)
    es = _escale(lat)
    phl = ki.random_phase(lat.n, 1, 3000, lat.active)[:, 0]
    phr = ki.random_phase(lat.n, 1, 3100, lat.active)[:, 0]
    nm = 64
    idx, ev, q = _active_eig(lat, es)
    cl, cr = q.T @ phl[idx], q.T @ phr[idx]
    tn = np.cos(np.outer(np.arange(nm), np.arccos(ev)))
    ref = tn @ (np.conj(cl) * cr)
    got = oracle.moments(lat, es, phl, phr, nm)
    scale = np.linalg.norm(phl) * np.linalg.norm(phr)
    assert np.max(np.abs(got - ref)) / scale < 1e-13
    same = oracle.moments(lat, es, phl, phl, nm)
    assert abs(same[0] - np.count_nonzero(lat.active)) < 1e-12   # <phi|phi> = N
    assert np.max(np.abs(same.imag)) < 1e-12
    assert np.all(np.abs(same.real) <= same[0].real * (1 + 1e-12))


def test_pristine_exact_trace_odd_moments_vanish():
    lat = _lat(8, 4)
    es = _escale(lat)
    tot = np.zeros(9, dtype=complex)
    for k in range(lat.n):
        e = np.zeros(lat.n, complex)
        e[k] = 1.0
        tot += oracle.moments(lat, es, e, e, 9)
    ev = np.linalg.eigvalsh(oracle.dense_h(lat)) / es
    ref = [np.sum(np.cos(m * np.arccos(ev))) for m in range(9)]
    assert np.allclose(tot.real, ref, atol=1e-12)
    assert np.allclose(tot.real[1::2], 0.0, atol=1e-12)


# --------------------------------------------------------------------------- Bessel / U(dt)

@pytest.mark.parametrize("x", [0.0, 1e-3, 0.5, 1.25, np.pi, 3.0494, 3.2170, 10.0, 47.5])
def test_bessel_against_scipy(x):
    m = int(max(60, x + 40))
    got = oracle.bessel_j(m, x)
    ref = sps.jv(np.arange(m), x)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-15)
    assert abs(got[0] + 2 * got[2::2].sum() - 1.0) < 1e-14


def test_bessel_terms_printed_in_paper(golden_rows):
    (x, nterms, acc), = golden_rows("bessel_terms.txt")
    x, nterms, acc = float(x), int(nterms), float(acc)
    j = oracle.bessel_j(nterms + 30, x)
    tail = 2 * np.abs(j[nterms:]).sum()            # neglected terms, |T_m| <= 1
    assert tail < 10 * acc                         # "about 20 terms for 1e-15"
    assert 2 * np.abs(j[nterms - 4:]).sum() > acc  # and clearly fewer do not suffice


def _expm_u(lat, es, t_fs):
    h = oracle.dense_h(lat)
    return sla.expm(-1j * h * t_fs / HBAR)


@pytest.mark.parametrize("geometry,sign", [("sheet", 1), ("sheet", -1), ("zgnr", 1), ("agnr", -1)])
def test_evolve_matches_matrix_exponential(geometry, sign):
    lat = _lat(8, 6, geometry, w=1.0, vac=0.05, seed=5) if geometry != "agnr" else \
        _lat(7, 6, geometry, w=1.0, vac=0.05, seed=5)
    es = _escale(lat)
    phi = ki.random_phase(lat.n, 1, 3000, lat.active)[:, 0]
    dt = 0.5
    got = oracle.evolve(lat, es, phi, dt, sign, 40)
    ref = _expm_u(lat, es, sign * dt) @ phi
    assert np.max(np.abs(got - ref)) < 1e-12
    assert abs(np.vdot(got, got).real - np.vdot(phi, phi).real) < 1e-11
    back = oracle.evolve(lat, es, got, dt, -sign, 40)
    assert np.max(np.abs(back - phi)) < 1e-12


def test_evolve_truncation_is_controlled_by_bessel_tail():
    """Too few terms must show an error of the size of the dropped coefficients."""
    lat = _lat(8, 4, w=1.0)
    es = _escale(lat)
    phi = ki.random_phase(lat.n, 1, 3000)[:, 0]
    dt = 1.0
    x = es * dt / HBAR
    ref = _expm_u(lat, es, dt) @ phi
    for npoly in (8, 12, 16):
        err = np.max(np.abs(oracle.evolve(lat, es, phi, dt, 1, npoly) - ref))
        tail = 2 * np.abs(sps.jv(np.arange(npoly, npoly + 40), x)).sum()
        assert err <= tail * np.abs(phi).sum() + 1e-13
        assert err > 1e-3 * 2 * abs(sps.jv(npoly, x))


# --------------------------------------------------------------------------- [X, U(dt)]

def _divided_difference_u(ev, x):
    """U^{[1]}(e_a, e_b) for U(e) = exp(-i x e), with -i x exp(-i x e) on ties."""
    fa = np.exp(-1j * x * ev)
    d = ev[:, None] - ev[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        dd = (fa[:, None] - fa[None, :]) / d
    tie = np.abs(d) < 1e-9
    dd[tie] = (-1j * x * np.exp(-1j * x * (ev[:, None] + 0 * ev[None, :])))[tie]
    return dd


@pytest.mark.parametrize("geometry", ["sheet", "zgnr", "agnr"])
def test_commutator_propagator_daleckii_krein(geometry):
    """[X, U(dt)] is the derivation generated by D = [X, H~] applied to U:
    in the eigenbasis of H~ its entries are U^{[1]}(e_a, e_b) (Q^T D Q)_ab."""
    lat = _lat(8, 6, geometry, w=1.0, seed=9) if geometry != "agnr" else _lat(7, 6, geometry, w=1.0, seed=9)
    es = _escale(lat)
    phi = ki.random_phase(lat.n, 1, 3000)[:, 0]
    dt = 0.4
    x = es * dt / HBAR
    ev, q = np.linalg.eigh(oracle.dense_h(lat) / es)
    dq = q.T @ (oracle.dense_d(lat) / es) @ q
    ref = q @ ((_divided_difference_u(ev, x) * dq) @ (q.T @ phi))
    outx, outu = oracle.evolve_x(lat, es, phi, dt, 40)
    assert np.max(np.abs(outx - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(outu - _expm_u(lat, es, dt) @ phi)) < 1e-12


def test_commutator_is_xu_minus_ux_without_wrap():
    """Away from any periodic wrap the derivation is the plain commutator with
    the position operator: on an AGNR (transport along y), a state confined to
    the middle of a long ribbon gives [X, U] phi = (X U - U X) phi with
    absolute y positions, since nothing reaches the wrap within dt."""
    lat = _lat(6, 40, "agnr", w=0.5, seed=2)
    es = _escale(lat)
    _, y = _positions(6, 40)
    # a state localised in the middle of the ribbon
    phi = np.zeros(lat.n, complex)
    mid = (np.arange(lat.n) // 6 >= 18) & (np.arange(lat.n) // 6 < 22)
    phi[mid] = ki.random_phase(int(mid.sum()), 1, 3000)[:, 0]
    dt = 0.2
    xop = np.diag(y)
    u = _expm_u(lat, es, dt)
    ref = (xop @ u - u @ xop) @ phi
    outx, _ = oracle.evolve_x(lat, es, phi, dt, 40)
    assert np.max(np.abs(outx - ref)) < 1e-10


# --------------------------------------------------------------------------- VAC and MSD

def test_vac_matches_direct_evaluation():
    lat = _lat(8, 4, w=1.0, seed=4)
    es = _escale(lat)
    phi = ki.random_phase(lat.n, 1, 3000)[:, 0]
    dt, steps, nm = 0.3, 3, 24
    got = oracle.vac(lat, es, phi, steps, dt, 40, nm)
    v = -1j * oracle.dense_d(lat) / HBAR                 # V = (i/hbar)[H, X]
    ev, q = np.linalg.eigh(oracle.dense_h(lat) / es)
    tn = np.cos(np.outer(np.arange(nm), np.arccos(ev)))
    for k in range(steps + 1):
        ud = _expm_u(lat, es, -k * dt)                   # U^dagger(t_k)
        left = v @ (ud @ phi)
        right = ud @ (v @ phi)
        ref = tn @ (np.conj(q.T @ left) * (q.T @ right))
        assert np.allclose(got[k], ref.real, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_msd_matches_direct_commutator():
    lat = _lat(8, 4, w=1.0, seed=6)
    es = _escale(lat)
    phi = ki.random_phase(lat.n, 1, 3000)[:, 0]
    dt, steps, nm = 0.25, 4, 24
    got = oracle.msd(lat, es, phi, steps, dt, 40, nm)
    ev, q = np.linalg.eigh(oracle.dense_h(lat) / es)
    dq = q.T @ (oracle.dense_d(lat) / es) @ q
    tn = np.cos(np.outer(np.arange(nm), np.arccos(ev)))
    assert np.all(got[0] == 0.0)
    for k in range(1, steps + 1):
        x = es * k * dt / HBAR
        y = q @ ((_divided_difference_u(ev, x) * dq) @ (q.T @ phi))
        c = q.T @ y
        ref = tn @ (np.abs(c) ** 2)
        assert np.allclose(got[k], ref, rtol=0, atol=1e-11 * ref.max())


def test_msd_second_derivative_is_twice_vac_exact_trace():
    """Under the exact trace MSD_n''(t) = 2 VAC_n(t) for every moment n."""
    lat = _lat(8, 4, w=1.0, seed=8)
    es = _escale(lat)
    h, nm = 2e-3, 8
    msd = np.zeros((3, nm))
    vac = np.zeros((3, nm))
    for k in range(lat.n):
        e = np.zeros(lat.n, complex)
        e[k] = 1.0
        msd += oracle.msd(lat, es, e, 2, h, 30, nm)
        vac += oracle.vac(lat, es, e, 2, h, 30, nm)
    d2 = (msd[2] - 2 * msd[1] + msd[0]) / h ** 2
    assert np.allclose(d2, 2 * vac[1], rtol=2e-3, atol=2e-3 * np.abs(vac[1]).max())


# --------------------------------------------------------------------------- reconstruction

def test_jackson_is_normalised_autocorrelation():
    """Jackson's factors are the autocorrelation of a_v = sin(pi (v+1)/(N+1))."""
    for n in (5, 64, 500):
        a = np.sin(np.pi * (np.arange(n) + 1) / (n + 1))
        ref = np.array([a[: n - k] @ a[k:] for k in range(n)]) / (a @ a)
        assert np.allclose(oracle.jackson(n), ref, atol=1e-13)


def test_kpm_sum_normalisation_and_positivity():
    """With exact-trace moments the reconstructed DOS is >= 0 and integrates to
    2 N / Omega; its first Chebyshev moment is g_1 times the exact one."""
    lat = _lat(8, 4, w=1.0, seed=1)
    es = _escale(lat)
    ev = np.linalg.eigvalsh(oracle.dense_h(lat)) / es
    nm = 40
    mu = np.array([np.sum(np.cos(m * np.arccos(ev))) for m in range(nm)])
    kq = 2000                                           # Chebyshev-Gauss nodes
    th = np.pi * (np.arange(kq) + 0.5) / kq
    e_ev = np.cos(th) * es
    rho = oracle.dos(mu, e_ev, es, lat.area_nm2)
    assert np.all(rho > -1e-12)
    # int f(E) dE = E_s int f(eps) deps, and int g(eps)/sqrt(1-eps^2) deps = (pi/K) sum g(cos th)
    w = np.sqrt(1 - np.cos(th) ** 2) * np.pi / kq * es
    assert abs(np.sum(rho * w) - 2 * lat.n / lat.area_nm2) < 1e-10 * lat.n / lat.area_nm2
    first = np.sum(rho * w * np.cos(th)) * lat.area_nm2 / 2
    assert abs(first - oracle.jackson(nm)[1] * mu[1]) < 1e-10


def test_running_conductivity_forms():
    dt = 0.1
    t = dt * np.arange(200)
    v2 = 0.7
    rho_msd = (v2 * t ** 2)[:, None]
    e1 = oracle.sigma_e1(rho_msd, dt)
    e2 = oracle.sigma_e2(rho_msd, dt)
    assert np.allclose(e1[1:-1, 0], np.pi * HBAR * 2 * v2 * t[1:-1], rtol=1e-12)
    ratio = float([r for r in __import__("conftest").golden("ballistic_ratio.txt")][0][1])
    assert np.allclose(e2[5:-1, 0] / e1[5:-1, 0], ratio, rtol=1e-12)
    # diffusive: MSD = D t  ->  E1 = E2 = pi hbar D
    dd = 3.0
    e1d = oracle.sigma_e1((dd * t)[:, None], dt)
    e2d = oracle.sigma_e2((dd * t)[:, None], dt)
    assert np.allclose(e1d[:, 0], np.pi * HBAR * dd, rtol=1e-12)
    assert np.allclose(e2d[1:, 0], np.pi * HBAR * dd, rtol=1e-12)
    # GK of a cosine VAC: the trapezoid sum of cos(w t) is sin(w t)/w times
    # (w dt/2)/tan(w dt/2) exactly
    w = 0.5
    gk = oracle.sigma_gk(np.cos(w * t)[:, None], dt)
    corr = (w * dt / 2) / np.tan(w * dt / 2)
    assert np.allclose(gk[:, 0], 2 * np.pi * HBAR * np.sin(w * t) / w * corr, atol=1e-12)


def test_einstein_equals_green_kubo_exact_trace():
    """sigma_E1 from the MSD equals sigma_GK from the VAC (Sec. 5.2) when both
    use the exact trace; the residual is the time-discretisation error."""
    lat = _lat(8, 4, w=1.0, seed=8)
    es = _escale(lat)
    dt, steps, nm = 0.02, 40, 16
    msd = np.zeros((steps + 1, nm))
    vac = np.zeros((steps + 1, nm))
    for k in range(lat.n):
        e = np.zeros(lat.n, complex)
        e[k] = 1.0
        msd += oracle.msd(lat, es, e, steps, dt, 30, nm)
        vac += oracle.vac(lat, es, e, steps, dt, 30, nm)
    en = np.array([-3.0, -1.0, 0.5, 2.0])
    rm = oracle.kpm_sum(msd, en, es, lat.area_nm2)
    rv = oracle.kpm_sum(vac, en, es, lat.area_nm2)
    e1 = oracle.sigma_e1(rm, dt)
    gk = oracle.sigma_gk(rv, dt)
    scale = np.abs(gk).max()
    assert np.max(np.abs(e1[1:-1] - gk[1:-1])) < 2e-3 * scale


# --------------------------------------------------------------------------- Fourier moments

def test_fourier_moments_match_eigendecomposition():
    """F_n = sum_a conj(<a|L>) <a|R> exp(-i e_a x n), x = E_s dtau / hbar (Eq. 25)."""
    lat = _lat(12, 6, w=1.0, vac=0.05, seed=12)
    es = _escale(lat)
    phl = ki.random_phase(lat.n, 1, 3000, lat.active)[:, 0]
    phr = ki.random_phase(lat.n, 1, 3100, lat.active)[:, 0]
    nm, dtau = 12, np.pi * HBAR / es          # Bessel argument pi (Sec. 4.2)
    got = oracle.fourier_moments(lat, es, phl, phr, nm, dtau, 40)
    idx, ev, q = _active_eig(lat, es)
    cl, cr = q.T @ phl[idx], q.T @ phr[idx]
    n = np.arange(-nm, nm + 1)
    ref = np.exp(-1j * np.outer(n, ev) * np.pi) @ (np.conj(cl) * cr)
    assert np.max(np.abs(got - ref)) < 1e-11 * np.linalg.norm(phl) * np.linalg.norm(phr)
    same = oracle.fourier_moments(lat, es, phl, phl, nm, dtau, 40)
    assert np.allclose(same[::-1], np.conj(same), atol=1e-10)     # F_-n = conj(F_n)


def test_hanning_window_and_ftm_normalisation():
    """The Hanning-windowed Fourier DOS integrates to 2N/Omega over one period of
    the energy axis (only n = 0 survives), and w_0 = 1 (Eq. 28)."""
    lat = _lat(8, 4, w=1.0, seed=1)
    es = _escale(lat)
    nm = 30
    dtau = np.pi * HBAR / es                   # period of E: 2 pi hbar / dtau = 2 E_s
    ftot = np.zeros(2 * nm + 1, complex)
    for k in range(lat.n):
        e = np.zeros(lat.n, complex)
        e[k] = 1.0
        ftot += oracle.fourier_moments(lat, es, e, e, nm, dtau, 40)
    w = oracle.hanning(nm)
    assert w[nm] == 1.0 and np.allclose(w, w[::-1])
    kq = 4 * nm + 7                            # uniform periodic grid: exact for |n| <= nm
    en = -es + 2 * es * np.arange(kq) / kq
    rho = oracle.ftm_sum(ftot, en, dtau, lat.area_nm2)
    integral = np.sum(rho) * 2 * es / kq
    assert abs(integral - 2 * lat.n / lat.area_nm2) < 1e-10 * lat.n / lat.area_nm2


def test_ftm_and_kpm_dos_agree():
    """Sec. 4.2: the FTM and KPM give consistent DOS curves; with the exact
    trace the integrated densities of states agree across the band."""
    lat = _lat(16, 8, w=1.0, seed=2)
    es = _escale(lat)
    nm_k, nm_f = 300, 150
    dtau = np.pi * HBAR / es
    mu = np.zeros(nm_k)
    ftot = np.zeros(2 * nm_f + 1, complex)
    ev = np.linalg.eigvalsh(oracle.dense_h(lat)) / es
    mu = np.array([np.sum(np.cos(m * np.arccos(ev))) for m in range(nm_k)])
    n = np.arange(-nm_f, nm_f + 1)
    ftot = np.exp(-1j * np.outer(n, ev) * np.pi).sum(axis=1)   # exact-trace F_n
    en = np.linspace(-0.95 * es, 0.95 * es, 4001)
    rk = oracle.dos(mu, en, es, lat.area_nm2)
    rf = oracle.ftm_sum(ftot, en, dtau, lat.area_nm2)
    ck = np.cumsum(rk) * (en[1] - en[0]) * lat.area_nm2 / 2
    cf = np.cumsum(rf) * (en[1] - en[0]) * lat.area_nm2 / 2
    assert np.max(np.abs(ck - cf)) < 0.02 * lat.n


def test_threaded_oracle_equals_serial_bit_for_bit():
    """The oracle's row loops may run on several threads; every value is then
    computed by the same operations in the same order and the inner products
    stay serial, so moments, propagators and both time loops are bit-identical
    for 1 and 4 threads (on a lattice long enough for the loops to split)."""
    nx, ny = 256, 160
    n = nx * ny
    act = ki.vacancy_mask(n, 0.02, 2000)
    lat = oracle.graphene(nx, ny, "sheet", -2.7, ki.anderson_onsite(n, 1.0, 1000), act)
    es = 1.01 * (3 * 2.7 + 0.5)
    phi = ki.random_phase(n, 1, 3000, act)[:, 0]
    psi = ki.random_phase(n, 1, 3001, act)[:, 0]
    prev = oracle.set_threads()
    out = {}
    try:
        for th in (1, 4):
            oracle.set_threads(th)
            out[th] = (oracle.moments(lat, es, psi, phi, 90),
                       oracle.evolve(lat, es, phi, 0.3, -1, 17),
                       *oracle.evolve_x(lat, es, phi, 0.3, 17),
                       oracle.vac(lat, es, phi, 2, 0.3, 17, 40),
                       oracle.msd(lat, es, phi, 2, 0.3, 17, 40),
                       oracle.fourier_moments(lat, es, psi, phi, 3, 0.2, 12))
    finally:
        oracle.set_threads(prev)
    for a, b in zip(out[1], out[4]):
        assert np.array_equal(a, b)
