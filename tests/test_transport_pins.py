"""Pins of the transport post-processing (Sec. 5) in the oracle: quantised
ballistic conductance of pristine nanoribbons (Eq. 50-52, Sec. 5.1), the
confinement of the length under open boundaries (Sec. 5.1), and closed forms
of sigma_sc (Eq. 53, 55), the Pade fit (Eq. 58) and G_typ (Eq. 60).

The ribbons use the exact trace: for a translation-invariant pristine ribbon
the unit vectors of one translation cell, weighted by the number of cells,
give the trace over all sites (no stochastic error).  In the ballistic regime
Delta X^2 = v^2 t^2, and with one open subband per direction the two
crossings +-k have equal speed, so G = (W/L) sigma_E1 = 2 e^2/h exactly in
the continuum limit (spin-degenerate single channel per direction).
"""
import numpy as np
import pytest

import oracle
from oracle import transport as tr
from oracle.core import Lattice
from cases import cell_trace_states

HBAR = oracle.HBAR_EV_FS
ES = 1.01 * 3 * 2.7


def _ribbon_transport(geometry, nx, ny, nm, n_steps, dt, nb, energies):
    lat = oracle.graphene(nx, ny, geometry, -2.7)
    phi, cells = cell_trace_states(geometry, nx, ny)
    mu = np.zeros(nm)
    ms = np.zeros((n_steps + 1, nm))
    for c in range(phi.shape[1]):
        mu += oracle.moments(lat, ES, phi[:, c], phi[:, c], nm).real
        ms += oracle.msd(lat, ES, phi[:, c], n_steps, dt, nb, nm)
    mu *= cells
    ms *= cells
    rho = oracle.dos(mu, energies, ES, lat.area_nm2)
    rm = oracle.kpm_sum(ms, energies, ES, lat.area_nm2)
    s1 = oracle.sigma_e1(rm, dt)
    lg = tr.length(rm, rho)
    g = tr.conductance(s1, lg, lat.width_nm)
    gb = tr.ballistic_conductance(rm, rho, dt, lat.width_nm)
    return lat, rho, rm, g, gb


def test_quantised_ballistic_conductance_zgnr():
    """Pristine ZGNR, 4 zigzag chains, periodic along x (1024 sites per chain):
    G(E) = 2 e^2/h on the first plateau at every interior time point."""
    en = np.array([-1.5, -1.0, -0.5, 0.5, 1.0, 1.5])
    lat, rho, rm, g, gb = _ribbon_transport("zgnr", 1024, 4, 400, 10, 2.0, 40, en)
    # past the first few fs (interband terms of the MSD fade relative to v^2 t^2),
    # at centred-difference time points
    inner = g[4:-1]
    assert np.max(np.abs(inner - 2.0)) < 0.005, inner
    # Eq. 52 (ballistic form) gives the same plateau
    assert np.max(np.abs(gb[4:] - 2.0)) < 0.01     # v^2 = MSD / t^2 keeps the interband offset / t^2
    # symmetric spectrum of the bipartite lattice
    assert np.allclose(g[5], g[5][::-1], rtol=1e-8)


def test_quantised_ballistic_conductance_agnr():
    """Pristine AGNR, periodic along the transport axis y.  5 dimer lines
    (metallic): G = 2 e^2/h around E = 0.  4 dimer lines (semiconducting):
    G = 0 in the gap, then the plateaus 2 and 4 e^2/h."""
    en = np.array([-1.0, -0.5, 0.0, 0.5, 1.0])
    _, _, _, g, _ = _ribbon_transport("agnr", 5, 1024, 400, 10, 2.0, 40, en)
    assert np.max(np.abs(g[4:-1] - 2.0)) < 0.005, g[5]
    en = np.array([0.0, 0.25, 1.375, 2.0])
    _, _, _, g, _ = _ribbon_transport("agnr", 4, 1024, 400, 10, 2.0, 40, en)
    mid = g[5]
    assert abs(mid[0]) < 0.01 and abs(mid[1]) < 0.01, mid
    assert abs(mid[2] - 2.0) < 0.02, mid
    assert abs(mid[3] - 4.0) < 0.03, mid


def _open_along_x(lat):
    """The same sheet with the bonds that wrap around the x boundary removed
    (open boundary along the transport axis); remaining bonds keep their
    displacement, which is then the absolute-position difference."""
    rp, col, hop, dx = [0], [], [], []
    for r in range(lat.n):
        for e in range(lat.row_ptr[r], lat.row_ptr[r + 1]):
            c = lat.col[e]
            if abs(r % lat.nx - c % lat.nx) > 1:
                continue
            col.append(c)
            hop.append(lat.hop[e])
            dx.append(lat.dx[e])
        rp.append(len(col))
    return Lattice(lat.nx, lat.ny, lat.geometry, lat.t_ev, np.array(rp, np.int64),
                   np.array(col, np.int64), np.array(hop), np.array(dx), lat.onsite.copy(),
                   lat.active.copy())


def test_length_periodic_vs_open_boundary():
    """Sec. 5.1: with periodic boundaries along the transport direction the
    length L = 2 sqrt(Delta X^2) keeps growing (ballistic, L = 2 v t); with an
    open boundary it is confined to about the sample length."""
    nx, ny, nm, ns, dt, nb = 32, 4, 200, 40, 1.0, 40
    per = oracle.graphene(nx, ny, "sheet", -2.7)
    opn = _open_along_x(per)
    en = np.array([-1.0, -0.5, 0.5, 1.0])
    cells = ny // 2
    out = {}
    for name, lat in (("periodic", per), ("open", opn)):
        mu = np.zeros(nm)
        ms = np.zeros((ns + 1, nm))
        for j in (0, 1):
            for i in range(nx):
                e = np.zeros(lat.n, complex)
                e[j * nx + i] = 1.0
                mu += oracle.moments(lat, ES, e, e, nm).real
                ms += oracle.msd(lat, ES, e, ns, dt, nb, nm)
        rho = oracle.dos(mu * cells, en, ES, lat.area_nm2)
        out[name] = tr.length(oracle.kpm_sum(ms * cells, en, ES, lat.area_nm2), rho)
    lx = per.lx_nm
    assert np.all(out["periodic"][-1] > 4 * lx)
    # linear growth: L(t) / t nearly constant at late times
    slope = out["periodic"][-1] / out["periodic"][ns // 2]
    assert np.all(np.abs(slope - 2.0) < 0.05)
    # open: bounded by the sample (the paper: the largest length is the sample
    # length; here within 25 % on a 32-site-wide sample, where Delta X^2 <= L_x^2
    # is the strict bound, i.e. L <= 2 L_x)
    top = np.nanmax(out["open"], axis=0)
    assert np.all(top < 1.25 * lx) and np.all(top > 0.9 * lx), top / lx
    assert np.all(out["open"][-1] < 1.25 * lx)


def test_length_and_ballistic_closed_forms():
    """Delta X^2 = v^2 t^2 gives L = 2 v t, sigma_E2 = sigma_E1 / 2 at interior
    points, and G = (W/L) sigma_E1 = pi hbar W rho v (Eq. 51 = Eq. 52)."""
    dt, v, rho, w = 0.5, np.array([0.3, 0.8]), np.array([0.02, 0.05]), 3.0
    t = dt * np.arange(12)
    rm = rho * (v * t[:, None]) ** 2
    lg = tr.length(rm, rho)
    assert np.allclose(lg, 2 * v * t[:, None], rtol=1e-14, atol=1e-14)
    s1 = oracle.sigma_e1(rm, dt)
    s2 = oracle.sigma_e2(rm, dt)
    assert np.allclose(s2[1:-1], 0.5 * s1[1:-1], rtol=1e-12)
    g = tr.conductance(s1, lg, w)
    assert np.all(np.isnan(g[0]))
    assert np.allclose(g[1:-1], np.pi * HBAR * w * rho * v, rtol=1e-12)
    gb = tr.ballistic_conductance(rm, rho, dt, w)
    assert np.allclose(gb[1:], np.pi * HBAR * w * rho * v, rtol=1e-12)


def test_sigma_sc_closed_forms():
    t = np.arange(11, dtype=float)
    sig = np.stack([5.0 + 0 * t, 2.0 * t, -(t - 4.0) ** 2 + 9.0], axis=1)
    sig[0] = 100.0                        # t = 0 is excluded from the maximum
    assert np.allclose(tr.sigma_sc_max(sig), [5.0, 20.0, 9.0])
    avg = tr.sigma_sc_average(sig, 2, 8)
    assert avg[0] == pytest.approx(5.0)
    assert avg[1] == pytest.approx(2.0 * 5.0)            # linear: the midpoint value
    # trapezoid on the parabola: exact integral 30, plus (h^2/12)(f'(8) - f'(2)) = -1
    assert avg[2] == pytest.approx((30.0 - 1.0) / 6.0)
    with pytest.raises(ValueError):
        tr.sigma_sc_average(sig, 3, 3)


def test_pade_recovers_rational_function():
    a = np.array([0.5, 3.0, 40.0])
    b = np.array([0.2, 0.1])
    t = np.linspace(0.0, 50.0, 40)
    y = (a[0] + a[1] * t + a[2] * t ** 2) / (1 + b[0] * t + b[1] * t ** 2)
    fa, fb = tr.pade_fit(t, y, 2, 2)
    assert np.allclose(fa, a, rtol=1e-8)
    assert np.allclose(fb, b, rtol=1e-8)
    val, der = tr.pade_eval(fa, fb, t)
    exact_der = ((a[1] + 2 * a[2] * t) * (1 + b[0] * t + b[1] * t ** 2)
                 - (a[0] + a[1] * t + a[2] * t ** 2) * (b[0] + 2 * b[1] * t)) \
        / (1 + b[0] * t + b[1] * t ** 2) ** 2
    assert np.allclose(val, y, rtol=1e-10)
    assert np.allclose(der, exact_der, rtol=1e-7, atol=1e-10)
    # sigma_E1 of the fitted MSD: pi hbar rho d(Delta X^2)/dt
    assert np.allclose(tr.sigma_e1_pade(0.03, fa, fb, t), np.pi * HBAR * 0.03 * der)


def test_pade_smooths_a_noisy_saturating_msd():
    """A saturating MSD (localised regime, Sec. 5.3) with small noise: the [2/2]
    fit tracks the clean curve far better than the noise amplitude allows a
    finite difference to."""
    t = np.linspace(100.0, 2000.0, 200)
    clean = 400.0 * t ** 2 / (1e5 + 0.5 * t + t ** 2)
    rng = np.random.default_rng(0)
    y = clean * (1 + 1e-3 * rng.standard_normal(t.shape))
    fa, fb = tr.pade_fit(t, y, 2, 2)
    val, der = tr.pade_eval(fa, fb, t)
    assert np.max(np.abs(val - clean)) / np.max(clean) < 5e-4
    exact_der = np.gradient(clean, t)
    fd = np.gradient(y, t)
    assert np.max(np.abs(der - exact_der)) < 0.3 * np.max(np.abs(fd - exact_der))
    # without the re-weighting sweeps the linearised fit is an order of magnitude worse
    fa0, fb0 = tr.pade_fit(t, y, 2, 2, sweeps=0)
    assert np.max(np.abs(tr.pade_eval(fa0, fb0, t)[0] - clean)) / np.max(clean) > 5e-3


def test_typical_conductance_of_exponential_decay():
    """G = G0 exp(-L / xi) over lengths L: G_typ = G0 exp(-<L> / xi) (Eq. 60-61)."""
    lengths = np.array([10.0, 20.0, 35.0, 50.0])
    g = 2.0 * np.exp(-lengths[:, None] / np.array([15.0, 40.0]))
    assert np.allclose(tr.typical_conductance(g), 2.0 * np.exp(-lengths.mean() / np.array([15.0, 40.0])))
