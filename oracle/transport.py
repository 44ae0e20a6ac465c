"""Transport quantities derived from the running conductivities (test
infrastructure only): the length and conductance of Sec. 5.1, the
semi-classical conductivity of Sec. 5.2, the Pade fit of the saturating MSD
and the typical conductance of Sec. 5.3.  Plain float64 numpy written from
the definitions; arrays are [T, K] (time points t_k = k dt by energies).

Units: MSD in nm^2, rho in 1/(eV nm^2), widths and lengths in nm, time in fs,
conductivities and conductances in e^2/h.
"""
from __future__ import annotations

import numpy as np

from .core import HBAR_EV_FS


def msd_per_state(rho_msd, rho):
    """Delta X^2(E, t) = [rho Delta X^2](E, t) / rho(E): the trace ratio that
    defines the MSD next to Eq. 9.  NaN where rho(E) = 0."""
    rho_msd = np.asarray(rho_msd, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(rho != 0, rho_msd / rho, np.nan)


def length(rho_msd, rho):
    """L(E, t) = 2 sqrt(Delta X^2(E, t)) (Eq. 50).  Negative MSD values
    (possible from a stochastic trace) give NaN."""
    x2 = msd_per_state(rho_msd, rho)
    with np.errstate(invalid="ignore"):
        return np.where(x2 >= 0, 2.0 * np.sqrt(np.where(x2 >= 0, x2, 0.0)), np.nan)


def conductance(sigma, length_nm, width_nm: float):
    """G(E, L) = (W / L(E, t)) sigma(E, t) in e^2/h (Eq. 51 and Eq. 59).
    NaN where L is zero or undefined (t = 0)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    lg = np.asarray(length_nm, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(lg > 0, width_nm * sigma / lg, np.nan)


def ballistic_conductance(rho_msd, rho, dt_fs: float, width_nm: float,
                          hbar: float = HBAR_EV_FS):
    """G(E) = (W/2) e^2 rho(E) sqrt(v^2(E)) in e^2/h (Eq. 52), with
    v^2(E, t_k) = Delta X^2(E, t_k) / t_k^2 from each time point t_k > 0 (the
    ballistic form Delta X^2 = v^2 t^2).  e^2 / (e^2/h) = h = 2 pi hbar, so
    G/(e^2/h) = pi hbar W rho sqrt(v^2).  Row 0 (t = 0) is NaN."""
    rho = np.asarray(rho, dtype=np.float64)
    x2 = msd_per_state(rho_msd, rho)
    t = dt_fs * np.arange(x2.shape[0], dtype=np.float64)
    out = np.full_like(x2, np.nan)
    with np.errstate(invalid="ignore"):
        v = np.sqrt(np.where(x2[1:] >= 0, x2[1:], np.nan)) / t[1:, None]
    out[1:] = np.pi * hbar * width_nm * rho * v
    return out


def sigma_sc_max(sigma):
    """sigma_sc(E) = max over t > 0 of sigma(E, t) (Eq. 53): rows 1 .. T-1."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.shape[0] < 2:
        raise ValueError("need at least one time point with t > 0")
    return np.max(sigma[1:], axis=0)


def sigma_sc_average(sigma, k1: int, k2: int):
    """sigma_sc(E) = (1/(t2 - t1)) int_{t1}^{t2} sigma_GK(E, t) dt (Eq. 55), with
    t1 = k1 dt, t2 = k2 dt on the time grid and the trapezoid rule (the time
    step cancels)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if not 0 <= k1 < k2 < sigma.shape[0]:
        raise ValueError("need 0 <= k1 < k2 < T")
    s = sigma[k1:k2 + 1]
    return (0.5 * (s[0] + s[-1]) + s[1:-1].sum(axis=0)) / (k2 - k1)


def pade_fit(t, y, m: int, n: int, sweeps: int = 8):
    """Coefficients of the [m/n] Pade approximant of Eq. 58,
    y(t) ~ sum_{j=0}^{m} a_j t^j / (1 + sum_{k=1}^{n} b_k t^k),
    fitted in the least-squares sense.  The paper does not say how; here the
    linearised residual y q - p (q, p: denominator and numerator) is minimised
    and then re-weighted by 1 / q of the previous solution, `sweeps` times
    (the Sanathanan-Koerner iteration), which approaches the least-squares fit
    of y - p/q itself.  Each solve runs in tau = t / t_max (an exact change of
    variable); the coefficients are returned for t: a_j / t_max^j, b_k / t_max^k."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if t.shape != y.shape or t.ndim != 1 or t.shape[0] < m + n + 1:
        raise ValueError("need 1-D t, y with at least m + n + 1 points")
    ts = float(np.max(np.abs(t)))
    tau = t / ts
    cols = [tau ** j for j in range(m + 1)] + [-y * tau ** k for k in range(1, n + 1)]
    a_mat = np.stack(cols, axis=1)
    w = np.ones_like(t)
    for _ in range(sweeps + 1):
        sol = np.linalg.lstsq(a_mat * w[:, None], y * w, rcond=None)[0]
        q = 1.0 + sum(sol[m + k] * tau ** k for k in range(1, n + 1))
        if np.any(q == 0):
            raise ValueError("pole at a data point")
        w = 1.0 / np.abs(q)
    a = sol[:m + 1] / ts ** np.arange(m + 1)
    b = sol[m + 1:] / ts ** np.arange(1, n + 1)
    return a, b


def pade_eval(a, b, t):
    """Value and time derivative of the Pade approximant at t."""
    t = np.asarray(t, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    p = sum(a[j] * t ** j for j in range(len(a)))
    dp = sum(j * a[j] * t ** (j - 1) for j in range(1, len(a)))
    q = 1.0 + sum(b[k - 1] * t ** k for k in range(1, len(b) + 1))
    dq = sum(k * b[k - 1] * t ** (k - 1) for k in range(1, len(b) + 1))
    return p / q, (dp * q - p * dq) / q ** 2


def sigma_e1_pade(rho, a, b, t, hbar: float = HBAR_EV_FS):
    """sigma_E1 (Eq. 9) of a Pade-fitted MSD: pi hbar rho d(Delta X^2_fit)/dt in
    e^2/h, at one energy (rho scalar) and the times t."""
    return np.pi * hbar * rho * pade_eval(a, b, t)[1]


def typical_conductance(g, axis: int = 0):
    """G_typ = exp(<ln G>) over realisations (Eq. 60)."""
    return np.exp(np.mean(np.log(np.asarray(g, dtype=np.float64)), axis=axis))
