"""Host-side reconstruction from Chebyshev moments (test infrastructure only).

Jackson damping (Eq. 35), the KPM sums of Eq. 29-31 and the running
electrical conductivities of Eq. 6 (Green-Kubo), Eq. 9 (Einstein E1) and
Eq. 11 (Einstein E2).  Plain float64 numpy, written from the definitions.

Conventions (readings of points the paper leaves open):
  * H~ = H / E_s with no shift; the Jacobian of delta(E - H) =
    delta(E/E_s - H~) / E_s is applied in every sum.
  * T_n(e) = cos(n arccos e) on |e| < 1.
  * Time integrals use the cumulative trapezoid rule, time derivatives the
    centred difference (one-sided at the two ends).
  * Conductivities are returned in units of e^2/h: with hbar in eV fs, time
    in fs, rho in 1/(eV nm^2), VAC in nm^2/fs^2 and MSD in nm^2,
    sigma_GK/(e^2/h) = 2 pi hbar int rho C_vv dt and
    sigma_E1/(e^2/h) = pi hbar d(rho MSD)/dt.
"""
from __future__ import annotations

import numpy as np

from .core import HBAR_EV_FS


def jackson(n_moments: int) -> np.ndarray:
    """Jackson damping factors g_n, n < n_moments, alpha = 1/(N_m + 1) (Eq. 35)."""
    n = np.arange(n_moments, dtype=np.float64)
    a = 1.0 / (n_moments + 1)
    return (1 - n * a) * np.cos(np.pi * n * a) + a * np.sin(np.pi * n * a) / np.tan(np.pi * a)


def hanning(n_moments: int) -> np.ndarray:
    """Hanning window w_n = (1 + cos(pi n / (N_m + 1))) / 2, n = -N_m .. N_m (Eq. 28)."""
    n = np.arange(-n_moments, n_moments + 1, dtype=np.float64)
    return 0.5 * (1.0 + np.cos(np.pi * n / (n_moments + 1)))


def ftm_sum(fmom, energies_ev, dtau_fs: float, area_nm2: float, window=None,
            hbar: float = HBAR_EV_FS) -> np.ndarray:
    """(dtau / (pi hbar Omega)) sum_n w_n Re[exp(i E n dtau / hbar) F_n] (Eq. 22-24).

    fmom: [..., 2 N_m + 1] complex Fourier moments F_{-N_m} .. F_{N_m}.
    """
    fmom = np.asarray(fmom, dtype=np.complex128)
    nm = (fmom.shape[-1] - 1) // 2
    w = hanning(nm) if window is None else np.asarray(window)
    n = np.arange(-nm, nm + 1, dtype=np.float64)
    ph = np.exp(1j * np.outer(n, np.asarray(energies_ev, dtype=np.float64)) * dtau_fs / hbar)
    s = np.real(np.tensordot(fmom * w, ph, axes=([-1], [0])))
    return s * dtau_fs / (np.pi * hbar * area_nm2)


def energies_grid(n_energies: int, e_scale: float, frac: float = 0.95) -> np.ndarray:
    """Uniform energies on [-frac E_s, frac E_s] (eV)."""
    return np.linspace(-frac * e_scale, frac * e_scale, n_energies)


def kpm_sum(mom, energies_ev, e_scale: float, area_nm2: float, damping=None) -> np.ndarray:
    """(2/Omega) <.|delta(E - H)|.> from moments (Eq. 29-31).

    mom: [..., N_m] real (or complex: the real part of the sum is taken, as in
    Eq. 30).  Returns [..., K] in 1/(eV nm^2) times the unit of the moments.
    """
    mom = np.asarray(mom)
    nm = mom.shape[-1]
    g = jackson(nm) if damping is None else np.asarray(damping)
    w = g * np.where(np.arange(nm) == 0, 1.0, 2.0)
    eps = np.asarray(energies_ev, dtype=np.float64) / e_scale
    if np.any(np.abs(eps) >= 1):
        raise ValueError("energies must lie inside the scaled band")
    tn = np.cos(np.outer(np.arange(nm), np.arccos(eps)))            # [N_m, K]
    s = np.real(np.tensordot(mom * w, tn, axes=([-1], [0])))
    pref = 2.0 / (np.pi * area_nm2 * e_scale * np.sqrt(1.0 - eps ** 2))
    return s * pref


def dos(mu, energies_ev, e_scale, area_nm2):
    """rho(E) (Eq. 29)."""
    return kpm_sum(mu, energies_ev, e_scale, area_nm2)


def _cumtrapz(y, dt):
    out = np.zeros_like(y)
    if y.shape[0] > 1:
        out[1:] = np.cumsum(0.5 * (y[1:] + y[:-1]) * dt, axis=0)
    return out


def sigma_gk(rho_cvv, dt_fs: float, hbar: float = HBAR_EV_FS):
    """sigma_GK(E, t_k) in e^2/h from rho*C_vv [T, K] sampled at t_k = k dt (Eq. 6)."""
    return 2.0 * np.pi * hbar * _cumtrapz(np.asarray(rho_cvv, dtype=np.float64), dt_fs)


def sigma_e1(rho_msd, dt_fs: float, hbar: float = HBAR_EV_FS):
    """sigma_E1(E, t_k) in e^2/h from rho*MSD [T, K] (Eq. 9)."""
    y = np.asarray(rho_msd, dtype=np.float64)
    d = np.gradient(y, dt_fs, axis=0, edge_order=1) if y.shape[0] > 1 else np.zeros_like(y)
    return np.pi * hbar * d


def sigma_e2(rho_msd, dt_fs: float, hbar: float = HBAR_EV_FS):
    """sigma_E2(E, t_k) in e^2/h from rho*MSD [T, K] (Eq. 11); zero at t = 0."""
    y = np.asarray(rho_msd, dtype=np.float64)
    t = dt_fs * np.arange(y.shape[0], dtype=np.float64)
    out = np.zeros_like(y)
    out[1:] = np.pi * hbar * y[1:] / t[1:, None] if y.ndim == 2 else np.pi * hbar * y[1:] / t[1:]
    return out
