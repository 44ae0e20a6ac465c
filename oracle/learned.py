"""Learned moment-to-spectrum reconstruction (test infrastructure only).

Not part of the paper: a small fully connected network maps the first
n_in Chebyshev moments of a sample (DOS moments of Eq. 46 and MSD moments of
Eq. 44 at one correlation time t*) to the spectra that Jackson-damped KPM sums
of many more moments give (Eq. 29-31): the DOS and sigma_E2(E, t*) of Eq. 11.
Plain float64 numpy, written from the definitions below.

Network: widths d_0 .. d_L; hidden layers a_{l+1} = tanh(a_l W_l^T + b_l),
linear output; loss = mean over batch and outputs of (y_pred - y)^2; Adam
(Kingma and Ba, ICLR 2015) with bias-corrected moments.

Features of a sample (moments averaged over its random vectors first):
  x = [mu_n / mu_0, n < n_in] + [c_n / c_0, n < n_in] + [ln(c_0 / mu_0)]
with mu the DOS moments and c the MSD moments at t*.
Targets on an energy grid E_k (eV), with Omega the sample area:
  y = [DOS_SCALE * rho(E_k) Omega / (2 mu_0)] + [SIGMA_SCALE * sigma_E2(E_k, t*)]
rho and rho * Delta X^2 being the KPM sums of all the moments given.
"""
from __future__ import annotations

import numpy as np

from .core import HBAR_EV_FS
from .recon import kpm_sum

DOS_SCALE = 10.0       # eV: per-state DOS (about 0.1 / eV) to order one
SIGMA_SCALE = 0.25     # sigma_E2 in e^2/h (a few) to order one


# ------------------------------------------------------------------ network
def forward(params, x):
    """Activations [a_0 = x, a_1, .., a_L] of the network on a batch x [B, d_0]."""
    acts = [np.asarray(x, dtype=np.float64)]
    for l, (w, b) in enumerate(params):
        z = acts[-1] @ w.T + b
        acts.append(np.tanh(z) if l < len(params) - 1 else z)
    return acts


def loss_and_grads(params, x, y):
    """Mean squared error and its gradient with respect to every W_l and b_l
    (backpropagation through the layers above)."""
    acts = forward(params, x)
    y = np.asarray(y, dtype=np.float64)
    diff = acts[-1] - y
    loss = float(np.mean(diff ** 2))
    g = 2.0 * diff / diff.size                  # d loss / d z_L
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        w, _ = params[l]
        grads[l] = (g.T @ acts[l], g.sum(axis=0))
        if l > 0:
            g = (g @ w) * (1.0 - acts[l] ** 2)    # through tanh of layer l
    return loss, grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; state = (t, m, v) with m, v shaped like params.
    Returns (new params, new state)."""
    t, m, v = state
    t += 1
    new_p, new_m, new_v = [], [], []
    for (w, b), (gw, gb), (mw, mb), (vw, vb) in zip(params, grads, m, v):
        out = []
        for p, g, mm, vv in ((w, gw, mw, vw), (b, gb, mb, vb)):
            mm = beta1 * mm + (1 - beta1) * g
            vv = beta2 * vv + (1 - beta2) * g * g
            mhat = mm / (1 - beta1 ** t)
            vhat = vv / (1 - beta2 ** t)
            out.append((p - lr * mhat / (np.sqrt(vhat) + eps), mm, vv))
        new_p.append((out[0][0], out[1][0]))
        new_m.append((out[0][1], out[1][1]))
        new_v.append((out[0][2], out[1][2]))
    return new_p, (t, new_m, new_v)


def adam_init(params):
    z = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    return (0, z, [(np.zeros_like(w), np.zeros_like(b)) for w, b in params])


def flatten(params) -> np.ndarray:
    """[W_0, b_0, W_1, b_1, ...] row-major in one vector."""
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def unflatten(vec, sizes):
    out, o = [], 0
    for l in range(len(sizes) - 1):
        fi, fo = sizes[l], sizes[l + 1]
        w = np.asarray(vec[o:o + fi * fo], dtype=np.float64).reshape(fo, fi)
        o += fi * fo
        b = np.asarray(vec[o:o + fo], dtype=np.float64)
        o += fo
        out.append((w, b))
    return out


# ------------------------------------------------------------------ features and targets
def features(mu_dos, mu_msd, n_in: int) -> np.ndarray:
    """x for each sample from moments [S, R, >= n_in] (averaged over R)."""
    mu = np.real(np.asarray(mu_dos)).astype(np.float64).mean(axis=1)
    c = np.real(np.asarray(mu_msd)).astype(np.float64).mean(axis=1)
    return np.concatenate([mu[:, :n_in] / mu[:, :1], c[:, :n_in] / c[:, :1],
                           np.log(c[:, :1] / mu[:, :1])], axis=1)


def targets(mu_dos, mu_msd, energies_ev, e_scale: float, area_nm2: float, t_star_fs: float,
            hbar: float = HBAR_EV_FS) -> np.ndarray:
    """y for each sample from all the moments given [S, R, N_m] (averaged over R)."""
    mu = np.real(np.asarray(mu_dos)).astype(np.float64).mean(axis=1)
    c = np.real(np.asarray(mu_msd)).astype(np.float64).mean(axis=1)
    rho = kpm_sum(mu, energies_ev, e_scale, area_nm2)              # [S, K]
    rho_x2 = kpm_sum(c, energies_ev, e_scale, area_nm2)
    dos = DOS_SCALE * rho * area_nm2 / (2.0 * mu[:, :1])
    sig = SIGMA_SCALE * np.pi * hbar * rho_x2 / t_star_fs          # sigma_E2, Eq. 11
    return np.concatenate([dos, sig], axis=1)


def spectra_error(y_pred, y_ref, n_energies: int):
    """Per sample: (max|d DOS| / max|DOS|, max|d sigma| / max|sigma|)."""
    y_pred, y_ref = np.asarray(y_pred), np.asarray(y_ref)
    out = []
    for part in (slice(0, n_energies), slice(n_energies, 2 * n_energies)):
        d = np.max(np.abs(y_pred[:, part] - y_ref[:, part]), axis=1)
        out.append(d / np.max(np.abs(y_ref[:, part]), axis=1))
    return out[0], out[1]
