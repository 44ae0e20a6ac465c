"""Seeded synthetic inputs shared by the oracle and the GPU library.

This module draws random numbers and nothing else: it holds none of the
method's arithmetic (no lattice, no Hamiltonian, no recursion).  Both sides
of every parity test receive the arrays produced here, so that the two
implementations see bit-identical inputs.

Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used in counter mode: the k-th draw of a
stream with seed s is mix(s + (k + 1) * 0x9E3779B97F4A7C15).  The top 53 bits
of a draw give a uniform double in [0, 1).

Site index convention shared with both lattice builders: site (i, j) with
i in [0, nx) along the zigzag chains and j in [0, ny) across them has index
n = j * nx + i.

Seed recipe for the standard workloads: on-site disorder 1000 + sample,
vacancies 2000 + sample, random vectors 3000 + vector index.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Draws offset .. offset+count-1 of the SplitMix64 stream ``seed`` (uint64)."""
    k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits each."""
    return (splitmix64(seed, count, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def anderson_onsite(n_sites: int, w_ev: float, seed: int) -> np.ndarray:
    """On-site energies uniform in [-W/2, W/2) eV, one per site index (float64)."""
    if w_ev == 0.0:
        return np.zeros(n_sites, dtype=np.float64)
    return w_ev * (uniform(seed, n_sites) - 0.5)


def vacancy_mask(n_sites: int, fraction: float, seed: int) -> np.ndarray:
    """Active-site mask (uint8, 0 = vacancy) with exactly round(fraction*N) vacancies.

    The vacancies are a uniform draw without replacement: the sites holding the
    N_v smallest keys of an i.i.d. uniform key per site (ties broken by index).
    """
    n_vac = int(round(fraction * n_sites))
    active = np.ones(n_sites, dtype=np.uint8)
    if n_vac <= 0:
        return active
    if n_vac > n_sites:
        raise ValueError("vacancy fraction above 1")
    keys = splitmix64(seed, n_sites)
    order = np.argsort(keys, kind="stable")
    active[order[:n_vac]] = 0
    return active


def random_phase(n_sites: int, n_vec: int, seeds, active=None) -> np.ndarray:
    """Random-phase vectors exp(i*theta), theta uniform in [0, 2*pi).

    Returns complex128 of shape [n_sites, n_vec] (vector index fastest), zero
    on inactive sites, so <phi|phi> equals the number of active sites.
    ``seeds`` is an int (vector r uses seed + r) or a sequence of n_vec seeds.
    """
    if np.isscalar(seeds):
        seeds = [int(seeds) + r for r in range(n_vec)]
    if len(seeds) != n_vec:
        raise ValueError("one seed per vector required")
    out = np.empty((n_sites, n_vec), dtype=np.complex128)
    for r, s in enumerate(seeds):
        theta = 2.0 * np.pi * uniform(int(s), n_sites)
        out[:, r] = np.cos(theta) + 1j * np.sin(theta)
    if active is not None:
        out[np.asarray(active) == 0, :] = 0.0
    return out


def ragged_specs(count: int, seed: int, n_min: float = 1e4, n_max: float = 1e6,
                 w_min: int = 20, w_max: int = 400) -> list:
    """Sizes of a ragged batch: per sample a geometry (AGNR, ZGNR or sheet), a
    width in cells (ZGNR: zigzag chains; AGNR: twice as many dimer lines), a
    length giving a log-uniform site count in [n_min, n_max], and an Anderson
    strength W in {0.5, 1, 2} eV.  Periodic directions get even sizes."""
    u = uniform(seed, 4 * count).reshape(count, 4)
    out = []
    for s in range(count):
        geo = ("agnr", "zgnr", "sheet")[int(3 * u[s, 0])]
        width = w_min + int(u[s, 1] * (w_max - w_min + 1))
        n_target = float(np.exp(np.log(n_min) + u[s, 2] * (np.log(n_max) - np.log(n_min))))
        w_ev = (0.5, 1.0, 2.0)[int(3 * u[s, 3])]
        if geo == "zgnr":
            ny = width
            nx = max(4, 2 * int(round(n_target / ny / 2)))
        elif geo == "agnr":
            nx = 2 * width
            ny = max(2, 2 * int(round(n_target / nx / 2)))
        else:
            half = max(2, 2 * int(round(np.sqrt(n_target / 2) / 2)))
            nx, ny = 2 * half, half
        out.append(dict(geometry=geo, nx=nx, ny=ny, w=w_ev))
    return out


def sheet_config(name: str) -> dict:
    """Parameters of the named synthetic workloads (sizes in sites, energies in eV)."""
    hbar = 0.6582119569  # eV fs
    if name == "small":
        # 32x32 two-atom cells = 64x32 sites, W = 1 eV, no vacancies.
        return dict(geometry="sheet", nx=64, ny=32, t=-2.7, w=1.0, vac=0.0,
                    e_scale=1.01 * (3 * 2.7 + 0.5), n_moments=500, n_steps=10,
                    dt_fs=hbar / 2.7, n_bessel=30, n_vec=1)
    if name == "paper":
        # 1414x1414 two-atom cells = 2828x1414 sites, 0.5 % vacancies, W = 0.1 eV.
        return dict(geometry="sheet", nx=2828, ny=1414, t=-2.7, w=0.1, vac=0.005,
                    e_scale=1.01 * (3 * 2.7 + 0.05), n_moments=3000, n_steps=20,
                    dt_fs=hbar / 2.7, n_bessel=40, n_vec=1)
    if name == "ragged":
        # 32 samples of 1e4..1e6 sites, 8 vectors each, 1000 moments.
        return dict(count=32, seed=4000, n_min=1e4, n_max=1e6, w_min=20, w_max=400,
                    n_vec=8, n_moments=1000, t=-2.7)
    raise KeyError(name)


def learned_sample_specs(count: int, seed: int) -> list:
    """Disordered sheets for the learned reconstruction: per sample a vacancy
    fraction uniform in [0, 0.02) and an Anderson width W uniform in [0, 2) eV,
    and the seeds of its disorder, vacancies and random vectors (1000 + k,
    2000 + k, 3000 + 100 k with k = seed + index)."""
    u = uniform(seed, 2 * count)
    out = []
    for s in range(count):
        k = seed + s
        out.append(dict(vac=float(0.02 * u[2 * s]),
                        w=float(2.0 * u[2 * s + 1]),
                        onsite_seed=1000 + k, vac_seed=2000 + k, vec_seed=3000 + 100 * k))
    return out


def mlp_init(sizes, seed: int) -> list:
    """Initial weights of a fully connected network with layer widths `sizes`
    (Glorot-uniform W_l in [-a, a), a = sqrt(6 / (fan_in + fan_out)), zero
    biases), as float32 values held in float64: [(W_l [out, in], b_l [out])]."""
    params = []
    for l in range(len(sizes) - 1):
        fi, fo = sizes[l], sizes[l + 1]
        a = np.sqrt(6.0 / (fi + fo))
        w = (a * (2.0 * uniform(seed + l, fi * fo) - 1.0)).astype(np.float32).astype(np.float64)
        params.append((w.reshape(fo, fi), np.zeros(fo)))
    return params
