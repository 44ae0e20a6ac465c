"""Workload of the host-sanitizer test: every host-side routine of the C oracle
and of the library's host-only part (lattice builder, descriptor validation,
running conductivities, transport post-processing) on small seeded inputs.

run(orc, host) takes the two loaded libraries and returns the results as one
flat dict of float lists.  As a script (`python sanitized_host.py ORC HOST`)
it loads the instrumented builds at those paths, runs the workload and prints
the dict as JSON; the test compares that with run() on the ordinary builds.
"""
import ctypes as C
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import kpm_inputs as ki                       # noqa: E402
import oracle                                 # noqa: E402
import oracle.core as ocore                   # noqa: E402
from paper_1307_0288_amd import kpm as kb     # noqa: E402

HOST_SYMBOLS = ("kpm_build_graphene", "kpm_validate", "kpm_sigma_gk", "kpm_sigma_e1",
                "kpm_sigma_e2", "kpm_length", "kpm_conductance", "kpm_ballistic_conductance",
                "kpm_sigma_sc_max", "kpm_sigma_sc_average", "kpm_pade_fit", "kpm_pade_eval",
                "kpm_typical_conductance")


def load_host(path):
    """The host-only part of the library built at `path`, typed like libkpm."""
    lib = C.CDLL(path)
    sig = kb._signatures()
    for name in HOST_SYMBOLS:
        f = getattr(lib, name)
        f.argtypes = sig[name]
        f.restype = C.c_int
    lib.kpm_last_error.restype = C.c_char_p
    return lib


def _flat(x):
    return [float(v) for v in np.ravel(np.asarray(x, dtype=np.complex128).view(np.float64))]


def _oracle_part(out):
    for k, geo in enumerate(("sheet", "zgnr", "agnr")):
        nx, ny = 8, 6
        act = ki.vacancy_mask(nx * ny, 0.05, 70 + k)
        ons = ki.anderson_onsite(nx * ny, 1.0, 80 + k)
        lat = oracle.graphene(nx, ny, geo, -2.7, ons, act)
        es = 1.01 * (3 * 2.7 + 0.5)
        phi = ki.random_phase(nx * ny, 1, 90 + k, act)[:, 0]
        out[f"orc_moments_{geo}"] = _flat(oracle.moments(lat, es, phi, phi, 24))
        out[f"orc_evolve_{geo}"] = _flat(oracle.evolve(lat, es, phi, 0.7, 1, 14))
        ox, ou = oracle.evolve_x(lat, es, phi, 0.7, 14)
        out[f"orc_evolve_x_{geo}"] = _flat(ox) + _flat(ou)
        out[f"orc_vac_{geo}"] = _flat(oracle.vac(lat, es, phi, 2, 0.5, 12, 16))
        out[f"orc_msd_{geo}"] = _flat(oracle.msd(lat, es, phi, 2, 0.5, 12, 16))
        out[f"orc_fourier_{geo}"] = _flat(oracle.fourier_moments(lat, es, phi, phi, 6, 0.8, 14))
    out["orc_bessel"] = _flat(oracle.bessel_j(20, 3.7))


def _host_part(out):
    for geo in ("sheet", "zgnr", "agnr"):
        for vac in (0.0, 0.1):
            act = ki.vacancy_mask(10 * 8, vac, 5) if vac else None
            nbr, dx = kb.kpm_build_graphene(10, 8, geo, act)
            out[f"graphene_{geo}_{vac}"] = _flat(nbr) + _flat(dx)
            out[f"bound_{geo}_{vac}"] = [kb.kpm_validate(nbr, dx=dx,
                                                        onsite=ki.anderson_onsite(80, 0.4, 6))]
    nbr, dx = kb.kpm_build_graphene(10, 8, "sheet")
    bad = {"range": nbr.copy(), "asym": nbr.copy()}
    bad["range"][2, 5] = 80
    bad["asym"][0, 3] = 7
    for name, nb in bad.items():
        try:
            kb.kpm_validate(nb, e_scale=9.0)
            out[f"invalid_{name}"] = [0.0]
        except kb.KpmError as e:
            out[f"invalid_{name}"] = [float(e.status)]
    try:
        kb.kpm_validate(nbr, e_scale=9.0, onsite=np.full(80, np.nan))
        out["invalid_nan"] = [0.0]
    except kb.KpmError as e:
        out["invalid_nan"] = [float(e.status)]

    rng = np.random.default_rng(11)
    t_n, k_n = 12, 5
    vacf = rng.standard_normal((t_n, k_n))
    msd = np.cumsum(rng.random((t_n, k_n)), axis=0)
    rho = rng.random(k_n) + 0.1
    out["sigma_gk"] = _flat(kb.kpm_sigma_gk(vacf, 0.5))
    out["sigma_e1"] = _flat(kb.kpm_sigma_e1(msd, 0.5))
    s2 = kb.kpm_sigma_e2(msd, 0.5)
    out["sigma_e2"] = _flat(s2)
    length = kb.kpm_length(msd, rho)
    out["length"] = _flat(length)
    out["conductance"] = _flat(kb.kpm_conductance(s2[1:], length[1:], 3.0))
    out["ballistic"] = _flat(kb.kpm_ballistic_conductance(msd, rho, 0.5, 3.0))
    out["sc_max"] = _flat(kb.kpm_sigma_sc_max(s2))
    out["sc_avg"] = _flat(kb.kpm_sigma_sc_average(s2, 3, 9))
    t = np.linspace(0.5, 40.0, 30)
    y = 2.0 * t * (1 + 0.3 * t) / (1 + 0.5 * t + 0.05 * t * t)
    a, b = kb.kpm_pade_fit(t, y, 2, 2)
    v, d = kb.kpm_pade_eval(a, b, t)
    out["pade"] = _flat(a) + _flat(b) + _flat(v) + _flat(d)
    out["typical"] = _flat(kb.kpm_typical_conductance(rng.random((7, k_n)) + 0.05))


def run(orc, host):
    """Both parts with the given libraries in place of the ordinary ones."""
    ocore._LIB = orc
    kb._lib = host
    out = {}
    _oracle_part(out)
    _host_part(out)
    return out


if __name__ == "__main__":
    with open("/proc/self/maps") as f:
        if "libasan" not in f.read():
            sys.exit("the AddressSanitizer runtime is not loaded")
    res = run(ocore.load(sys.argv[1]), load_host(sys.argv[2]))
    print(json.dumps(res))
