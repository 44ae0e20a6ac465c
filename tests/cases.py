"""Matched test inputs: one seeded recipe feeds both the oracle and the GPU library."""
import numpy as np

import kpm_inputs as ki
import oracle


def recipe(geometry, nx, ny, w=0.0, vac=0.0, seed=0, e_scale=None, onsite="f64"):
    """Seeded on-site disorder, vacancies and E_s for an nx x ny sample.

    onsite="f32" is the float-exact disorder variant of a test case: the same
    draw rounded to the nearest float32 (the library then stores the on-site
    terms in 4 bytes); both sides of a comparison receive the rounded values."""
    n = nx * ny
    act = ki.vacancy_mask(n, vac, 2000 + seed) if vac else None
    ons = ki.anderson_onsite(n, w, 1000 + seed)
    if onsite == "f32":
        ons = float_exact(ons)
    elif onsite != "f64":
        raise ValueError(onsite)
    es = 1.01 * (3 * 2.7 + w / 2) if e_scale is None else e_scale
    return dict(geometry=geometry, nx=nx, ny=ny, onsite=ons, active=act, e_scale=es)


def float_exact(values):
    """Values rounded to the nearest float32, held in float64."""
    return np.asarray(values, dtype=np.float64).astype(np.float32).astype(np.float64)


def onsite_bytes(c):
    """Bytes per row the library stores for the on-site term of case c."""
    ons = np.asarray(c["onsite"])
    return 4 if np.array_equal(float_exact(ons), ons) else 8


def oracle_lattice(c):
    return oracle.graphene(c["nx"], c["ny"], c["geometry"], -2.7, c["onsite"], c["active"])


def gpu_system(c, precision="fp64"):
    import paper_1307_0288_amd as kp
    return kp.graphene_system(c["nx"], c["ny"], c["geometry"], -2.7, c["onsite"], c["active"],
                              c["e_scale"], precision)


def phases(c, n_vec=1, seed=3000):
    act = c["active"]
    return ki.random_phase(c["nx"] * c["ny"], n_vec, seed, act)


def rel_err(got, ref, scale=None):
    got, ref = np.asarray(got), np.asarray(ref)
    s = np.max(np.abs(ref)) if scale is None else scale
    return float(np.max(np.abs(got - ref)) / s) if s > 0 else float(np.max(np.abs(got - ref)))


def cell_trace_states(geometry, nx, ny):
    """Unit vectors on one translation cell of a pristine ribbon, and the number
    of cells: for an operator that commutes with the lattice translations the
    trace over all sites is that number times the sum of the cell's diagonal
    elements, so these states give the exact trace.  ZGNR (periodic along x)
    repeats every 2 sites along x, AGNR (periodic along y) every 2 chains."""
    n = nx * ny
    if geometry == "zgnr":
        sites = [j * nx + i for j in range(ny) for i in (0, 1)]
        cells = nx // 2
    elif geometry == "agnr":
        sites = [j * nx + i for j in (0, 1) for i in range(nx)]
        cells = ny // 2
    else:
        raise ValueError(geometry)
    phi = np.zeros((n, len(sites)), dtype=np.complex128)
    for c, s in enumerate(sites):
        phi[s, c] = 1.0
    return phi, cells
