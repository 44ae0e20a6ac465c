"""ctypes front end of the C oracle (test infrastructure only).

Each function follows the paper's statement of the step it names; the
arithmetic itself lives in kpm_oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HBAR_EV_FS = 0.6582119569          # reduced Planck constant, eV fs
BOND_NM = 0.142                    # carbon-carbon distance a (Sec. 2)
GEOMETRIES = {"sheet": 0, "zgnr": 1, "agnr": 2}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liborc.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        _LIB = load(path)
    return _LIB


def load(path):
    """The C oracle built at `path` (liborc.so, or an instrumented build of the
    same source), with its argument types set."""
    lib = C.CDLL(path)
    i64, dp, ip = C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int64)
    up = C.POINTER(C.c_ubyte)
    lib.orc_set_threads.restype = C.c_int
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_graphene.restype = i64
    lib.orc_graphene.argtypes = [i64, i64, C.c_int, C.c_double, up, ip, ip, dp, dp]
    ham = [i64, ip, ip, dp, dp, dp, C.c_double]
    lib.orc_moments.restype = C.c_int
    lib.orc_moments.argtypes = ham + [dp, dp, C.c_int, dp]
    lib.orc_bessel_j.restype = C.c_int
    lib.orc_bessel_j.argtypes = [C.c_int, C.c_double, dp]
    lib.orc_evolve.restype = C.c_int
    lib.orc_evolve.argtypes = ham + [C.c_double, C.c_double, C.c_int, C.c_int, dp, dp]
    lib.orc_evolve_x.restype = C.c_int
    lib.orc_evolve_x.argtypes = ham + [C.c_double, C.c_double, C.c_int, dp, dp, dp]
    lib.orc_fourier.restype = C.c_int
    lib.orc_fourier.argtypes = ham + [C.c_double, dp, dp, C.c_int, C.c_double, C.c_int, dp]
    for f in (lib.orc_vac, lib.orc_msd):
        f.restype = C.c_int
        f.argtypes = ham + [C.c_double, dp, C.c_int, C.c_double, C.c_int, C.c_int, dp]
    return lib


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's parallel row loops (n >= 1 sets them); returns
    the count in use.  Results are the same for every count."""
    return _lib().orc_set_threads(int(n))


def _p(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


@dataclass
class Lattice:
    """Graphene sample as a CSR matrix over all nx*ny site indices (Sec. 2).

    hop[e] = H_nm in eV, dx[e] = X_n - X_m (nm) along the transport axis,
    onsite[n] in eV; a vacancy has an empty row and no bond points to it.
    """
    nx: int
    ny: int
    geometry: str
    t_ev: float
    row_ptr: np.ndarray
    col: np.ndarray
    hop: np.ndarray
    dx: np.ndarray
    onsite: np.ndarray
    active: np.ndarray

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def lx_nm(self) -> float:
        return np.sqrt(3.0) * self.nx * BOND_NM / 2.0

    @property
    def ly_nm(self) -> float:
        return 3.0 * self.ny * BOND_NM / 2.0

    @property
    def area_nm2(self) -> float:
        return self.lx_nm * self.ly_nm

    @property
    def width_nm(self) -> float:
        """Width across the transport direction."""
        return self.lx_nm if self.geometry == "agnr" else self.ly_nm

    def _ham(self):
        return (self.n, _p(self.row_ptr, C.c_int64), _p(self.col, C.c_int64),
                _p(self.hop), _p(self.dx), _p(self.onsite))


def graphene(nx: int, ny: int, geometry: str = "sheet", t_ev: float = -2.7,
             onsite=None, active=None) -> Lattice:
    """Build the nearest-neighbour lattice (Sec. 2 and Eq. 13)."""
    n = nx * ny
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(3 * n, dtype=np.int64)
    hop = np.zeros(3 * n, dtype=np.float64)
    dx = np.zeros(3 * n, dtype=np.float64)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    nnz = _lib().orc_graphene(nx, ny, GEOMETRIES[geometry], t_ev, _p(act, C.c_ubyte),
                              _p(row_ptr, C.c_int64), _p(col, C.c_int64), _p(hop), _p(dx))
    if nnz < 0:
        raise ValueError(f"invalid lattice {nx}x{ny} {geometry}")
    ons = np.zeros(n) if onsite is None else np.ascontiguousarray(onsite, dtype=np.float64).copy()
    if act is not None:
        ons[act == 0] = 0.0
    return Lattice(nx, ny, geometry, t_ev, row_ptr, col[:nnz].copy(), hop[:nnz].copy(),
                   dx[:nnz].copy(), ons, np.ones(n, np.uint8) if act is None else act)


def dense_h(lat: Lattice) -> np.ndarray:
    """Dense H (eV) over all site indices, for exact-diagonalisation tests."""
    h = np.zeros((lat.n, lat.n))
    for r in range(lat.n):
        for e in range(lat.row_ptr[r], lat.row_ptr[r + 1]):
            h[r, lat.col[e]] += lat.hop[e]
        h[r, r] += lat.onsite[r]
    return h


def dense_d(lat: Lattice) -> np.ndarray:
    """Dense (X_n - X_m) H_nm (eV nm): [X, H] with minimum-image bonds (Eq. 15)."""
    d = np.zeros((lat.n, lat.n))
    for r in range(lat.n):
        for e in range(lat.row_ptr[r], lat.row_ptr[r + 1]):
            d[r, lat.col[e]] += lat.dx[e] * lat.hop[e]
    return d


def _cvec(phi, n):
    a = np.ascontiguousarray(phi, dtype=np.complex128).reshape(-1)
    if a.shape[0] != n:
        raise ValueError("state length mismatch")
    return a


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed ({rc})")


def moments(lat: Lattice, e_scale: float, phi_l, phi_r, n_moments: int) -> np.ndarray:
    """C_m = <phi_L|T_m(H/E_s)|phi_R>, m < n_moments (Eq. 46, Alg. 5). complex128."""
    l, r = _cvec(phi_l, lat.n), _cvec(phi_r, lat.n)
    mu = np.zeros(n_moments, dtype=np.complex128)
    _check(_lib().orc_moments(*lat._ham(), e_scale, _p(l.view(np.float64)),
                              _p(r.view(np.float64)), n_moments, _p(mu.view(np.float64))),
           "moments")
    return mu


def bessel_j(count: int, x: float) -> np.ndarray:
    """J_0(x) .. J_{count-1}(x) by Miller's backward recurrence."""
    out = np.zeros(count)
    _check(_lib().orc_bessel_j(count, x, _p(out)), "bessel")
    return out


def evolve(lat: Lattice, e_scale: float, phi, dt_fs: float, sign: int, n_bessel: int,
           hbar: float = HBAR_EV_FS) -> np.ndarray:
    """U(sign*dt) phi by the Chebyshev-Bessel expansion (Eq. 36, Alg. 6)."""
    a = _cvec(phi, lat.n)
    out = np.zeros(lat.n, dtype=np.complex128)
    _check(_lib().orc_evolve(*lat._ham(), e_scale, hbar, dt_fs, sign, n_bessel,
                             _p(a.view(np.float64)), _p(out.view(np.float64))), "evolve")
    return out


def evolve_x(lat: Lattice, e_scale: float, phi, dt_fs: float, n_bessel: int,
             hbar: float = HBAR_EV_FS):
    """([X, U(dt)] phi, U(dt) phi) by Eq. 37 and the recursion of Eq. 38-41 (Alg. 7)."""
    a = _cvec(phi, lat.n)
    ox = np.zeros(lat.n, dtype=np.complex128)
    ou = np.zeros(lat.n, dtype=np.complex128)
    _check(_lib().orc_evolve_x(*lat._ham(), e_scale, hbar, dt_fs, n_bessel,
                               _p(a.view(np.float64)), _p(ox.view(np.float64)),
                               _p(ou.view(np.float64))), "evolve_x")
    return ox, ou


def vac(lat: Lattice, e_scale: float, phi, n_steps: int, dt_fs: float, n_bessel: int,
        n_moments: int, hbar: float = HBAR_EV_FS) -> np.ndarray:
    """Re <V U^dag(t_k) phi| T_m(H~) |U^dag(t_k) V phi>, shape [n_steps+1, n_moments] (Alg. 2)."""
    a = _cvec(phi, lat.n)
    out = np.zeros((n_steps + 1, n_moments))
    _check(_lib().orc_vac(*lat._ham(), e_scale, hbar, _p(a.view(np.float64)), n_steps, dt_fs,
                          n_bessel, n_moments, _p(out)), "vac")
    return out


def msd(lat: Lattice, e_scale: float, phi, n_steps: int, dt_fs: float, n_bessel: int,
        n_moments: int, hbar: float = HBAR_EV_FS) -> np.ndarray:
    """Re <[X,U(t_k)] phi| T_m(H~) |[X,U(t_k)] phi>, shape [n_steps+1, n_moments] (Alg. 3)."""
    a = _cvec(phi, lat.n)
    out = np.zeros((n_steps + 1, n_moments))
    _check(_lib().orc_msd(*lat._ham(), e_scale, hbar, _p(a.view(np.float64)), n_steps, dt_fs,
                          n_bessel, n_moments, _p(out)), "msd")
    return out


def fourier_moments(lat: Lattice, e_scale: float, phi_l, phi_r, n_moments: int, dtau_fs: float,
                    n_bessel: int, hbar: float = HBAR_EV_FS) -> np.ndarray:
    """F_n = <phi_L|U(n dtau)|phi_R>, n = -N_m .. N_m (Alg. 4). complex128 [2 N_m + 1]."""
    l, r = _cvec(phi_l, lat.n), _cvec(phi_r, lat.n)
    f = np.zeros(2 * n_moments + 1, dtype=np.complex128)
    _check(_lib().orc_fourier(*lat._ham(), e_scale, hbar, _p(l.view(np.float64)),
                              _p(r.view(np.float64)), n_moments, dtau_fs, n_bessel,
                              _p(f.view(np.float64))), "fourier")
    return f
