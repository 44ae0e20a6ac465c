"""Python binding of the C ABI in include/kpm.h (ctypes; argument marshalling only).

Every computation runs in libkpm.so.  PyTorch provides device memory (state
tensors) and the stream: each call runs on torch's current HIP stream.

States are torch tensors on the GPU of shape [n_sites, n_vec] and dtype
complex128 (KPM_FP64 systems) or complex64 (KPM_FP32_STATES and KPM_FP32 systems), or the
equivalent real view [n_sites, n_vec, 2]; n_vec is a power of two <= 64.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libkpm.so")

KPM_OK, KPM_ERR_INVALID, KPM_ERR_OOM, KPM_ERR_DEVICE, KPM_ERR_UNSUPPORTED, KPM_ERR_NUMERIC = range(6)
KPM_FP64, KPM_FP32_STATES, KPM_FP32 = 0, 1, 2
# precision names of the binding: FP64 states; FP32 states (FP64 arithmetic);
# FP32 states with the strips' recursion arithmetic in FP32
PRECISIONS = {"fp64": KPM_FP64, "fp32": KPM_FP32_STATES, "fp32_arith": KPM_FP32}
GEOMETRIES = {"sheet": 0, "zgnr": 1, "agnr": 2}
HBAR_EV_FS = 0.6582119569
BOND_NM = 0.142

# Every symbol declared in include/kpm.h.
ABI_SYMBOLS = ("kpm_build_graphene", "kpm_validate", "kpm_system_create", "kpm_system_destroy",
               "kpm_system_set_stream", "kpm_system_n_sites", "kpm_batch_create",
               "kpm_system_n_samples", "kpm_system_offsets", "kpm_moments",
               "kpm_moments_noalloc", "kpm_moments_doubled", "kpm_evolve", "kpm_evolve_x", "kpm_vac", "kpm_msd",
               "kpm_msd_doubled", "kpm_vac_msd", "kpm_dos_vac_msd", "kpm_fourier_moments",
               "kpm_ftm_sum",
               "kpm_kpm_sum", "kpm_sigma_gk",
               "kpm_sigma_e1", "kpm_sigma_e2", "kpm_length", "kpm_conductance",
               "kpm_ballistic_conductance", "kpm_sigma_sc_max", "kpm_sigma_sc_average",
               "kpm_pade_fit", "kpm_pade_eval", "kpm_typical_conductance",
               "kpm_mlp_create", "kpm_mlp_destroy", "kpm_mlp_n_params", "kpm_mlp_set_params",
               "kpm_mlp_get_params", "kpm_mlp_forward", "kpm_mlp_gradients",
               "kpm_mlp_train_step", "kpm_learned_features", "kpm_learned_targets",
               "kpm_xu_state", "kpm_vac_continue", "kpm_msd_continue",
               "kpm_default_launch", "kpm_set_launch", "kpm_get_launch", "kpm_set_launch_doubled",
               "kpm_get_launch_doubled",
               "kpm_autotune", "kpm_autotune_candidates", "kpm_set_graphs", "kpm_set_timing", "kpm_get_stats",
               "kpm_reset_stats",
               "kpm_last_error", "kpm_version")


class KpmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"kpm status {status}: {msg}")
        self.status = status


class _Desc(C.Structure):
    _fields_ = [("n_sites", C.c_int64), ("width", C.c_int32),
                ("nbr", C.POINTER(C.c_int32)), ("hop", C.POINTER(C.c_double)),
                ("t_uniform", C.c_double), ("onsite", C.POINTER(C.c_double)),
                ("dx", C.POINTER(C.c_double)), ("active", C.POINTER(C.c_uint8)),
                ("e_scale", C.c_double)]


class Launch(C.Structure):
    _fields_ = [("groups_per_cu", C.c_int32), ("ilp", C.c_int32), ("streaming", C.c_int32),
                ("compact", C.c_int32), ("tiled", C.c_int32), ("steps", C.c_int32),
                ("vectors_per_wave", C.c_int32), ("plane_groups", C.c_int32),
                ("group_size", C.c_int32)]

    def as_dict(self) -> dict:
        """The shape's fields; the two vector-layout fields only when set."""
        d = dict(groups_per_cu=self.groups_per_cu, ilp=self.ilp, streaming=self.streaming,
                 compact=self.compact, tiled=self.tiled, steps=self.steps)
        if self.vectors_per_wave or self.plane_groups:
            d.update(vectors_per_wave=self.vectors_per_wave, plane_groups=self.plane_groups)
        if self.group_size:
            d.update(group_size=self.group_size)
        return d


class Adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class Stats(C.Structure):
    _fields_ = [("step_ms", C.c_double), ("step_launches", C.c_int64),
                ("step_rows", C.c_int64), ("site_updates", C.c_int64),
                ("step_bytes", C.c_int64), ("step_bytes_total", C.c_int64),
                ("wide_ms", C.c_double), ("wide_launches", C.c_int64), ("wide_rows", C.c_int64)]


_lib = None


def _signatures():
    """Argument types of every compute entry point (all return kpm_status)."""
    vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
    fp = C.POINTER(C.c_float)
    return {
        "kpm_build_graphene": [i64, i64, C.c_int, C.POINTER(C.c_uint8), C.POINTER(C.c_int32), dp],
        "kpm_validate": [C.POINTER(_Desc), dp],
        "kpm_system_create": [C.POINTER(_Desc), C.c_int, C.c_int, vp, C.POINTER(vp)],
        "kpm_batch_create": [C.c_int, C.POINTER(_Desc), C.c_int, C.c_int, vp, C.POINTER(vp)],
        "kpm_system_offsets": [vp, C.POINTER(C.c_int64)],
        "kpm_system_destroy": [vp],
        "kpm_system_set_stream": [vp, vp],
        "kpm_moments": [vp, C.c_int, vp, vp, C.c_int, dp],
        "kpm_moments_noalloc": [vp, C.c_int, vp, vp, C.c_int, dp],
        "kpm_moments_doubled": [vp, C.c_int, vp, C.c_int, dp],
        "kpm_evolve": [vp, C.c_int, vp, C.c_double, C.c_int, C.c_int],
        "kpm_evolve_x": [vp, C.c_int, vp, vp, vp, C.c_double, C.c_int],
        "kpm_vac": [vp, C.c_int, vp, C.c_int, C.c_double, C.c_int, C.c_int, dp],
        "kpm_msd": [vp, C.c_int, vp, C.c_int, C.c_double, C.c_int, C.c_int, dp],
        "kpm_msd_doubled": [vp, C.c_int, vp, C.c_int, C.c_double, C.c_int, C.c_int, dp],
        "kpm_vac_msd": [vp, C.c_int, vp, C.c_int, C.c_double, C.c_int, C.c_int, dp, dp],
        "kpm_dos_vac_msd": [vp, C.c_int, vp, C.c_int, C.c_double, C.c_int, C.c_int, dp, dp, dp],
        "kpm_kpm_sum": [C.c_int, C.c_int, dp, C.c_int, dp, C.c_double, C.c_double,
                        C.c_int, vp, dp],
        "kpm_fourier_moments": [vp, C.c_int, vp, vp, C.c_int, C.c_double, C.c_int, dp],
        "kpm_ftm_sum": [C.c_int, C.c_int, dp, C.c_int, dp, C.c_double, C.c_double,
                        C.c_int, vp, dp],
        "kpm_sigma_gk": [C.c_int, C.c_int, dp, C.c_double, dp],
        "kpm_sigma_e1": [C.c_int, C.c_int, dp, C.c_double, dp],
        "kpm_sigma_e2": [C.c_int, C.c_int, dp, C.c_double, dp],
        "kpm_length": [C.c_int, C.c_int, dp, dp, dp],
        "kpm_conductance": [C.c_int, C.c_int, dp, dp, C.c_double, dp],
        "kpm_ballistic_conductance": [C.c_int, C.c_int, dp, dp, C.c_double, C.c_double, dp],
        "kpm_sigma_sc_max": [C.c_int, C.c_int, dp, dp],
        "kpm_sigma_sc_average": [C.c_int, C.c_int, dp, C.c_int, C.c_int, dp],
        "kpm_pade_fit": [C.c_int, dp, dp, C.c_int, C.c_int, C.c_int, dp, dp],
        "kpm_pade_eval": [C.c_int, C.c_int, dp, dp, C.c_int, dp, dp, dp],
        "kpm_typical_conductance": [C.c_int, C.c_int, dp, dp],
        "kpm_mlp_create": [C.c_int, C.POINTER(C.c_int32), C.c_int, C.c_int, vp,
                           C.POINTER(vp)],
        "kpm_mlp_destroy": [vp],
        "kpm_mlp_set_params": [vp, fp],
        "kpm_mlp_get_params": [vp, fp],
        "kpm_mlp_forward": [vp, C.c_int, vp, vp],
        "kpm_mlp_gradients": [vp, C.c_int, vp, vp, dp, fp],
        "kpm_mlp_train_step": [vp, C.c_int, vp, vp, C.POINTER(Adam), dp],
        "kpm_learned_features": [C.c_int, C.c_int, C.c_int, dp, dp, C.c_int, fp],
        "kpm_learned_targets": [C.c_int, C.c_int, C.c_int, dp, dp, C.c_int, dp, C.c_double,
                                C.c_double, C.c_double, vp, fp],
        "kpm_xu_state": [vp, C.c_int, vp, C.c_int, C.c_double, C.c_int, vp],
        "kpm_vac_continue": [vp, C.c_int, vp, vp, C.c_int, C.c_int, C.c_double, C.c_int,
                             C.c_int, dp],
        "kpm_msd_continue": [vp, C.c_int, vp, vp, C.c_int, C.c_int, C.c_double, C.c_int,
                             C.c_int, C.c_int, dp],
        "kpm_default_launch": [C.c_int, C.c_int, C.POINTER(Launch)],
        "kpm_set_launch": [vp, C.c_int, C.POINTER(Launch)],
        "kpm_get_launch": [vp, C.c_int, C.POINTER(Launch)],
        "kpm_set_launch_doubled": [vp, C.c_int, C.POINTER(Launch)],
        "kpm_get_launch_doubled": [vp, C.c_int, C.POINTER(Launch)],
        "kpm_autotune": [vp, C.c_int, vp, C.c_int, C.POINTER(Launch)],
        "kpm_autotune_candidates": [vp, C.c_int, C.POINTER(Launch), C.c_int32,
                                    C.POINTER(C.c_int32)],
        "kpm_set_graphs": [vp, C.c_int],
        "kpm_set_timing": [vp, C.c_int],
        "kpm_get_stats": [vp, C.POINTER(Stats)],
        "kpm_reset_stats": [vp],
    }


def lib():
    """The loaded libkpm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1307_0288_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        sig = _signatures()
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.kpm_system_n_sites.argtypes = [vp]
        L.kpm_system_n_sites.restype = C.c_int64
        L.kpm_mlp_n_params.argtypes = [vp]
        L.kpm_mlp_n_params.restype = C.c_int64
        L.kpm_system_n_samples.argtypes = [vp]
        L.kpm_system_n_samples.restype = C.c_int32
        L.kpm_last_error.restype = C.c_char_p
        L.kpm_version.restype = C.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != KPM_OK:
        raise KpmError(status, lib().kpm_last_error().decode())


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ host helpers
def kpm_build_graphene(nx: int, ny: int, geometry: str = "sheet", active=None):
    """Neighbour list [3][nx*ny] (int32, -1 empty) and dx [3][nx*ny] (nm)."""
    n = nx * ny
    nbr = np.empty((3, n), dtype=np.int32)
    dx = np.empty((3, n), dtype=np.float64)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    _check(lib().kpm_build_graphene(nx, ny, GEOMETRIES[geometry],
                                    None if act is None else act.ctypes.data_as(C.POINTER(C.c_uint8)),
                                    nbr.ctypes.data_as(C.POINTER(C.c_int32)), _dp(dx)))
    return nbr, dx


def kpm_kpm_sum(moments, energies_ev, e_scale: float, area_nm2: float, jackson: bool = True):
    """KPM sum of Eq. 29-31 on the device: moments [rows, N_m] -> [rows, K]."""
    mom = np.ascontiguousarray(np.real(moments), dtype=np.float64)
    squeeze = mom.ndim == 1
    mom = mom.reshape(-1, mom.shape[-1])
    en = np.ascontiguousarray(energies_ev, dtype=np.float64).reshape(-1)
    out = np.empty((mom.shape[0], en.shape[0]))
    _check(lib().kpm_kpm_sum(mom.shape[0], mom.shape[1], _dp(mom), en.shape[0], _dp(en),
                             e_scale, area_nm2, int(bool(jackson)), _stream(), _dp(out)))
    return out[0] if squeeze else out


def kpm_ftm_sum(fmom, energies_ev, dtau_fs: float, area_nm2: float, hanning: bool = True):
    """Fourier (FTM) sum of Eq. 22-24 on the device: F [rows, 2 N_m + 1] -> [rows, K]."""
    f = np.ascontiguousarray(fmom, dtype=np.complex128)
    squeeze = f.ndim == 1
    f = f.reshape(-1, f.shape[-1])
    nm = (f.shape[1] - 1) // 2
    en = np.ascontiguousarray(energies_ev, dtype=np.float64).reshape(-1)
    out = np.empty((f.shape[0], en.shape[0]))
    _check(lib().kpm_ftm_sum(f.shape[0], nm, _dp(f.view(np.float64)), en.shape[0], _dp(en),
                             dtau_fs, area_nm2, int(bool(hanning)), _stream(), _dp(out)))
    return out[0] if squeeze else out


def _sigma(fn, rows, dt_fs):
    a = np.ascontiguousarray(rows, dtype=np.float64)
    a2 = a.reshape(a.shape[0], -1)
    out = np.empty_like(a2)
    _check(fn(a2.shape[0], a2.shape[1], _dp(a2), dt_fs, _dp(out)))
    return out.reshape(a.shape)


def kpm_sigma_gk(rho_vac, dt_fs):
    """sigma_GK(E, t_k) / (e^2/h) from rho*C_vv [T, K] (Eq. 6)."""
    return _sigma(lib().kpm_sigma_gk, rho_vac, dt_fs)


def kpm_sigma_e1(rho_msd, dt_fs):
    """sigma_E1(E, t_k) / (e^2/h) from rho*MSD [T, K] (Eq. 9)."""
    return _sigma(lib().kpm_sigma_e1, rho_msd, dt_fs)


def kpm_sigma_e2(rho_msd, dt_fs):
    """sigma_E2(E, t_k) / (e^2/h) from rho*MSD [T, K] (Eq. 11)."""
    return _sigma(lib().kpm_sigma_e2, rho_msd, dt_fs)


def _rows(a):
    """[T, K] float64 C-contiguous view of a [T, K] or [T] array."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(a.shape[0], -1)


def kpm_length(rho_msd, rho):
    """L(E, t) = 2 sqrt(rho_msd / rho) in nm (Eq. 50); rho_msd [T, K], rho [K]."""
    m = _rows(rho_msd)
    r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    if r.shape[0] != m.shape[1]:
        raise ValueError("rho must have one entry per energy")
    out = np.empty_like(m)
    _check(lib().kpm_length(m.shape[0], m.shape[1], _dp(m), _dp(r), _dp(out)))
    return out.reshape(np.shape(rho_msd))


def kpm_conductance(sigma, length_nm, width_nm: float):
    """G(E, L) = (W / L) sigma in e^2/h (Eq. 51, Eq. 59); [T, K] arrays."""
    s, lg = _rows(sigma), _rows(length_nm)
    if s.shape != lg.shape:
        raise ValueError("sigma and length differ in shape")
    out = np.empty_like(s)
    _check(lib().kpm_conductance(s.shape[0], s.shape[1], _dp(s), _dp(lg), width_nm, _dp(out)))
    return out.reshape(np.shape(sigma))


def kpm_ballistic_conductance(rho_msd, rho, dt_fs: float, width_nm: float):
    """G(E) = (W/2) e^2 rho sqrt(v^2) in e^2/h with v^2 = Delta X^2 / t^2 (Eq. 52)."""
    m = _rows(rho_msd)
    r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    if r.shape[0] != m.shape[1]:
        raise ValueError("rho must have one entry per energy")
    out = np.empty_like(m)
    _check(lib().kpm_ballistic_conductance(m.shape[0], m.shape[1], _dp(m), _dp(r), dt_fs,
                                           width_nm, _dp(out)))
    return out.reshape(np.shape(rho_msd))


def kpm_sigma_sc_max(sigma):
    """sigma_sc(E) = max over t > 0 of sigma(E, t) (Eq. 53): [T, K] -> [K]."""
    s = _rows(sigma)
    out = np.empty(s.shape[1])
    _check(lib().kpm_sigma_sc_max(s.shape[0], s.shape[1], _dp(s), _dp(out)))
    return out


def kpm_sigma_sc_average(sigma, k1: int, k2: int):
    """sigma_sc(E) = time-block average of sigma over [k1 dt, k2 dt] (Eq. 55)."""
    s = _rows(sigma)
    out = np.empty(s.shape[1])
    _check(lib().kpm_sigma_sc_average(s.shape[0], s.shape[1], _dp(s), k1, k2, _dp(out)))
    return out


def kpm_pade_fit(t, y, m: int, n: int, sweeps: int = 8):
    """[m/n] Pade coefficients (a [m+1], b [n]) of Eq. 58 by re-weighted
    linearised least squares (`sweeps` re-weightings)."""
    t = np.ascontiguousarray(t, dtype=np.float64).reshape(-1)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
    if t.shape != y.shape:
        raise ValueError("t and y differ in length")
    a, b = np.empty(m + 1), np.empty(max(n, 1))
    _check(lib().kpm_pade_fit(t.shape[0], _dp(t), _dp(y), m, n, sweeps, _dp(a), _dp(b)))
    return a, b[:n]


def kpm_pade_eval(a, b, t):
    """Value and d/dt of the Pade approximant (a, b) at the times t."""
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    t = np.ascontiguousarray(t, dtype=np.float64).reshape(-1)
    bb = b if b.shape[0] else np.zeros(1)
    v, d = np.empty_like(t), np.empty_like(t)
    _check(lib().kpm_pade_eval(a.shape[0] - 1, b.shape[0], _dp(a), _dp(bb), t.shape[0], _dp(t),
                               _dp(v), _dp(d)))
    return v, d


def kpm_typical_conductance(g):
    """G_typ(E) = exp(<ln G(E)>) over realisations (Eq. 60): [R, K] -> [K]."""
    gg = _rows(g)
    out = np.empty(gg.shape[1])
    _check(lib().kpm_typical_conductance(gg.shape[0], gg.shape[1], _dp(gg), _dp(out)))
    return out


# ------------------------------------------------------------------ system
def _make_desc(nbr, e_scale, t_uniform=-2.7, hop=None, onsite=None, dx=None, active=None,
               keep=None):
    """A kpm_system_desc over numpy arrays (kept alive in `keep`)."""
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    if nbr.ndim != 2:
        raise ValueError("nbr must be [width][n_sites]")
    keep.append(nbr)
    width, n = nbr.shape

    def arr(a, dt, shape):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dt)
        if a.shape != shape:
            raise ValueError(f"array shape {a.shape} != {shape}")
        keep.append(a)
        return a

    hop = arr(hop, np.float64, nbr.shape)
    onsite = arr(onsite, np.float64, (n,))
    dx = arr(dx, np.float64, nbr.shape)
    active = arr(active, np.uint8, (n,))
    return _Desc(n, width, nbr.ctypes.data_as(C.POINTER(C.c_int32)), _dp(hop), t_uniform,
                 _dp(onsite), _dp(dx),
                 None if active is None else active.ctypes.data_as(C.POINTER(C.c_uint8)),
                 e_scale)


def kpm_validate(nbr, e_scale: float = 0.0, t_uniform: float = -2.7, hop=None, onsite=None,
                 dx=None, active=None):
    """Host check of a descriptor (the rules of kpm_system_create); returns the
    Gershgorin bound in eV.  With e_scale = 0 only the structure is checked."""
    keep = []
    d = _make_desc(nbr, e_scale, t_uniform, hop, onsite, dx, active, keep)
    bound = C.c_double(float("nan"))
    st = lib().kpm_validate(C.byref(d), C.byref(bound))
    if st != KPM_OK and not (e_scale == 0.0 and np.isfinite(bound.value)):
        _check(st)
    return bound.value


class System:
    """A Hamiltonian resident on one GPU (wraps kpm_system_create), or a ragged
    batch of samples (System.batch, wraps kpm_batch_create)."""

    def __init__(self, nbr, e_scale: float, t_uniform: float = -2.7, hop=None, onsite=None,
                 dx=None, active=None, precision: str = "fp64", device: int | None = None):
        keep = []
        d = _make_desc(nbr, e_scale, t_uniform, hop, onsite, dx, active, keep)
        self._create([d], precision, device)

    @classmethod
    def batch(cls, samples, precision: str = "fp64", device: int | None = None):
        """samples: list of dicts with the keyword arguments of System()."""
        keep = []
        descs = [_make_desc(keep=keep, **smp) for smp in samples]
        obj = cls.__new__(cls)
        obj._create(descs, precision, device)
        return obj

    def _create(self, descs, precision, device):
        import torch
        self.precision = precision
        self.e_scale = float(descs[0].e_scale)
        self.device = torch.cuda.current_device() if device is None else int(device)
        self._h = C.c_void_p()
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        prec = PRECISIONS[precision]
        arr = (_Desc * len(descs))(*descs)
        with torch.cuda.device(self.device):
            _check(lib().kpm_batch_create(len(descs), arr, prec, self.device, _stream(),
                                          C.byref(self._h)))
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.n_sites = int(lib().kpm_system_n_sites(self._h))
        self.n_samples = int(lib().kpm_system_n_samples(self._h))
        off = np.zeros(self.n_samples + 1, dtype=np.int64)
        _check(lib().kpm_system_offsets(self._h, off.ctypes.data_as(C.POINTER(C.c_int64))))
        self.offsets = off
        self.width = max(int(d.width) for d in descs)

    def _shape(self, out):
        """Drop the leading sample axis of a host output for a single system."""
        return out[0] if self.n_samples == 1 else out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().kpm_system_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _sync_stream(self):
        _check(lib().kpm_system_set_stream(self._h, _stream()))

    def _state(self, t, name):
        """(data pointer, n_vec) of a state tensor, after checking it."""
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a GPU tensor")
        if t.dtype in (torch.float64, torch.float32):
            if t.dim() != 3 or t.shape[-1] != 2:
                raise ValueError(f"{name}: real view must be [n_sites, n_vec, 2]")
            t = torch.view_as_complex(t)
        if t.dtype != self.cdtype:
            raise TypeError(f"{name} must be {self.cdtype} for a {self.precision} system")
        if t.dim() == 1:
            t = t.unsqueeze(1)
        if t.dim() != 2 or t.shape[0] != self.n_sites or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous [n_sites={self.n_sites}, n_vec]")
        if t.device.index != self.device:
            raise ValueError(f"{name} is on device {t.device.index}, system on {self.device}")
        return C.c_void_p(t.data_ptr()), int(t.shape[1])

    def new_state(self, n_vec: int = 1):
        import torch
        return torch.zeros((self.n_sites, n_vec), dtype=self.cdtype, device=f"cuda:{self.device}")

    def upload(self, phi):
        """Host complex array [n_sites] or [n_sites, n_vec] -> device state tensor."""
        import torch
        a = np.asarray(phi)
        if a.ndim == 1:
            a = a[:, None]
        npdt = np.complex128 if self.precision == "fp64" else np.complex64
        return torch.from_numpy(np.ascontiguousarray(a, dtype=npdt)).to(f"cuda:{self.device}")


def kpm_moments(sys: System, phi_l, phi_r, n_moments: int) -> np.ndarray:
    """C_m = <phi_L|T_m(H~)|phi_R>, complex128 [n_vec, n_moments] (Eq. 46);
    [n_samples, n_vec, n_moments] for a batch."""
    pl, nv = sys._state(phi_l, "phi_l")
    pr, nv2 = sys._state(phi_r, "phi_r")
    if nv != nv2:
        raise ValueError("phi_l and phi_r differ in n_vec")
    out = np.empty((sys.n_samples, nv, n_moments, 2))
    sys._sync_stream()
    _check(lib().kpm_moments(sys.handle, nv, pl, pr, n_moments, _dp(out)))
    return sys._shape(out[..., 0] + 1j * out[..., 1])


def kpm_moments_noalloc(sys: System, phi_l, phi_r, n_moments: int) -> np.ndarray:
    """kpm_moments through the entry point that allocates no device memory
    (its scratch is the library's fixed per-GPU array)."""
    pl, nv = sys._state(phi_l, "phi_l")
    pr, nv2 = sys._state(phi_r, "phi_r")
    if nv != nv2:
        raise ValueError("phi_l and phi_r differ in n_vec")
    out = np.empty((sys.n_samples, nv, n_moments, 2))
    sys._sync_stream()
    _check(lib().kpm_moments_noalloc(sys.handle, nv, pl, pr, n_moments, _dp(out)))
    return sys._shape(out[..., 0] + 1j * out[..., 1])


def kpm_moments_doubled(sys: System, phi, n_moments: int) -> np.ndarray:
    """kpm_moments(sys, phi, phi, n_moments) from about half the recursion
    steps (product identities of T_n); same shape and values up to rounding."""
    p, nv = sys._state(phi, "phi")
    out = np.empty((sys.n_samples, nv, n_moments, 2))
    sys._sync_stream()
    _check(lib().kpm_moments_doubled(sys.handle, nv, p, n_moments, _dp(out)))
    return sys._shape(out[..., 0] + 1j * out[..., 1])


def kpm_fourier_moments(sys: System, phi_l, phi_r, n_moments: int, dtau_fs: float,
                        n_bessel: int) -> np.ndarray:
    """F_n = <phi_L|U(n dtau)|phi_R>, n = -N_m .. N_m (Alg. 4): complex128
    [n_vec, 2 N_m + 1]; leading sample axis for a batch."""
    pl, nv = sys._state(phi_l, "phi_l")
    pr, nv2 = sys._state(phi_r, "phi_r")
    if nv != nv2:
        raise ValueError("phi_l and phi_r differ in n_vec")
    out = np.empty((sys.n_samples, nv, 2 * n_moments + 1, 2))
    sys._sync_stream()
    _check(lib().kpm_fourier_moments(sys.handle, nv, pl, pr, n_moments, dtau_fs, n_bessel,
                                     _dp(out)))
    return sys._shape(out[..., 0] + 1j * out[..., 1])


def kpm_evolve(sys: System, phi, dt_fs: float, sign: int, n_bessel: int):
    """phi <- U(sign dt) phi in place (Eq. 36)."""
    p, nv = sys._state(phi, "phi")
    sys._sync_stream()
    _check(lib().kpm_evolve(sys.handle, nv, p, dt_fs, sign, n_bessel))
    return phi


def kpm_evolve_x(sys: System, phi, out_x, out_u, dt_fs: float, n_bessel: int):
    """out_x <- [X, U(dt)] phi, out_u <- U(dt) phi (Eq. 37); out_u may be None."""
    p, nv = sys._state(phi, "phi")
    px, nx_ = sys._state(out_x, "out_x")
    pu = None
    if out_u is not None:
        pu, nu = sys._state(out_u, "out_u")
        if nu != nv:
            raise ValueError("n_vec mismatch")
    if nx_ != nv:
        raise ValueError("n_vec mismatch")
    sys._sync_stream()
    _check(lib().kpm_evolve_x(sys.handle, nv, p, px, pu, dt_fs, n_bessel))


def _loop(fn, sys, phi, n_steps, dt_fs, n_bessel, n_moments):
    p, nv = sys._state(phi, "phi")
    out = np.empty((sys.n_samples, nv, n_steps + 1, n_moments))
    sys._sync_stream()
    _check(fn(sys.handle, nv, p, n_steps, dt_fs, n_bessel, n_moments, _dp(out)))
    return sys._shape(out)


def kpm_vac_msd(sys: System, phi, n_steps: int, dt_fs: float, n_bessel: int, n_moments: int):
    """(VAC, MSD) moments of kpm_vac and kpm_msd from one call, each
    [n_vec, n_steps+1, n_moments]; leading sample axis for a batch."""
    p, nv = sys._state(phi, "phi")
    vac = np.empty((sys.n_samples, nv, n_steps + 1, n_moments))
    msd = np.empty_like(vac)
    sys._sync_stream()
    _check(lib().kpm_vac_msd(sys.handle, nv, p, n_steps, dt_fs, n_bessel, n_moments, _dp(vac),
                             _dp(msd)))
    return sys._shape(vac), sys._shape(msd)


def kpm_dos_vac_msd(sys: System, phi, n_steps: int, dt_fs: float, n_bessel: int,
                    n_moments: int):
    """(DOS, VAC, MSD) moments of one call: the DOS moments <phi|T_m|phi> (real)
    [n_vec, n_moments] and kpm_vac_msd's two arrays; leading sample axis for a
    batch."""
    p, nv = sys._state(phi, "phi")
    dos = np.empty((sys.n_samples, nv, n_moments))
    vac = np.empty((sys.n_samples, nv, n_steps + 1, n_moments))
    msd = np.empty_like(vac)
    sys._sync_stream()
    _check(lib().kpm_dos_vac_msd(sys.handle, nv, p, n_steps, dt_fs, n_bessel, n_moments,
                                 _dp(dos), _dp(vac), _dp(msd)))
    return sys._shape(dos), sys._shape(vac), sys._shape(msd)


def kpm_vac(sys: System, phi, n_steps: int, dt_fs: float, n_bessel: int, n_moments: int):
    """VAC moments [n_vec, n_steps+1, n_moments] in nm^2/fs^2 (Alg. 2); leading
    sample axis for a batch."""
    return _loop(lib().kpm_vac, sys, phi, n_steps, dt_fs, n_bessel, n_moments)


def kpm_msd(sys: System, phi, n_steps: int, dt_fs: float, n_bessel: int, n_moments: int):
    """MSD moments [n_vec, n_steps+1, n_moments] in nm^2 (Alg. 3); leading
    sample axis for a batch."""
    return _loop(lib().kpm_msd, sys, phi, n_steps, dt_fs, n_bessel, n_moments)


def kpm_msd_doubled(sys: System, phi, n_steps: int, dt_fs: float, n_bessel: int,
                    n_moments: int):
    """kpm_msd with the moments of each state in the doubling form."""
    return _loop(lib().kpm_msd_doubled, sys, phi, n_steps, dt_fs, n_bessel, n_moments)


def _continue(fn, sys, a, b, start, n_steps, dt_fs, n_bessel, n_moments, *extra):
    pa, nv = sys._state(a, "psi")
    pb, nv2 = sys._state(b, "second state")
    if nv != nv2:
        raise ValueError("state buffers differ in n_vec")
    out = np.empty((sys.n_samples, nv, n_steps + int(bool(start)), n_moments))
    sys._sync_stream()
    _check(fn(sys.handle, nv, pa, pb, int(bool(start)), n_steps, dt_fs, n_bessel, n_moments,
              *extra, _dp(out)))
    return sys._shape(out)


def kpm_vac_continue(sys: System, psi, r, start: bool, n_steps: int, dt_fs: float,
                     n_bessel: int, n_moments: int):
    """VAC loop from the state (psi, r), both updated in place (see kpm.h)."""
    return _continue(lib().kpm_vac_continue, sys, psi, r, start, n_steps, dt_fs, n_bessel,
                     n_moments)


def kpm_msd_continue(sys: System, psi, y, start: bool, n_steps: int, dt_fs: float,
                     n_bessel: int, n_moments: int, doubled: bool = False):
    """MSD loop from the state (psi, y), both updated in place (see kpm.h)."""
    return _continue(lib().kpm_msd_continue, sys, psi, y, start, n_steps, dt_fs, n_bessel,
                     n_moments, int(bool(doubled)))


def kpm_set_launch(sys: System, n_vec: int, groups_per_cu: int, ilp: int, streaming: int = 0,
                   compact: int = 1, tiled: int = 0, steps: int = 1, vectors_per_wave: int = 0,
                   plane_groups: int = 0, group_size: int = 0):
    """Launch shape of the moment step for n_vec vectors (see kpm_launch in kpm.h)."""
    _check(lib().kpm_set_launch(sys.handle, n_vec,
                                C.byref(Launch(groups_per_cu, ilp, int(bool(streaming)),
                                               int(bool(compact)), int(tiled), int(steps),
                                               int(vectors_per_wave), int(plane_groups),
                                               int(group_size)))))


def kpm_default_launch(n_vec: int, precision: str = "fp64") -> dict:
    """Launch shape a new system starts with (environment overrides applied);
    host only."""
    out = Launch()
    _check(lib().kpm_default_launch(n_vec, PRECISIONS[precision], C.byref(out)))
    return out.as_dict()


def kpm_get_launch(sys: System, n_vec: int) -> dict:
    out = Launch()
    _check(lib().kpm_get_launch(sys.handle, n_vec, C.byref(out)))
    return out.as_dict()


def kpm_set_launch_doubled(sys: System, n_vec: int, groups_per_cu: int, ilp: int,
                           streaming: int = 0, compact: int = 1, tiled: int = 0, steps: int = 1,
                           vectors_per_wave: int = 0, plane_groups: int = 0, group_size: int = 0):
    """Launch shape of doubling-form moment sets (kpm_set_launch sets both forms)."""
    _check(lib().kpm_set_launch_doubled(sys.handle, n_vec,
                                        C.byref(Launch(groups_per_cu, ilp, int(bool(streaming)),
                                                       int(bool(compact)), int(tiled),
                                                       int(steps), int(vectors_per_wave),
                                                       int(plane_groups), int(group_size)))))


def kpm_get_launch_doubled(sys: System, n_vec: int) -> dict:
    out = Launch()
    _check(lib().kpm_get_launch_doubled(sys.handle, n_vec, C.byref(out)))
    return out.as_dict()


def kpm_autotune(sys: System, phi, reps: int = 10) -> dict:
    """Time every candidate launch shape on `phi` and keep the fastest for its n_vec."""
    p, nv = sys._state(phi, "phi")
    out = Launch()
    sys._sync_stream()
    _check(lib().kpm_autotune(sys.handle, nv, p, reps, C.byref(out)))
    return out.as_dict()


def kpm_autotune_candidates(sys: System, n_vec: int) -> list:
    """The launch shapes kpm_autotune times for n_vec vectors on this system."""
    cnt = C.c_int32()
    _check(lib().kpm_autotune_candidates(sys.handle, n_vec, None, 0, C.byref(cnt)))
    arr = (Launch * max(cnt.value, 1))()
    _check(lib().kpm_autotune_candidates(sys.handle, n_vec, arr, cnt.value, C.byref(cnt)))
    return [arr[q].as_dict() for q in range(cnt.value)]


def kpm_set_graphs(sys: System, enable: bool = True):
    """Capture each moment set as a hipGraph once and replay it."""
    _check(lib().kpm_set_graphs(sys.handle, int(bool(enable))))


def kpm_set_timing(sys: System, enable: bool = True):
    _check(lib().kpm_set_timing(sys.handle, int(bool(enable))))


def kpm_get_stats(sys: System) -> dict:
    s = Stats()
    _check(lib().kpm_get_stats(sys.handle, C.byref(s)))
    return dict(step_ms=s.step_ms, step_launches=s.step_launches, step_rows=s.step_rows,
                site_updates=s.site_updates, step_bytes=s.step_bytes,
                step_bytes_total=s.step_bytes_total, wide_ms=s.wide_ms,
                wide_launches=s.wide_launches, wide_rows=s.wide_rows)


def kpm_reset_stats(sys: System):
    _check(lib().kpm_reset_stats(sys.handle))


def graphene_system(nx: int, ny: int, geometry: str = "sheet", t_ev: float = -2.7,
                    onsite=None, active=None, e_scale: float | None = None,
                    precision: str = "fp64", device: int | None = None) -> System:
    """System for an nx x ny graphene sample (Sec. 2), built with kpm_build_graphene."""
    nbr, dx = kpm_build_graphene(nx, ny, geometry, active)
    if e_scale is None:
        wmax = 0.0 if onsite is None else float(np.max(np.abs(onsite)))
        e_scale = 1.01 * (3 * abs(t_ev) + wmax)
    s = System(nbr, e_scale, t_uniform=t_ev, onsite=onsite, dx=dx, active=active,
               precision=precision, device=device)
    s.nx, s.ny, s.geometry = nx, ny, geometry
    lx = np.sqrt(3.0) * nx * BOND_NM / 2.0
    ly = 3.0 * ny * BOND_NM / 2.0
    s.area_nm2 = lx * ly
    s.width_nm = lx if geometry == "agnr" else ly
    return s


def graphene_batch(samples, precision: str = "fp64", device: int | None = None) -> System:
    """Ragged batch of graphene samples (Sec. 2).  samples: list of dicts with
    nx, ny, geometry, and optionally t_ev, onsite, active, e_scale."""
    descs = []
    meta = []
    for smp in samples:
        nx, ny, geo = smp["nx"], smp["ny"], smp.get("geometry", "sheet")
        t_ev = smp.get("t_ev", -2.7)
        onsite, active = smp.get("onsite"), smp.get("active")
        nbr, dx = kpm_build_graphene(nx, ny, geo, active)
        es = smp.get("e_scale")
        if es is None:
            wmax = 0.0 if onsite is None else float(np.max(np.abs(onsite)))
            es = 1.01 * (3 * abs(t_ev) + wmax)
        descs.append(dict(nbr=nbr, e_scale=es, t_uniform=t_ev, onsite=onsite, dx=dx,
                          active=active))
        lx = np.sqrt(3.0) * nx * BOND_NM / 2.0
        ly = 3.0 * ny * BOND_NM / 2.0
        meta.append(dict(nx=nx, ny=ny, geometry=geo, e_scale=es, area_nm2=lx * ly,
                         width_nm=lx if geo == "agnr" else ly))
    s = System.batch(descs, precision, device)
    s.samples = meta
    return s


# ------------------------------------------------------------------ learned reconstruction
def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _f32_gpu(t, name, width):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 \
            or t.dim() != 2 or t.shape[1] != width or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 GPU tensor [batch, {width}]")
    return C.c_void_p(t.data_ptr())


class MLP:
    """Network of the learned reconstruction (kpm_mlp_create): widths d_0 .. d_L,
    tanh hidden layers, linear output, FP32, on the current torch stream."""

    def __init__(self, widths, max_batch: int, device: int | None = None):
        import torch
        self.widths = [int(w) for w in widths]
        self.device = torch.cuda.current_device() if device is None else device
        arr = (C.c_int32 * len(self.widths))(*self.widths)
        h = C.c_void_p()
        _check(lib().kpm_mlp_create(len(self.widths) - 1, arr, max_batch, self.device,
                                    _stream(), C.byref(h)))
        self._h = h
        self.max_batch = max_batch

    @property
    def n_params(self) -> int:
        return int(lib().kpm_mlp_n_params(self._h))

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != self.n_params:
            raise ValueError("parameter count mismatch")
        _check(lib().kpm_mlp_set_params(self._h, _fp(a)))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.n_params, dtype=np.float32)
        _check(lib().kpm_mlp_get_params(self._h, _fp(a)))
        return a

    def forward(self, x):
        import torch
        b = x.shape[0]
        y = torch.empty((b, self.widths[-1]), dtype=torch.float32, device=x.device)
        _check(lib().kpm_mlp_forward(self._h, b, _f32_gpu(x, "x", self.widths[0]),
                                     _f32_gpu(y, "y", self.widths[-1])))
        return y

    def gradients(self, x, y):
        loss = C.c_double()
        g = np.empty(self.n_params, dtype=np.float32)
        _check(lib().kpm_mlp_gradients(self._h, x.shape[0], _f32_gpu(x, "x", self.widths[0]),
                                       _f32_gpu(y, "y", self.widths[-1]), C.byref(loss), _fp(g)))
        return loss.value, g

    def train_step(self, x, y, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                   eps: float = 1e-8, want_loss: bool = True):
        """One Adam step; returns the loss before it (a host sync), or None
        without synchronising when want_loss is False."""
        loss = C.c_double()
        opt = Adam(lr, beta1, beta2, eps)
        _check(lib().kpm_mlp_train_step(self._h, x.shape[0], _f32_gpu(x, "x", self.widths[0]),
                                        _f32_gpu(y, "y", self.widths[-1]), C.byref(opt),
                                        C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().kpm_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _moments_real(mu):
    """Real parts of moments [S, R, N] (or [R, N] for one sample) as float64."""
    a = np.real(np.asarray(mu))
    if a.ndim == 2:
        a = a[None]
    return np.ascontiguousarray(a, dtype=np.float64)


def kpm_learned_features(mu_dos, mu_msd, n_in: int) -> np.ndarray:
    """Features [S, 2 n_in + 1] (float32) of the learned reconstruction."""
    d, c = _moments_real(mu_dos), _moments_real(mu_msd)
    if d.shape != c.shape:
        raise ValueError("DOS and MSD moments differ in shape")
    x = np.empty((d.shape[0], 2 * n_in + 1), dtype=np.float32)
    _check(lib().kpm_learned_features(d.shape[0], d.shape[1], d.shape[2], _dp(d), _dp(c), n_in,
                                      _fp(x)))
    return x


def kpm_learned_targets(mu_dos, mu_msd, energies_ev, e_scale: float, area_nm2: float,
                        t_star_fs: float) -> np.ndarray:
    """Targets [S, 2 K] (float32): scaled DOS and sigma_E2(t*) from all the moments."""
    d, c = _moments_real(mu_dos), _moments_real(mu_msd)
    if d.shape != c.shape:
        raise ValueError("DOS and MSD moments differ in shape")
    en = np.ascontiguousarray(energies_ev, dtype=np.float64).reshape(-1)
    y = np.empty((d.shape[0], 2 * en.size), dtype=np.float32)
    _check(lib().kpm_learned_targets(d.shape[0], d.shape[1], d.shape[2], _dp(d), _dp(c), en.size,
                                     _dp(en), e_scale, area_nm2, t_star_fs, _stream(), _fp(y)))
    return y


def kpm_xu_state(sys: System, phi, n_steps: int, dt_fs: float, n_bessel: int):
    """[X, U(n_steps dt)] phi (Eq. 44) as a new device state."""
    p, nv = sys._state(phi, "phi")
    out = sys.new_state(nv)
    sys._sync_stream()
    _check(lib().kpm_xu_state(sys.handle, nv, p, n_steps, dt_fs, n_bessel,
                              C.c_void_p(out.data_ptr())))
    return out
