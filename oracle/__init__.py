"""CPU oracle for the Kubo-Greenwood hot path -- TEST INFRASTRUCTURE ONLY.

Plain complex128 code written from the paper (Fan et al., linear-scaling
Kubo-Greenwood transport on GPUs): a C core (kpm_oracle.c) for the lattice,
the Chebyshev/Bessel recursions and the VAC/MSD loops, and numpy for the
host-side reconstruction (Jackson damping, KPM sums, running conductivities).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never does, and this package never
imports the GPU library.
"""
from .core import (HBAR_EV_FS, BOND_NM, Lattice, graphene, moments, bessel_j,
                   evolve, evolve_x, vac, msd, dense_h, dense_d, fourier_moments, set_threads)
from .recon import (jackson, kpm_sum, dos, sigma_gk, sigma_e1, sigma_e2,
                    energies_grid, hanning, ftm_sum)

__all__ = ["HBAR_EV_FS", "BOND_NM", "Lattice", "graphene", "moments", "bessel_j",
           "evolve", "evolve_x", "vac", "msd", "dense_h", "dense_d", "fourier_moments", "set_threads",
           "jackson", "kpm_sum", "dos", "sigma_gk", "sigma_e1", "sigma_e2", "energies_grid",
           "hanning", "ftm_sum"]
