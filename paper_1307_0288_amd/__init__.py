"""MI355X library for the Chebyshev hot path of linear-scaling Kubo-Greenwood
transport (Fan, Uppstu, Siro, Harju): KPM moments, Chebyshev-Bessel time
evolution, commutator propagation, and the VAC / MSD time loops, computed by
hand-written gfx950 kernels behind the C ABI of include/kpm.h.

This package is the Python binding of that ABI.  The shared library
(libkpm.so, built in-tree by `python -m paper_1307_0288_amd.build`) is loaded
on first use; every entry point raises ImportError when it is missing.  There
is no CPU fallback.
"""
from .kpm import (ABI_SYMBOLS, HBAR_EV_FS, BOND_NM, KpmError, System, graphene_batch,
                  graphene_system,
                  kpm_autotune, kpm_autotune_candidates, kpm_build_graphene, kpm_validate, kpm_evolve, kpm_evolve_x, kpm_fourier_moments,
                  kpm_ftm_sum, kpm_default_launch, kpm_get_launch, kpm_get_launch_doubled, kpm_set_launch_doubled,
                  kpm_get_stats, kpm_kpm_sum, kpm_set_graphs, kpm_set_launch,
                  kpm_moments, kpm_moments_doubled, kpm_moments_noalloc, kpm_msd, kpm_reset_stats, kpm_set_timing, kpm_sigma_e1,
                  kpm_sigma_e2, kpm_sigma_gk, kpm_vac, kpm_vac_msd, kpm_dos_vac_msd, kpm_length,
                  kpm_conductance,
                  kpm_ballistic_conductance, kpm_sigma_sc_max, kpm_sigma_sc_average,
                  kpm_pade_fit, kpm_pade_eval, kpm_typical_conductance, kpm_msd_doubled,
                  MLP, kpm_learned_features, kpm_learned_targets, kpm_xu_state,
                  kpm_vac_continue, kpm_msd_continue, lib)

__all__ = ["ABI_SYMBOLS", "HBAR_EV_FS", "BOND_NM", "KpmError", "System", "graphene_batch",
           "graphene_system",
           "kpm_autotune", "kpm_autotune_candidates", "kpm_build_graphene", "kpm_validate", "kpm_evolve", "kpm_fourier_moments", "kpm_ftm_sum",
           "kpm_default_launch", "kpm_get_launch", "kpm_get_launch_doubled", "kpm_set_launch_doubled", "kpm_set_launch",
           "kpm_set_graphs", "kpm_evolve_x", "kpm_get_stats",
           "kpm_kpm_sum", "kpm_moments", "kpm_moments_doubled", "kpm_moments_noalloc", "kpm_msd", "kpm_reset_stats", "kpm_set_timing",
           "kpm_sigma_e1", "kpm_sigma_e2", "kpm_sigma_gk", "kpm_vac", "kpm_vac_msd",
           "kpm_dos_vac_msd", "kpm_length",
           "kpm_conductance", "kpm_ballistic_conductance", "kpm_sigma_sc_max",
           "kpm_sigma_sc_average", "kpm_pade_fit", "kpm_pade_eval", "kpm_typical_conductance",
           "kpm_msd_doubled", "MLP", "kpm_learned_features", "kpm_learned_targets",
           "kpm_xu_state", "kpm_vac_continue", "kpm_msd_continue", "lib"]
