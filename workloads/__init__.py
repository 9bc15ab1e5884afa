"""Seeded synthetic inputs shared by the product path and the oracle.

This package holds input generation only: initial states in tensor-train form (cores
built from separable closed forms, or a TT-SVD of a sampled piecewise-constant field)
and grid descriptions. It holds none of the WENO-TT method's arithmetic (no fluxes, no
reconstruction, no cross, no rounding) and imports neither the product nor the oracle.
"""
from .flows import (Flow, config1_smooth_wave_2d, config2_quadrants_2d, config3_wave_3d, config4_blast_3d,
                    config5_tilted_sod_3d, random_positive_tt, sod_1d_like, sod_exact_rho, tt_svd_input,
                    scalar_linadv_3d, scalar_burgers_3d, burgers_exact)

__all__ = ["Flow", "config1_smooth_wave_2d", "config2_quadrants_2d", "config3_wave_3d", "config4_blast_3d",
           "config5_tilted_sod_3d", "random_positive_tt", "sod_1d_like", "sod_exact_rho", "tt_svd_input",
           "scalar_linadv_3d", "scalar_burgers_3d", "burgers_exact"]
