"""MI355X-native density-fitted Coulomb/exchange (J/K) build.

The compute path is libdfjk.so (HIP kernels for gfx950 behind the C-ABI in
include/dfjk.h); this package only loads it and marshals arguments.
"""
from .dfjk import (  # noqa: F401
    DFJK_BF16, DFJK_F16, DFJK_F32, DFJK_F64, DFJKError, Handle, dfjk_build_J, dfjk_build_J_diag, dfjk_build_J_multi, dfjk_build_K, dfjk_form_B,
    dfjk_build_K_factored, dfjk_build_K_pair, dfjk_destroy, dfjk_init, dfjk_profile, dfjk_profile_read, dfjk_set_tile, dfjk_tile_count,
    dfjk_tile_info, DFJK_TILE_GEMM1, DFJK_TILE_J_OUT, DFJK_TILE_K16, DFJK_TILE_K16_SYRK, dfjk_scf_step, dfjk_scf_reset, dfjk_aufbau, dfjk_probe_mfma, dfjk_probe_hbm_read, DFJK_SCF_C_VALID, ScfInfo, Batch, MLP, dfjk_guess_features,
    dfjk_guess_assemble, dfjk_last_error, dfjk_quantize,
    dfjk_workspace_bytes, lib, lib_path,
)
