"""MI355X hot path of mixed real/momentum-space cylinder DMRG (arXiv:1512.03318).

Thin ctypes binding of ``libmrdmrg.so``; the functions keep the C ABI's names
(``heff_apply``, ``lanczos_ground``, ``env_update_left``, ``env_update_right``,
``lanczos_ground_batched``) and only marshal arguments: charges and bonds into C
structs, torch device tensors into pointers, numpy block dictionaries into the
library's canonical layouts (offsets come from ``dm_layout``).  Every arithmetic step
runs in the library.  Importing this package fails if the library is missing.
"""
from .binding import (Split, MPS, dmrg_sweeps, idmrg, entanglement, DM_BF16X3, DM_FP32, DM_FP64, DM_REAL, Bond, HeffPlan, Batch, HofstadterMPO,
                      LibraryError, MpoSite, env_flops, env_update_left, env_update_left_noalloc,
                      env_update_right, heff_apply,
                      lanczos_ground, lanczos_ground_batched, layout, lib, pack, unpack,
                      LAYOUT_SITE, LAYOUT_THETA, LAYOUT_ENV_L, LAYOUT_ENV_R, DM_OK, DM_ERR_ARG,
                      DM_ERR_CHARGE, DM_ERR_DIM, DM_ERR_LAYOUT, DM_ERR_DTYPE, DM_ERR_ALLOC,
                      DM_ERR_HIP, DM_ERR_NONFINITE)

__all__ = ["Split", "MPS", "dmrg_sweeps", "idmrg", "entanglement", "DM_BF16X3", "DM_FP32", "DM_FP64", "DM_REAL", "Bond", "HeffPlan", "Batch", "HofstadterMPO",
           "LibraryError", "MpoSite", "env_flops", "env_update_left", "env_update_left_noalloc",
           "env_update_right", "heff_apply",
           "lanczos_ground", "lanczos_ground_batched", "layout", "lib", "pack", "unpack",
           "LAYOUT_SITE", "LAYOUT_THETA", "LAYOUT_ENV_L", "LAYOUT_ENV_R", "DM_OK", "DM_ERR_ARG",
           "DM_ERR_CHARGE", "DM_ERR_DIM", "DM_ERR_LAYOUT", "DM_ERR_DTYPE", "DM_ERR_ALLOC",
           "DM_ERR_HIP", "DM_ERR_NONFINITE"]
