"""Adaptive data-parallel regions on MI355X (gfx950).

A region declares several variants (launch geometries, tilings, execution
targets); each execution is profiled and a learned cost model picks the
variant.  All computation happens in ``libadaptomp.so`` (hand-written HIP
kernels and a C++ runtime); this package only marshals arguments to its C
ABI (``include/adaptomp.h``).  Importing it fails loudly when the library
has not been built: there is no fallback path.
"""
from __future__ import annotations

from ._lib import (  # noqa: F401
    AO_CSR_RELAX_F64, AO_CSR_SPMV_F64, AO_JACOBI7_F64, AO_MAX_FEATURES, AO_MAX_VARIANTS, AO_MLP_PARAMS,
    AO_OK, AO_NOTE_FALLBACK, AO_NOTE_UNTRAINED, AO_PROFILE_RECORD, AO_TARGET_GPU,
    AO_TARGET_HOST, AO_VF_HALO_PREFETCH, AO_VF_NT_STORE, AO_VF_OCCUPANCY, AO_VF_STAGED,
    AO_VF_LDS_SWEEPS, AO_VF_FILL_Z, FAM_JACOBI_DIRECT,
    FAM_JACOBI_HOST, FAM_JACOBI_ZMARCH, FAM_JACOBI_ZREG, FAM_JACOBI_ZREG_T2, FAM_JACOBI_ZREG_T3,
    FAM_JACOBI_ZREG_T4, FAM_JACOBI_COSCHED,
    FAM_SPMV_XSLICE, FAM_SPMV_MERGE_PATH, FAM_SPMV_THREAD_ROW, FAM_SPMV_WAVE_ROW, AdaptError, Args, Stats,
    TrainOpts, Variant, lib, lib_path, ao_last_error, ao_device_cus, ao_jacobi_planes,
    ao_gather_probe, ao_hbm_copy, gather_probe_out_len, ao_mlp_adam, ao_mlp_forward,
    ao_mlp_grad, batch_autotune, batch_candidates, batch_create, batch_destroy, batch_info,
    batch_min_traffic, batch_run, batch_set_tiles,
    region_clear_memo, region_declare_variants, region_destroy, region_features, region_load, region_profile,
    region_record, region_records, region_run, region_run_noalloc, region_save, region_stats, selector_select, selector_train,
    jacobi_args, relax_args, spmv_args)
from .variants import (  # noqa: F401
    jacobi_sweep_gpu, jacobi_sweep_host, jacobi_variants_blocks, jacobi_variants_sweep, spmv_variants)
