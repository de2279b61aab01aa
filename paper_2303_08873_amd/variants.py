"""Variant tables of the region workloads (declaration order = variant id,
as categorical variants are numbered from 0 in the order given, Sec. 3.1
model_output clause)."""
from __future__ import annotations

from ._lib import (AO_TARGET_GPU, AO_TARGET_HOST, AO_VF_FILL_Z, AO_VF_LDS_SWEEPS, AO_VF_NT_STORE,
                   AO_VF_STAGED,
                   FAM_JACOBI_DIRECT, FAM_JACOBI_HOST, FAM_JACOBI_ZREG_T3,
                   FAM_JACOBI_ZREG_T4, FAM_SPMV_XSLICE,
                   FAM_SPMV_MERGE_PATH, FAM_SPMV_THREAD_ROW, FAM_SPMV_WAVE_ROW, Variant)


def jacobi_variants_blocks():
    """Threads-per-block variants 64 / 256 / 1024 of the one-point-per-thread
    Jacobi kernel (the GPU-threads use case, Sec. 3.2 / Sec. 5)."""
    return [Variant(AO_TARGET_GPU, FAM_JACOBI_DIRECT, 64, 1, 1, 0),
            Variant(AO_TARGET_GPU, FAM_JACOBI_DIRECT, 64, 4, 1, 0),
            Variant(AO_TARGET_GPU, FAM_JACOBI_DIRECT, 64, 16, 1, 0)]


# ids 0..5 run on the GPU, 6..10 on the host CPU (device-selection use case)
JACOBI_SWEEP_GPU = [(FAM_JACOBI_ZREG_T3, 64, 1, 1, AO_VF_STAGED), (FAM_JACOBI_DIRECT, 64, 4, 1, 0),
                    (FAM_JACOBI_ZREG_T3, 64, 4, 22, AO_VF_STAGED | AO_VF_FILL_Z),
                    (FAM_JACOBI_ZREG_T4, 64, 4, 74, AO_VF_NT_STORE | AO_VF_STAGED | AO_VF_FILL_Z),
                    (FAM_JACOBI_ZREG_T3, 64, 2, 22, AO_VF_STAGED | AO_VF_FILL_Z),
                    (FAM_JACOBI_DIRECT, 64, 16, 1, AO_VF_LDS_SWEEPS)]
JACOBI_SWEEP_HOST = [(0, 1), (256, 4), (64, 16), (0, 8), (128, 32)]
STATIC_DEFAULT = 1  # 64x4 = 256 threads, the OpenMP offload default team size


def jacobi_variants_sweep():
    """11 variants: 6 GPU kernels (the three-sweep register z-march with
    level 0 staged, 1 row per wave and 1 plane per block for small grids;
    one point per thread with 64x4 threads, the static default; the staged
    three-sweep march with 4 rows per wave and up to 22 planes per block,
    the staged four-sweep march with 4 rows and up to 74 planes, and the
    staged three-sweep march with 2 rows and up to 22 planes, each launch
    taking the chunk that fills the device; one point per thread with 64x16
    threads and small grids' sweeps all in one workgroup's LDS) and 5
    host-CPU cache-block shapes."""
    out = [Variant(AO_TARGET_GPU, f, bx, by, bz, fl) for f, bx, by, bz, fl in JACOBI_SWEEP_GPU]
    out += [Variant(AO_TARGET_HOST, FAM_JACOBI_HOST, bx, by, 1, 0) for bx, by in JACOBI_SWEEP_HOST]
    return out


def jacobi_sweep_gpu():
    """The GPU variants of the size-sweep table (its first ids)."""
    return jacobi_variants_sweep()[:len(JACOBI_SWEEP_GPU)]


def jacobi_sweep_host():
    """The host-CPU variants of the size-sweep table (its last ids)."""
    return jacobi_variants_sweep()[len(JACOBI_SWEEP_GPU):]


def spmv_variants(blocks=(64, 256, 1024), wave_lanes: int = 64, xslice=()):
    """{thread-per-row, wavefront-per-row, merge-path} x block sizes, then the
    x-slice family for each log2 slice width (13 or 14) in `xslice`."""
    out = []
    for fam in (FAM_SPMV_THREAD_ROW, FAM_SPMV_WAVE_ROW, FAM_SPMV_MERGE_PATH):
        for b in blocks:
            out.append(Variant(AO_TARGET_GPU, fam, b, wave_lanes if fam == FAM_SPMV_WAVE_ROW else 0,
                               1, 0))
    for swl in xslice:
        out.append(Variant(AO_TARGET_GPU, FAM_SPMV_XSLICE, 0, swl, 1, 0))
    return out
