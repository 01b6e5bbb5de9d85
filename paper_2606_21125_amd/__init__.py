"""MI355X-native divide-and-conquer DFT fragment SCF (HIP library + thin binding).

The compute lives in ``libdcdft.so`` (HIP, gfx950), declared in
``include/dcdft.h``.  This package only marshals arguments to it; importing a
symbol that needs the library raises if the library has not been built.
"""
from .binding import (DCDFT, DcdftError, DcdftParams, DcdftScfInfo, DcdftSpecies,  # noqa: F401
                      EXPORTED, LIB_PATH, PREC_FP64, PREC_MIXED, FIELD_VLOC, FIELD_VH,
                      FIELD_RHO_IN, FIELD_RHO_OUT, FFIELD_VEFF, FFIELD_RHO_IN, FFIELD_RHO_OUT,
                      KERNEL_HLOC, KERNEL_GRAM, KERNEL_ROTATE, KERNEL_GRAM_FUSED, KERNEL_KB,
                      HLOC_VARIANTS, DcdftTuneInfo, MIX_LINEAR, MIX_PULAY,
                      load_library, dcdft_setup, dcdft_scf_step, dcdft_destroy,
                      dcdft_last_error)
