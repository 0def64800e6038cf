"""MI355X-native CCSD non-adiabatic derivative couplings (HIP for gfx950).

The computation lives in libnacme.so (C ABI, include/nacme.h); this package
only builds and binds it.
"""
from ._lib import (CC_BF16X3_REFINE, CC_BOTH, CC_FP32_REFINE, CC_FP64, CC_LEFT,  # noqa: F401
                   CC_NOT_CONVERGED, CC_OK, CC_RIGHT,
                   CCError, MLP, Context, contract, default_opts, eig_host, gemm, lib, pair_interleave)
