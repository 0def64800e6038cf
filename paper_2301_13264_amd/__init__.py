"""MI355X-native CCSD non-adiabatic derivative couplings (HIP for gfx950).

The computation lives in libnacme.so (C ABI, include/nacme.h); this package
only builds and binds it.
"""
from ._lib import (CC_BOTH, CC_LEFT, CC_RIGHT, CCError, Context, contract,  # noqa: F401
                   default_opts, eig_host, lib)
