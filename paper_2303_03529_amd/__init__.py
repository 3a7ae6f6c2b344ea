"""MI355X-native spin-charge Krylov kernel (hot path of spin-polarized XL-BOMD).

The compute lives in the HIP library libkrylov_kernel.so (C ABI in
include/krylov_kernel.h); `krylov` is its Python binding and `setup` builds
the expansion point a caller hands to the library.
"""

__all__ = ["krylov", "setup"]
