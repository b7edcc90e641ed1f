"""MI355X-native Chebyshev-filtered plane-wave eigensolver hot path.

The compute path is the HIP library ``libchebfi.so`` (C ABI in
``include/chebfi.h``); :mod:`.binding` marshals torch tensors into it.
Importing this package does not load the library; :func:`binding.lib` does,
and raises when the library has not been built.
"""

__all__ = ["binding", "build"]
