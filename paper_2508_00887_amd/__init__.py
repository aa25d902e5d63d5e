"""MI355X-native FRAM: Python binding of libfram.so (see include/fram.h).

The binding only marshals arguments; every step of the method runs in the
HIP kernels of libfram.so.  Importing succeeds without the library, but any
call raises if libfram.so has not been built (no CPU fallback exists).
"""
from .fram import (  # noqa: F401
    Context, FramError, Stats, Options, load_library, library_path,
    FRAM_OK, FRAM_EINVAL, FRAM_ENOMEM, FRAM_EDEVICE, FRAM_ENUMERIC, FRAM_EBUSY,
    FRAM_FP32, FRAM_BF16, FRAM_FP16, PRECISIONS,
)
